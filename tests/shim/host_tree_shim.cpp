// Test shim: exposes the library's host-side ghost-face builder (no GPU calls) to CPU tests.
// The tree arrays come from the caller (leaf anchors and levels in Morton order, anchor keys,
// 8 slot nodes and the 8 x 8 constraint matrix C[vertex][slot] of every leaf).
#include <cstring>
#include <string>
#include <vector>

#include "../../paper_2606_09275_amd/csrc/geom.h"

namespace mpm {
void set_error(int32_t, const std::string&, int64_t) {}
int32_t hip_fail(hipError_t, const char*) { return MPM_EHIP; }
}  // namespace mpm

static mpm::GhostHost g_ghost;

extern "C" int64_t shim_ghost(int64_t nl, const int32_t* leaf, const uint64_t* leaf_key, const int32_t* cell_nodes,
                              const double* cell_cmat, const double* lo, double hmin, int32_t lmax, const int32_t* lat,
                              const uint8_t* pop) {
  mpm::HostTree T;
  T.leaf.assign(leaf, leaf + 4 * nl);
  T.leaf_key.assign(leaf_key, leaf_key + nl);
  T.cell_nodes.assign(cell_nodes, cell_nodes + 8 * nl);
  T.cell_cmat.assign(cell_cmat, cell_cmat + 64 * nl);
  mpm::LeafGeo G;
  G.leaf = T.leaf.data();
  G.leaf_key = T.leaf_key.data();
  G.cellmap = nullptr;
  G.n_leaf = nl;
  for (int a = 0; a < 3; ++a) {
    G.lo[a] = lo[a];
    G.lat[a] = lat[a];
  }
  G.hmin = hmin;
  G.lmax = lmax;
  std::vector<uint8_t> p(pop, pop + nl);
  g_ghost = mpm::GhostHost();
  return mpm::ghost_faces_host(T, G, p, &g_ghost);
}

extern "C" void shim_ghost_arrays(int32_t* face, int32_t* leaf2, int32_t* nodes, double* h, double* G) {
  std::memcpy(face, g_ghost.face.data(), g_ghost.face.size() * 4);
  std::memcpy(leaf2, g_ghost.leaf2.data(), g_ghost.leaf2.size() * 4);
  std::memcpy(nodes, g_ghost.nodes.data(), g_ghost.nodes.size() * 4);
  std::memcpy(h, g_ghost.h.data(), g_ghost.h.size() * 8);
  std::memcpy(G, g_ghost.G.data(), g_ghost.G.size() * 8);
}
