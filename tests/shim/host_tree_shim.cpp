// Test shim: exposes the library's host octree construction (no GPU calls) to CPU tests.
#include <cstring>
#include <string>

#include "../../paper_2606_09275_amd/csrc/geom.h"

namespace mpm {
int32_t build_tree(const mpm_refine_t& c, HostTree& T, int lat_out[3], double* hmin_out);
void set_error(int32_t, const std::string&, int64_t) {}
int32_t hip_fail(hipError_t, const char*) { return MPM_EHIP; }
}  // namespace mpm

static mpm::HostTree g_tree;

extern "C" int32_t shim_build(const mpm_refine_t* c, int64_t* counts) {
  g_tree = mpm::HostTree();
  int lat[3];
  double hmin;
  int32_t rc = mpm::build_tree(*c, g_tree, lat, &hmin);
  if (rc) return rc;
  counts[0] = int64_t(g_tree.leaf_key.size());
  counts[1] = int64_t(g_tree.node_ijk.size() / 3);
  counts[2] = int64_t(g_tree.hang_owner.size());
  return 0;
}

extern "C" void shim_arrays(int32_t* leaf, int32_t* node_ijk, int32_t* hang_ijk, int32_t* hang_sup, double* hang_w,
                            int32_t* hang_owner, int32_t* cell_nodes, int32_t* cell_code, double* cell_cmat) {
  std::memcpy(leaf, g_tree.leaf.data(), g_tree.leaf.size() * 4);
  std::memcpy(node_ijk, g_tree.node_ijk.data(), g_tree.node_ijk.size() * 4);
  std::memcpy(hang_ijk, g_tree.hang_ijk.data(), g_tree.hang_ijk.size() * 4);
  std::memcpy(hang_sup, g_tree.hang_sup.data(), g_tree.hang_sup.size() * 4);
  std::memcpy(hang_w, g_tree.hang_w.data(), g_tree.hang_w.size() * 8);
  std::memcpy(hang_owner, g_tree.hang_owner.data(), g_tree.hang_owner.size() * 4);
  std::memcpy(cell_nodes, g_tree.cell_nodes.data(), g_tree.cell_nodes.size() * 4);
  std::memcpy(cell_code, g_tree.cell_code.data(), g_tree.cell_code.size() * 4);
  std::memcpy(cell_cmat, g_tree.cell_cmat.data(), g_tree.cell_cmat.size() * 8);
}

// ghost faces of the last tree for the populated flags pop [n_leaf]; returns the face count
static mpm::GhostHost g_ghost;
extern "C" int64_t shim_ghost(const mpm_refine_t* c, const uint8_t* pop) {
  int lat[3];
  double hmin;
  mpm::HostTree T;
  if (mpm::build_tree(*c, T, lat, &hmin)) return -1;
  mpm::LeafGeo G;
  G.leaf = T.leaf.data();
  G.leaf_key = T.leaf_key.data();
  G.cellmap = nullptr;
  G.n_leaf = int64_t(T.leaf_key.size());
  for (int a = 0; a < 3; ++a) {
    G.lo[a] = c->lo[a];
    G.lat[a] = lat[a];
  }
  G.hmin = hmin;
  G.lmax = c->lvl_max;
  std::vector<uint8_t> p(pop, pop + G.n_leaf);
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
