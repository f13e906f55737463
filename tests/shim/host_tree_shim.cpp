// Test shim: exposes the library's host octree construction (no GPU calls) to CPU tests.
#include <cstring>
#include <string>

#include "../../paper_2606_09275_amd/csrc/internal.h"

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
