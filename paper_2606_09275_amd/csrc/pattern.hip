// Point-dependent part of the mesh construction on the GPU: the CSR pattern of the tangent
// (a node pair is coupled iff some point's support holds both; ghost faces couple the nodes of
// their two leaves), the wavefront segments of the sorted points, the per-node lists of the
// (segment record, slot) contributions that the row gather sums, and the block column of
// every slot pair of a populated leaf. Node pairs are 64-bit keys (row << 32 | column) sorted
// and deduplicated on the device; rows and columns follow from the sorted keys in closed form
// (every coupled pair is a dense 3x3 block, so row 3a + c starts at 9 off(a) + 3 c deg(a)).
#include <algorithm>

#include "geom.h"

namespace mpm {

namespace {

inline dim3 grid_of(int64_t n, int threads = 256) { return dim3(unsigned(std::max<int64_t>(1, (n + threads - 1) / threads))); }

__global__ void k_fill32(int32_t* __restrict__ a, int64_t n, int32_t v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_strad_flags(const uint8_t* __restrict__ pnleaf, int64_t n, int32_t* __restrict__ cnt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = pnleaf[i] > 1 ? 1 : 0;
}
__global__ void k_compact_index(const int32_t* __restrict__ cnt, const int64_t* __restrict__ off, int64_t n,
                                int64_t* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n && cnt[i]) out[off[i]] = i;
}
// the points whose domain lies in one leaf (flags), and their leaves in list order
__global__ void k_fast_flags(const uint8_t* __restrict__ pnleaf, int64_t n, int32_t* __restrict__ cnt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = pnleaf[i] == 1 ? 1 : 0;
}
__global__ void k_fast_leaf(const int64_t* __restrict__ fidx, int64_t nf, const int32_t* __restrict__ pleaf,
                            int32_t* __restrict__ fleaf) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j < nf) fleaf[j] = pleaf[fidx[j]];
}

// group of a straddling point by its number of leaves (2, 3-4, 5-8) as a sort key
__global__ void k_strad_group(const int64_t* __restrict__ strad, int64_t ns, const uint8_t* __restrict__ pnleaf,
                              uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= ns) return;
  const int nl = pnleaf[strad[t]];
  key[t] = nl <= 2 ? 0u : (nl <= 4 ? 1u : 2u);
  val[t] = uint32_t(strad[t]);
}
__global__ void k_group_init(int64_t* __restrict__ first) {
  if (threadIdx.x < 3) first[threadIdx.x] = -1;
}
// the grouped order back into the straddler list, and the first index of each group present
__global__ void k_strad_grouped(const uint32_t* __restrict__ key, const uint32_t* __restrict__ val, int64_t ns,
                                int64_t* __restrict__ strad, int64_t* __restrict__ first) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= ns) return;
  strad[t] = int64_t(val[t]);
  if (t == 0 || key[t] != key[t - 1]) first[key[t]] = t;
}

// populated leaves: a point whose domain lies in one leaf (pop), or any point (anypop)
__global__ void k_populated(const int32_t* __restrict__ pleaf, const uint8_t* __restrict__ pnleaf, int64_t n,
                            int32_t* __restrict__ pop) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n && pnleaf[i] == 1) pop[pleaf[i]] = 1;
}
__global__ void k_strad_pop(const int32_t* __restrict__ sleaf, int64_t ns, int32_t* __restrict__ anypop) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= ns) return;
  for (int k = 0; k < kMaxPointLeaves; ++k) {
    const int32_t e = sleaf[t * kMaxPointLeaves + k];
    if (e < 0) break;
    anypop[e] = 1;
  }
}

// support of a straddling point: union of the slot nodes of its leaves, in ascending node
// order (so that the nodes after a given one are a contiguous range of slots)
__device__ int strad_support(const int32_t* __restrict__ sleaf, int64_t t, const int32_t* __restrict__ cell_nodes,
                             int32_t sup[kMaxPointLeaves * 8]) {
  int ns = 0;
  for (int k = 0; k < kMaxPointLeaves; ++k) {
    const int32_t e = sleaf[t * kMaxPointLeaves + k];
    if (e < 0) break;
    for (int v = 0; v < 8; ++v) {
      const int32_t id = cell_nodes[8 * int64_t(e) + v];
      bool f = false;
      for (int z = 0; z < ns; ++z) f |= sup[z] == id;
      if (!f) sup[ns++] = id;
    }
  }
  for (int z = 1; z < ns; ++z) {  // insertion sort of at most 64 ids
    const int32_t id = sup[z];
    int y = z;
    for (; y > 0 && sup[y - 1] > id; --y) sup[y] = sup[y - 1];
    sup[y] = id;
  }
  return ns;
}
__global__ void k_strad_count(const int32_t* __restrict__ sleaf, int64_t ns, const int32_t* __restrict__ cell_nodes,
                              int32_t* __restrict__ cnt, int32_t* __restrict__ maxsup) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= ns) return;
  int32_t sup[kMaxPointLeaves * 8];
  const int k = strad_support(sleaf, t, cell_nodes, sup);
  cnt[t] = k * k;
  atomicMax(maxsup, k);
}
__global__ void k_strad_pairs(const int32_t* __restrict__ sleaf, int64_t ns, const int32_t* __restrict__ cell_nodes,
                              const int64_t* __restrict__ off, uint64_t* __restrict__ pairs) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= ns) return;
  int32_t sup[kMaxPointLeaves * 8];
  const int k = strad_support(sleaf, t, cell_nodes, sup);
  uint64_t* o = pairs + off[t];
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) o[a * k + b] = (uint64_t(uint32_t(sup[a])) << 32) | uint32_t(sup[b]);
}

__global__ void k_strad_nsup(const int32_t* __restrict__ sleaf, int64_t ns, const int32_t* __restrict__ cell_nodes,
                             int32_t* __restrict__ cnt) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= ns) return;
  int32_t sup[kMaxPointLeaves * 8];
  cnt[t] = strad_support(sleaf, t, cell_nodes, sup);
}
// support of each straddling point in slot order, and for each slot the leaves of the point
// that hold its node (bit q) with the node's vertex in each (3 bits at 8 + 3 q)
__global__ void k_strad_slots(const int32_t* __restrict__ sleaf, int64_t ns, const int32_t* __restrict__ cell_nodes,
                              const int64_t* __restrict__ off, int32_t* __restrict__ sup_id,
                              uint32_t* __restrict__ sup_src) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= ns) return;
  int32_t sup[kMaxPointLeaves * 8];
  const int k = strad_support(sleaf, t, cell_nodes, sup);
  for (int z = 0; z < k; ++z) {
    uint32_t src = 0;
    for (int q = 0; q < kMaxPointLeaves; ++q) {
      const int32_t e = sleaf[t * kMaxPointLeaves + q];
      if (e < 0) break;
      for (int v = 0; v < 8; ++v)
        if (cell_nodes[8 * int64_t(e) + v] == sup[z]) src |= (1u << q) | (uint32_t(v) << (8 + 3 * q));
    }
    sup_id[off[t] + z] = sup[z];
    sup_src[off[t] + z] = src;
  }
}

// Transposed block positions for the rows reached by straddling points: for block j of row a
// whose column node c is above a, the block column of a in the row of c (the pattern is
// symmetric and each row's columns ascend: bisection); -1 if absent, which the row kernel
// reports. One wavefront per row, lanes over its blocks.
__global__ void k_tpos(const int32_t* __restrict__ snode, const int64_t* __restrict__ row_ptr,
                       const int32_t* __restrict__ col, int32_t* __restrict__ tpos) {
  const int64_t a = snode[blockIdx.x];
  const int64_t r0 = row_ptr[3 * a];
  const int deg = int((row_ptr[3 * a + 1] - r0) / 3);
  for (int j = threadIdx.x; j < deg; j += 64) {
    const int64_t c = col[r0 + 3 * j] / 3;
    if (c <= a) continue;
    const int64_t s0 = row_ptr[3 * c];
    int lo = 0, hi = int((row_ptr[3 * c + 1] - s0) / 3) - 1, m = -1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int64_t b = col[s0 + 3 * mid] / 3;
      if (b == a) {
        m = mid;
        break;
      }
      if (b < a) lo = mid + 1;
      else hi = mid - 1;
    }
    tpos[r0 / 9 + j] = m;
  }
}

// (support node, straddling point) incidences
__global__ void k_strad_inc(const int32_t* __restrict__ sleaf, int64_t ns, const int32_t* __restrict__ cell_nodes,
                            const int64_t* __restrict__ off, uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= ns) return;
  int32_t sup[kMaxPointLeaves * 8];
  const int k = strad_support(sleaf, t, cell_nodes, sup);
  for (int z = 0; z < k; ++z) {  // the point and the node's slot in its support
    key[off[t] + z] = uint32_t(sup[z]);
    val[off[t] + z] = (uint32_t(t) << 6) | uint32_t(z);
  }
}
__global__ void k_key_runs(const uint32_t* __restrict__ key, int64_t n, int32_t* __restrict__ cnt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}
__global__ void k_run_tables(const uint32_t* __restrict__ key, const uint32_t* __restrict__ val,
                             const int32_t* __restrict__ cnt, const int64_t* __restrict__ off, int64_t n,
                             int32_t* __restrict__ node, int64_t* __restrict__ start, int32_t* __restrict__ items) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (cnt[i]) {
    node[off[i]] = int32_t(key[i]);
    start[off[i]] = i;
  }
  if (i == n - 1) start[off[n]] = n;
  items[i] = int32_t(val[i]);
}

__global__ void k_leaf_pairs(const int32_t* __restrict__ pop, const int64_t* __restrict__ poff, int64_t nl,
                             const int32_t* __restrict__ cell_nodes, uint64_t* __restrict__ pairs) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= 64 * nl) return;
  const int64_t e = t >> 6;
  if (!pop[e]) return;
  const int a = int(t >> 3) & 7, b = int(t & 7);
  pairs[64 * poff[e] + 8 * a + b] =
      (uint64_t(uint32_t(cell_nodes[8 * e + a])) << 32) | uint32_t(cell_nodes[8 * e + b]);
}

// 256 pairs per ghost face (pairs with a padding slot repeat the face's first pair)
__global__ void k_ghost_pairs(const int32_t* __restrict__ gnodes, int64_t nf, uint64_t* __restrict__ pairs) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= 256 * nf) return;
  const int64_t f = t >> 8;
  const int a = int(t >> 4) & 15, b = int(t & 15);
  const int32_t* id = gnodes + 16 * f;
  const int32_t x = id[a] >= 0 && id[b] >= 0 ? id[a] : id[0], y = id[a] >= 0 && id[b] >= 0 ? id[b] : id[0];
  pairs[t] = (uint64_t(uint32_t(x)) << 32) | uint32_t(y);
}

__global__ void k_unique_flags64(const uint64_t* __restrict__ k, int64_t n, int32_t* __restrict__ cnt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = (i == 0 || k[i] != k[i - 1]) ? 1 : 0;
}
__global__ void k_compact64(const uint64_t* __restrict__ k, const int32_t* __restrict__ cnt,
                            const int64_t* __restrict__ off, int64_t n, uint64_t* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n && cnt[i]) out[off[i]] = k[i];
}

__device__ inline int64_t lower_bound64(const uint64_t* __restrict__ a, int64_t lo, int64_t hi, uint64_t key) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// first pair of every row (node) a in [0, nn]
__global__ void k_row_starts(const uint64_t* __restrict__ up, int64_t npu, int64_t nn, int64_t* __restrict__ nb_off) {
  const int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (a <= nn) nb_off[a] = lower_bound64(up, 0, npu, uint64_t(a) << 32);
}

__global__ void k_rows(const int64_t* __restrict__ nb_off, int64_t nn, int64_t* __restrict__ row_ptr,
                       int32_t* __restrict__ stats /* [0] widest row, [1] active DOF rows */) {
  const int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (a >= nn) return;
  const int64_t deg = nb_off[a + 1] - nb_off[a];
  for (int c = 0; c < 3; ++c) row_ptr[3 * a + c] = 9 * nb_off[a] + 3 * c * deg;
  if (a == nn - 1) row_ptr[3 * nn] = 9 * nb_off[nn];
  if (deg) {
    atomicMax(stats, int32_t(deg > 0x7fffffff ? 0x7fffffff : deg));
    atomicAdd(stats + 1, 3);
  }
}

__global__ void k_cols(const uint64_t* __restrict__ up, int64_t npu, const int64_t* __restrict__ nb_off,
                       int32_t* __restrict__ col) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= npu) return;
  const int64_t a = int64_t(up[t] >> 32);
  const int32_t b = int32_t(up[t] & 0xffffffffu);
  const int64_t deg = nb_off[a + 1] - nb_off[a], j = t - nb_off[a], base = 9 * nb_off[a];
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k < 3; ++k) col[base + 3 * c * deg + 3 * j + k] = 3 * b + k;
}

// segments: maximal runs of one leaf inside each 64-point wavefront of the sorted points
__global__ void k_seg_flags(const int32_t* __restrict__ pleaf, int64_t n, int32_t* __restrict__ cnt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = ((i & 63) == 0 || pleaf[i] != pleaf[i - 1]) ? 1 : 0;
}
__global__ void k_seg_first(const int32_t* __restrict__ pleaf, int64_t n, const int64_t* __restrict__ soff,
                            int64_t n_wave, int32_t* __restrict__ wave_seg, int32_t* __restrict__ leaf_seg0) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if ((i & 63) == 0) wave_seg[i >> 6] = int32_t(soff[i]);
  if (i == 0) wave_seg[n_wave] = int32_t(soff[n]);
  if (i == 0 || pleaf[i - 1] != pleaf[i]) leaf_seg0[pleaf[i]] = int32_t(soff[i]);
}
__global__ void k_seg_count(const int32_t* __restrict__ pleaf, int64_t n, const int64_t* __restrict__ soff,
                            const int32_t* __restrict__ leaf_seg0, int32_t* __restrict__ leaf_nseg) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (i == n - 1 || pleaf[i + 1] != pleaf[i]) leaf_nseg[pleaf[i]] = int32_t(soff[i + 1] - leaf_seg0[pleaf[i]]);
}

// (node, leaf * 8 + slot) incidences of the populated leaves, in leaf order
__global__ void k_incidences(const int32_t* __restrict__ pop, const int64_t* __restrict__ poff, int64_t nl,
                             const int32_t* __restrict__ cell_nodes, uint32_t* __restrict__ key,
                             uint32_t* __restrict__ val) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= 8 * nl) return;
  const int64_t e = t >> 3;
  if (!pop[e]) return;
  const int a = int(t & 7);
  const int64_t o = 8 * poff[e] + a;
  key[o] = uint32_t(cell_nodes[t]);
  val[o] = uint32_t(t);
}

__device__ inline int32_t leaf_ncon(const int32_t* __restrict__ leaf_rec, const int32_t* __restrict__ leaf_nseg,
                                    int64_t e) {
  return leaf_rec[e] >= 0 ? 1 : leaf_nseg[e];
}
__global__ void k_con_count(const uint32_t* __restrict__ val, int64_t ninc, const int32_t* __restrict__ leaf_rec,
                            const int32_t* __restrict__ leaf_nseg, int32_t* __restrict__ cnt) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < ninc) cnt[t] = leaf_ncon(leaf_rec, leaf_nseg, int64_t(val[t] >> 3));
}
__global__ void k_con_off(const uint32_t* __restrict__ key, int64_t ninc, const int64_t* __restrict__ cpos,
                          int64_t nn, int32_t* __restrict__ con_off) {
  const int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (a > nn) return;
  int64_t lo = 0, hi = ninc;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (int64_t(key[mid]) < a) lo = mid + 1;
    else hi = mid;
  }
  con_off[a] = int32_t(cpos[lo]);
}
__global__ void k_con_fill(const uint32_t* __restrict__ val, int64_t ninc, const int64_t* __restrict__ cpos,
                           const int32_t* __restrict__ leaf_rec, const int32_t* __restrict__ leaf_seg0,
                           const int32_t* __restrict__ leaf_nseg, int32_t* __restrict__ con_seg,
                           int32_t* __restrict__ con_bp) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= ninc) return;
  const int64_t e = int64_t(val[t] >> 3);
  const int a = int(val[t] & 7);
  const int32_t nc = leaf_ncon(leaf_rec, leaf_nseg, e);
  for (int32_t g = 0; g < nc; ++g) {
    const int64_t rec = leaf_rec[e] >= 0 ? leaf_rec[e] : leaf_seg0[e] + g;
    con_seg[cpos[t] + g] = int32_t((rec << 3) | a);
    con_bp[cpos[t] + g] = int32_t(64 * e + 8 * a);
  }
}

// block column of slot b's node in the row of slot a's node, for every populated leaf
__global__ void k_bpos(const int32_t* __restrict__ pop, int64_t nl, const int32_t* __restrict__ cell_nodes,
                       const uint64_t* __restrict__ up, const int64_t* __restrict__ nb_off, int16_t* __restrict__ bpos) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= 64 * nl) return;
  const int64_t e = t >> 6;
  if (!pop[e]) {
    bpos[t] = -1;
    return;
  }
  const int a = int(t >> 3) & 7, b = int(t & 7);
  const int64_t na = cell_nodes[8 * e + a];
  const uint64_t key = (uint64_t(na) << 32) | uint32_t(cell_nodes[8 * e + b]);
  bpos[t] = int16_t(lower_bound64(up, nb_off[na], nb_off[na + 1], key) - nb_off[na]);
}

__global__ void k_ghost_bpos(const int32_t* __restrict__ gnodes, int64_t nf, const uint64_t* __restrict__ up,
                             const int64_t* __restrict__ nb_off, int16_t* __restrict__ gbpos) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= 256 * nf) return;
  const int64_t f = t >> 8;
  const int a = int(t >> 4) & 15, b = int(t & 15);
  const int32_t* id = gnodes + 16 * f;
  if (id[a] < 0 || id[b] < 0) {
    gbpos[t] = 0;
    return;
  }
  const int64_t na = id[a];
  const uint64_t key = (uint64_t(na) << 32) | uint32_t(id[b]);
  gbpos[t] = int16_t(lower_bound64(up, nb_off[na], nb_off[na + 1], key) - nb_off[na]);
}

template <typename T>
int32_t download(std::vector<T>& h, const T* d, int64_t n, const char* what) {
  h.resize(size_t(n));
  if (n) {
    const hipError_t e = hipMemcpy(h.data(), d, size_t(n) * sizeof(T), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, what);
  }
  return MPM_OK;
}
template <typename T>
int32_t upload_vec(T** dst, const std::vector<T>& v, const char* what) {
  const hipError_t e = hipMalloc(dst, std::max<size_t>(1, v.size()) * sizeof(T));
  if (e != hipSuccess) return hip_fail(e, what);
  if (!v.empty()) {
    const hipError_t e2 = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e2 != hipSuccess) return hip_fail(e2, what);
  }
  return MPM_OK;
}
int32_t read64(const int64_t* d, int64_t* out) {
  MPM_HIP(hipMemcpy(out, d, 8, hipMemcpyDeviceToHost));
  return MPM_OK;
}
int bits_for(int64_t v) {
  int b = 1;
  while ((int64_t(1) << b) <= v) ++b;
  return b;
}

}  // namespace

// Builds, for the sorted and classified points of the mesh (perm, point leaf, overlap counts
// on the device), the straddler lists, the CSR pattern, segments, records, contribution lists
// and slot block columns, and the ghost faces when the criterion asks for them.
int32_t gpu_build_pattern(mpm_mesh* m, const double* dx, const double* dl, hipStream_t st) {
  const int64_t n = m->n_point, nl = m->n_leaf, nn = m->n_node;
  int32_t rc = MPM_OK;
  // straddling points (domain over several leaves) and their leaves
  m->n_straddle = 0;
  if (n) {
    DevBuf cnt, off;
    if ((rc = cnt.alloc(size_t(n) * 4, "octree_build: straddle flags")) ||
        (rc = off.alloc(size_t(n + 1) * 8, "octree_build: straddle offsets")))
      return rc;
    hipLaunchKernelGGL(k_strad_flags, grid_of(n), dim3(256), 0, st, m->d_pnleaf, n, cnt.as<int32_t>());
    if ((rc = scan_counts(cnt.as<int32_t>(), n, off.as<int64_t>(), st))) return rc;
    if ((rc = read64(off.as<int64_t>() + n, &m->n_straddle))) return rc;
    if (m->n_straddle) {
      MPM_HIP(hipMalloc(&m->d_strad, size_t(m->n_straddle) * 8));
      MPM_HIP(hipMalloc(&m->d_strad_leaf, size_t(m->n_straddle) * kMaxPointLeaves * 4));
      MPM_HIP(hipMalloc(&m->d_grec, size_t(m->n_straddle) * kGenRec * 8));
      hipLaunchKernelGGL(k_compact_index, grid_of(n), dim3(256), 0, st, cnt.as<int32_t>(), off.as<int64_t>(), n,
                         m->d_strad);
      // grouped by their number of leaves (a stable sort keeps point order inside a group), so
      // that the wavefronts of the per-point kernels loop over similar numbers of leaves
      const int64_t ns0 = m->n_straddle;
      const int64_t nblk = (ns0 + kRsTile - 1) / kRsTile;
      if (n >= (int64_t(1) << 32)) {  // the grouping sorts 32-bit point indices
        set_error(MPM_EARG, "octree_build: 2^32 points or more with domains over several leaves");
        return MPM_EARG;
      }
      DevBuf gk, gv, gkt, gvt, gh, gf;
      if ((rc = gk.alloc(size_t(ns0) * 4, "octree_build: straddler groups")) ||
          (rc = gv.alloc(size_t(ns0) * 4, "octree_build: straddler groups")) ||
          (rc = gkt.alloc(size_t(ns0) * 4, "octree_build: straddler groups")) ||
          (rc = gvt.alloc(size_t(ns0) * 4, "octree_build: straddler groups")) ||
          (rc = gh.alloc(size_t(nblk) * 1024 + 1024, "octree_build: straddler groups")) ||
          (rc = gf.alloc(3 * 8, "octree_build: straddler groups")))
        return rc;
      hipLaunchKernelGGL(k_strad_group, grid_of(ns0), dim3(256), 0, st, m->d_strad, ns0, m->d_pnleaf,
                         gk.as<uint32_t>(), gv.as<uint32_t>());
      uint32_t *gk2 = gk.as<uint32_t>(), *gv2 = gv.as<uint32_t>();
      if ((rc = radix_sort(gk.as<uint32_t>(), gv.as<uint32_t>(), ns0, 2, gkt.as<uint32_t>(), gvt.as<uint32_t>(),
                           gh.as<uint32_t>(), gh.as<uint32_t>() + size_t(nblk) * 256, st, &gk2, &gv2)))
        return rc;
      hipLaunchKernelGGL(k_group_init, dim3(1), dim3(64), 0, st, gf.as<int64_t>());
      hipLaunchKernelGGL(k_strad_grouped, grid_of(ns0), dim3(256), 0, st, gk2, gv2, ns0, m->d_strad,
                         gf.as<int64_t>());
      int64_t first[3] = {-1, -1, -1};
      MPM_HIP(hipMemcpyAsync(first, gf.as<int64_t>(), sizeof(first), hipMemcpyDeviceToHost, st));
      MPM_HIP(hipStreamSynchronize(st));
      m->strad_grp[3] = ns0;
      for (int g = 2; g >= 0; --g) m->strad_grp[g] = first[g] >= 0 ? first[g] : m->strad_grp[g + 1];
      MPM_HIP(hipStreamCreateWithFlags(&m->side, hipStreamNonBlocking));
      MPM_HIP(hipEventCreateWithFlags(&m->fork_ev, hipEventDisableTiming));
      MPM_HIP(hipEventCreateWithFlags(&m->join_ev, hipEventDisableTiming));
      if ((rc = strad_leaves(m, dx, dl, st))) return rc;
    }
  }
  const int64_t ns = m->n_straddle;
  // populated leaves
  DevBuf pop, poff, anypop;
  if ((rc = pop.alloc(size_t(nl) * 4, "octree_build: populated flags")) ||
      (rc = poff.alloc(size_t(nl + 1) * 8, "octree_build: populated ranks")))
    return rc;
  hipLaunchKernelGGL(k_fill32, grid_of(nl), dim3(256), 0, st, pop.as<int32_t>(), nl, 0);
  if (n) hipLaunchKernelGGL(k_populated, grid_of(n), dim3(256), 0, st, m->d_pleaf, m->d_pnleaf, n, pop.as<int32_t>());
  if ((rc = scan_counts(pop.as<int32_t>(), nl, poff.as<int64_t>(), st))) return rc;
  int64_t npop = 0;
  if ((rc = read64(poff.as<int64_t>() + nl, &npop))) return rc;

  // ghost faces: populated here means overlapped by any point domain
  if (m->crit.ghost && n) {
    if ((rc = anypop.alloc(size_t(nl) * 4, "octree_build: overlapped flags"))) return rc;
    MPM_HIP(hipMemcpyAsync(anypop.p, pop.p, size_t(nl) * 4, hipMemcpyDeviceToDevice, st));
    if (ns) hipLaunchKernelGGL(k_strad_pop, grid_of(ns), dim3(256), 0, st, m->d_strad_leaf, ns, anypop.as<int32_t>());
    if ((rc = gpu_ghost_faces(m, anypop.as<int32_t>(), st))) return rc;
  }
  const int64_t nf = m->n_gface;

  // node pairs: populated leaves (64 each), straddlers (support squared), ghost faces (256)
  DevBuf scnt, soff;
  int64_t n_spair = 0;
  int32_t* d_stats = nullptr;  // [0] widest row, [1] active rows, [2] largest straddler support
  DevBuf stats;
  if ((rc = stats.alloc(16, "octree_build: counters"))) return rc;
  d_stats = stats.as<int32_t>();
  MPM_HIP(hipMemsetAsync(d_stats, 0, 16, st));
  if (ns) {
    if ((rc = scnt.alloc(size_t(ns) * 4, "octree_build: straddle pair counts")) ||
        (rc = soff.alloc(size_t(ns + 1) * 8, "octree_build: straddle pair offsets")))
      return rc;
    hipLaunchKernelGGL(k_strad_count, grid_of(ns), dim3(256), 0, st, m->d_strad_leaf, ns, m->d_cell_nodes,
                       scnt.as<int32_t>(), d_stats + 2);
    if ((rc = scan_counts(scnt.as<int32_t>(), ns, soff.as<int64_t>(), st))) return rc;
    if ((rc = read64(soff.as<int64_t>() + ns, &n_spair))) return rc;
  }
  const int64_t n_lpair = 64 * npop, n_gpair = 256 * nf;
  const int64_t npair = n_lpair + n_spair + n_gpair;
  DevBuf pairs, ucnt, uoff, upairs, nb_off;
  if ((rc = pairs.alloc(size_t(npair) * 8, "octree_build: node pairs"))) return rc;
  hipLaunchKernelGGL(k_leaf_pairs, grid_of(64 * nl), dim3(256), 0, st, pop.as<int32_t>(), poff.as<int64_t>(), nl,
                     m->d_cell_nodes, pairs.as<uint64_t>());
  if (ns)
    hipLaunchKernelGGL(k_strad_pairs, grid_of(ns), dim3(256), 0, st, m->d_strad_leaf, ns, m->d_cell_nodes,
                       soff.as<int64_t>(), pairs.as<uint64_t>() + n_lpair);
  if (nf)
    hipLaunchKernelGGL(k_ghost_pairs, grid_of(n_gpair), dim3(256), 0, st, m->d_gf_nodes, nf,
                       pairs.as<uint64_t>() + n_lpair + n_spair);
  MPM_HIP(hipGetLastError());
  if ((rc = sort_u64(pairs.as<uint64_t>(), npair, 32 + bits_for(nn), st))) return rc;
  if ((rc = ucnt.alloc(size_t(npair) * 4, "octree_build: pair flags")) ||
      (rc = uoff.alloc(size_t(npair + 1) * 8, "octree_build: pair offsets")))
    return rc;
  hipLaunchKernelGGL(k_unique_flags64, grid_of(npair), dim3(256), 0, st, pairs.as<uint64_t>(), npair,
                     ucnt.as<int32_t>());
  if ((rc = scan_counts(ucnt.as<int32_t>(), npair, uoff.as<int64_t>(), st))) return rc;
  int64_t npu = 0;
  if ((rc = read64(uoff.as<int64_t>() + npair, &npu))) return rc;
  if ((rc = upairs.alloc(size_t(npu) * 8, "octree_build: coupled pairs")) ||
      (rc = nb_off.alloc(size_t(nn + 1) * 8, "octree_build: row starts")))
    return rc;
  hipLaunchKernelGGL(k_compact64, grid_of(npair), dim3(256), 0, st, pairs.as<uint64_t>(), ucnt.as<int32_t>(),
                     uoff.as<int64_t>(), npair, upairs.as<uint64_t>());
  pairs.alloc(8, "octree_build: node pairs");  // release the unsorted pairs
  ucnt.alloc(8, "octree_build: pair flags");
  uoff.alloc(8, "octree_build: pair offsets");
  hipLaunchKernelGGL(k_row_starts, grid_of(nn + 1), dim3(256), 0, st, upairs.as<uint64_t>(), npu, nn,
                     nb_off.as<int64_t>());
  m->nnz = 9 * npu;
  MPM_HIP(hipMalloc(&m->d_row_ptr, size_t(3 * nn + 1) * 8));
  MPM_HIP(hipMalloc(&m->d_col, size_t(std::max<int64_t>(1, m->nnz)) * 4));
  if (nn) hipLaunchKernelGGL(k_rows, grid_of(nn), dim3(256), 0, st, nb_off.as<int64_t>(), nn, m->d_row_ptr, d_stats);
  else MPM_HIP(hipMemsetAsync(m->d_row_ptr, 0, 8, st));
  hipLaunchKernelGGL(k_cols, grid_of(npu), dim3(256), 0, st, upairs.as<uint64_t>(), npu, nb_off.as<int64_t>(),
                     m->d_col);
  MPM_HIP(hipGetLastError());

  // segments of the points whose domain lies in one leaf: maximal runs of one leaf inside each
  // 64-point wavefront of their list (the sorted points themselves when no domain straddles)
  m->n_fast = n - ns;
  const int64_t nfast = m->n_fast;
  const int32_t* lf = m->d_pleaf;
  DevBuf fcnt, foff, fleaf;
  if (ns && nfast) {
    if ((rc = fcnt.alloc(size_t(n) * 4, "octree_build: one-leaf points")) ||
        (rc = foff.alloc(size_t(n + 1) * 8, "octree_build: one-leaf points")) ||
        (rc = fleaf.alloc(size_t(nfast) * 4, "octree_build: one-leaf points")))
      return rc;
    MPM_HIP(hipMalloc(&m->d_fidx, size_t(nfast) * 8));
    hipLaunchKernelGGL(k_fast_flags, grid_of(n), dim3(256), 0, st, m->d_pnleaf, n, fcnt.as<int32_t>());
    if ((rc = scan_counts(fcnt.as<int32_t>(), n, foff.as<int64_t>(), st))) return rc;
    int64_t cnt1 = 0;
    if ((rc = read64(foff.as<int64_t>() + n, &cnt1))) return rc;
    if (cnt1 != nfast) {  // every point overlaps at least one leaf once classified
      set_error(MPM_EARG, "octree_build: point overlap counts do not add up");
      return MPM_EARG;
    }
    hipLaunchKernelGGL(k_compact_index, grid_of(n), dim3(256), 0, st, fcnt.as<int32_t>(), foff.as<int64_t>(), n,
                       m->d_fidx);
    hipLaunchKernelGGL(k_fast_leaf, grid_of(nfast), dim3(256), 0, st, m->d_fidx, nfast, m->d_pleaf, fleaf.as<int32_t>());
    lf = fleaf.as<int32_t>();
  }
  m->n_wave = (nfast + 63) / 64;
  DevBuf segc, segoff;
  MPM_HIP(hipMalloc(&m->d_wave_seg, size_t(m->n_wave + 1) * 4));
  MPM_HIP(hipMalloc(&m->d_leaf_seg0, size_t(std::max<int64_t>(1, nl)) * 4));
  MPM_HIP(hipMalloc(&m->d_leaf_nseg, size_t(std::max<int64_t>(1, nl)) * 4));
  hipLaunchKernelGGL(k_fill32, grid_of(nl), dim3(256), 0, st, m->d_leaf_seg0, nl, 0);
  hipLaunchKernelGGL(k_fill32, grid_of(nl), dim3(256), 0, st, m->d_leaf_nseg, nl, 0);
  int64_t nseg = 0;
  if (nfast) {
    if ((rc = segc.alloc(size_t(nfast) * 4, "octree_build: segment flags")) ||
        (rc = segoff.alloc(size_t(nfast + 1) * 8, "octree_build: segment offsets")))
      return rc;
    hipLaunchKernelGGL(k_seg_flags, grid_of(nfast), dim3(256), 0, st, lf, nfast, segc.as<int32_t>());
    if ((rc = scan_counts(segc.as<int32_t>(), nfast, segoff.as<int64_t>(), st))) return rc;
    if ((rc = read64(segoff.as<int64_t>() + nfast, &nseg))) return rc;
    hipLaunchKernelGGL(k_seg_first, grid_of(nfast), dim3(256), 0, st, lf, nfast, segoff.as<int64_t>(), m->n_wave,
                       m->d_wave_seg, m->d_leaf_seg0);
    hipLaunchKernelGGL(k_seg_count, grid_of(nfast), dim3(256), 0, st, lf, nfast, segoff.as<int64_t>(),
                       m->d_leaf_seg0, m->d_leaf_nseg);
  } else {
    MPM_HIP(hipMemsetAsync(m->d_wave_seg, 0, 4, st));
  }
  m->n_seg = nseg;
  if (nseg >= (int64_t(1) << 31)) {
    set_error(MPM_EARG, "octree_build: too many point segments");
    return MPM_EARG;
  }

  // Leaves holding more than kHeavySeg segments (a leaf with many points, which spans
  // several wavefronts) are summed into one record first, so that every node row gathers a
  // bounded number of records: chunks of up to kRedChunk segments are summed in parallel,
  // then the chunk sums of each leaf, always in ascending record order (host: one pass over
  // the leaves).
  constexpr int kHeavySeg = 4, kRedChunk = 64;
  std::vector<int32_t> hpop, hseg0, hnseg;
  MPM_HIP(hipStreamSynchronize(st));
  if ((rc = download(hpop, pop.as<int32_t>(), nl, "octree_build: populated flags")) ||
      (rc = download(hseg0, m->d_leaf_seg0, nl, "octree_build: leaf segments")) ||
      (rc = download(hnseg, m->d_leaf_nseg, nl, "octree_build: leaf segments")))
    return rc;
  std::vector<int32_t> leaf_rec(size_t(nl), -1), red1, red2;
  int64_t nrec = nseg;
  for (int64_t e = 0; e < nl; ++e)
    if (hpop[e] && hnseg[e] > kHeavySeg) leaf_rec[e] = int32_t(nrec++);
  for (int64_t e = 0; e < nl; ++e) {
    if (leaf_rec[e] < 0) continue;
    const int32_t nse = hnseg[e];
    if (nse <= kRedChunk) {
      red1.insert(red1.end(), {hseg0[e], nse, leaf_rec[e]});
      continue;
    }
    const int32_t first_chunk = int32_t(nrec);
    const int32_t nch = (nse + kRedChunk - 1) / kRedChunk;
    for (int32_t c = 0; c < nch; ++c)
      red1.insert(red1.end(), {hseg0[e] + c * kRedChunk, std::min(kRedChunk, nse - c * kRedChunk), int32_t(nrec++)});
    red2.insert(red2.end(), {first_chunk, nch, leaf_rec[e]});
  }
  m->n_rec = nrec;
  m->n_red1 = int64_t(red1.size() / 3);
  m->n_red2 = int64_t(red2.size() / 3);
  if (nrec >= (int64_t(1) << 28)) {
    set_error(MPM_EARG, "octree_build: too many segment records");
    return MPM_EARG;
  }
  DevBuf drec;
  {
    int32_t* p = nullptr;
    if ((rc = upload_vec(&p, leaf_rec, "octree_build: leaf records"))) return rc;
    drec.p = p;
  }
  if (!red1.empty() && (rc = upload_vec(&m->d_red1, red1, "octree_build: record reductions"))) return rc;
  if (!red2.empty() && (rc = upload_vec(&m->d_red2, red2, "octree_build: record reductions"))) return rc;

  // contributions (record, slot) per node, ascending leaf then segment
  const int64_t ninc = 8 * npop;
  DevBuf ik, iv, ikt, ivt, hist, ccnt, cpos;
  const int64_t nblk = (ninc + kRsTile - 1) / kRsTile;
  if ((rc = ik.alloc(size_t(ninc) * 4, "octree_build: incidences")) ||
      (rc = iv.alloc(size_t(ninc) * 4, "octree_build: incidences")) ||
      (rc = ikt.alloc(size_t(ninc) * 4, "octree_build: incidences")) ||
      (rc = ivt.alloc(size_t(ninc) * 4, "octree_build: incidences")) ||
      (rc = hist.alloc(size_t(nblk) * 1024 + 1024, "octree_build: incidence counts")) ||
      (rc = ccnt.alloc(size_t(ninc) * 4, "octree_build: contribution counts")) ||
      (rc = cpos.alloc(size_t(ninc + 1) * 8, "octree_build: contribution offsets")))
    return rc;
  hipLaunchKernelGGL(k_incidences, grid_of(8 * nl), dim3(256), 0, st, pop.as<int32_t>(), poff.as<int64_t>(), nl,
                     m->d_cell_nodes, ik.as<uint32_t>(), iv.as<uint32_t>());
  uint32_t *ks = ik.as<uint32_t>(), *vs = iv.as<uint32_t>();
  if ((rc = radix_sort(ik.as<uint32_t>(), iv.as<uint32_t>(), ninc, bits_for(nn), ikt.as<uint32_t>(),
                       ivt.as<uint32_t>(), hist.as<uint32_t>(), hist.as<uint32_t>() + size_t(nblk) * 256, st, &ks,
                       &vs)))
    return rc;
  hipLaunchKernelGGL(k_con_count, grid_of(ninc), dim3(256), 0, st, vs, ninc, drec.as<int32_t>(), m->d_leaf_nseg,
                     ccnt.as<int32_t>());
  if ((rc = scan_counts(ccnt.as<int32_t>(), ninc, cpos.as<int64_t>(), st))) return rc;
  if ((rc = read64(cpos.as<int64_t>() + ninc, &m->n_con))) return rc;
  if (m->n_con >= (int64_t(1) << 31)) {
    set_error(MPM_EARG, "octree_build: too many segment contributions");
    return MPM_EARG;
  }
  MPM_HIP(hipMalloc(&m->d_con_off, size_t(nn + 1) * 4));
  MPM_HIP(hipMalloc(&m->d_con_seg, size_t(std::max<int64_t>(1, m->n_con)) * 4));
  MPM_HIP(hipMalloc(&m->d_con_bp, size_t(std::max<int64_t>(1, m->n_con)) * 4));
  MPM_HIP(hipMalloc(&m->d_bpos, size_t(std::max<int64_t>(1, nl)) * 64 * 2));
  hipLaunchKernelGGL(k_con_off, grid_of(nn + 1), dim3(256), 0, st, ks, ninc, cpos.as<int64_t>(), nn, m->d_con_off);
  hipLaunchKernelGGL(k_con_fill, grid_of(ninc), dim3(256), 0, st, vs, ninc, cpos.as<int64_t>(), drec.as<int32_t>(),
                     m->d_leaf_seg0, m->d_leaf_nseg, m->d_con_seg, m->d_con_bp);
  hipLaunchKernelGGL(k_bpos, grid_of(64 * nl), dim3(256), 0, st, pop.as<int32_t>(), nl, m->d_cell_nodes,
                     upairs.as<uint64_t>(), nb_off.as<int64_t>(), m->d_bpos);
  MPM_HIP(hipGetLastError());

  int32_t hstats[4] = {0, 0, 0, 0};
  MPM_HIP(hipStreamSynchronize(st));
  MPM_HIP(hipMemcpy(hstats, d_stats, 16, hipMemcpyDeviceToHost));
  m->max_deg = hstats[0];
  m->n_active_rows = hstats[1];
  m->max_support = std::max(npop ? 8 : 0, hstats[2]);
  if (m->max_deg > 1024 || nl >= (int64_t(1) << 25)) {
    set_error(MPM_ESTENCIL, "octree_build: node row too wide or too many leaves for the gather");
    return MPM_ESTENCIL;
  }
  // the row gather's launch order when some rows are wide (the LDS of a launch is sized for
  // its widest row): narrow rows first, from their widths on the host
  if (m->max_deg > kGatherNarrow && nn) {
    std::vector<int64_t> rp(size_t(3 * nn + 1));
    MPM_HIP(hipMemcpyAsync(rp.data(), m->d_row_ptr, rp.size() * 8, hipMemcpyDeviceToHost, st));
    MPM_HIP(hipStreamSynchronize(st));
    std::vector<int32_t> order;
    order.reserve(size_t(nn));
    m->n_gnarrow = 0;
    for (int pass = 0; pass < 2; ++pass)
      for (int64_t a = 0; a < nn; ++a) {
        const bool narrow = (rp[size_t(3 * a + 1)] - rp[size_t(3 * a)]) / 3 <= kGatherNarrow;
        if (narrow != (pass == 0)) continue;
        order.push_back(int32_t(a));
        if (narrow) ++m->n_gnarrow;
      }
    MPM_HIP(hipMalloc(&m->d_gorder, order.size() * 4));
    MPM_HIP(hipMemcpyAsync(m->d_gorder, order.data(), order.size() * 4, hipMemcpyHostToDevice, st));
    MPM_HIP(hipStreamSynchronize(st));
  }

  // ghost couplings: block column of every face node pair in the first node's row
  if (nf) {
    MPM_HIP(hipMalloc(&m->d_gf_bpos, size_t(nf) * 256 * 2));
    hipLaunchKernelGGL(k_ghost_bpos, grid_of(256 * nf), dim3(256), 0, st, m->d_gf_nodes, nf, upairs.as<uint64_t>(),
                       nb_off.as<int64_t>(), m->d_gf_bpos);
    MPM_HIP(hipMalloc(&m->d_gbeta, size_t(nl) * 8));
    MPM_HIP(hipMalloc(&m->d_gsegmax, size_t(std::max<int64_t>(1, m->n_seg)) * 8));
    MPM_HIP(hipMalloc(&m->d_gf_sc, size_t(nf) * 8));
  }

  // rows reached by straddling points, each with its points in ascending order; an entry
  // holds the point and the slot of the row's node in its support (t 64 + slot)
  m->n_snode = 0;
  if (ns >= (int64_t(1) << 26)) {
    set_error(MPM_ESTENCIL, "octree_build: more than 2^26 point domains overlap several leaves");
    return MPM_ESTENCIL;
  }
  if (ns) {
    DevBuf sc, so, sk, sv, skt, svt, sh, rcn, ro;
    if ((rc = sc.alloc(size_t(ns) * 4, "octree_build: straddle supports")) ||
        (rc = so.alloc(size_t(ns + 1) * 8, "octree_build: straddle supports")))
      return rc;
    hipLaunchKernelGGL(k_strad_nsup, grid_of(ns), dim3(256), 0, st, m->d_strad_leaf, ns, m->d_cell_nodes,
                       sc.as<int32_t>());
    if ((rc = scan_counts(sc.as<int32_t>(), ns, so.as<int64_t>(), st))) return rc;
    int64_t ninc = 0;
    if ((rc = read64(so.as<int64_t>() + ns, &ninc))) return rc;
    const int64_t nblk2 = (ninc + kRsTile - 1) / kRsTile;
    if ((rc = sk.alloc(size_t(ninc) * 4, "octree_build: straddle incidences")) ||
        (rc = sv.alloc(size_t(ninc) * 4, "octree_build: straddle incidences")) ||
        (rc = skt.alloc(size_t(ninc) * 4, "octree_build: straddle incidences")) ||
        (rc = svt.alloc(size_t(ninc) * 4, "octree_build: straddle incidences")) ||
        (rc = sh.alloc(size_t(nblk2) * 1024 + 1024, "octree_build: straddle incidence counts")) ||
        (rc = rcn.alloc(size_t(ninc) * 4, "octree_build: straddle rows")) ||
        (rc = ro.alloc(size_t(ninc + 1) * 8, "octree_build: straddle rows")))
      return rc;
    hipLaunchKernelGGL(k_strad_inc, grid_of(ns), dim3(256), 0, st, m->d_strad_leaf, ns, m->d_cell_nodes,
                       so.as<int64_t>(), sk.as<uint32_t>(), sv.as<uint32_t>());
    // the support of each point in slot order, kept with the mesh for the row kernel
    MPM_HIP(hipMalloc(&m->d_sup_off, size_t(ns + 1) * 8));
    MPM_HIP(hipMalloc(&m->d_sup_id, size_t(std::max<int64_t>(1, ninc)) * 4));
    MPM_HIP(hipMalloc(&m->d_sup_src, size_t(std::max<int64_t>(1, ninc)) * 4));
    MPM_HIP(hipMalloc(&m->d_sup_g, size_t(std::max<int64_t>(1, ninc)) * 4 * 8));
    MPM_HIP(hipMemcpyAsync(m->d_sup_off, so.as<int64_t>(), size_t(ns + 1) * 8, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_strad_slots, grid_of(ns), dim3(256), 0, st, m->d_strad_leaf, ns, m->d_cell_nodes,
                       so.as<int64_t>(), m->d_sup_id, m->d_sup_src);
    uint32_t *ks2 = sk.as<uint32_t>(), *vs2 = sv.as<uint32_t>();
    if ((rc = radix_sort(sk.as<uint32_t>(), sv.as<uint32_t>(), ninc, bits_for(nn), skt.as<uint32_t>(),
                         svt.as<uint32_t>(), sh.as<uint32_t>(), sh.as<uint32_t>() + size_t(nblk2) * 256, st, &ks2,
                         &vs2)))
      return rc;
    hipLaunchKernelGGL(k_key_runs, grid_of(ninc), dim3(256), 0, st, ks2, ninc, rcn.as<int32_t>());
    if ((rc = scan_counts(rcn.as<int32_t>(), ninc, ro.as<int64_t>(), st))) return rc;
    if ((rc = read64(ro.as<int64_t>() + ninc, &m->n_snode))) return rc;
    MPM_HIP(hipMalloc(&m->d_snode, size_t(std::max<int64_t>(1, m->n_snode)) * 4));
    MPM_HIP(hipMalloc(&m->d_sinc_off, size_t(m->n_snode + 1) * 8));
    MPM_HIP(hipMalloc(&m->d_sinc, size_t(std::max<int64_t>(1, ninc)) * 4));
    hipLaunchKernelGGL(k_run_tables, grid_of(ninc), dim3(256), 0, st, ks2, vs2, rcn.as<int32_t>(), ro.as<int64_t>(),
                       ninc, m->d_snode, m->d_sinc_off, m->d_sinc);
    MPM_HIP(hipGetLastError());
    // launch order of those rows: narrow rows first (stable), from their widths on the host
    std::vector<int32_t> node(size_t(m->n_snode));
    std::vector<int64_t> rp(size_t(3 * m->n_node + 1));
    MPM_HIP(hipMemcpyAsync(node.data(), m->d_snode, node.size() * 4, hipMemcpyDeviceToHost, st));
    MPM_HIP(hipMemcpyAsync(rp.data(), m->d_row_ptr, rp.size() * 8, hipMemcpyDeviceToHost, st));
    MPM_HIP(hipStreamSynchronize(st));
    std::vector<int32_t> order;
    order.reserve(node.size());
    for (int pass = 0; pass < 2; ++pass)
      for (size_t b = 0; b < node.size(); ++b) {
        const int64_t a = node[b];
        const bool narrow = (rp[size_t(3 * a + 1)] - rp[size_t(3 * a)]) / 3 <= kNarrowRow;
        if (narrow == (pass == 0)) order.push_back(int32_t(b));
        if (pass == 0 && narrow) ++m->n_snode_narrow;
      }
    MPM_HIP(hipMalloc(&m->d_srow, std::max<size_t>(1, order.size()) * 4));
    MPM_HIP(hipMemcpyAsync(m->d_srow, order.data(), order.size() * 4, hipMemcpyHostToDevice, st));
    MPM_HIP(hipMalloc(&m->d_tpos, size_t(std::max<int64_t>(1, m->nnz / 9)) * 4));
    if (m->n_snode)
      hipLaunchKernelGGL(k_tpos, dim3(unsigned(m->n_snode)), dim3(64), 0, st, m->d_snode, m->d_row_ptr, m->d_col,
                         m->d_tpos);
    MPM_HIP(hipGetLastError());
    MPM_HIP(hipStreamSynchronize(st));
  }

  MPM_HIP(hipMalloc(&m->d_segK, size_t(std::max<int64_t>(1, nrec)) * 324 * 8));
  MPM_HIP(hipMalloc(&m->d_segF, size_t(std::max<int64_t>(1, nrec)) * 24 * 8));
  MPM_HIP(hipMalloc(&m->d_segM, size_t(std::max<int64_t>(1, nrec)) * 36 * 8));
  MPM_HIP(hipMalloc(&m->d_partial, 4096 * sizeof(double)));
  MPM_HIP(hipGetLastError());
  MPM_HIP(hipStreamSynchronize(st));
  return MPM_OK;
}

}  // namespace mpm
