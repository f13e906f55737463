// Mesh construction entry points and point order: octree_build (tree in tree.hip, then point
// keys, LSD radix sort by leaf, overlap classification here, then the pattern in pattern.hip),
// the point sort and state permutation of later steps, mesh queries and error reporting.
#include <algorithm>
#include <cmath>
#include <utility>
#include <cstring>
#include <mutex>

#include "geom.h"

namespace mpm {

// ------------------------------------------------------------------ errors
namespace {
thread_local std::string g_msg;
thread_local int64_t g_index = -1;
}  // namespace

void set_error(int32_t code, const std::string& msg, int64_t index) {
  g_msg = "[" + std::to_string(code) + "] " + msg;
  g_index = index;
}
int32_t hip_fail(hipError_t e, const char* what) {
  set_error(MPM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  return MPM_EHIP;
}

int32_t gpu_build_tree(mpm_mesh* m, const mpm_refine_t& c, hipStream_t st);
int32_t gpu_build_pattern(mpm_mesh* m, const double* dx, const double* dl, hipStream_t st);

// ------------------------------------------------------------------ point keys
// key = rank of the leaf containing the point's centre, value = original index; a stable
// sort by key gives the point order (leaf, original index).
__global__ void k_point_keys(const double* __restrict__ x, int64_t n, LeafGeo G, uint32_t* __restrict__ keys,
                             uint32_t* __restrict__ idx, DevErr* err) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double xp[3];
  bool bad = false;
  for (int a = 0; a < 3; ++a) {
    xp[a] = x[a * n + p];
    bad |= !isfinite(xp[a]);
  }
  idx[p] = uint32_t(p);
  if (bad) {
    if (atomicCAS(&err->code, 0, MPM_ENONFINITE) == 0) err->index = p;
    keys[p] = 0;
    return;
  }
  int64_t e = leaf_of_point(G, xp[0], xp[1], xp[2]);
  if (e < 0 || e >= G.n_leaf) {  // the leaves tile the box: never taken for a consistent tree
    if (atomicCAS(&err->code, 0, MPM_ETREE) == 0) err->index = p;
    e = 0;
  }
  keys[p] = uint32_t(e);
}

// leaf rank of every finest lattice cell: one workgroup per leaf fills its block
__global__ __launch_bounds__(256) void k_fill_cellmap(const int32_t* __restrict__ leaf, int lmax, int nx, int ny,
                                                      int32_t* __restrict__ map) {
  const int64_t e = blockIdx.x;
  const int32_t* q = leaf + 4 * e;
  const int s = 1 << (lmax - q[3]);
  const int64_t cells = int64_t(s) * s * s;
  for (int64_t c = threadIdx.x; c < cells; c += blockDim.x) {
    const int cx = int(c % s), cy = int((c / s) % s), cz = int(c / (int64_t(s) * s));
    map[(int64_t(q[2] + cz) * ny + (q[1] + cy)) * nx + (q[0] + cx)] = int32_t(e);
  }
}

// ------------------------------------------------------------------ stable LSD radix sort
// 8-bit digits; 32-bit keys with 32-bit values. Per pass: per-tile digit counts, one scan
// per digit over the tiles, then a scatter that ranks equal digits inside each wavefront
// with ballots (stable: tiles, wavefronts and lanes keep their input order).

__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                        uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * kRsTile;
  for (int i = threadIdx.x; i < kRsTile; i += kRsThreads) {
    const int64_t j = base + i;
    if (j < n) atomicAdd(&h[(keys[j] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[int64_t(threadIdx.x) * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// exclusive prefix sum over the 256 threads of a workgroup (thread t holds digit t's value):
// inclusive sums inside each wavefront by shuffles, then the wavefront totals; all threads
// call it; *total (if given) receives the sum of all 256 values
static_assert(kRsThreads == 256, "the radix kernels give thread t digit t");
__device__ __forceinline__ uint32_t block_exclusive_256(uint32_t v, uint32_t* wtot, uint32_t* total = nullptr) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(inc, off);
    if (lane >= off) inc += t;
  }
  if (lane == 63) wtot[wave] = inc;
  __syncthreads();
  uint32_t before = 0;
  for (int w = 0; w < wave; ++w) before += wtot[w];
  if (total) *total = wtot[0] + wtot[1] + wtot[2] + wtot[3];
  __syncthreads();  // wtot may be reused by the caller's next scan
  return before + inc - v;
}

// exclusive scan of one digit's per-block counts (one workgroup per digit); total -> tot[d]
__global__ __launch_bounds__(kRsThreads) void k_rs_scan_digit(uint32_t* __restrict__ hist, int nblk,
                                                              uint32_t* __restrict__ tot) {
  __shared__ uint32_t wtot[kRsThreads / 64];
  uint32_t* row = hist + int64_t(blockIdx.x) * nblk;
  uint32_t carry = 0;
  for (int base = 0; base < nblk; base += kRsThreads) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < nblk ? row[i] : 0u;
    uint32_t chunk;
    const uint32_t ex = block_exclusive_256(v, wtot, &chunk);
    if (i < nblk) row[i] = carry + ex;
    carry += chunk;
  }
  if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

// Ranks each element among equal digits of its tile (ballots per wavefront, counts per
// wavefront in LDS), stages the tile in LDS in digit order, then writes it out: the elements
// of one digit leave the tile as one contiguous run.
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
                                                           uint32_t* __restrict__ vout, int64_t n, int shift,
                                                           const uint32_t* __restrict__ hist,
                                                           const uint32_t* __restrict__ tot) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[kRsThreads / 64][256];
  __shared__ uint32_t start[256];  // first output position of the tile's elements of digit d
  __shared__ uint32_t lbase[256];  // first staging slot of digit d in the tile
  __shared__ uint32_t lk[kRsTile], lv[kRsTile];
  __shared__ uint32_t wtot[kRsThreads / 64];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t nblk = gridDim.x, blk = blockIdx.x;
  {
    // digit d's elements start at (all elements of smaller digits) + (digit d in earlier
    // tiles); inside the tile's staging copy at (the tile's elements of smaller digits)
    const uint32_t h0 = hist[int64_t(tid) * nblk + blk];
    const uint32_t h1 = blk + 1 < nblk ? hist[int64_t(tid) * nblk + blk + 1] : tot[tid];
    const uint32_t db = block_exclusive_256(tot[tid], wtot);
    const uint32_t lb = block_exclusive_256(h1 - h0, wtot);
    start[tid] = db + h0;
    run[tid] = db + h0;
    lbase[tid] = lb;
  }
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = blk * kRsTile;
  uint32_t kk[kRsRounds];  // the whole tile is loaded up front: one memory latency per tile
  uint32_t vv[kRsRounds];
#pragma unroll
  for (int r = 0; r < kRsRounds; ++r) {
    const int64_t j = base + int64_t(r) * kRsThreads + tid;
    kk[r] = j < n ? kin[j] : 0u;
    vv[r] = j < n ? vin[j] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kRsRounds; ++r) {
    for (int i = tid; i < (kRsThreads / 64) * 256; i += kRsThreads) (&wcnt[0][0])[i] = 0u;
    const int64_t j = base + int64_t(r) * kRsThreads + tid;
    const bool valid = j < n;
    const uint32_t k = kk[r];
    const uint32_t v = vv[r];
    const uint32_t d = uint32_t(k >> shift) & 255u;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      const uint64_t bb = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? bb : ~bb;
    }
    const uint32_t rank = __popcll(peers & lt);
    __syncthreads();
    if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t off = run[d] + rank;
      for (int w = 0; w < wave; ++w) off += wcnt[w][d];
      const uint32_t slot = off - start[d] + lbase[d];
      lk[slot] = k;
      lv[slot] = v;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kRsThreads / 64; ++w) add += wcnt[w][tid];
    run[tid] += add;
    __syncthreads();
  }
  const int64_t rem = n - base;
  const int cnt = int(rem < kRsTile ? rem : kRsTile);
  for (int i = tid; i < cnt; i += kRsThreads) {
    const uint32_t k = lk[i];
    const uint32_t d = (k >> shift) & 255u;
    const uint32_t out = start[d] + (uint32_t(i) - lbase[d]);
    kout[out] = k;
    vout[out] = lv[i];
  }
}

// sorts (keys, vals) by the low `bits` bits of keys; the result ends in whichever of the
// two buffers the last pass wrote, returned through *kres / *vres
int32_t radix_sort(uint32_t* keys, uint32_t* vals, int64_t n, int bits, uint32_t* ktmp, uint32_t* vtmp, uint32_t* hist,
                   uint32_t* tot, hipStream_t st, uint32_t** kres, uint32_t** vres) {
  uint32_t *ka = keys, *kb = ktmp;
  uint32_t *va = vals, *vb = vtmp;
  if (n > 1) {
    const int nblk = int((n + kRsTile - 1) / kRsTile);
    const int passes = (bits + 7) / 8;
    for (int ps = 0; ps < passes; ++ps) {
      const int shift = 8 * ps;
      hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(kRsThreads), 0, st, ka, n, shift, hist);
      hipLaunchKernelGGL(k_rs_scan_digit, dim3(256), dim3(kRsThreads), 0, st, hist, nblk, tot);
      hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(kRsThreads), 0, st, ka, va, kb, vb, n, shift, hist, tot);
      std::swap(ka, kb);
      std::swap(va, vb);
    }
  }
  *kres = ka;
  *vres = va;
  MPM_HIP(hipGetLastError());
  return MPM_OK;
}

__global__ void k_unpack_keys(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals, int64_t n,
                              int32_t* __restrict__ leaf, int64_t* __restrict__ perm) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    leaf[i] = int32_t(keys[i]);
    perm[i] = int64_t(vals[i]);
  }
}

// overlap classification in sorted order: number of leaves each domain overlaps
__global__ void k_classify(const double* __restrict__ x, const double* __restrict__ l, int64_t n,
                           const int64_t* __restrict__ perm, const int32_t* __restrict__ pleaf, LeafGeo G,
                           uint8_t* __restrict__ nleaf, DevErr* err) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t p = perm[i];
  double xp[3], lp[3];
  bool bad = false;
  for (int a = 0; a < 3; ++a) {
    xp[a] = x[a * n + p];
    lp[a] = l[a * n + p];
    bad |= !isfinite(lp[a]) || !(lp[a] > 0.0);
  }
  if (bad) {
    if (atomicCAS(&err->code, 0, MPM_ENONFINITE) == 0) err->index = i;
    nleaf[i] = 0;
    return;
  }
  int32_t lv[kMaxPointLeaves];
  const int c = domain_leaves(G, pleaf[i], xp, lp, lv);
  if (c < 0) {
    if (atomicCAS(&err->code, 0, c) == 0) err->index = i;
    nleaf[i] = 0;
    return;
  }
  nleaf[i] = uint8_t(c);
}

__global__ void k_strad_leaves(const double* __restrict__ x, const double* __restrict__ l, int64_t n,
                               const int64_t* __restrict__ perm, const int32_t* __restrict__ pleaf,
                               const int64_t* __restrict__ strad, int64_t ns, LeafGeo G, int32_t* __restrict__ out) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= ns) return;
  const int64_t i = strad[t], p = perm[i];
  double xp[3], lp[3];
  for (int a = 0; a < 3; ++a) {
    xp[a] = x[a * n + p];
    lp[a] = l[a * n + p];
  }
  int32_t lv[kMaxPointLeaves];
  const int c = domain_leaves(G, pleaf[i], xp, lp, lv);
  for (int k = 0; k < kMaxPointLeaves; ++k) out[t * kMaxPointLeaves + k] = k < c ? lv[k] : -1;
}

__global__ void k_permute(const int64_t* __restrict__ perm, const double* __restrict__ src, double* __restrict__ dst,
                          int64_t n, int ncomp) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t p = perm[i];
  for (int c = 0; c < ncomp; ++c) dst[c * n + i] = src[c * n + p];
}

// A random permutation of a [ncomp][n] array touches one cache line per component and
// point; staging a record-major copy makes each point's record one contiguous read. Both
// steps are instantiated per component count so that all loads of a thread are issued
// before the first wait.
// Step 1: tiled [ncomp][n] -> [n][ncomp] transpose through LDS (coalesced on both sides).
constexpr int kPermTile = 128, kPermMaxComp = 32;
//
// Permutations of points that moved little since the last sort are made of long runs of
// consecutive indices; then a direct gather is coalesced and moves half the bytes. A first
// kernel counts the run breaks on the device; the staged and the direct kernels are all
// launched and each returns at once unless the count selects it (no host round trip).
__global__ void k_perm_zero(unsigned long long* brk) { *brk = 0; }
// grid-stride count, one atomic per workgroup (atomics on one address serialise)
constexpr int kBreakBlocks = 1024;
__global__ __launch_bounds__(256) void k_perm_breaks(const int64_t* __restrict__ perm, int64_t n,
                                                     unsigned long long* brk) {
  __shared__ unsigned long long wsum[4];
  unsigned long long c = 0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x + 1; i < n; i += int64_t(gridDim.x) * blockDim.x)
    c += perm[i] != perm[i - 1] + 1;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long t = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (t) atomicAdd(brk, t);
  }
}
// direct mode: at most one run break per 64 points on average
__device__ __forceinline__ bool perm_direct(const unsigned long long* brk, int64_t n) {
  return (unsigned long long)(n / 64) >= *brk;
}
template <int NC>
__global__ __launch_bounds__(256) void k_permute_runs(const int64_t* __restrict__ perm, const double* __restrict__ src,
                                                      double* __restrict__ dst, int64_t n,
                                                      const unsigned long long* brk) {
  if (!perm_direct(brk, n)) return;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t p = perm[i];
  double v[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) v[c] = src[c * n + p];
#pragma unroll
  for (int c = 0; c < NC; ++c) dst[c * n + i] = v[c];
}

template <int NC>
__global__ __launch_bounds__(kPermTile) void k_soa_to_aos(const double* __restrict__ src, double* __restrict__ aos,
                                                          int64_t n, const unsigned long long* brk) {
  if (perm_direct(brk, n)) return;
  __shared__ double tile[NC * kPermTile];
  const int64_t p0 = int64_t(blockIdx.x) * kPermTile;
  const int t = threadIdx.x;
  const int cnt = int(n - p0 < kPermTile ? n - p0 : kPermTile);
  if (t < cnt) {
    double v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = src[c * n + p0 + t];
#pragma unroll
    for (int c = 0; c < NC; ++c) tile[t * NC + c] = v[c];
  }
  __syncthreads();
  double* out = aos + p0 * NC;
  if (cnt == kPermTile) {
    double v[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) v[q] = tile[q * kPermTile + t];
#pragma unroll
    for (int q = 0; q < NC; ++q) out[q * kPermTile + t] = v[q];
  } else {
    for (int j = t; j < cnt * NC; j += kPermTile) out[j] = tile[j];
  }
}
// Step 2: gather one record per sorted position, write component rows (coalesced).
template <int NC>
__global__ __launch_bounds__(256) void k_aos_gather(const int64_t* __restrict__ perm, const double* __restrict__ aos,
                                                    double* __restrict__ dst, int64_t n, const unsigned long long* brk) {
  if (perm_direct(brk, n)) return;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* r = aos + perm[i] * NC;
  if constexpr (NC % 2 == 0) {  // records start on 16-byte boundaries: 16-byte loads
    const double2* r2 = reinterpret_cast<const double2*>(r);
    double2 v[NC / 2];
#pragma unroll
    for (int c = 0; c < NC / 2; ++c) v[c] = r2[c];
#pragma unroll
    for (int c = 0; c < NC / 2; ++c) {
      dst[(2 * c) * n + i] = v[c].x;
      dst[(2 * c + 1) * n + i] = v[c].y;
    }
  } else {
    double v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = r[c];
#pragma unroll
    for (int c = 0; c < NC; ++c) dst[c * n + i] = v[c];
  }
}

template <int NC>
static void launch_permute(const int64_t* pm, const double* src, double* aos, double* dst, int64_t n,
                           const unsigned long long* brk, hipStream_t st) {
  hipLaunchKernelGGL(k_permute_runs<NC>, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, pm, src, dst, n, brk);
  hipLaunchKernelGGL(k_soa_to_aos<NC>, dim3(unsigned((n + kPermTile - 1) / kPermTile)), dim3(kPermTile), 0, st, src,
                     aos, n, brk);
  hipLaunchKernelGGL(k_aos_gather<NC>, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, pm, aos, dst, n, brk);
}

template <int... NC>
static bool dispatch_permute(int ncomp, const int64_t* pm, const double* src, double* aos, double* dst, int64_t n,
                             const unsigned long long* brk, hipStream_t st, std::integer_sequence<int, NC...>) {
  bool done = false;
  ((ncomp == NC + 2 ? (launch_permute<NC + 2>(pm, src, aos, dst, n, brk, st), done = true) : false), ...);
  return done;
}

LeafGeo make_geo(const mpm_mesh* m) {
  LeafGeo G;
  G.leaf = m->d_leaf;
  G.leaf_key = m->d_leaf_key;
  G.cellmap = m->d_cellmap;
  G.n_leaf = m->n_leaf;
  for (int a = 0; a < 3; ++a) G.lo[a] = m->crit.lo[a];
  G.hmin = m->hmin;
  G.lmax = m->crit.lvl_max;
  G.lat[0] = m->nx;
  G.lat[1] = m->ny;
  G.lat[2] = m->nz;
  return G;
}


// Copies the device error word to pinned host memory and waits for it by polling an event
// (a blocking stream synchronisation can leave the device idle for hundreds of microseconds
// after the work has finished, before the host thread is woken).
int32_t read_error(mpm_mesh* m, hipStream_t st, const char* what) {
  if (!m->h_err) MPM_HIP(hipHostMalloc((void**)&m->h_err, sizeof(DevErr), hipHostMallocDefault));
  if (!m->err_ev) MPM_HIP(hipEventCreateWithFlags(&m->err_ev, hipEventDisableTiming));
  MPM_HIP(hipMemcpyAsync(m->h_err, m->d_err, sizeof(DevErr), hipMemcpyDeviceToHost, st));
  MPM_HIP(hipEventRecord(m->err_ev, st));
  hipError_t q;
  while ((q = hipEventQuery(m->err_ev)) == hipErrorNotReady) {
  }
  if (q != hipSuccess) return hip_fail(q, what);
  const DevErr e = *m->h_err;
  if (e.code != 0) {
    static const char* names[] = {"", "bad argument", "det(dF) <= 0 or non-positive trial eigenvalue",
                                  "domain spans more than one leaf boundary per axis or key overflow",
                                  "point domain outside the mesh", "tree inconsistency", "HIP error",
                                  "non-finite input"};
    const int c = -e.code;
    set_error(e.code, std::string(what) + ": " + (c >= 0 && c < 8 ? names[c] : "error"), int64_t(e.index));
    MPM_HIP(hipMemsetAsync(m->d_err, 0, sizeof(DevErr), st));
    return e.code;
  }
  return MPM_OK;
}

int32_t read_word(mpm_mesh* m, const int64_t* d, int64_t* out, hipStream_t st, const char* what) {
  if (!m->h_word) MPM_HIP(hipHostMalloc((void**)&m->h_word, sizeof(int64_t), hipHostMallocDefault));
  if (!m->err_ev) MPM_HIP(hipEventCreateWithFlags(&m->err_ev, hipEventDisableTiming));
  MPM_HIP(hipMemcpyAsync(m->h_word, d, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  MPM_HIP(hipEventRecord(m->err_ev, st));
  hipError_t q;
  while ((q = hipEventQuery(m->err_ev)) == hipErrorNotReady) {
  }
  if (q != hipSuccess) return hip_fail(q, what);
  *out = *m->h_word;
  return MPM_OK;
}

// Grows a work buffer of the mesh to at least `bytes` (the old contents are dropped). The
// stream is drained first: work already queued may still read the old buffer.
int32_t ensure_buffer(void** buf, size_t* have, size_t bytes, hipStream_t st, const char* what) {
  if (*have >= bytes && *buf) return MPM_OK;
  MPM_HIP(hipStreamSynchronize(st));
  if (*buf) MPM_HIP(hipFree(*buf));
  *buf = nullptr;
  *have = 0;
  const hipError_t e = hipMalloc(buf, bytes);
  if (e != hipSuccess) {
    *buf = nullptr;
    return hip_fail(e, what);
  }
  *have = bytes;
  return MPM_OK;
}

// sort points (device x [3][n]) into perm / leaf with the mesh's leaves
int32_t sort_points(const mpm_mesh* mc, const double* dx, int64_t n, int64_t* perm, int32_t* leaf, hipStream_t st) {
  if (n == 0) return MPM_OK;
  if (n > int64_t(UINT32_MAX)) {
    set_error(MPM_EARG, "point sort: more than 2^32 - 1 points");
    return MPM_EARG;
  }
  mpm_mesh* m = const_cast<mpm_mesh*>(mc);
  const int bits = m->leaf_bits;
  const int nblk = int((n + kRsTile - 1) / kRsTile);
  const size_t na = (size_t(n) * 4 + 255) / 256 * 256;  // one 32-bit array, 256-byte aligned
  const size_t need = 4 * na + size_t(nblk) * 256 * 4 + 256 * 4;
  int32_t rc = ensure_buffer(&m->d_scratch, &m->scratch_bytes, need, st, "point sort: work buffer");
  if (rc) return rc;
  char* w = static_cast<char*>(m->d_scratch);
  uint32_t* keys = reinterpret_cast<uint32_t*>(w);
  uint32_t* ktmp = reinterpret_cast<uint32_t*>(w + na);
  uint32_t* vals = reinterpret_cast<uint32_t*>(w + 2 * na);
  uint32_t* vtmp = reinterpret_cast<uint32_t*>(w + 3 * na);
  uint32_t* hist = reinterpret_cast<uint32_t*>(w + 4 * na);
  uint32_t* tot = hist + size_t(nblk) * 256;
  const LeafGeo G = make_geo(m);
  hipLaunchKernelGGL(k_point_keys, dim3((n + 255) / 256), dim3(256), 0, st, dx, n, G, keys, vals, m->d_err);
  uint32_t* ks = nullptr;
  uint32_t* vs = nullptr;
  rc = radix_sort(keys, vals, n, bits, ktmp, vtmp, hist, tot, st, &ks, &vs);
  if (!rc) hipLaunchKernelGGL(k_unpack_keys, dim3((n + 255) / 256), dim3(256), 0, st, ks, vs, n, leaf, perm);
  if (!rc) MPM_HIP(hipGetLastError());
  return rc;
}

static bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

}  // namespace mpm

using namespace mpm;

extern "C" int32_t mpm_last_error(char* buf, size_t n) {
  if (buf && n) {
    std::strncpy(buf, g_msg.c_str(), n - 1);
    buf[n - 1] = 0;
  }
  return int32_t(g_msg.size());
}
extern "C" int64_t mpm_last_error_index(void) { return g_index; }

extern "C" void mpm_mesh_free(mpm_mesh_t* m) {
  if (!m) return;
  void* ptrs[] = {m->d_leaf, m->d_leaf_key, m->d_cell_nodes, m->d_cell_code, m->d_cell_cmat, m->d_node_ijk,
                  m->d_hang_ijk, m->d_hang_sup, m->d_hang_w, m->d_hang_owner, m->d_perm, m->d_pleaf, m->d_pnleaf,
                  m->d_row_ptr, m->d_col, m->d_wave_seg, m->d_leaf_seg0, m->d_leaf_nseg, m->d_con_off, m->d_con_seg, m->d_con_bp, m->d_bpos,
                  m->d_segK, m->d_segF, m->d_segM, m->d_red1, m->d_red2, m->d_strad, m->d_strad_leaf, m->d_grec, m->d_err,
                  m->d_partial, m->d_scratch, m->d_stage, m->d_cellmap, m->d_cg, m->d_gm, m->d_split, m->d_snode, m->d_srow, m->d_sinc_off, m->d_sinc, m->d_sup_off, m->d_sup_id, m->d_sup_src, m->d_sup_g, m->d_tpos, m->d_fidx, m->d_gorder, m->d_gf_leaf, m->d_gf_nodes,
                  m->d_gf_G, m->d_gf_h, m->d_gf_sc, m->d_gf_bpos, m->d_gnode, m->d_gcon_off, m->d_gcon, m->d_gbeta, m->d_gsegmax};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (hipEvent_t e : m->ev)
    if (e) (void)hipEventDestroy(e);
  if (m->h_err) (void)hipHostFree(m->h_err);
  if (m->err_ev) (void)hipEventDestroy(m->err_ev);
  if (m->h_cg) (void)hipHostFree(m->h_cg);
  if (m->h_word) (void)hipHostFree(m->h_word);
  if (m->cg_ev) (void)hipEventDestroy(m->cg_ev);
  if (m->side) {
    (void)hipStreamSynchronize(m->side);
    (void)hipStreamDestroy(m->side);
  }
  if (m->fork_ev) (void)hipEventDestroy(m->fork_ev);
  if (m->join_ev) (void)hipEventDestroy(m->join_ev);
  delete m;
}

extern "C" int32_t octree_build(const mpm_refine_t* crit, const double* x, const double* l, int64_t n, void* stream,
                                mpm_mesh_t** out_mesh) {
  if (!crit || !out_mesh || n < 0 || (n > 0 && (!x || !l))) {
    set_error(MPM_EARG, "octree_build: null argument or negative n");
    return MPM_EARG;
  }
  *out_mesh = nullptr;
  // criterion checks come before any device call
  if (crit->lvl_max < crit->lvl_base || crit->lvl_max - crit->lvl_base > 13 || !(crit->h0 > 0) ||
      !std::isfinite(crit->h0) || crit->base[0] <= 0 || crit->base[1] <= 0 || crit->base[2] <= 0 ||
      crit->lvl_base < 0 || crit->lvl_max > 31 || crit->body_kind < MPM_BODY_NONE || crit->body_kind > MPM_BODY_BOX ||
      !std::isfinite(crit->dx_region) || crit->dx_region < 0.0) {
    set_error(MPM_EARG, "octree_build: bad refinement levels, base grid, h0, body kind or dx_region");
    return MPM_EARG;
  }
  for (int a = 0; a < 3; ++a)
    if (int64_t(crit->base[a]) << (crit->lvl_max - crit->lvl_base) >= (int64_t(1) << 13)) {
      set_error(MPM_ESTENCIL, "octree_build: finest lattice exceeds 8191 cells per axis");
      return MPM_ESTENCIL;
    }
  hipStream_t st = (hipStream_t)stream;
  mpm_mesh* m = new mpm_mesh();
  m->crit = *crit;
  if (hipMalloc(&m->d_err, sizeof(DevErr)) != hipSuccess || hipMemsetAsync(m->d_err, 0, sizeof(DevErr), st) != hipSuccess) {
    mpm_mesh_free(m);
    return hip_fail(hipErrorOutOfMemory, "octree_build: error word");
  }
  int32_t rc = gpu_build_tree(m, *crit, st);
  if (rc) {
    mpm_mesh_free(m);
    return rc;
  }
  while ((int64_t(1) << m->leaf_bits) < m->n_leaf + 1) ++m->leaf_bits;
  if (m->leaf_bits > 31) {
    set_error(MPM_ESTENCIL, "octree_build: too many leaves for 32-bit point keys");
    mpm_mesh_free(m);
    return MPM_ESTENCIL;
  }
  // dense leaf map of the finest cells when it takes at most 1 GiB (else the leaf search
  // bisects the sorted leaf keys)
  const int64_t ncell = int64_t(m->nx) * m->ny * m->nz;
  if (ncell > 0 && ncell <= (int64_t(1) << 28) && m->n_leaf > 0) {
    if (hipMalloc(&m->d_cellmap, size_t(ncell) * 4) != hipSuccess ||
        hipMemsetAsync(m->d_cellmap, 0xff, size_t(ncell) * 4, st) != hipSuccess) {
      mpm_mesh_free(m);
      return hip_fail(hipErrorOutOfMemory, "octree_build: cell map");
    }
    hipLaunchKernelGGL(k_fill_cellmap, dim3(unsigned(m->n_leaf)), dim3(256), 0, st, m->d_leaf, crit->lvl_max, m->nx,
                       m->ny, m->d_cellmap);
  }
  m->n_point = n;
  const double *dx = x, *dl = l;
  DevBuf tx, tl;
  if (n > 0) {
    if (!is_device_ptr(x) || !is_device_ptr(l)) {
      if ((rc = tx.alloc(size_t(3 * n) * 8, "octree_build: point upload")) ||
          (rc = tl.alloc(size_t(3 * n) * 8, "octree_build: point upload"))) {
        mpm_mesh_free(m);
        return rc;
      }
      (void)hipMemcpyAsync(tx.p, x, size_t(3 * n) * 8, hipMemcpyHostToDevice, st);
      (void)hipMemcpyAsync(tl.p, l, size_t(3 * n) * 8, hipMemcpyHostToDevice, st);
      dx = tx.as<double>();
      dl = tl.as<double>();
    }
    hipError_t e = hipMalloc(&m->d_perm, size_t(n) * 8);
    if (e == hipSuccess) e = hipMalloc(&m->d_pleaf, size_t(n) * 4);
    if (e == hipSuccess) e = hipMalloc(&m->d_pnleaf, size_t(n));
    if (e != hipSuccess) {
      mpm_mesh_free(m);
      return hip_fail(e, "octree_build: point arrays");
    }
    rc = sort_points(m, dx, n, m->d_perm, m->d_pleaf, st);
    if (!rc) rc = read_error(m, st, "octree_build (point keys)");
    if (!rc) {
      const LeafGeo G = make_geo(m);
      hipLaunchKernelGGL(k_classify, dim3((n + 255) / 256), dim3(256), 0, st, dx, dl, n, m->d_perm, m->d_pleaf, G,
                         m->d_pnleaf, m->d_err);
      rc = read_error(m, st, "octree_build (domain overlaps)");
    }
    if (rc) {
      mpm_mesh_free(m);
      return rc;
    }
  }
  // pattern, segments, records and contribution lists of the points
  rc = gpu_build_pattern(m, dx, dl, st);
  if (!rc) rc = read_error(m, st, "octree_build (pattern)");
  if (rc) {
    (void)hipStreamSynchronize(st);
    mpm_mesh_free(m);
    return rc;
  }
  *out_mesh = m;
  return MPM_OK;
}

namespace mpm {
int32_t strad_leaves(mpm_mesh* m, const double* dx, const double* dl, hipStream_t st) {
  const LeafGeo G = make_geo(m);
  hipLaunchKernelGGL(k_strad_leaves, dim3(unsigned((m->n_straddle + 255) / 256)), dim3(256), 0, st, dx, dl,
                     m->n_point, m->d_perm, m->d_pleaf, m->d_strad, m->n_straddle, G, m->d_strad_leaf);
  MPM_HIP(hipGetLastError());
  return MPM_OK;
}

}  // namespace mpm

extern "C" int32_t mpm_mesh_info(const mpm_mesh_t* m, mpm_mesh_info_t* o) {
  if (!m || !o) {
    set_error(MPM_EARG, "mpm_mesh_info: null argument");
    return MPM_EARG;
  }
  o->n_leaf = m->n_leaf;
  o->n_node = m->n_node;
  o->n_hang = m->n_hang;
  o->n_dof = 3 * m->n_node;
  o->nnz = m->nnz;
  o->n_point = m->n_point;
  o->n_straddle = m->n_straddle;
  o->n_active_rows = m->n_active_rows;
  o->max_support = m->max_support;
  o->lattice[0] = m->nx;
  o->lattice[1] = m->ny;
  o->lattice[2] = m->nz;
  o->h_min = m->hmin;
  o->n_ghost_face = m->n_gface;
  return MPM_OK;
}

extern "C" int32_t mpm_ghost_faces(const mpm_mesh_t* m, int32_t* out) {
  if (!m || (!out && m->n_gface)) {
    set_error(MPM_EARG, "mpm_ghost_faces: null argument");
    return MPM_EARG;
  }
  if (m->n_gface) std::memcpy(out, m->h_gface.data(), m->h_gface.size() * sizeof(int32_t));
  return MPM_OK;
}

extern "C" int32_t mpm_mesh_arrays(const mpm_mesh_t* m, mpm_mesh_arrays_t* o) {
  if (!m || !o) {
    set_error(MPM_EARG, "mpm_mesh_arrays: null argument");
    return MPM_EARG;
  }
  o->leaf = m->d_leaf;
  o->node_ijk = m->d_node_ijk;
  o->hang_ijk = m->d_hang_ijk;
  o->hang_support = m->d_hang_sup;
  o->hang_weight = m->d_hang_w;
  o->hang_owner = m->d_hang_owner;
  o->cell_nodes = m->d_cell_nodes;
  o->cell_cmat = m->d_cell_cmat;
  o->perm = m->d_perm;
  o->point_leaf = m->d_pleaf;
  o->point_nleaf = m->d_pnleaf;
  o->row_ptr = m->d_row_ptr;
  o->col = m->d_col;
  return MPM_OK;
}

extern "C" int32_t mpm_point_sort(const mpm_mesh_t* m, const double* x, int64_t n, int64_t* perm_out,
                                  int32_t* leaf_out, void* stream) {
  if (!m || n != m->n_point || (n > 0 && (!x || !perm_out || !leaf_out))) {
    set_error(MPM_EARG, "mpm_point_sort: null argument or n differs from the mesh's point count");
    return MPM_EARG;
  }
  hipStream_t st = (hipStream_t)stream;
  int32_t rc = sort_points(m, x, n, perm_out, leaf_out, st);
  return rc;
}

extern "C" int32_t mpm_permute(const mpm_mesh_t* m, const int64_t* perm, const double* src, double* dst,
                               int32_t ncomp, void* stream) {
  if (!m || ncomp <= 0 || (m->n_point > 0 && (!src || !dst))) {
    set_error(MPM_EARG, "mpm_permute: null argument");
    return MPM_EARG;
  }
  const int64_t n = m->n_point;
  if (n == 0) return MPM_OK;
  hipStream_t st = (hipStream_t)stream;
  const int64_t* pm = perm ? perm : m->d_perm;
  mpm_mesh* mm = const_cast<mpm_mesh*>(m);
  if (ncomp >= 2 && ncomp <= kPermMaxComp &&
      ensure_buffer(&mm->d_stage, &mm->stage_bytes, size_t(n) * ncomp * 8 + 256, st, "mpm_permute: staging") ==
          MPM_OK) {
    // the run-break counter sits after the staging copy
    double* aos = static_cast<double*>(mm->d_stage);
    unsigned long long* brk = reinterpret_cast<unsigned long long*>(aos + size_t(n) * ncomp);
    hipLaunchKernelGGL(k_perm_zero, dim3(1), dim3(1), 0, st, brk);
    hipLaunchKernelGGL(k_perm_breaks, dim3(unsigned(std::min<int64_t>(kBreakBlocks, (n + 255) / 256))), dim3(256), 0,
                       st, pm, n, brk);
    dispatch_permute(ncomp, pm, src, aos, dst, n, brk, st, std::make_integer_sequence<int, kPermMaxComp - 1>{});
  } else {
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_permute, dim3((n + 255) / 256), dim3(256), 0, st, pm, src, dst, n, ncomp);
  }
  MPM_HIP(hipGetLastError());
  return MPM_OK;
}

extern "C" int32_t mpm_kernel_timing(mpm_mesh_t* m, int32_t enable, double* ms_out) {
  if (!m || enable < -1 || enable > 1) {
    set_error(MPM_EARG, "mpm_kernel_timing: null mesh or bad flag");
    return MPM_EARG;
  }
  if (enable == 1 && !m->ev[0])
    for (auto& e : m->ev) MPM_HIP(hipEventCreate(&e));
  if (enable >= 0) m->timing = enable == 1;
  if (ms_out) {
    ms_out[0] = m->t_asm;
    ms_out[1] = double(m->n_asm);
    ms_out[2] = m->t_adj;
    ms_out[3] = double(m->n_adj);
    ms_out[4] = m->t_gat;
    ms_out[5] = double(m->n_gat);
    m->t_asm = m->t_adj = m->t_gat = 0;
    m->n_asm = m->n_adj = m->n_gat = 0;
  }
  return MPM_OK;
}
