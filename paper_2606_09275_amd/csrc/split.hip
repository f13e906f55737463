// GIMP refinement of the adaptive strategy (Section 5). The criterion splits a GIMP when a
// leaf its domain overlaps (positive volume) has half side l_K < beta l_p, l_p the largest
// of the domain's three half sides. A split GIMP becomes 8 GIMPs that tile its domain: child
// c sits at x_a + s_a l_a / 2 (s_a = +1 if bit a of c is set, else -1) with half sides l / 2,
// volume and mass / 8; data constant over the domain is copied; data defined by the
// reference position is evaluated at the child's reference position X + F_n^{-1} (x_c - x)
// (F constant over the domain makes the current-to-reference map affine there).
//
// The output keeps the input order (a point, or its 8 children in child order): blocks of
// 256 points count their splits, one workgroup scans the block counts, each block then scans
// its own points to place their first outputs, and one thread per output point finds its
// parent by bisection of those offsets and writes every field (coalesced stores).
#include "geom.h"

namespace mpm {

constexpr int kSplitBlock = 256;

// The criterion only needs to know whether the domain overlaps a leaf finer than L*, the
// finest level whose leaves are large enough (0.5 h_L >= beta l_p; the condition is monotone
// in the level). Leaves of level <= L* are unions of level-L* lattice cells, so the domain
// overlaps a finer leaf iff one of the level-L* cells it overlaps with positive volume lies in
// a leaf of a level above L* (the cell is subdivided, and the leaves inside it cover the
// overlapped part). The domain is at most S / beta wide for cells of side S, so a few cells
// per axis are checked, each by the leaf holding its first finest cell.
constexpr int kSplitMaxCells = 4096;

__device__ int split_flag(const LeafGeo& G, int lbase, const double x[3], const double l[3], double beta) {
#pragma clang fp contract(off)
  const double lmax = fmax(fmax(l[0], l[1]), l[2]);
  double thr[3], a0[3], a1[3];
  for (int a = 0; a < 3; ++a) {
    a0[a] = x[a] - l[a];
    a1[a] = x[a] + l[a];
    thr[a] = 1e-12 * (2.0 * l[a]);
    const double mlo = G.lo[a], mhi = G.lo[a] + double(G.lat[a]) * G.hmin;
    if (mlo - a0[a] > thr[a] || a1[a] - mhi > thr[a]) return MPM_EOUTSIDE;
  }
  int Ls = lbase - 1;  // finest level whose leaves do not trigger the split
  for (int L = lbase; L <= G.lmax; ++L)
    if (!(0.5 * double(1 << (G.lmax - L)) * G.hmin < beta * lmax)) Ls = L;
  if (Ls >= G.lmax) return 0;  // no leaf is small enough to split the point
  if (Ls < lbase) return 1;    // every leaf is (the domain overlaps at least one)
  const int s = 1 << (G.lmax - Ls);
  const double S = double(s) * G.hmin;
  int c0[3], c1[3];
  int64_t ncell = 1;
  for (int a = 0; a < 3; ++a) {
    const int nc = G.lat[a] / s;
    c0[a] = int(floor((a0[a] - G.lo[a]) / S));
    c1[a] = int(floor((a1[a] - G.lo[a]) / S));
    c0[a] = c0[a] < 0 ? 0 : (c0[a] > nc - 1 ? nc - 1 : c0[a]);
    c1[a] = c1[a] < 0 ? 0 : (c1[a] > nc - 1 ? nc - 1 : c1[a]);
    ncell *= int64_t(c1[a] - c0[a] + 1);
  }
  if (ncell > kSplitMaxCells) return MPM_ESTENCIL;
  for (int k = c0[2]; k <= c1[2]; ++k)
    for (int j = c0[1]; j <= c1[1]; ++j)
      for (int i = c0[0]; i <= c1[0]; ++i) {
        const int c[3] = {i, j, k};
        bool pos = true;
        for (int a = 0; a < 3; ++a) {
          const double lo = G.lo[a] + double(c[a]) * S, hi = lo + S;
          const double o = (a1[a] < hi ? a1[a] : hi) - (a0[a] > lo ? a0[a] : lo);
          pos = pos && o > thr[a];
        }
        if (!pos) continue;
        const double p0 = G.lo[0] + (double(i * s) + 0.5) * G.hmin, p1 = G.lo[1] + (double(j * s) + 0.5) * G.hmin,
                     p2 = G.lo[2] + (double(k * s) + 0.5) * G.hmin;
        const int64_t e = leaf_of_point(G, p0, p1, p2);
        if (G.leaf[4 * e + 3] > Ls) return 1;
      }
  return 0;
}

__global__ __launch_bounds__(kSplitBlock) void k_split_mark(const double* __restrict__ x, const double* __restrict__ l,
                                                            int64_t n, double beta, LeafGeo G, int lbase,
                                                            uint8_t* __restrict__ split, int64_t* __restrict__ blk,
                                                            DevErr* err) {
  __shared__ int wsum[kSplitBlock / 64];
  const int64_t i = int64_t(blockIdx.x) * kSplitBlock + threadIdx.x;
  int s = 0;
  if (i < n) {
    double xp[3], lp[3];
    bool bad = false;
    for (int a = 0; a < 3; ++a) {
      xp[a] = x[a * n + i];
      lp[a] = l[a * n + i];
      bad |= !isfinite(xp[a]) || !isfinite(lp[a]) || !(lp[a] > 0.0);
    }
    if (bad) {
      if (atomicCAS(&err->code, 0, MPM_ENONFINITE) == 0) err->index = i;
    } else {
      const int f = split_flag(G, lbase, xp, lp, beta);
      if (f < 0) {
        if (atomicCAS(&err->code, 0, f) == 0) err->index = i;
      } else {
        s = f;
      }
    }
    split[i] = uint8_t(s);
  }
  int v = s;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kSplitBlock / 64; ++w) t += wsum[w];
    blk[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kSplitBlock) void k_split_count(const uint8_t* __restrict__ split, int64_t n,
                                                             int64_t* __restrict__ blk) {
  __shared__ int wsum[kSplitBlock / 64];
  const int64_t i = int64_t(blockIdx.x) * kSplitBlock + threadIdx.x;
  int v = i < n ? int(split[i] != 0) : 0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kSplitBlock / 64; ++w) t += wsum[w];
    blk[blockIdx.x] = t;
  }
}

// exclusive scan of nb block counts in place; blk[nb] receives the total
__global__ __launch_bounds__(1024) void k_split_scan(int64_t* blk, int64_t nb) {
  __shared__ int64_t wtot[16];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t base = 0; base < nb; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = i < nb ? blk[i] : 0;
    int64_t inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t o = __shfl_up(inc, off);
      if (lane >= off) inc += o;
    }
    if (lane == 63) wtot[wv] = inc;
    __syncthreads();
    int64_t pre = carry;
    for (int w = 0; w < wv; ++w) pre += wtot[w];
    if (i < nb) blk[i] = pre + inc - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry = pre + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) blk[nb] = carry;
}

struct SplitIO {
  mpm_state_t in;
  const double *X, *v;
  mpm_state_out_t out;
  double *Xo, *vo;
  double props[12];
  int32_t mask;
  int64_t n, n_out;
};

// first output of every input point (offs[n] = n_out): the block offset of the counts scan
// plus the point's rank inside its block
__global__ __launch_bounds__(kSplitBlock) void k_split_offsets(const uint8_t* __restrict__ split, int64_t n,
                                                               const int64_t* __restrict__ blk,
                                                               int64_t* __restrict__ offs, int64_t nb) {
  __shared__ int wtot[kSplitBlock / 64];
  const int64_t i = int64_t(blockIdx.x) * kSplitBlock + threadIdx.x;
  const int cnt = i < n ? (split[i] != 0 ? 8 : 1) : 0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int inc = cnt;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(inc, off);
    if (lane >= off) inc += o;
  }
  if (lane == 63) wtot[wv] = inc;
  __syncthreads();
  int pre = 0;
  for (int w = 0; w < wv; ++w) pre += wtot[w];
  // outputs before this block: its points, plus 7 per split among them
  if (i < n) offs[i] = int64_t(blockIdx.x) * kSplitBlock + 7 * blk[blockIdx.x] + pre + inc - cnt;
  if (i == 0) offs[n] = n + 7 * blk[nb];
}

// parent input point of every output point: input i owns outputs offs[i] .. offs[i + 1] - 1
__global__ __launch_bounds__(256) void k_split_parent(const int64_t* __restrict__ offs, int64_t n,
                                                      int64_t* __restrict__ parent) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o0 = offs[i], o1 = offs[i + 1];
  for (int64_t o = o0; o < o1; ++o) parent[o] = i;
}

// One thread per output point (coalesced stores): its parent from k_split_parent, its child
// index the distance to the parent's first output.
__global__ __launch_bounds__(256) void k_split_emit(SplitIO io, const uint8_t* __restrict__ split,
                                                    const int64_t* __restrict__ offs,
                                                    const int64_t* __restrict__ parent) {
  const int64_t n = io.n, n_out = io.n_out;
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n_out) return;
  const int64_t i = parent[j];
  const int c = int(j - offs[i]);
  const bool s = split[i] != 0;
  const mpm_state_t& S = io.in;
  const mpm_state_out_t& D = io.out;
  // data constant over the domain
  if (D.Jn) D.Jn[j] = S.Jn[i];
  if (D.bn)
    for (int k = 0; k < 6; ++k) D.bn[k * n_out + j] = S.bn[k * n + i];
  if (D.Fn)
    for (int k = 0; k < 9; ++k) D.Fn[k * n_out + j] = S.Fn[k * n + i];
  if (io.vo)
    for (int k = 0; k < 3; ++k) io.vo[k * n_out + j] = io.v[k * n + i];
  const double* prm[3] = {S.E, S.nu, S.sy};
  double* prmo[3] = {D.E, D.nu, D.sy};
  if (!s) {
    for (int a = 0; a < 3; ++a) {
      D.x[a * n_out + j] = S.x[a * n + i];
      D.l[a * n_out + j] = S.l[a * n + i];
      if (io.Xo) io.Xo[a * n_out + j] = io.X[a * n + i];
    }
    D.vol[j] = S.vol[i];
    D.mass[j] = S.mass[i];
    for (int r = 0; r < 3; ++r)
      if (prmo[r]) prmo[r][j] = prm[r][i];
    return;
  }
  double d[3];
  for (int a = 0; a < 3; ++a) {
    const double xp = S.x[a * n + i], h = 0.5 * S.l[a * n + i];
    d[a] = ((c >> a) & 1) ? h : -h;
    D.x[a * n_out + j] = xp + d[a];
    D.l[a * n_out + j] = h;
  }
  D.vol[j] = S.vol[i] * 0.125;
  D.mass[j] = S.mass[i] * 0.125;
  double Xc[3] = {0.0, 0.0, 0.0};
  if (io.Xo) {
    double F[9];
    for (int k = 0; k < 9; ++k) F[k] = S.Fn[k * n + i];
    // inverse by cofactors (F row-major)
    const double c00 = F[4] * F[8] - F[5] * F[7], c01 = F[5] * F[6] - F[3] * F[8], c02 = F[3] * F[7] - F[4] * F[6];
    const double det = F[0] * c00 + F[1] * c01 + F[2] * c02, r = 1.0 / det;
    double Fi[9];
    Fi[0] = c00 * r;
    Fi[3] = c01 * r;
    Fi[6] = c02 * r;
    Fi[1] = (F[2] * F[7] - F[1] * F[8]) * r;
    Fi[4] = (F[0] * F[8] - F[2] * F[6]) * r;
    Fi[7] = (F[1] * F[6] - F[0] * F[7]) * r;
    Fi[2] = (F[1] * F[5] - F[2] * F[4]) * r;
    Fi[5] = (F[2] * F[3] - F[0] * F[5]) * r;
    Fi[8] = (F[0] * F[4] - F[1] * F[3]) * r;
    for (int a = 0; a < 3; ++a) {
      Xc[a] = io.X[a * n + i] + (Fi[3 * a] * d[0] + Fi[3 * a + 1] * d[1] + Fi[3 * a + 2] * d[2]);
      io.Xo[a * n_out + j] = Xc[a];
    }
  }
  for (int r = 0; r < 3; ++r) {
    if (!prmo[r]) continue;
    if ((io.mask >> r) & 1) {
      const double* q = io.props + 4 * r;
      prmo[r][j] = q[0] + q[1] * Xc[0] + q[2] * Xc[1] + q[3] * Xc[2];
    } else {
      prmo[r][j] = prm[r][i];
    }
  }
}

// work buffer: nb + 1 block counts, then (apply) n + 1 output offsets
static int32_t split_buffers(mpm_mesh* m, int64_t nb, int64_t n_offs, hipStream_t st) {
  return ensure_buffer(&m->d_split, &m->split_bytes, size_t(nb + 1 + n_offs) * 8, st, "GIMP split: work buffer");
}

}  // namespace mpm

using namespace mpm;

extern "C" int32_t mpm_split_mark(const mpm_mesh_t* mc, const double* x, const double* l, int64_t n, double beta,
                                  uint8_t* split, int64_t* n_split, void* stream) {
  if (!mc || n < 0 || (n > 0 && (!x || !l || !split)) || !n_split || !std::isfinite(beta) || !(beta > 0.0)) {
    set_error(MPM_EARG, "mpm_split_mark: null argument, negative n or bad beta");
    return MPM_EARG;
  }
  *n_split = 0;
  if (n == 0) return MPM_OK;
  mpm_mesh* m = const_cast<mpm_mesh*>(mc);
  hipStream_t st = (hipStream_t)stream;
  const int64_t nb = (n + kSplitBlock - 1) / kSplitBlock;
  if (nb > int64_t(UINT32_MAX)) {
    set_error(MPM_EARG, "mpm_split_mark: too many points");
    return MPM_EARG;
  }
  if (const int32_t rc = split_buffers(m, nb, 0, st)) return rc;
  int64_t* blk = static_cast<int64_t*>(m->d_split);
  hipLaunchKernelGGL(k_split_mark, dim3(unsigned(nb)), dim3(kSplitBlock), 0, st, x, l, n, beta, make_geo(m),
                     int(m->crit.lvl_base), split, blk, m->d_err);
  hipLaunchKernelGGL(k_split_scan, dim3(1), dim3(1024), 0, st, blk, nb);
  MPM_HIP(hipGetLastError());
  if (const int32_t rc = read_error(m, st, "mpm_split_mark")) return rc;
  return read_word(m, blk + nb, n_split, st, "mpm_split_mark: count");
}

extern "C" int32_t mpm_split_apply(const mpm_mesh_t* mc, int64_t n, const uint8_t* split, const mpm_state_t* in,
                                   const double* X_in, const double* v_in, const double* props, int32_t prop_mask,
                                   const mpm_state_out_t* out, double* X_out, double* v_out, int64_t n_out,
                                   void* stream) {
  const bool need_state = n > 0 && (!split || !in || !out || !in->x || !in->l || !in->vol || !in->mass || !out->x ||
                                    !out->l || !out->vol || !out->mass);
  const bool opt_bad = n > 0 && !need_state &&
                       ((!in->Jn != !out->Jn) || (!in->bn != !out->bn) || (!in->Fn != !out->Fn) ||
                        (!in->E != !out->E) || (!in->nu != !out->nu) || (!in->sy != !out->sy) ||
                        (!X_in != !X_out) || (!v_in != !v_out));
  const bool prop_bad = n > 0 && !need_state && prop_mask &&
                        (!props || !X_in || !in->Fn || ((prop_mask & 1) && !in->E) || ((prop_mask & 2) && !in->nu) ||
                         ((prop_mask & 4) && !in->sy));
  const bool ref_bad = n > 0 && !need_state && X_in && !in->Fn;
  if (!mc || n < 0 || n_out < n || need_state || opt_bad || prop_bad || ref_bad || (prop_mask & ~7)) {
    set_error(MPM_EARG, "mpm_split_apply: null or unpaired argument, bad sizes, reference positions "
                        "without F_n, or reference-position parameters without X");
    return MPM_EARG;
  }
  if (n == 0) return MPM_OK;
  mpm_mesh* m = const_cast<mpm_mesh*>(mc);
  hipStream_t st = (hipStream_t)stream;
  const int64_t nb = (n + kSplitBlock - 1) / kSplitBlock;
  if (n_out < n || n_out > 8 * n) {
    set_error(MPM_EARG, "mpm_split_apply: n_out differs from n + 7 * (flagged points)");
    return MPM_EARG;
  }
  if (const int32_t rc = split_buffers(m, nb, n + 1 + n_out, st)) return rc;
  int64_t* blk = static_cast<int64_t*>(m->d_split);
  int64_t* offs = blk + nb + 1;
  int64_t* parent = offs + n + 1;
  // block counts of the flags (the scan of the marking call may belong to other flags)
  hipLaunchKernelGGL(k_split_count, dim3(unsigned(nb)), dim3(kSplitBlock), 0, st, split, n, blk);
  hipLaunchKernelGGL(k_split_scan, dim3(1), dim3(1024), 0, st, blk, nb);
  int64_t total = 0;
  if (const int32_t rc = read_word(m, blk + nb, &total, st, "mpm_split_apply: count")) return rc;
  if (n + 7 * total != n_out) {
    set_error(MPM_EARG, "mpm_split_apply: n_out differs from n + 7 * (flagged points)");
    return MPM_EARG;
  }
  SplitIO io;
  io.in = *in;
  io.X = X_in;
  io.v = v_in;
  io.out = *out;
  io.Xo = X_out;
  io.vo = v_out;
  for (int k = 0; k < 12; ++k) io.props[k] = prop_mask ? props[k] : 0.0;
  io.mask = prop_mask;
  io.n = n;
  io.n_out = n_out;
  hipLaunchKernelGGL(k_split_offsets, dim3(unsigned(nb)), dim3(kSplitBlock), 0, st, split, n, blk, offs, nb);
  hipLaunchKernelGGL(k_split_parent, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, offs, n, parent);
  hipLaunchKernelGGL(k_split_emit, dim3(unsigned((n_out + 255) / 256)), dim3(256), 0, st, io, split, offs, parent);
  MPM_HIP(hipGetLastError());
  return read_error(m, st, "mpm_split_apply");
}
