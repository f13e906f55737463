// Assembly kernels: fused per-point GIMP basis -> kinematics -> Hencky/von Mises return ->
// consistent tangent -> per-leaf segmented reduction in LDS -> segment records -> (records
// of heavily populated leaves summed) -> one workgroup per node row writes f_int and the CSR
// values; rows gathered from per-node lists of the points whose domain overlaps several
// leaves; body force; residual and its FP64 norm; the adjoint gather.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "point_math.h"

namespace mpm {

struct AsmArgs {
  LeafGeo G;
  const int32_t* cell_nodes;
  const int32_t* cell_code;
  const int32_t* pleaf;
  const uint8_t* pnleaf;
  const int32_t* wave_seg;
  const int32_t* gorder;     // the row gather's node order (null: ascending)
  const int32_t* leaf_seg0;
  const int32_t* leaf_nseg;
  const int32_t* con_off;
  const int32_t* con_seg;
  const int32_t* con_bp;
  const int16_t* bpos;
  void* segK;
  double* segF;
  void* segM;  // inertia: per record the 36 sums of (2 m / dt^2) S_a S_b (a <= b), or null
  const int64_t* row_ptr;
  const int32_t* col;
  const int64_t* strad;
  const int64_t* fidx;       // points whose domain lies in one leaf, in sorted order (null: all points)
  const int32_t* strad_leaf;
  const int32_t* snode;      // rows reached by straddling points
  const int32_t* srow;       // their launch order (indices into snode)
  const int64_t* sinc_off;   // per such row: its straddling points
  const int32_t* sinc;
  double* grec;              // per straddling point: tangent record of the general path
  const int64_t* sup_off;    // per straddling point: its support slots
  const int32_t* sup_id;     // node of each slot
  const uint32_t* sup_src;   // leaves of the point holding the slot's node, and its vertex in each
  double* sup_g;             // per slot: S and the spatial gradient (written by k_general_support)
  const int32_t* tpos;       // per block of those rows above the diagonal: column of the row's node in the
                             // row of the block's node
  int64_t n, n_strad, n_fast;
  mpm_state_t s;
  const double* u;
  const double* lam;  // adjoint
  double* f;
  void* K;
  double* sigma;
  double* Fnew;
  double* be;
  double *dE, *dnu, *dsy, *dV;
  // Newmark inertia (gamma = 1, beta = 1/2): point velocities at the start of the step [3][n]
  // (null: quasi-static), step size, optional point accelerations / velocities out [3][n]
  const double* vel;
  double dt;
  double* a_new;
  double* v_new;
  DevErr* err;
};

__device__ __forceinline__ void raise(DevErr* err, int code, int64_t idx) {
  if (atomicCAS(&err->code, 0, code) == 0) err->index = (unsigned long long)idx;
}

// Basis of a point over one leaf overlap box, accumulated into the 8 slots of that leaf.
template <typename T>
__device__ __forceinline__ void leaf_overlap_basis(const LeafGeo& G, int64_t e, int32_t code, const double x[3],
                                                   const double l[3], T S[8], T dS[8][3]) {
  double lo[3], hi[3], h;
  leaf_bounds(G, e, lo, hi, &h);
  double ctr[3], wgt = 1.0;
  for (int a = 0; a < 3; ++a) {
    const double a0 = x[a] - l[a] > lo[a] ? x[a] - l[a] : lo[a];
    const double a1 = x[a] + l[a] < hi[a] ? x[a] + l[a] : hi[a];
    ctr[a] = 0.5 * (a0 + a1);
    wgt *= (a1 - a0) / (2.0 * l[a]);
  }
  T xi[3];
  for (int a = 0; a < 3; ++a) xi[a] = T((ctr[a] - lo[a]) / h);
  slot_basis<T>(xi, T(1.0 / h), code, T(wgt), S, dS);
}

template <typename T>
__device__ __forceinline__ void load_B(const mpm_state_t& s, int64_t n, int64_t i, T B[3][3]) {
  const double b0 = s.bn[i], b1 = s.bn[n + i], b2 = s.bn[2 * n + i];
  const double b3 = s.bn[3 * n + i], b4 = s.bn[4 * n + i], b5 = s.bn[5 * n + i];
  B[0][0] = T(b0 - 1.0);
  B[1][1] = T(b1 - 1.0);
  B[2][2] = T(b2 - 1.0);
  B[0][1] = B[1][0] = T(b3);
  B[1][2] = B[2][1] = T(b4);
  B[0][2] = B[2][0] = T(b5);
}

// write sigma and (optionally) the committed state of one point: the elastic left
// Cauchy-Green tensor b_e = sum_a exp(2 eps_e,a) n_a n_a^T of the returned elastic strains
// (Section 2.2) and F_new = dF F_n (Section 2.1, updated Lagrangian). Both are formed from
// their increments so that the FP32 working precision costs relative accuracy of the strain,
// not of the unit tensor: b_e = I + sum_a expm1(2 eps_e,a) n_a n_a^T (the n_a are orthonormal)
// and F_new = F_n + H F_n with H = dF - I, the unit parts added in FP64.
template <typename T>
__device__ __forceinline__ void write_point(const AsmArgs& A, int64_t i, const PointMat<T>& P, const T H[3][3],
                                            double J) {
  const int64_t n = A.n;
  if (A.sigma) {
    const double iJ = 1.0 / J;
    A.sigma[i] = double(P.tau[0][0]) * iJ;
    A.sigma[n + i] = double(P.tau[1][1]) * iJ;
    A.sigma[2 * n + i] = double(P.tau[2][2]) * iJ;
    A.sigma[3 * n + i] = double(P.tau[0][1]) * iJ;
    A.sigma[4 * n + i] = double(P.tau[1][2]) * iJ;
    A.sigma[5 * n + i] = double(P.tau[0][2]) * iJ;
  }
  if (A.be) {
    // eps_e = eps - (1 - r) s_trial / (2 G). The return keeps the volumetric strain and scales
    // the deviator to the surface, so at a plastic point eps_e = tr(eps)/3 + r s_trial / (2 G)
    // with r |s_trial| = sqrt(2/3) sigma_y: formed from the unit deviator, this avoids the
    // cancellation of eps against the returned part (large when sigma_y is small against the
    // trial stress), which costs FP32 most of its digits
    T ee[3];
    if (P.plastic) {
      const T tr3 = (P.eps[0] + P.eps[1] + P.eps[2]) / T(3);
      const T rs = t_sqrt<T>(T(2) / T(3)) * T(A.s.sy[i]) / (T(2) * P.G);
      for (int a = 0; a < 3; ++a) ee[a] = t_expm1<T>(T(2) * (tr3 + rs * P.s_hat[a]));
    } else {
      for (int a = 0; a < 3; ++a) ee[a] = t_expm1<T>(T(2) * P.eps[a]);
    }
    const int ii[6] = {0, 1, 2, 0, 1, 0}, jj[6] = {0, 1, 2, 1, 2, 2};
    for (int c = 0; c < 6; ++c) {
      T v = 0;
      for (int a = 0; a < 3; ++a) v += ee[a] * P.N[ii[c]][a] * P.N[jj[c]][a];
      A.be[c * n + i] = double(v) + (c < 3 ? 1.0 : 0.0);
    }
  }
  if (A.Fnew && A.s.Fn) {
    double Fn[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) Fn[r][c] = A.s.Fn[(3 * r + c) * n + i];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double v = 0;
        for (int m = 0; m < 3; ++m) v += double(H[r][m]) * Fn[m][c];
        A.Fnew[(3 * r + c) * n + i] = Fn[r][c] + v;
      }
  }
}

// ------------------------------------------------------------------ fast path
// One 64-lane workgroup = one wavefront = 64 consecutive sorted points. Points whose domain
// lies in one leaf share that leaf's 8-node stencil; each lane computes its point's force
// (24 values) and upper-triangle stiffness blocks (36 x 9); the values are reduced per leaf
// segment (run of one leaf inside the wavefront) through LDS, 36 values per round, and each
// segment's sums are stored once, contiguously, in the segment buffer: a record holds the 36
// upper-triangle blocks (a <= b) in production order (b outer, a inner; then r, k), 324
// values, so a round's 36 sums land at consecutive offsets. No atomics: the row-gather kernel
// below turns segment sums into f_int and the CSR values.

// sum of row[0..len) with four independent accumulators (a fixed order for a given len)
template <typename T>
__device__ __forceinline__ T seg_sum(const T* row, int len) {
  T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  int j = 0;
  for (; j + 8 <= len; j += 8) {  // eight loads in flight per step
    T t[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) t[q] = row[j + q];
    s0 += t[0];
    s1 += t[1];
    s2 += t[2];
    s3 += t[3];
    s0 += t[4];
    s1 += t[5];
    s2 += t[6];
    s3 += t[7];
  }
  for (; j + 4 <= len; j += 4) {
    s0 += row[j];
    s1 += row[j + 1];
    s2 += row[j + 2];
    s3 += row[j + 3];
  }
  for (; j < len; ++j) s0 += row[j];
  return (s0 + s1) + (s2 + s3);
}

// Segment sums of one reduction round: the nseg x NV grid of (segment, value) sums is dealt
// to the lanes in order (value fastest), lane l taking entries l, l + 64, ...; the (segment,
// value) pair is advanced incrementally. store(sg, v, sum) receives each sum.
template <typename T, int NV, int NR, typename Store>
__device__ __forceinline__ void round_sums(const T (*red)[NR], const int32_t* seg_start, int nseg, Store store) {
  const int lane = threadIdx.x;
  constexpr int dsg = 64 / NV, dv = 64 % NV;
  int sg = lane / NV, v = lane % NV;
  for (int pp = lane; pp < nseg * NV; pp += 64) {
    const int s0 = seg_start[sg], s1 = seg_start[sg + 1];
    store(sg, v, seg_sum<T>(&red[v][s0], s1 - s0));
    v += dv;
    sg += dsg;
    if (v >= NV) {
      v -= NV;
      ++sg;
    }
  }
}

// LDS rows of the reduction are padded by one element: lanes that sum different values of
// one segment read one element per row, and a row stride of 65 elements spreads them over
// the banks (a stride of 64 would put them all in one bank).
constexpr int kRow = 65;

// stiffness values of a segment record: the 36 upper-triangle 3x3 slot blocks
constexpr int kRec = 324;

// Values per reduction round: four 3x3 blocks (36 values); forces in FP64, 24 per round in
// the FP64 kernel and 12 in the FP32 kernel, whose LDS then holds four wavefronts per SIMD.
template <typename T>
struct Rounds {
  static constexpr int kBlocks = 4;
  static constexpr int kVals = 9 * kBlocks;
  static constexpr int kForce = sizeof(T) == 8 ? 24 : 12;  // force values per round
  static constexpr int kBytes = (kVals * kRow * int(sizeof(T)) > kForce * kRow * 8) ? kVals * kRow * int(sizeof(T))
                                                                                 : kForce * kRow * 8;
};

// Segments of this wavefront's 64 points (runs of one leaf): seg_start[s] is the first lane
// of segment s and seg_start[nseg] the number of points; all 64 lanes must call it.
__device__ __forceinline__ void wave_segments(int32_t leaf, bool inr, int64_t n, int32_t* seg_start,
                                              int32_t* seg_cnt) {
  const int lane = threadIdx.x;
  const int32_t prev = __shfl_up(leaf, 1);
  const bool head = inr && (lane == 0 || prev != leaf);
  const uint64_t heads = __ballot(head);
  const uint64_t le = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
  const int my_seg = __popcll(heads & le) - 1;
  if (lane == 0) *seg_cnt = __popcll(heads);
  __syncthreads();
  if (head) seg_start[my_seg] = lane;
  if (lane == 0) {
    const int64_t rem = n - int64_t(blockIdx.x) * 64;
    seg_start[__popcll(heads)] = int32_t(rem < 64 ? rem : 64);
  }
}

// Register budget: two wavefronts per SIMD in FP64 (256 registers), four in FP32 (128).
// DYN adds the Newmark inertia term: f_v += S_v m_p a_p, and the tangent's (2 m_p / dt^2) S_a S_b
// (FP64: as 36 per-segment sums in their own record, which the row gather adds to the block
// diagonals; FP32: in the block values).
template <typename T, bool DYN>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 2 : 4)))
void k_assemble_fast(AsmArgs A) {
  constexpr int kRound = Rounds<T>::kVals, kBPR = Rounds<T>::kBlocks, kFR = Rounds<T>::kForce;
  __shared__ __align__(16) unsigned char red_raw[Rounds<T>::kBytes];
  __shared__ int32_t seg_start[65];
  __shared__ int32_t seg_cnt;
  T(*red)[kRow] = reinterpret_cast<T(*)[kRow]>(red_raw);
  double(*redd)[kRow] = reinterpret_cast<double(*)[kRow]>(red_raw);

  const int lane = threadIdx.x;
  const int64_t j = int64_t(blockIdx.x) * 64 + lane;  // position in the list of one-leaf points
  const int64_t n = A.n;
  const bool inr = j < A.n_fast;
  const int64_t i = inr ? (A.fidx ? A.fidx[j] : j) : 0;  // the point (sorted order)
  const int32_t leaf = inr ? A.pleaf[i] : -1;
  bool act = inr && A.pnleaf[i] == 1;
  wave_segments(leaf, inr, A.n_fast, seg_start, &seg_cnt);

  // ---------------- per-point arithmetic
  T S[8], dS[8][3], g[8][3];
  PointMat<T> P;
  T c = 0;
  T F[3][3];
  int32_t nodes[8];
  double acc[3] = {0.0, 0.0, 0.0}, mp = 0.0;  // inertia: point acceleration, mass
  if (act) {
    const int32_t code = A.cell_code[leaf];
    for (int v = 0; v < 8; ++v) nodes[v] = A.cell_nodes[8 * int64_t(leaf) + v];
    double x[3], l[3];
    for (int a = 0; a < 3; ++a) {
      x[a] = A.s.x[a * n + i];
      l[a] = A.s.l[a * n + i];
    }
    leaf_overlap_basis<T>(A.G, leaf, code, x, l, S, dS);
    T H[3][3];
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) H[r][q] = 0;
    double du[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const double* uv = A.u + 3 * int64_t(nodes[v]);
      const T u0 = T(uv[0]), u1 = T(uv[1]), u2 = T(uv[2]);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        H[0][q] += u0 * dS[v][q];
        H[1][q] += u1 * dS[v][q];
        H[2][q] += u2 * dS[v][q];
      }
      if constexpr (DYN) {
        du[0] += double(S[v]) * uv[0];
        du[1] += double(S[v]) * uv[1];
        du[2] += double(S[v]) * uv[2];
      }
    }
    if constexpr (DYN) {
      // Newmark, gamma = 1, beta = 1/2: a = 2 (du - dt v_n) / dt^2, v_new = v_n + dt a
      const double c2 = 2.0 / (A.dt * A.dt);
      mp = A.s.mass[i];
      for (int r = 0; r < 3; ++r) {
        const double vr = A.vel[r * n + i];
        acc[r] = c2 * (du[r] - A.dt * vr);
        if (A.a_new) A.a_new[r * n + i] = acc[r];
        if (A.v_new) A.v_new[r * n + i] = vr + A.dt * acc[r];
      }
    }
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) F[r][q] = H[r][q] + (r == q ? T(1) : T(0));
    T Fi[3][3];
    const T Jd = inv3(F, Fi);
    const double Jn = A.s.Jn[i];
    if (!isfinite(double(Jd)) || !isfinite(Jn)) {
      raise(A.err, MPM_ENONFINITE, i);
      act = false;
    } else if (!(Jd > T(0))) {
      raise(A.err, MPM_EDET, i);
      act = false;
    }
    if (act) {
#pragma unroll
      for (int v = 0; v < 8; ++v)
#pragma unroll
        for (int q = 0; q < 3; ++q) g[v][q] = Fi[0][q] * dS[v][0] + Fi[1][q] * dS[v][1] + Fi[2][q] * dS[v][2];
      T B[3][3];
      load_B<T>(A.s, n, i, B);
      const int st = material<T>(H, B, A.s.E[i], A.s.nu[i], A.s.sy[i], P);
      if (st) {
        raise(A.err, st, i);
        act = false;
      } else {
        c = T(A.s.vol[i] / Jn);
        write_point<T>(A, i, P, H, double(Jd) * Jn);
      }
    }
  }
  if (!act) {
    c = 0;
    mp = 0.0;
    for (int v = 0; v < 8; ++v) {
      nodes[v] = 0;
      S[v] = 0;
      for (int q = 0; q < 3; ++q) g[v][q] = 0;
    }
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) {
        P.tau[r][q] = 0;
        P.N[r][q] = r == q ? T(1) : T(0);
        P.D[r][q] = 0;
      }
    P.Geff = 0;
    P.th01 = P.th02 = P.th12 = 0;
    for (int a = 0; a < 3; ++a) P.x[a] = 1;
  }
  const int nseg = seg_cnt;

  // ---------------- force: f_v = c tau g_v (FP64 accumulation)
  const int64_t seg0 = A.wave_seg[blockIdx.x];
#pragma unroll
  for (int part = 0; part < 24 / kFR; ++part) {  // 24 force values in rounds of kFR
#pragma unroll
    for (int v = part * (kFR / 3); v < (part + 1) * (kFR / 3); ++v)
#pragma unroll
      for (int r = 0; r < 3; ++r)
        redd[3 * v + r - part * kFR][lane] =
            double(c) * double(P.tau[r][0] * g[v][0] + P.tau[r][1] * g[v][1] + P.tau[r][2] * g[v][2]) +
            (DYN ? double(S[v]) * mp * acc[r] : 0.0);
    __syncthreads();
    round_sums<double, kFR>(redd, seg_start, nseg, [&](int sg, int v, double sum) {
      A.segF[(seg0 + sg) * 24 + part * kFR + v] = sum;
    });
    __syncthreads();
  }
  if (!A.K) return;
  // FP64: the inertia tangent (2 m / dt^2) S_a S_b on the diagonal of block (a, b) is one scalar
  // per upper-triangle block, summed per segment like the stiffness values and added to the
  // block diagonals by the row gather, so the basis values are dead in the block loop (they
  // would spill there). FP32 adds it to the block values in the loop.
  constexpr bool kMassRec = DYN && sizeof(T) == 8;
  if constexpr (kMassRec) {
    const T cm = T(2.0 * mp / (A.dt * A.dt));
    int q = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int a = 0; a <= b; ++a, ++q) red[q][lane] = cm * S[a] * S[b];
    __syncthreads();
    T* segM = reinterpret_cast<T*>(A.segM);
    round_sums<T, kRound>(red, seg_start, nseg, [&](int sg, int v, T sum) { segM[(seg0 + sg) * 36 + v] = sum; });
    __syncthreads();
  }

  // ---------------- stiffness: K_(a,i)(b,k) = c [ (dtau(b,k) g_a)_i - (tau g_b)_i g_a,k ]
  // = sum_j X[k][i][j] g_a,j with X[k][i][j] = c dtau(b,k)_ij - (c tau g_b)_i delta_jk.
  // FP64 forms the 6x9 tangent matrix once (fewer operations); FP32 rotates each direction
  // from the principal frame (fewer live registers: four wavefronts per SIMD).
  constexpr bool kMatrix = sizeof(T) == 8;
  T* segK = reinterpret_cast<T*>(A.segK);
  T C[6][9];
  if constexpr (kMatrix) spatial_tangent<T>(P, c, C);
  T tau6[6] = {P.tau[0][0], P.tau[1][1], P.tau[2][2], P.tau[0][1], P.tau[1][2], P.tau[0][2]};
  int blk = 0;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    T X[3][3][3];
    if constexpr (kMatrix) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        T d6[6];
#pragma unroll
        for (int q = 0; q < 6; ++q)
          d6[q] = C[q][3 * k] * g[b][0] + C[q][3 * k + 1] * g[b][1] + C[q][3 * k + 2] * g[b][2];
        X[k][0][0] = d6[0];
        X[k][1][1] = d6[1];
        X[k][2][2] = d6[2];
        X[k][0][1] = X[k][1][0] = d6[3];
        X[k][1][2] = X[k][2][1] = d6[4];
        X[k][0][2] = X[k][2][0] = d6[5];
      }
    } else {
      T gt[3];
#pragma unroll
      for (int al = 0; al < 3; ++al) gt[al] = P.N[0][al] * g[b][0] + P.N[1][al] * g[b][1] + P.N[2][al] * g[b][2];
#pragma unroll
      for (int k = 0; k < 3; ++k) dtau_rank1<T>(P, k, gt, c, X[k]);
    }
    {
      const T tg0 = c * (tau6[0] * g[b][0] + tau6[3] * g[b][1] + tau6[5] * g[b][2]);
      const T tg1 = c * (tau6[3] * g[b][0] + tau6[1] * g[b][1] + tau6[4] * g[b][2]);
      const T tg2 = c * (tau6[5] * g[b][0] + tau6[4] * g[b][1] + tau6[2] * g[b][2]);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        X[k][0][k] -= tg0;
        X[k][1][k] -= tg1;
        X[k][2][k] -= tg2;
      }
    }
    const T msb = (DYN && !kMassRec) ? T(2.0 * mp / (A.dt * A.dt)) * S[b] : T(0);  // inertia: (2 m / dt^2) S_b
#pragma unroll
    for (int a = 0; a <= b; ++a) {
      const int slotv = (blk % kBPR) * 9;
      T vd[3][3];  // diagonal block (a == b): symmetric like K, its lower entries are copies
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          T val;
          if (a == b && k < r) {
            val = vd[k][r];
          } else {
            val = X[k][r][0] * g[a][0] + X[k][r][1] * g[a][1] + X[k][r][2] * g[a][2];
            if constexpr (DYN && !kMassRec)
              if (r == k) val += msb * S[a];
          }
          vd[r][k] = val;
          red[slotv + 3 * r + k][lane] = val;
        }
      if (blk % kBPR == kBPR - 1) {
        __syncthreads();
        const int rnd = blk / kBPR;
        round_sums<T, kRound>(red, seg_start, nseg,
                              [&](int sg, int v, T sum) { segK[(seg0 + sg) * kRec + rnd * kRound + v] = sum; });
        __syncthreads();
      }
      ++blk;
    }
  }
}

// ------------------------------------------------------------------ record reduction
// Task t = (first, count, out): record out = sum of records first .. first+count-1 (K values
// when wantK, forces always), summed in ascending order. 192 threads x 2 K values.
template <typename T>
__global__ __launch_bounds__(192) void k_rec_reduce(void* segK_, double* __restrict__ segF, void* segM_,
                                                    const int32_t* __restrict__ task, bool wantK) {
  const int64_t first = task[3 * blockIdx.x], out = task[3 * blockIdx.x + 2];
  const int cnt = task[3 * blockIdx.x + 1];
  const int t = threadIdx.x;
  if (wantK) {
    T* segK = reinterpret_cast<T*>(segK_);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (t + 192 * q >= kRec) break;
      const T* p = segK + first * kRec + t + 192 * q;
      T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
      int j = 0;
      for (; j + 4 <= cnt; j += 4) {
        s0 += p[int64_t(j) * kRec];
        s1 += p[int64_t(j + 1) * kRec];
        s2 += p[int64_t(j + 2) * kRec];
        s3 += p[int64_t(j + 3) * kRec];
      }
      for (; j < cnt; ++j) s0 += p[int64_t(j) * kRec];
      segK[out * kRec + t + 192 * q] = (s0 + s1) + (s2 + s3);
    }
  }
  if (t < 24) {
    double s = 0;
    for (int j = 0; j < cnt; ++j) s += segF[(first + j) * 24 + t];
    segF[out * 24 + t] = s;
  }
  if (wantK && segM_ && t >= 64 && t < 64 + 36) {  // inertia sums (dynamic assembly)
    T* segM = reinterpret_cast<T*>(segM_);
    T s = 0;
    for (int j = 0; j < cnt; ++j) s += segM[(first + j) * 36 + (t - 64)];
    segM[out * 36 + (t - 64)] = s;
  }
}

template <typename T>
static void launch_rec_reduce(const mpm_mesh* m, hipStream_t st, bool wantK, void* segM) {
  if (m->n_red1)
    hipLaunchKernelGGL(k_rec_reduce<T>, dim3(unsigned(m->n_red1)), dim3(192), 0, st, m->d_segK, m->d_segF, segM,
                       m->d_red1, wantK);
  if (m->n_red2)
    hipLaunchKernelGGL(k_rec_reduce<T>, dim3(unsigned(m->n_red2)), dim3(192), 0, st, m->d_segK, m->d_segF, segM,
                       m->d_red2, wantK);
}

// Workgroups are dealt to the chip's 8 XCDs (each with its own L2) in turn: workgroup w runs
// on XCD w % 8. This maps them so that XCD x takes one contiguous range of items (the first
// N % 8 XCDs one more): neighbouring items, which read the same records, share an L2.
__device__ __forceinline__ int64_t xcd_block(int64_t w, int64_t n) {
  const int64_t x = w & 7, q = w >> 3, m = n >> 3, r = n & 7;
  return x * m + (x < r ? x : r) + q;
}

// ------------------------------------------------------------------ row gather
// One workgroup per independent node n: the three CSR rows of n are accumulated in LDS from
// the reduced segment blocks of every (populated leaf, slot a) incidence of n, in ascending
// leaf order, and written once. A contribution is row a of a segment record: blocks (a, b)
// for b >= a as stored, blocks (b, a) for b < a read transposed. Rows and f_int are
// overwritten. The loads of a batch of contributions are
// issued without branches (indices past the end repeat the last one and are not added), so
// that they are all in flight together.
template <typename T, bool WANTK, bool MASS>
__global__ __launch_bounds__(64) void k_gather(AsmArgs A, int64_t row0) {
  extern __shared__ __align__(16) unsigned char gsm[];
  T* acc = reinterpret_cast<T*>(gsm);
  constexpr int kBatch = 4;  // contributions in flight per step: 52 registers, eight wavefronts per SIMD
  const int64_t q = row0 + xcd_block(blockIdx.x, gridDim.x);
  const int64_t nd = A.gorder ? A.gorder[q] : q;
  const int lane = threadIdx.x;
  const int64_t base = A.row_ptr[3 * nd];
  const int deg = int((A.row_ptr[3 * nd + 1] - base) / 3);
  const int len = 9 * deg;
  if (WANTK)
    for (int j = lane; j < len; j += 64) acc[j] = T(0);
  double fsum = 0.0;
  __syncthreads();
  const T* segK = reinterpret_cast<const T*>(A.segK);
  // lane -> (b, r, k) of the 72 values a contribution adds; lanes 0..7 also take values 64..71
  // (the other lanes load a duplicate of their first value and do not add it)
  const bool has1 = lane < 8;
  const int v0 = lane, v1 = has1 ? lane + 64 : lane;
  const int b0 = v0 / 9, r0 = (v0 % 9) / 3, k0 = v0 % 3;
  const int b1 = v1 / 9, r1 = (v1 % 9) / 3, k1 = v1 % 3;
  // record offset of value (r, k) of block (a, b): block (a, b) = 9 (b (b + 1) / 2 + a) + 3r + k
  // for a <= b; for a > b the transpose of block (b, a): 9 (a (a + 1) / 2 + b) + 3k + r
  const int up0 = 9 * (b0 * (b0 + 1) / 2) + 3 * r0 + k0, lo0 = 9 * b0 + 3 * k0 + r0;
  const int up1 = 9 * (b1 * (b1 + 1) / 2) + 3 * r1 + k1, lo1 = 9 * b1 + 3 * k1 + r1;
  // dynamic assembly: the inertia sum of block (a, b) (index b (b + 1)/2 + a, a <= b) is added to
  // the block's diagonal values
  const T* segM = reinterpret_cast<const T*>(A.segM);
  const bool dg0 = r0 == k0, dg1 = has1 && r1 == k1;
  const int fl = lane < 3 ? lane : 0;
  const int c0 = A.con_off[nd], c1 = A.con_off[nd + 1];
  // lane j holds contribution cl + j of the node (64 at a time, indices past the end repeat the
  // last one); every lane reads a batch's entries back as uniform values
  int cl = c0;
  int32_t my_cs = 0, my_cp = 0;  // record * 8 + slot, bpos offset
  for (int cb = c0; cb < c1; cb += kBatch) {
    const int nb = c1 - cb < kBatch ? c1 - cb : kBatch;
    if (cb == c0 || cb - cl + kBatch > 64) {
      cl = cb;
      const int jl = cb + lane < c1 ? cb + lane : c1 - 1;
      my_cs = A.con_seg[jl];
      my_cp = A.con_bp[jl];
    }
    int32_t cs[kBatch], cp[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int q = cb - cl + (j < nb ? j : nb - 1);
      cs[j] = __builtin_amdgcn_readlane(my_cs, q);
      cp[j] = __builtin_amdgcn_readlane(my_cp, q);
    }
    T val0[kBatch], val1[kBatch], mv0[kBatch], mv1[kBatch];
    int16_t p0[kBatch], p1[kBatch];
    double fv[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int64_t rec = cs[j] >> 3;
      const int slot = cs[j] & 7;
      if (WANTK) {
        const T* src = segK + rec * kRec;
        const int16_t* bp = A.bpos + cp[j];
        const int tri = 9 * (slot * (slot + 1) / 2);
        val0[j] = src[slot <= b0 ? up0 + 9 * slot : lo0 + tri];
        val1[j] = src[slot <= b1 ? up1 + 9 * slot : lo1 + tri];
        if constexpr (MASS) {  // loaded with the batch, added below (no wait inside the load loop)
          const T m0 = segM[rec * 36 + (slot <= b0 ? b0 * (b0 + 1) / 2 + slot : tri / 9 + b0)];
          const T m1 = segM[rec * 36 + (slot <= b1 ? b1 * (b1 + 1) / 2 + slot : tri / 9 + b1)];
          mv0[j] = dg0 ? m0 : T(0);
          mv1[j] = dg1 ? m1 : T(0);
        }
        p0[j] = bp[b0];
        p1[j] = bp[b1];
      }
      fv[j] = A.segF[rec * 24 + 3 * slot + fl];
    }
    // accumulate in contribution order; the 72 destinations of one contribution are distinct
    // and a single wavefront executes its LDS operations in program order
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      if (j >= nb) break;
      if (WANTK) {
        T a0 = val0[j], a1 = val1[j];
        if constexpr (MASS) {  // dynamic assembly: the block's inertia sum on its diagonal values
          a0 += mv0[j];
          a1 += mv1[j];
        }
        acc[r0 * 3 * deg + 3 * p0[j] + k0] += a0;
        if (has1) acc[r1 * 3 * deg + 3 * p1[j] + k1] += a1;
      }
      fsum += fv[j];
    }
  }
  __syncthreads();
  if (WANTK) {
    T* Kout = reinterpret_cast<T*>(A.K);
    for (int j = lane; j < len; j += 64) Kout[base + j] = acc[j];
  }
  if (lane < 3) A.f[3 * nd + lane] = fsum;
}

// nodes [row0, row0 + count) of the gather order, LDS for rows of at most deg block columns
template <typename T>
static void gather_part(hipStream_t st, const AsmArgs& A, int64_t row0, int64_t count, int64_t deg) {
  if (count <= 0) return;
  const dim3 grid(static_cast<unsigned>(count));
  const size_t lds = size_t(9) * size_t(deg) * sizeof(T);
  if (A.K && A.segM) hipLaunchKernelGGL((k_gather<T, true, true>), grid, dim3(64), lds, st, A, row0);
  else if (A.K) hipLaunchKernelGGL((k_gather<T, true, false>), grid, dim3(64), lds, st, A, row0);
  else hipLaunchKernelGGL((k_gather<T, false, false>), grid, dim3(64), 0, st, A, row0);
}
template <typename T>
static void launch_gather(const mpm_mesh* m, hipStream_t st, const AsmArgs& A) {
  if (!m->n_node) return;
  if (!m->d_gorder) {  // every row narrow: one launch in node order
    gather_part<T>(st, A, 0, m->n_node, m->max_deg);
    return;
  }
  gather_part<T>(st, A, 0, m->n_gnarrow, std::min<int64_t>(kGatherNarrow, m->max_deg));
  gather_part<T>(st, A, m->n_gnarrow, m->n_node - m->n_gnarrow, m->max_deg);
}

// ------------------------------------------------------------------ general path
// Points whose domain overlaps several leaves (up to 8 leaves, so at most 64 support nodes).
constexpr int kMaxSup = kMaxPointLeaves * 8;

// A first kernel takes one lane per such point: its update from the leaves it overlaps
// (basis, deformation, material), the point outputs (stress, committed state, Newmark
// kinematics) and a record of what the rows need, so that the update is computed once per
// point rather than once per row the point reaches:
// (symmetric 3x3 matrices as 6 values in the order xx, yy, zz, xy, yz, xz)
//   [0, 54)    c dtau for the direction e_k (x) N^T e_j, symmetric, at (3 j + k) 6
//   [54, 60)   c tau, symmetric                              (c = V_n / J_n)
//   [60, 69)   dF^-1, entry (r, k) at 60 + 3 r + k
//   [69, 72)   m_p a_p (Newmark inertia; zero when quasi-static)
//   [72]       2 m_p / dt^2 (zero when quasi-static)
__device__ constexpr int kSym6[3][3] = {{0, 3, 5}, {3, 1, 4}, {5, 4, 2}};
// the same index computed, for indices known only at run time (no table load): with
// s = r + m, the off-diagonal pairs (0,1), (1,2), (0,2) have s = 1, 3, 2
__device__ __forceinline__ int sym6(int r, int m) {
  const int sum = r + m;
  return r == m ? r : (sum == 2 ? 5 : 2 + ((sum + 1) >> 1));
}
// LDS written by one lane of a wavefront and read by another lane of the same wavefront: the
// wavefront's LDS operations are performed in order, so only the compiler must not move them
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The wavefront's 64 records are contiguous; they are written through LDS in four rounds
// (tangent direction rows j = 0, 1, 2: 18 values each; then the last 20 values), so that
// consecutive lanes store consecutive values of one record instead of 64 records at once.
constexpr int kRecStage = 21;  // LDS row of one lane's round (20 values, odd stride)
template <typename T>
__global__ __launch_bounds__(64) void k_general_points(AsmArgs A) {
  __shared__ double stage[64][kRecStage];
  const int lane = threadIdx.x;
  const int64_t t = int64_t(blockIdx.x) * 64 + lane;
  const bool live = t < A.n_strad;
  const int64_t n = A.n;
  PointMat<T> P;
  T Fi[3][3];
  T c = 0;
  double ma[3] = {0.0, 0.0, 0.0}, c2m = 0.0;
  bool okp = false;  // the point's record holds its values (else zeros: the call fails)
  if (live) {
    const int64_t i = A.strad[t];
    double x[3], l[3];
    for (int q = 0; q < 3; ++q) {
      x[q] = A.s.x[q * n + i];
      l[q] = A.s.l[q * n + i];
    }
    const int32_t* lv = A.strad_leaf + t * kMaxPointLeaves;
    T H[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double du[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < kMaxPointLeaves && lv[q] >= 0; ++q) {
      T s8[8], d8[8][3];
      leaf_overlap_basis<T>(A.G, lv[q], A.cell_code[lv[q]], x, l, s8, d8);
      for (int v = 0; v < 8; ++v) {
        const double* uv = A.u + 3 * int64_t(A.cell_nodes[8 * int64_t(lv[q]) + v]);
        for (int r = 0; r < 3; ++r) {
          for (int cc = 0; cc < 3; ++cc) H[r][cc] += T(uv[r]) * d8[v][cc];
          du[r] += double(s8[v]) * uv[r];
        }
      }
    }
    int stc = 0;
    T F[3][3];
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc) F[r][cc] = H[r][cc] + (r == cc ? T(1) : T(0));
    const T Jd = inv3(F, Fi);
    const double Jn = A.s.Jn[i];
    if (!isfinite(double(Jd)) || !isfinite(Jn)) stc = MPM_ENONFINITE;
    else if (!(Jd > T(0))) stc = MPM_EDET;
    else {
      T B[3][3];
      load_B<T>(A.s, n, i, B);
      stc = material<T>(H, B, A.s.E[i], A.s.nu[i], A.s.sy[i], P);
    }
    if (stc) {
      raise(A.err, stc, i);
    } else {
      okp = true;
      write_point<T>(A, i, P, H, double(Jd) * Jn);
      c = T(A.s.vol[i] / Jn);
      if (A.vel) {  // Newmark inertia, gamma = 1, beta = 1/2
        const double c2 = 2.0 / (A.dt * A.dt), mp = A.s.mass[i];
        for (int r = 0; r < 3; ++r) {
          const double vr = A.vel[r * n + i];
          const double ar = c2 * (du[r] - A.dt * vr);
          if (A.a_new) A.a_new[r * n + i] = ar;
          if (A.v_new) A.v_new[r * n + i] = vr + A.dt * ar;
          ma[r] = mp * ar;
        }
        c2m = double(T(2.0 * mp / (A.dt * A.dt)));
      }
    }
  }
  double* rec0 = A.grec + int64_t(blockIdx.x) * 64 * kGenRec;
  const int64_t left = A.n_strad - int64_t(blockIdx.x) * 64;
  const int nrec = int(left < 64 ? left : 64);
  // one round: lane l stages nv values at stage[l][0..nv), then the wavefront stores value v of
  // record r at rec0[r kGenRec + o + v]
  auto flush = [&](int o, int nv) {
    wave_lds_sync();
    for (int e = lane; e < nrec * nv; e += 64) {
      const int r = e / nv, v = e - nv * r;
      rec0[int64_t(r) * kGenRec + o + v] = stage[r][v];
    }
    wave_lds_sync();
  };
  // c dtau for the direction e_k (x) N^T e_j, symmetric, at (3 j + k) 6
  for (int j = 0; j < 3; ++j) {
    if (okp) {
      const T gt[3] = {P.N[j][0], P.N[j][1], P.N[j][2]};  // N^T e_j
      for (int k = 0; k < 3; ++k) {
        T dtk[3][3];
        dtau_rank1<T>(P, k, gt, T(1), dtk);
        for (int r = 0; r < 3; ++r)
          for (int m = r; m < 3; ++m) stage[lane][6 * k + kSym6[r][m]] = double(c * dtk[r][m]);
      }
    } else {
      for (int q = 0; q < 18; ++q) stage[lane][q] = 0.0;
    }
    flush(18 * j, 18);
  }
  // c tau (symmetric), dF^-1, the inertia terms
  for (int r = 0; r < 3; ++r)
    for (int j = 0; j < 3; ++j) {
      if (j >= r) stage[lane][kSym6[r][j]] = okp ? double(c * P.tau[r][j]) : 0.0;
      stage[lane][6 + 3 * r + j] = okp ? double(Fi[r][j]) : 0.0;
    }
  for (int r = 0; r < 3; ++r) stage[lane][15 + r] = ma[r];
  stage[lane][18] = c2m;
  stage[lane][19] = 0.0;
  flush(54, 20);
}

// Merged support of each straddling point, once per assembly: one lane per (point, leaf),
// launched per group of straddling points t0 .. t1 whose leaf counts are at most 2^lg, with
// 2^lg lanes per point. Each lane evaluates its leaf's 8 slot functions at the overlap box
// (values and reference gradients), maps the gradients to the current configuration with the
// point's dF^-1 (from its record), and stages them in LDS; then each support slot sums the
// entries of the leaves that hold its node, in ascending leaf order (a fixed order), and
// writes (S, grad_x S) to the slot. The row kernel below reads these.
template <typename T>
__global__ __launch_bounds__(64) void k_general_support(AsmArgs A, int64_t t0, int64_t t1, int lg) {
  __shared__ double stg[64][8][4];  // 16 KB: lane l stages its leaf at row l
  const int lp = 1 << lg;
  const int pp = threadIdx.x >> lg, q = threadIdx.x & (lp - 1);
  const int64_t t = t0 + int64_t(blockIdx.x) * (64 >> lg) + pp;
  const bool ok = t < t1;
  const int32_t e = ok ? A.strad_leaf[t * kMaxPointLeaves + q] : -1;
  if (e >= 0) {
    const int64_t n = A.n, i = A.strad[t];
    double x[3], l[3];
    for (int a = 0; a < 3; ++a) {
      x[a] = A.s.x[a * n + i];
      l[a] = A.s.l[a * n + i];
    }
    T s8[8], d8[8][3];
    leaf_overlap_basis<T>(A.G, e, A.cell_code[e], x, l, s8, d8);
    const double* rec = A.grec + t * kGenRec;
    T Fi[3][3];
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) Fi[r][k] = T(rec[60 + 3 * r + k]);
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      stg[threadIdx.x][v][0] = double(s8[v]);
#pragma unroll
      for (int k = 0; k < 3; ++k)
        stg[threadIdx.x][v][1 + k] = double(Fi[0][k] * d8[v][0] + Fi[1][k] * d8[v][1] + Fi[2][k] * d8[v][2]);
    }
  }
  __syncthreads();
  if (!ok) return;
  const int64_t off = A.sup_off[t];
  const int ns = int(A.sup_off[t + 1] - off);
  for (int z = q; z < ns; z += lp) {
    const uint32_t src = A.sup_src[off + z];
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    for (int qq = 0; qq < lp; ++qq)  // the point has at most lp leaves
      if ((src >> qq) & 1u) {
        const int v = int((src >> (8 + 3 * qq)) & 7u);
        for (int c = 0; c < 4; ++c) g[c] += stg[pp * lp + qq][v][c];
      }
    double* o = A.sup_g + (off + z) * 4;
    for (int c = 0; c < 4; ++c) o[c] = g[c];
  }
}

// The rows those points reach: one workgroup of W wavefronts per node a, which share the
// row's accumulator; each wavefront takes batches of 16 of the node's straddling points (batch
// b of the node goes to wavefront b mod W). For K_ab = V grad_x S_a . a . grad_x S_b a batch
// first forms, for each of its points, the 27 values
//   Mb[r][k][j] = (c dtau(j,k) g_a)_r - (c tau)_rj g_a,k
// from the point's record and the slot of node a in its support (four lanes per point, into
// the wavefront's part of LDS), and adds the point's force on node a. Then the (point,
// support slot) pairs of the batch with slot node b >= a are dealt to the lanes in order:
// each lane forms the 3x3 block sum_j Mb[r][k][j] g_b,j (+ the inertia term on the diagonal)
// and adds it to that node's column of the row. All loads of a batch are independent of
// each other, so they overlap; lanes of different points (and wavefronts) can add to one
// column at once, so the row additions are LDS atomics (the only unordered sums of the
// assembly: the fast path and the forces are summed in a fixed order). The row and the force
// are then added to the values the fast path wrote, and each new upper block is also stored,
// transposed, as block (b, a) of the row of b (K is symmetric). The column of a node in row a
// comes from an open-addressing table of the row's columns in LDS (at least half of it empty,
// so a probe sequence always ends).
__host__ __device__ constexpr int col_table_size(int deg) {
  int p = 2;
  while (p < 2 * deg) p <<= 1;
  return p;
}
__device__ __forceinline__ unsigned col_hash(int32_t id, int p) { return (unsigned(id) * 2654435761u) & unsigned(p - 1); }

// wavefronts per row of k_general_rows: rows of at most kNarrowRow columns take two (more rows
// in flight per CU; two beat one, four and eight), wider rows four (their LDS admits fewer
// workgroups per CU)
constexpr int kRowWavesNarrow = 2, kRowWavesWide = 4;
constexpr int kRowBatch = 16;  // straddling points per batch of one wavefront
// per point: Mb (27 values), S_a, 2 m / dt^2; the stride keeps 16-byte alignment and starts
// consecutive points 4 banks apart, so the lanes of the points of one task group (which read
// different points' values at once) do not meet in one bank
constexpr int kMbStride = 34;

// LDS of one wavefront's batch: Mb of its points
__host__ __device__ constexpr size_t row_batch_lds(int tb) {
  return size_t(kRowBatch * kMbStride) * size_t(tb);
}
// LDS bytes of k_general_rows with w wavefronts for rows of at most deg block columns, working
// type of size tb
__host__ __device__ constexpr size_t general_rows_lds(int deg, int tb, int w) {
  return size_t(w) * row_batch_lds(tb) + size_t(w * 4 * 8) + size_t(8) * col_table_size(deg) + size_t(9 * 8) * size_t(deg);
}

// marks an entry of the row that no straddling point reached (a NaN no arithmetic produces)
constexpr long long kUntouched = 0x7ff4d00d0000beefll;

template <typename T, int W>
__global__ __launch_bounds__(64 * W) void k_general_rows(AsmArgs A, int64_t row0) {
  extern __shared__ __align__(16) unsigned char gsm[];
  // the row's entry in the straddler tables; each XCD takes one contiguous range of rows, so
  // that rows sharing straddling points read them through one L2
  const int64_t rb = A.srow[row0 + xcd_block(blockIdx.x, gridDim.x)];
  const int64_t na = A.snode[rb];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t r0 = A.row_ptr[3 * na];
  const int deg = int((A.row_ptr[3 * na + 1] - r0) / 3);
  const int tp = col_table_size(deg);
  // LDS: the wavefronts' batch buffers (fixed size, first, so their alignment is known), the
  // wavefronts' forces, the column table and the row
  unsigned char* wb = gsm + size_t(wave) * row_batch_lds(sizeof(T));
  double* fsum = reinterpret_cast<double*>(gsm + size_t(W) * row_batch_lds(sizeof(T)));  // [W][3]
  // table entries: node id (high 32 bits) and column (low 32 bits); empty = all ones
  unsigned long long* ctab = reinterpret_cast<unsigned long long*>(fsum + W * 4);
  // the row in FP64, entry (r, k) of block column c at (3 r + k) deg + c: the lanes of one
  // addition (one entry, different columns) fall into consecutive banks
  double* acc = reinterpret_cast<double*>(ctab + tp);
  T* mbuf = reinterpret_cast<T*>(wb);  // [kRowBatch][kMbStride]
  const bool wantK = A.K != nullptr;
  if (wantK) {
    for (int j = tid; j < 9 * deg; j += 64 * W) acc[j] = 0.0;
    for (int j = tid; j < tp; j += 64 * W) ctab[j] = ~0ull;
  }
  __syncthreads();
  // the block column of a itself (the last of the force slots, unused by the forces)
  int* sja = reinterpret_cast<int*>(fsum + W * 4 - 1);
  if (wantK) {
    for (int j = tid; j < deg; j += 64 * W) {
      const int32_t id = A.col[r0 + 3 * j] / 3;
      if (id == na) *sja = j;
      const unsigned long long ent = (static_cast<unsigned long long>(unsigned(id)) << 32) | unsigned(j);
      for (unsigned hh = col_hash(id, tp);; hh = (hh + 1) & unsigned(tp - 1))
        if (atomicCAS(ctab + hh, ~0ull, ent) == ~0ull) break;
    }
  }
  __syncthreads();
  double fa[3] = {0.0, 0.0, 0.0};
  const int64_t c0 = A.sinc_off[rb], c1 = A.sinc_off[rb + 1];
  constexpr int64_t kStep = int64_t(W) * kRowBatch;
  // lanes pi, pi + 16, pi + 32, pi + 48 hold the batch's point pi: the point, the slot of node
  // a in its support, its support slots; the next batch's are loaded while this one runs
  const int pi = lane & (kRowBatch - 1), part = lane >> 4;
  auto entry = [&](int64_t cb, int64_t& t, int& za, int64_t& off, int& ns) {
    t = 0;
    za = 0;
    off = 0;
    ns = 0;
    if (cb + pi < c1) {
      const uint32_t ent = uint32_t(A.sinc[cb + pi]);
      t = int64_t(ent >> 6);
      za = int(ent & 63u);
      off = A.sup_off[t];
      ns = int(A.sup_off[t + 1] - off);
    }
  };
  int64_t t, off;
  int za, ns;
  entry(c0 + int64_t(wave) * kRowBatch, t, za, off, ns);
  // the wavefront's batches (its own trip count: only wavefront-level synchronisation inside)
  for (int64_t cb = c0 + int64_t(wave) * kRowBatch; cb < c1; cb += kStep) {
    const int nb = int(c1 - cb < kRowBatch ? c1 - cb : kRowBatch);
    if (pi < nb) {
      // the record is read in 16-byte pieces: the point's c tau and g_a by each of its four
      // lanes, and the six values of tangent direction dd = 3 j + k (48 bytes) by lane
      // dd mod 4, which forms Mb[r][k][j] for r = 0, 1, 2
      const double* rec = A.grec + t * kGenRec;
      const double2* gad = reinterpret_cast<const double2*>(A.sup_g + (off + za) * 4);
      const double2* tv = reinterpret_cast<const double2*>(rec + 54);
      const double2 g01 = gad[0], g23 = gad[1], t01 = tv[0], t23 = tv[1], t45 = tv[2];
      const T Sa = T(g01.x);
      const T ga[3] = {T(g01.y), T(g23.x), T(g23.y)};
      const T ct[6] = {T(t01.x), T(t01.y), T(t23.x), T(t23.y), T(t45.x), T(t45.y)};
      T* mb = mbuf + pi * kMbStride;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int dd = part + 4 * i;
        if (dd < 9) {
          const double2* dv = reinterpret_cast<const double2*>(rec + 6 * dd);
          const double2 d01 = dv[0], d23 = dv[1], d45 = dv[2];
          const T d6[6] = {T(d01.x), T(d01.y), T(d23.x), T(d23.y), T(d45.x), T(d45.y)};
          const int j = dd / 3, k = dd - 3 * j;
          const T gk = k == 0 ? ga[0] : (k == 1 ? ga[1] : ga[2]);
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            const int sj = sym6(r, j);
            const T trj = sj == 0 ? ct[0] : sj == 1 ? ct[1] : sj == 2 ? ct[2] : sj == 3 ? ct[3] : sj == 4 ? ct[4] : ct[5];
            mb[(3 * r + k) * 3 + j] = d6[kSym6[r][0]] * ga[0] + d6[kSym6[r][1]] * ga[1] + d6[kSym6[r][2]] * ga[2] -
                                      trj * gk;
          }
        }
      }
      if (part == 0) {
        mb[27] = Sa;
        mb[28] = T(rec[72]);
        for (int r = 0; r < 3; ++r)
          fa[r] += rec[54 + kSym6[r][0]] * double(ga[0]) + rec[54 + kSym6[r][1]] * double(ga[1]) +
                   rec[54 + kSym6[r][2]] * double(ga[2]) + double(Sa) * rec[69 + r];
      }
    }
    // this batch's support of the lane's point: the slots of nodes b >= a (the support is in
    // ascending node order and slot za holds a); K is symmetric, so the blocks (a, b) of the
    // nodes b < a are written by the rows of those nodes (below)
    const int64_t toff = off + za;
    const int tns = pi < nb ? ns - za : 0;
    // the lane's point's upper slots part, part + 4, ..., started at a per-point offset so that
    // points with the same support order add to different columns at once; each slot's node
    // and (S, grad_x S) are loaded one slot ahead of their use
    const int rot = tns > 0 ? (5 * pi) % tns : 0;
    auto slot_at = [&](int zz) {
      int z = zz + rot;
      if (z >= tns) z -= tns;
      return toff + z;
    };
    int32_t nid = 0;
    double2 n01 = {0.0, 0.0}, n23 = {0.0, 0.0};
    if (wantK && part < tns) {
      const int64_t o = slot_at(part);
      nid = A.sup_id[o];
      const double2* g = reinterpret_cast<const double2*>(A.sup_g + o * 4);
      n01 = g[0];
      n23 = g[1];
    }
    entry(cb + kStep, t, za, off, ns);  // the next batch of this wavefront
    wave_lds_sync();
    if (wantK && tns > 0) {
      // the point's Mb is read from LDS once
      const T* Mq = mbuf + pi * kMbStride;
      T M[29];
#pragma unroll
      for (int q = 0; q < 29; ++q) M[q] = Mq[q];
      const T ms0 = M[28] * M[27];  // inertia: (2 m / dt^2) S_a (times S_b below)
      for (int zz = part; zz < tns; zz += 4) {
        const int32_t id = nid;
        const double2 g01 = n01, g23 = n23;
        if (zz + 4 < tns) {
          const int64_t o = slot_at(zz + 4);
          nid = A.sup_id[o];
          const double2* g = reinterpret_cast<const double2*>(A.sup_g + o * 4);
          n01 = g[0];
          n23 = g[1];
        }
        const T sb = T(g01.x);
        const T gb[3] = {T(g01.y), T(g23.x), T(g23.y)};
        int lo = -1;  // block column of the slot's node in row a
        for (unsigned hh = col_hash(id, tp);; hh = (hh + 1) & unsigned(tp - 1)) {
          const unsigned long long en = ctab[hh];
          if (en == ~0ull) break;
          if (int32_t(en >> 32) == id) {
            lo = int(unsigned(en));
            break;
          }
        }
        if (lo < 0) {
          raise(A.err, MPM_ESTENCIL, na);
          continue;
        }
        const T ms = ms0 * sb;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const int rk = 3 * r + k;
            T val = M[3 * rk] * gb[0] + M[3 * rk + 1] * gb[1] + M[3 * rk + 2] * gb[2];
            if (r == k) val += ms;
            atomicAdd(acc + rk * deg + lo, double(val));
          }
      }
    }
    wave_lds_sync();  // the batch buffers are rewritten by the wavefront's next batch
  }
  // forces: lanes in a fixed order within each wavefront, then the wavefronts in order
#pragma unroll
  for (int off = 1; off < 64; off <<= 1)
    for (int r = 0; r < 3; ++r) fa[r] += __shfl_xor(fa[r], off);
  if (lane < 3) fsum[3 * wave + lane] = fa[lane];
  __syncthreads();
  if (tid < 3) {
    double f = 0.0;
    for (int w = 0; w < W; ++w) f += fsum[3 * w + tid];
    A.f[3 * na + tid] += f;
  }
  if (wantK) {
    // the blocks (a, c) of the columns c from a's own on (columns ascend), in CSR order (row r,
    // block column c, then k): K(a, c) += the row; the new value is kept in the row's LDS (an
    // entry no straddling point reaches is marked instead: it keeps the value of the one-leaf
    // gather, symmetric to rounding)
    T* Kout = reinterpret_cast<T*>(A.K);
    const int ja = *sja, nu = deg - ja;
    for (int q = tid; q < 9 * nu; q += 64 * W) {
      const int r = q / (3 * nu), rem = q - r * 3 * nu, cu = rem / 3, k = rem - 3 * cu, c = ja + cu;
      double* ap = acc + (3 * r + k) * deg + c;
      const double v = *ap;
      if (v == 0.0) {
        *ap = __longlong_as_double(kUntouched);
        continue;
      }
      const int64_t e = r0 + int64_t(r) * 3 * deg + 3 * c + k;
      const T kv = Kout[e] + T(v);
      Kout[e] = kv;
      *ap = double(kv);
    }
    __syncthreads();
    // for c above a the same values into block (c, a) of the row of c, entry (k, r) at the
    // block column the mesh keeps; lanes take (c, k, r) with r fastest, so that three lanes
    // store three consecutive values. That block is written by no other workgroup: the row of
    // c holds only its blocks from c on.
    const int64_t tb0 = r0 / 9;
    for (int q = tid; q < 9 * (nu - 1); q += 64 * W) {
      const int cu = 1 + q / 9, rem = q - 9 * (cu - 1), k = rem / 3, r = rem - 3 * k, c = ja + cu;
      const double kv = acc[(3 * r + k) * deg + c];
      if (__double_as_longlong(kv) == kUntouched) continue;
      const int64_t nc = A.col[r0 + 3 * c] / 3;
      const int32_t m = A.tpos[tb0 + c];
      if (m < 0) {  // the pattern is symmetric: cannot happen
        raise(A.err, MPM_ESTENCIL, na);
        continue;
      }
      Kout[A.row_ptr[3 * nc + k] + 3 * m + r] = T(kv);
    }
  }
}

// ------------------------------------------------------------------ body force
// f_ext,v = sum_p S_vp m_p g, through the same segment records and row gather as f_int.
__global__ __launch_bounds__(64) void k_external_fast(AsmArgs A) {
  __shared__ double redd[24][kRow];
  __shared__ int32_t seg_start[65];
  __shared__ int32_t seg_cnt;
  const int lane = threadIdx.x;
  const int64_t j = int64_t(blockIdx.x) * 64 + lane;  // position in the list of one-leaf points
  const int64_t n = A.n;
  const bool inr = j < A.n_fast;
  const int64_t i = inr ? (A.fidx ? A.fidx[j] : j) : 0;
  const int32_t leaf = inr ? A.pleaf[i] : -1;
  const bool act = inr && A.pnleaf[i] == 1;
  wave_segments(leaf, inr, A.n_fast, seg_start, &seg_cnt);
  double S[8], dS[8][3], mass = 0.0;
  if (act) {
    double x[3], l[3];
    for (int a = 0; a < 3; ++a) {
      x[a] = A.s.x[a * n + i];
      l[a] = A.s.l[a * n + i];
    }
    leaf_overlap_basis<double>(A.G, leaf, A.cell_code[leaf], x, l, S, dS);
    mass = A.s.mass[i];
  } else {
    for (int v = 0; v < 8; ++v) S[v] = 0.0;
  }
#pragma unroll
  for (int v = 0; v < 8; ++v)
#pragma unroll
    for (int r = 0; r < 3; ++r) redd[3 * v + r][lane] = S[v] * mass * A.s.g[r];
  __syncthreads();
  const int nseg = seg_cnt;
  const int64_t seg0 = A.wave_seg[blockIdx.x];
  round_sums<double, 24>(redd, seg_start, nseg,
                         [&](int sg, int v, double sum) { A.segF[(seg0 + sg) * 24 + v] = sum; });
}

// Body force of the points whose domain overlaps several leaves, gathered by rows in a fixed
// order: one wavefront per node a reached by such points; lane e takes the node's e-th
// point, whose support slot of a lists the point's leaves that hold a and a's vertex in each
// (the basis value S_a is the sum of those leaves' terms, in ascending leaf order); the
// lanes' S_a m_p g are summed in lane order and added to the gathered value.
__global__ __launch_bounds__(64) void k_external_rows(AsmArgs A) {
  const int64_t rb = blockIdx.x;
  const int64_t na = A.snode[rb];
  const int lane = threadIdx.x;
  const int64_t n = A.n;
  double fa[3] = {0.0, 0.0, 0.0};
  const int64_t c0 = A.sinc_off[rb], c1 = A.sinc_off[rb + 1];
  for (int64_t e = c0 + lane; e < c1; e += 64) {
    const uint32_t ent = uint32_t(A.sinc[e]);
    const int64_t t = int64_t(ent >> 6);
    const int za = int(ent & 63u);
    const uint32_t src = A.sup_src[A.sup_off[t] + za];
    const int64_t i = A.strad[t];
    double x[3], l[3];
    for (int c = 0; c < 3; ++c) {
      x[c] = A.s.x[c * n + i];
      l[c] = A.s.l[c * n + i];
    }
    double Sa = 0.0;
    for (int q = 0; q < kMaxPointLeaves; ++q)
      if ((src >> q) & 1u) {
        const int32_t lf = A.strad_leaf[t * kMaxPointLeaves + q];
        double S[8], dS[8][3];
        leaf_overlap_basis<double>(A.G, lf, A.cell_code[lf], x, l, S, dS);
        const int v = int((src >> (8 + 3 * q)) & 7u);
        for (int w = 0; w < 8; ++w) Sa += w == v ? S[w] : 0.0;  // select without dynamic register indexing
      }
    const double m = A.s.mass[i];
    for (int r = 0; r < 3; ++r) fa[r] += Sa * m * A.s.g[r];
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1)
    for (int r = 0; r < 3; ++r) fa[r] += __shfl_xor(fa[r], off);
  if (lane < 3) A.f[3 * na + lane] += fa[lane];
}

// ------------------------------------------------------------------ residual
constexpr int kResBlocks = 1024;
__global__ __launch_bounds__(256) void k_residual(const double* __restrict__ f, const double* __restrict__ fe,
                                                  const uint8_t* __restrict__ dir, double* __restrict__ r, int64_t nd,
                                                  double* __restrict__ partial) {
  __shared__ double s[256];
  double acc = 0;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < nd; k += int64_t(gridDim.x) * 256) {
    double v = f[k] - (fe ? fe[k] : 0.0);
    if (dir && dir[k]) v = 0.0;
    if (r) r[k] = v;
    acc += v * v;
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void k_norm_final(const double* __restrict__ partial, int np, double* out) {
  __shared__ double s[256];
  double acc = 0;
  for (int k = threadIdx.x; k < np; k += 256) acc += partial[k];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sqrt(s[0]);
}

// ------------------------------------------------------------------ adjoint
// L = lambda . f_int: per point L_p = c tau : G with c = V_n/J_n, G = sum_v lambda_v (x) grad_x S_v.
// dL/dV_n = tau:G / J_n; dL/dtheta = c sum_a (d tau_a / d theta) (n_a . G n_a): elastic points
// d tau_a/dE = tau_a/E, d tau_a/dnu = lam' tr(eps) + 2 G' eps_a; plastic points (radial return
// onto the von Mises circle, direction independent of E and nu) d tau_a/dE = tr(eps)/(3(1-2nu)),
// d tau_a/dnu = 2E tr(eps)/(3(1-2nu)^2), d tau_a/dsy = sqrt(2/3) s^_a.
// H += sum_v u_v (x) dS_v and Gp += sum_v lambda_v (x) dS_v over the 8 slots of one leaf
template <typename T>
__device__ __forceinline__ void adjoint_accumulate(const AsmArgs& A, const int32_t* nd, const T (*dS)[3], T H[3][3],
                                                   T Gp[3][3]) {
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const double* uv = A.u + 3 * int64_t(nd[v]);
    const double* lv = A.lam + 3 * int64_t(nd[v]);
    for (int r = 0; r < 3; ++r) {
      const T ur = T(uv[r]), lr = T(lv[r]);
      for (int q = 0; q < 3; ++q) {
        H[r][q] += ur * dS[v][q];
        Gp[r][q] += lr * dS[v][q];
      }
    }
  }
}

// the point's derivatives from H = sum_v u_v (x) dS_v and Gp = sum_v lambda_v (x) dS_v (both
// sums run over the point's (leaf, slot) terms, so domains over several leaves need no merged
// support; G = Gp dF^-1 below, and the basis gradients are dead before the material update)
template <typename T>
__device__ __forceinline__ void adjoint_point(const AsmArgs& A, int64_t i, const T H[3][3], const T Gp[3][3]) {
  const int64_t n = A.n;
  T F[3][3], Fi[3][3];
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) F[r][q] = H[r][q] + (r == q ? T(1) : T(0));
  const T Jd = inv3(F, Fi);
  T Gm[3][3];  // G = sum_v lambda_v (x) grad_x S_v, grad_x S_v = dF^-T dS_v
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) Gm[r][q] = Gp[r][0] * Fi[0][q] + Gp[r][1] * Fi[1][q] + Gp[r][2] * Fi[2][q];
  const double Jn = A.s.Jn[i];
  if (!isfinite(double(Jd)) || !isfinite(Jn)) {
    raise(A.err, MPM_ENONFINITE, i);
    return;
  }
  if (!(Jd > T(0))) {
    raise(A.err, MPM_EDET, i);
    return;
  }
  T B[3][3];
  load_B<T>(A.s, n, i, B);
  PointMat<T> P;
  const double Ed = A.s.E[i], nud = A.s.nu[i], syd = A.s.sy[i];
  const int st = material<T>(H, B, Ed, nud, syd, P);
  if (st) {
    raise(A.err, st, i);
    return;
  }
  double Ga[3], tauG = 0;
  for (int a = 0; a < 3; ++a) {
    T v = 0;
    for (int r = 0; r < 3; ++r)
      for (int q = 0; q < 3; ++q) v += P.N[r][a] * Gm[r][q] * P.N[q][a];
    Ga[a] = double(v);
    tauG += double(P.tp[a]) * Ga[a];
  }
  const double cc = A.s.vol[i] / Jn;
  double tr = 0;
  for (int a = 0; a < 3; ++a) tr += double(P.eps[a]);
  double dE = 0, dnu = 0, dsy = 0;
  if (P.plastic) {
    const double dKdE = 1.0 / (3.0 * (1.0 - 2.0 * nud));
    const double dKdnu = 2.0 * Ed / (3.0 * (1.0 - 2.0 * nud) * (1.0 - 2.0 * nud));
    const double sq = sqrt(2.0 / 3.0);
    for (int a = 0; a < 3; ++a) {
      dE += tr * dKdE * Ga[a];
      dnu += tr * dKdnu * Ga[a];
      dsy += sq * double(P.s_hat[a]) * Ga[a];
    }
  } else {
    const double opn = 1.0 + nud, omn = 1.0 - 2.0 * nud;
    const double dlam = Ed * (1.0 + 2.0 * nud * nud) / (opn * opn * omn * omn);
    const double dG = -Ed / (2.0 * opn * opn);
    for (int a = 0; a < 3; ++a) {
      dE += double(P.tp[a]) / Ed * Ga[a];
      dnu += (dlam * tr + 2.0 * dG * double(P.eps[a])) * Ga[a];
    }
  }
  A.dE[i] = cc * dE;
  A.dnu[i] = cc * dnu;
  A.dsy[i] = cc * dsy;
  A.dV[i] = tauG / Jn;
}

template <typename T>
__global__ __launch_bounds__(64) void k_adjoint_fast(AsmArgs A) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= A.n_fast) return;
  const int64_t i = A.fidx ? A.fidx[j] : j, n = A.n;
  if (A.pnleaf[i] != 1) return;
  double x[3], l[3];
  for (int a = 0; a < 3; ++a) {
    x[a] = A.s.x[a * n + i];
    l[a] = A.s.l[a * n + i];
  }
  const int32_t e = A.pleaf[i];
  int32_t nd[8];
  T S[8], dS[8][3];
  leaf_overlap_basis<T>(A.G, e, A.cell_code[e], x, l, S, dS);
  for (int v = 0; v < 8; ++v) nd[v] = A.cell_nodes[8 * int64_t(e) + v];
  T H[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  T Gp[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  adjoint_accumulate<T>(A, nd, dS, H, Gp);
  adjoint_point<T>(A, i, H, Gp);
}

template <typename T>
__global__ __launch_bounds__(64) void k_adjoint_general(AsmArgs A) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= A.n_strad) return;
  const int64_t i = A.strad[t], n = A.n;
  double x[3], l[3];
  for (int a = 0; a < 3; ++a) {
    x[a] = A.s.x[a * n + i];
    l[a] = A.s.l[a * n + i];
  }
  T H[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  T Gp[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  const int32_t* lv = A.strad_leaf + t * kMaxPointLeaves;
  for (int q = 0; q < kMaxPointLeaves && lv[q] >= 0; ++q) {
    int32_t nd[8];
    T S[8], dS[8][3];
    leaf_overlap_basis<T>(A.G, lv[q], A.cell_code[lv[q]], x, l, S, dS);
    for (int v = 0; v < 8; ++v) nd[v] = A.cell_nodes[8 * int64_t(lv[q]) + v];
    adjoint_accumulate<T>(A, nd, dS, H, Gp);
  }
  adjoint_point<T>(A, i, H, Gp);
}

static AsmArgs make_args(const mpm_mesh* m, const mpm_state_t* s) {
  AsmArgs A;
  std::memset(&A, 0, sizeof(A));
  A.G = make_geo(m);
  A.cell_nodes = m->d_cell_nodes;
  A.cell_code = m->d_cell_code;
  A.pleaf = m->d_pleaf;
  A.pnleaf = m->d_pnleaf;
  A.wave_seg = m->d_wave_seg;
  A.gorder = m->d_gorder;
  A.leaf_seg0 = m->d_leaf_seg0;
  A.leaf_nseg = m->d_leaf_nseg;
  A.con_off = m->d_con_off;
  A.con_seg = m->d_con_seg;
  A.con_bp = m->d_con_bp;
  A.bpos = m->d_bpos;
  A.segK = m->d_segK;
  A.segF = m->d_segF;
  A.row_ptr = m->d_row_ptr;
  A.col = m->d_col;
  A.strad = m->d_strad;
  A.strad_leaf = m->d_strad_leaf;
  A.snode = m->d_snode;
  A.srow = m->d_srow;
  A.sinc_off = m->d_sinc_off;
  A.sinc = m->d_sinc;
  A.grec = m->d_grec;
  A.sup_off = m->d_sup_off;
  A.sup_id = m->d_sup_id;
  A.sup_src = m->d_sup_src;
  A.sup_g = m->d_sup_g;
  A.tpos = m->d_tpos;
  A.n = m->n_point;
  A.n_strad = m->n_straddle;
  A.fidx = m->d_fidx;
  A.n_fast = m->n_fast;
  A.s = *s;
  A.err = m->d_err;
  return A;
}

// the per-point fields are required when the mesh has points (a mesh without points takes
// null or empty arrays)
static bool state_ok(const mpm_state_t* s, int64_t n) {
  return s && (n == 0 || (s->x && s->l && s->vol && s->Jn && s->bn && s->E && s->nu && s->sy));
}

}  // namespace mpm

using namespace mpm;

extern "C" int32_t mpm_external_force(const mpm_mesh_t* m, const mpm_state_t* s, double* f_ext, void* stream) {
  if (!m || !s || !f_ext || (m->n_point && (!s->x || !s->l || !s->mass))) {
    set_error(MPM_EARG, "mpm_external_force: null argument");
    return MPM_EARG;
  }
  hipStream_t st = (hipStream_t)stream;
  AsmArgs A = make_args(m, s);
  A.f = f_ext;
  A.K = nullptr;
  if (m->n_fast) hipLaunchKernelGGL(k_external_fast, dim3(unsigned((m->n_fast + 63) / 64)), dim3(64), 0, st, A);
  if (m->n_point) launch_rec_reduce<double>(m, st, false, nullptr);
  // every f_ext entry is written by the gather (zero where no point contributes)
  launch_gather<double>(m, st, A);
  if (m->n_snode) hipLaunchKernelGGL(k_external_rows, dim3(unsigned(m->n_snode)), dim3(64), 0, st, A);
  MPM_HIP(hipGetLastError());
  return read_error(const_cast<mpm_mesh*>(m), st, "mpm_external_force");
}

namespace mpm {
static int32_t assemble_impl(const mpm_mesh_t* m, const AsmArgs& A, int32_t precision, const double* f_ext,
                             const uint8_t* dirichlet, double* r, double* rnorm, hipStream_t st, const char* what);
}

extern "C" int32_t mpm_assemble(const mpm_mesh_t* m, const mpm_state_t* s, const double* u, int32_t precision,
                                const double* f_ext, const uint8_t* dirichlet, double* f_int, void* K_vals,
                                double* sigma6, double* r, double* rnorm, double* F_new, double* be_new,
                                void* stream) {
  if (!m || !state_ok(s, m->n_point) || !u || !f_int || (precision != MPM_F64 && precision != MPM_F32K) ||
      (F_new && m->n_point && !s->Fn)) {
    set_error(MPM_EARG, "mpm_assemble: null argument, bad precision or F_new without F_n");
    return MPM_EARG;
  }
  AsmArgs A = make_args(m, s);
  A.u = u;
  A.f = f_int;
  A.K = K_vals;
  A.sigma = sigma6;
  A.Fnew = F_new;
  A.be = be_new;
  return assemble_impl(m, A, precision, f_ext, dirichlet, r, rnorm, (hipStream_t)stream, "mpm_assemble");
}

extern "C" int32_t mpm_assemble_dynamic(const mpm_mesh_t* m, const mpm_state_t* s, const double* u,
                                        const double* v_n, double dt, int32_t precision, const double* f_ext,
                                        const uint8_t* dirichlet, double* f_int, void* K_vals, double* sigma6,
                                        double* r, double* rnorm, double* a_new, double* v_new, void* stream) {
  if (!m || !state_ok(s, m->n_point) || (m->n_point && (!s->mass || !v_n)) || !u || !f_int || !(dt > 0.0) ||
      !std::isfinite(dt) || (precision != MPM_F64 && precision != MPM_F32K)) {
    set_error(MPM_EARG, "mpm_assemble_dynamic: null argument, no mass, bad step size or bad precision");
    return MPM_EARG;
  }
  AsmArgs A = make_args(m, s);
  A.u = u;
  A.f = f_int;
  A.K = K_vals;
  A.sigma = sigma6;
  A.vel = v_n;
  A.dt = dt;
  A.segM = precision == MPM_F64 ? m->d_segM : nullptr;  // FP64 keeps the inertia sums in records
  A.a_new = a_new;
  A.v_new = v_new;
  return assemble_impl(m, A, precision, f_ext, dirichlet, r, rnorm, (hipStream_t)stream, "mpm_assemble_dynamic");
}

namespace mpm {
static int32_t assemble_impl(const mpm_mesh_t* m, const AsmArgs& A, int32_t precision, const double* f_ext,
                             const uint8_t* dirichlet, double* r, double* rnorm, hipStream_t st, const char* what) {
  double* f_int = A.f;
  void* K_vals = A.K;
  const int64_t n = m->n_point;
  mpm_mesh* mm = const_cast<mpm_mesh*>(m);
  const bool timed = mm->timing && n;
  if (m->n_snode && general_rows_lds(int(m->max_deg), 8, kRowWavesWide) > size_t(160) * 1024) {
    set_error(MPM_ESTENCIL, "assembly: a row couples more nodes than the general-path row kernel holds in LDS");
    return MPM_ESTENCIL;
  }
  // points whose domain overlaps several leaves: their update and tangent records, then their
  // merged supports, on the mesh's second stream beside the fast path (they write only their
  // own points' outputs and the mesh's per-point records)
  if (m->n_snode) {
    MPM_HIP(hipEventRecord(m->fork_ev, st));
    MPM_HIP(hipStreamWaitEvent(m->side, m->fork_ev, 0));
    const dim3 pgrid(unsigned((m->n_straddle + 63) / 64));
    if (precision == MPM_F64) hipLaunchKernelGGL(k_general_points<double>, pgrid, dim3(64), 0, m->side, A);
    else hipLaunchKernelGGL(k_general_points<float>, pgrid, dim3(64), 0, m->side, A);
    for (int g = 0; g < 3; ++g) {  // groups of at most 2, 4 and 8 leaves per point
      const int64_t t0 = m->strad_grp[g], t1 = m->strad_grp[g + 1];
      if (t1 <= t0) continue;
      const int ppw = 64 >> (g + 1);  // points per workgroup
      const dim3 sgrid(unsigned((t1 - t0 + ppw - 1) / ppw));
      if (precision == MPM_F64)
        hipLaunchKernelGGL(k_general_support<double>, sgrid, dim3(64), 0, m->side, A, t0, t1, g + 1);
      else hipLaunchKernelGGL(k_general_support<float>, sgrid, dim3(64), 0, m->side, A, t0, t1, g + 1);
    }
    MPM_HIP(hipEventRecord(m->join_ev, m->side));
  }
  if (timed) MPM_HIP(hipEventRecord(mm->ev[0], st));
  if (m->n_fast) {  // the points whose domain lies in one leaf
    const dim3 grid(unsigned((m->n_fast + 63) / 64));
    if (A.vel) {
      if (precision == MPM_F64) hipLaunchKernelGGL((k_assemble_fast<double, true>), grid, dim3(64), 0, st, A);
      else hipLaunchKernelGGL((k_assemble_fast<float, true>), grid, dim3(64), 0, st, A);
    } else {
      if (precision == MPM_F64) hipLaunchKernelGGL((k_assemble_fast<double, false>), grid, dim3(64), 0, st, A);
      else hipLaunchKernelGGL((k_assemble_fast<float, false>), grid, dim3(64), 0, st, A);
    }
  }
  if (timed) MPM_HIP(hipEventRecord(mm->ev[1], st));
  if (n) {
    if (precision == MPM_F64) launch_rec_reduce<double>(m, st, K_vals != nullptr, A.segM);
    else launch_rec_reduce<float>(m, st, K_vals != nullptr, A.segM);
  }
  // f_int and every CSR value are written by the gather (zero where no point contributes)
  if (precision == MPM_F64) launch_gather<double>(m, st, A);
  else launch_gather<float>(m, st, A);
  if (timed) MPM_HIP(hipEventRecord(mm->ev[4], st));
  if (m->n_snode) {  // rows reached by points whose domain overlaps several leaves
    MPM_HIP(hipStreamWaitEvent(st, m->join_ev, 0));  // their records and supports, and the gather
    // narrow rows with LDS for kNarrowRow columns, then the rest with LDS for the widest row
    const int64_t nn = m->n_snode_narrow, nw = m->n_snode - nn;
    const int tb = precision == MPM_F64 ? 8 : 4;
    const int dn = std::min<int>(kNarrowRow, int(m->max_deg));
    constexpr int wn = kRowWavesNarrow, ww = kRowWavesWide;
    if (precision == MPM_F64) {
      if (nn) hipLaunchKernelGGL((k_general_rows<double, wn>), dim3(unsigned(nn)), dim3(64 * wn),
                                 general_rows_lds(dn, tb, wn), st, A, int64_t(0));
      if (nw) hipLaunchKernelGGL((k_general_rows<double, ww>), dim3(unsigned(nw)), dim3(64 * ww),
                                 general_rows_lds(int(m->max_deg), tb, ww), st, A, nn);
    } else {
      if (nn) hipLaunchKernelGGL((k_general_rows<float, wn>), dim3(unsigned(nn)), dim3(64 * wn),
                                 general_rows_lds(dn, tb, wn), st, A, int64_t(0));
      if (nw) hipLaunchKernelGGL((k_general_rows<float, ww>), dim3(unsigned(nw)), dim3(64 * ww),
                                 general_rows_lds(int(m->max_deg), tb, ww), st, A, nn);
    }
  }
  // ghost penalty (Section 4): after every point term, before the residual
  if (const int32_t rg = ghost_apply(m, &A.s, A.u, precision, K_vals, f_int, st)) return rg;
  if (r || rnorm) {
    const int64_t nd = 3 * m->n_node;
    int nb = int(std::min<int64_t>(kResBlocks, (nd + 255) / 256));
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_residual, dim3(nb), dim3(256), 0, st, f_int, f_ext, dirichlet, r, nd, m->d_partial);
    if (rnorm) hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(256), 0, st, m->d_partial, nb, rnorm);
  }
  MPM_HIP(hipGetLastError());
  const int32_t rc = read_error(mm, st, what);
  if (timed) {
    float ms = 0, mg = 0;
    MPM_HIP(hipEventElapsedTime(&ms, mm->ev[0], mm->ev[1]));
    MPM_HIP(hipEventElapsedTime(&mg, mm->ev[1], mm->ev[4]));
    mm->t_asm += ms;
    mm->n_asm += 1;
    mm->t_gat += mg;
    mm->n_gat += 1;
  }
  return rc;
}
}  // namespace mpm

extern "C" int32_t mpm_assemble_adjoint(const mpm_mesh_t* m, const mpm_state_t* s, const double* u,
                                        const double* lambda, int32_t precision, double* dE, double* dnu,
                                        double* dsy, double* dV, void* stream) {
  if (!m || !state_ok(s, m->n_point) || !u || !lambda || (m->n_point && (!dE || !dnu || !dsy || !dV)) ||
      (precision != MPM_F64 && precision != MPM_F32K)) {
    set_error(MPM_EARG, "mpm_assemble_adjoint: null argument or bad precision");
    return MPM_EARG;
  }
  if (m->n_gface) {
    set_error(MPM_EARG, "mpm_assemble_adjoint: not defined on a mesh with ghost stabilisation");
    return MPM_EARG;
  }
  hipStream_t st = (hipStream_t)stream;
  AsmArgs A = make_args(m, s);
  A.u = u;
  A.lam = lambda;
  A.dE = dE;
  A.dnu = dnu;
  A.dsy = dsy;
  A.dV = dV;
  const int64_t n = m->n_point;
  mpm_mesh* mm = const_cast<mpm_mesh*>(m);
  const bool timed = mm->timing && n;
  // points whose domain overlaps several leaves on the mesh's second stream, beside the others
  if (m->n_straddle) {
    MPM_HIP(hipEventRecord(m->fork_ev, st));
    MPM_HIP(hipStreamWaitEvent(m->side, m->fork_ev, 0));
    const dim3 grid(unsigned((m->n_straddle + 63) / 64));
    if (precision == MPM_F64) hipLaunchKernelGGL(k_adjoint_general<double>, grid, dim3(64), 0, m->side, A);
    else hipLaunchKernelGGL(k_adjoint_general<float>, grid, dim3(64), 0, m->side, A);
    MPM_HIP(hipEventRecord(m->join_ev, m->side));
  }
  if (timed) MPM_HIP(hipEventRecord(mm->ev[2], st));
  if (m->n_fast) {  // the points whose domain lies in one leaf
    const dim3 grid(unsigned((m->n_fast + 63) / 64));
    if (precision == MPM_F64) hipLaunchKernelGGL(k_adjoint_fast<double>, grid, dim3(64), 0, st, A);
    else hipLaunchKernelGGL(k_adjoint_fast<float>, grid, dim3(64), 0, st, A);
  }
  if (timed) MPM_HIP(hipEventRecord(mm->ev[3], st));
  if (m->n_straddle) MPM_HIP(hipStreamWaitEvent(st, m->join_ev, 0));
  MPM_HIP(hipGetLastError());
  const int32_t rc = read_error(mm, st, "mpm_assemble_adjoint");
  if (timed) {
    float ms = 0;
    MPM_HIP(hipEventElapsedTime(&ms, mm->ev[2], mm->ev[3]));
    mm->t_adj += ms;
    mm->n_adj += 1;
  }
  return rc;
}
