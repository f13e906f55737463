// Per-material-point arithmetic of the assembly, templated on the working precision T.
//
//  - discrete GIMP basis (one-point rule on each domain/leaf overlap box, Section 3.2,
//    eq. GIMP numerical) mapped through the hanging-node constraints (Section 3.1, hanging
//    node basis): phi~_slot = sum_vertex C_K[vertex][slot] phi_vertex;
//  - Hencky elasticity with a von Mises perfect-plasticity return in principal logarithmic
//    strains (Section 2.2), computed from Y = b_tr - I so that small strains keep their
//    relative accuracy (eps_a = log1p(y_a) / 2);
//  - the linearisation of the Kirchhoff stress in the principal frame of b_tr: for a
//    displacement-gradient variation Z, dtau~_aa = sum_c D_ac Z~_cc and
//    dtau~_ab = G_eff theta_ab (Z~_ab x_b + x_a Z~_ba), theta_ab = (ln x_a - ln x_b)/(x_a - x_b).
#pragma once
#include "geom.h"

namespace mpm {

template <typename T>
__device__ __forceinline__ T t_log1p(T v);
template <>
__device__ __forceinline__ double t_log1p<double>(double v) { return log1p(v); }
template <>
__device__ __forceinline__ float t_log1p<float>(float v) { return log1pf(v); }
template <typename T>
__device__ __forceinline__ T t_sqrt(T v);
template <>
__device__ __forceinline__ double t_sqrt<double>(double v) { return sqrt(v); }
template <>
__device__ __forceinline__ float t_sqrt<float>(float v) { return sqrtf(v); }
template <typename T>
__device__ __forceinline__ T t_expm1(T v);
template <>
__device__ __forceinline__ double t_expm1<double>(double v) { return expm1(v); }
template <>
__device__ __forceinline__ float t_expm1<float>(float v) { return expm1f(v); }

// log1p(z)/z for |z| < 1/16 by the Mercator series log(1 + z) = z - z^2/2 + z^3/3 - ...
// (Horner form of sum_k (-z)^k / (k + 1)); the truncation error after degree n is below
// |z|^(n+1) / (n + 2) relative (an alternating series), i.e. under 2^-55 for FP64 at n = 12 and
// at most 2^-31 for FP32 at n = 6. Small logarithmic strains and the ratio of close eigenvalues take this path; larger
// arguments call log1p.
constexpr double kSeriesMax = 0.0625;
template <typename T>
__device__ __forceinline__ T log1p_over(T z) {
  constexpr int kDeg = sizeof(T) == 8 ? 12 : 6;
  T p = T(1) / T(kDeg + 1);
#pragma unroll
  for (int k = kDeg - 1; k >= 0; --k) p = T(1) / T(k + 1) - z * p;
  return p;
}
template <typename T>
__device__ __forceinline__ T log1p_fast(T y) {
  return fabs(y) < T(kSeriesMax) ? y * log1p_over<T>(y) : t_log1p<T>(y);
}

template <typename T>
struct Eps;
template <>
struct Eps<double> {
  static constexpr double v = 1e-16;
};
template <>
struct Eps<float> {
  static constexpr float v = 6e-8f;
};

// trilinear vertex functions and gradients of a leaf at local coordinates xi (vertex v has
// bit a = 1 at xi_a = 1), then the constraint map to the 8 slots of I(K)
template <typename T>
__device__ __forceinline__ void slot_basis(const T xi[3], T inv_h, int32_t code, T wgt, T S[8], T dS[8][3]) {
  T w[3][2];
  for (int a = 0; a < 3; ++a) {
    w[a][0] = T(1) - xi[a];
    w[a][1] = xi[a];
  }
  T ph[8], g0[8], g1[8], g2[8];
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int b0 = v & 1, b1 = (v >> 1) & 1, b2 = (v >> 2) & 1;
    const T s0 = b0 ? inv_h : -inv_h, s1 = b1 ? inv_h : -inv_h, s2 = b2 ? inv_h : -inv_h;
    ph[v] = w[0][b0] * w[1][b1] * w[2][b2];
    g0[v] = s0 * w[1][b1] * w[2][b2];
    g1[v] = w[0][b0] * s1 * w[2][b2];
    g2[v] = w[0][b0] * w[1][b1] * s2;
  }
  // Constraint map (Section 3.1, hanging node basis). A hanging vertex j of a child leaf
  // (child index cc in its parent) lies at the midpoint of a parent edge or face; its value
  // is the average of the 2^m parent corners of that edge or face, m = |j ^ cc|. Relative to
  // cc (j' = j ^ cc) those corners are the slots k with k' a subset of j'. So
  //   S[k] = [k not hanging] ph[k] + sum over hanging j with j' containing k' of ph[j] / 2^m_j,
  // a sum over supersets taken axis by axis (three passes of eight fused adds).
  const int hm = code_hmask(code);
  if (hm == 0) {  // no hanging vertex: the map is the identity
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      S[k] = ph[k] * wgt;
      dS[k][0] = g0[k] * wgt;
      dS[k][1] = g1[k] * wgt;
      dS[k][2] = g2[k] * wgt;
    }
    return;
  }
  const int cc = code_child(code);
  T wj[8], nh[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const bool hj = (hm >> j) & 1;
    const int m = __builtin_popcount((j ^ cc) & 7);
    wj[j] = hj ? (m == 1 ? T(0.5) : (m == 2 ? T(0.25) : T(0.125))) : T(0);
    nh[j] = hj ? T(0) : T(1);
  }
  T ax[3];  // 1 where slot k agrees with cc on the axis (it receives in that pass), else 0
#pragma unroll
  for (int a = 0; a < 3; ++a) ax[a] = ((cc >> a) & 1) ? T(1) : T(0);
  auto constrain = [&](const T* q, T* out, int stride) {
    T t[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) t[j] = wj[j] * q[j];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int bit = 1 << a;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (k & bit) continue;  // pair (k, k | bit): the member that agrees with cc receives
        const T lo = t[k], hi = t[k | bit];
        t[k] = lo + (T(1) - ax[a]) * hi;
        t[k | bit] = hi + ax[a] * lo;
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) out[k * stride] = (nh[k] * q[k] + t[k]) * wgt;
  };
  constrain(ph, S, 1);
  constrain(g0, &dS[0][0], 3);
  constrain(g1, &dS[0][1], 3);
  constrain(g2, &dS[0][2], 3);
}

// Reciprocal and reciprocal square root from the hardware estimates, refined by Newton steps
// (two for FP64: the error falls from the estimate's to about one unit in the last place; the
// FP32 estimates are already within one unit). Used for the Jacobi rotation parameters, which
// only need c^2 + s^2 = 1 to rounding.
template <typename T>
__device__ __forceinline__ T nr_rcp(T x);
template <>
__device__ __forceinline__ double nr_rcp<double>(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
template <>
__device__ __forceinline__ float nr_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <typename T>
__device__ __forceinline__ T nr_rsq(T x);
template <>
__device__ __forceinline__ double nr_rsq<double>(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int k = 0; k < 2; ++k) {  // y <- y (3 - x y^2) / 2
    const double h = 0.5 * y;
    y = fma(h, fma(-x * y, y, 1.0), y);
  }
  return y;
}
template <>
__device__ __forceinline__ float nr_rsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }

// one Jacobi rotation annihilating the (p,q) entry of the symmetric A (storage a[p][q]),
// accumulating the eigenvectors in the columns of V; t = tan of the rotation angle, the root
// of smaller magnitude of t^2 + 2 th t - 1 = 0
// (off-diagonals below the smallest normal range, whose reciprocal would overflow, are left
// as they are; for |th| beyond the range of th^2, t = 1 / (2 |th|))
template <typename T>
__device__ __forceinline__ void jrot(T A[3][3], T V[3][3], int p, int q, int r) {
  constexpr T kTiny = sizeof(T) == 8 ? T(1e-290) : T(1e-35), kBig = sizeof(T) == 8 ? T(1e150) : T(1e18);
  const T apq = A[p][q];
  if (!(fabs(apq) > kTiny)) return;
  const T th = (A[q][q] - A[p][p]) * (T(0.5) * nr_rcp<T>(apq));
  const T ath = fabs(th), q1 = T(1) + th * th;
  const T den = ath < kBig ? ath + q1 * nr_rsq<T>(q1) : T(2) * ath;  // |th| + sqrt(1 + th^2)
  const T t = (th >= T(0) ? T(1) : T(-1)) * nr_rcp<T>(den);
  const T c = nr_rsq<T>(T(1) + t * t), s = t * c;
  A[p][p] -= t * apq;
  A[q][q] += t * apq;
  A[p][q] = A[q][p] = T(0);
  const T arp = A[r][p], arq = A[r][q];
  A[r][p] = A[p][r] = c * arp - s * arq;
  A[r][q] = A[q][r] = s * arp + c * arq;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T vip = V[i][p], viq = V[i][q];
    V[i][p] = c * vip - s * viq;
    V[i][q] = s * vip + c * viq;
  }
}

template <typename T>
__device__ __forceinline__ void eig_sym3(T A[3][3], T y[3], T V[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) V[i][j] = i == j ? T(1) : T(0);
  const T scale = fabs(A[0][0]) + fabs(A[1][1]) + fabs(A[2][2]) + fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
  const T tol = Eps<T>::v * scale;
  for (int sweep = 0; sweep < 12; ++sweep) {
    const T off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
    if (!(off > tol)) break;
    jrot(A, V, 0, 1, 2);
    jrot(A, V, 0, 2, 1);
    jrot(A, V, 1, 2, 0);
  }
  y[0] = A[0][0];
  y[1] = A[1][1];
  y[2] = A[2][2];
}

// material state of one point after the return map
template <typename T>
struct PointMat {
  T N[3][3];     // eigenvectors of b_tr (columns)
  T x[3];        // eigenvalues of b_tr
  T tp[3];       // principal Kirchhoff stresses
  T D[3][3];     // algorithmic principal moduli d tau_a / d eps_b
  T Geff;        // shear modulus of the return (G or G r)
  T th01, th02, th12;
  T tau[3][3];   // Kirchhoff stress
  T eps[3], s_hat[3], r, lam, G;
  bool plastic;
};

template <typename T>
__device__ __forceinline__ T theta_pair(T ya, T yb) {
  // (ln x_a - ln x_b)/(x_a - x_b) with x = 1 + y: with z = (x_a - x_b)/x_b it is
  // log1p(z) / (z x_b), the series quotient for close eigenvalues (z = 0 included)
  const T d = ya - yb;
  const T ib = T(1) / (T(1) + yb);
  const T z = d * ib;
  if (fabs(z) < T(kSeriesMax)) return log1p_over<T>(z) * ib;
  return t_log1p<T>(z) / d;
}

// returns 0 or a negative status
template <typename T>
__device__ __forceinline__ int material(const T H[3][3], const T B[3][3], double Ed, double nud, double syd,
                                        PointMat<T>& P) {
  // Y = b_tr - I = H + H^T + H H^T + (I+H) (b_n - I) (I+H)^T
  T A1[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      T t = 0;
#pragma unroll
      for (int m = 0; m < 3; ++m) t += ((i == m ? T(1) : T(0)) + H[i][m]) * B[m][j];
      A1[i][j] = t;
    }
  T Y[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      T t = H[i][j] + H[j][i];
#pragma unroll
      for (int m = 0; m < 3; ++m) t += H[i][m] * H[j][m] + A1[i][m] * ((j == m ? T(1) : T(0)) + H[j][m]);
      Y[i][j] = Y[j][i] = t;
    }
  T y[3];
  eig_sym3(Y, y, P.N);
  if (!(y[0] > T(-1)) || !(y[1] > T(-1)) || !(y[2] > T(-1))) return MPM_EDET;
  const T E = T(Ed), nu = T(nud);
  const T lam = E * nu / ((T(1) + nu) * (T(1) - T(2) * nu));
  const T G = E / (T(2) * (T(1) + nu));
  const T Kb = lam + T(2) * G / T(3);
  P.lam = lam;
  P.G = G;
  T tr = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    P.x[a] = T(1) + y[a];
    P.eps[a] = T(0.5) * log1p_fast<T>(y[a]);
    tr += P.eps[a];
  }
  T t[3], s[3], p = 0, ns = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    t[a] = lam * tr + T(2) * G * P.eps[a];
    p += t[a];
  }
  p /= T(3);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    s[a] = t[a] - p;
    ns += s[a] * s[a];
  }
  ns = t_sqrt<T>(ns);
  const T q = t_sqrt<T>(T(1.5)) * ns;
  P.plastic = isfinite(syd) && (q - T(syd) > T(0));
  const T inv_ns = ns > T(0) ? T(1) / ns : T(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) P.s_hat[a] = s[a] * inv_ns;
  if (P.plastic) {
    const T r = t_sqrt<T>(T(2) / T(3)) * T(syd) * inv_ns;
    P.r = r;
    P.Geff = G * r;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      P.tp[a] = p + r * s[a];
#pragma unroll
      for (int b = 0; b < 3; ++b)
        P.D[a][b] = Kb + T(2) * G * r * ((a == b ? T(1) : T(0)) - T(1) / T(3) - P.s_hat[a] * P.s_hat[b]);
    }
  } else {
    P.r = T(1);
    P.Geff = G;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      P.tp[a] = t[a];
#pragma unroll
      for (int b = 0; b < 3; ++b) P.D[a][b] = lam + (a == b ? T(2) * G : T(0));
    }
  }
  P.th01 = theta_pair(y[0], y[1]);
  P.th02 = theta_pair(y[0], y[2]);
  P.th12 = theta_pair(y[1], y[2]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      T v = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) v += P.tp[a] * P.N[i][a] * P.N[j][a];
      P.tau[i][j] = P.tau[j][i] = v;
    }
  return 0;
}

// variation of tau for Z = e_k (x) g (principal-frame formula), scaled by `sc`, symmetric
// result dt[3][3] = sc N dtau~ N^T
template <typename T>
__device__ __forceinline__ void dtau_rank1(const PointMat<T>& P, int k, const T gt[3], T sc, T dt[3][3]) {
  // Z~ = (N^T e_k)(N^T g)^T: Z~_ab = N[k][a] gt[b]
  const T z0 = P.N[k][0] * gt[0], z1 = P.N[k][1] * gt[1], z2 = P.N[k][2] * gt[2];
  T m[3][3];
  m[0][0] = sc * (P.D[0][0] * z0 + P.D[0][1] * z1 + P.D[0][2] * z2);
  m[1][1] = sc * (P.D[1][0] * z0 + P.D[1][1] * z1 + P.D[1][2] * z2);
  m[2][2] = sc * (P.D[2][0] * z0 + P.D[2][1] * z1 + P.D[2][2] * z2);
  const T gs = sc * P.Geff;
  m[0][1] = m[1][0] = gs * P.th01 * (P.N[k][0] * gt[1] * P.x[1] + P.x[0] * P.N[k][1] * gt[0]);
  m[0][2] = m[2][0] = gs * P.th02 * (P.N[k][0] * gt[2] * P.x[2] + P.x[0] * P.N[k][2] * gt[0]);
  m[1][2] = m[2][1] = gs * P.th12 * (P.N[k][1] * gt[2] * P.x[2] + P.x[1] * P.N[k][2] * gt[1]);
  T W[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int b = 0; b < 3; ++b) W[i][b] = P.N[i][0] * m[0][b] + P.N[i][1] * m[1][b] + P.N[i][2] * m[2][b];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) dt[i][j] = dt[j][i] = W[i][0] * P.N[j][0] + W[i][1] * P.N[j][1] + W[i][2] * P.N[j][2];
}

// The same linearisation as a matrix: for Z = e_k (x) g, dtau_ij = sum_l C[q(i,j)][3k+l] g_l
// with q = 0..5 for (xx, yy, zz, xy, yz, xz), scaled by sc. With P^a = n_a n_a^T the normal
// part is sum_ac D_ac P^a_ij P^c_kl; each eigenvector pair (a,b) adds
// Geff theta_ab (n_a n_b^T + n_b n_a^T)_ij (x_b N_ka N_lb + x_a N_kb N_la). Forming C once
// per point replaces the per-direction rotations of dtau_rank1 by a 6x3 product per node.
template <typename T>
__device__ __forceinline__ void spatial_tangent(const PointMat<T>& P, T sc, T C[6][9]) {
  constexpr int vi[6] = {0, 1, 2, 0, 1, 0}, vj[6] = {0, 1, 2, 1, 2, 2};
  T M[6][3];  // M[q][c] = sc sum_a P^a_q D_ac
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    T pa[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) pa[a] = P.N[vi[q]][a] * P.N[vj[q]][a];
#pragma unroll
    for (int c = 0; c < 3; ++c) M[q][c] = sc * (pa[0] * P.D[0][c] + pa[1] * P.D[1][c] + pa[2] * P.D[2][c]);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = k; l < 3; ++l) {
      const T p0 = P.N[k][0] * P.N[l][0], p1 = P.N[k][1] * P.N[l][1], p2 = P.N[k][2] * P.N[l][2];
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const T v = M[q][0] * p0 + M[q][1] * p1 + M[q][2] * p2;
        C[q][3 * k + l] = v;
        C[q][3 * l + k] = v;
      }
    }
  const int pa_[3] = {0, 0, 1}, pb_[3] = {1, 2, 2};
  const T th[3] = {P.th01, P.th02, P.th12};
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const int a = pa_[t], b = pb_[t];
    const T gs = sc * P.Geff * th[t];
    T S[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) S[q] = gs * (P.N[vi[q]][a] * P.N[vj[q]][b] + P.N[vi[q]][b] * P.N[vj[q]][a]);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const T R = P.x[b] * P.N[k][a] * P.N[l][b] + P.x[a] * P.N[k][b] * P.N[l][a];
#pragma unroll
        for (int q = 0; q < 6; ++q) C[q][3 * k + l] += S[q] * R;
      }
  }
}

// kinematics from nodal displacements: H = sum u (x) dS, dF = I + H, inverse, det
template <typename T>
__device__ __forceinline__ T inv3(const T F[3][3], T R[3][3]) {
  const T c00 = F[1][1] * F[2][2] - F[1][2] * F[2][1];
  const T c01 = F[1][2] * F[2][0] - F[1][0] * F[2][2];
  const T c02 = F[1][0] * F[2][1] - F[1][1] * F[2][0];
  const T det = F[0][0] * c00 + F[0][1] * c01 + F[0][2] * c02;
  const T id = T(1) / det;
  R[0][0] = c00 * id;
  R[1][0] = c01 * id;
  R[2][0] = c02 * id;
  R[0][1] = (F[0][2] * F[2][1] - F[0][1] * F[2][2]) * id;
  R[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) * id;
  R[2][1] = (F[0][1] * F[2][0] - F[0][0] * F[2][1]) * id;
  R[0][2] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) * id;
  R[1][2] = (F[0][2] * F[1][0] - F[0][0] * F[1][2]) * id;
  R[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) * id;
  return det;
}

}  // namespace mpm
