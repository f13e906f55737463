/*
 * Oracle: per-point GIMP basis, Hencky / von Mises update, consistent tangent and the
 * parameter derivatives used by the adjoint. TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#include "orc_internal.h"
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- GIMP basis
 * S_vp = (1/V_p) sum_K int_{Omega_p cap Omega_K} phi~_vK dx (Section 3.2, GIMP basis),
 * evaluated here exactly: each overlap is a box, the trilinear phi_K is a product of 1D
 * linear factors, and each 1D factor is integrated with its antiderivative. The gradient
 * with respect to the point position is the same integral of grad phi~ (phi~ is C0, so
 * differentiation and convolution commute). phi~ = C_K^T phi (Section 3.1, hanging node
 * basis). V_p in the normaliser is the domain volume 8 l1 l2 l3. */
int32_t orc_point_basis(const orc_mesh* m, const double x[3], const double l[3], int32_t* node, double* S,
                        double* dS) {
  int32_t lv[ORC_MAXL];
  double box[6 * ORC_MAXL];
  int nl = orc_point_leaves(m, x, l, lv, box);
  if (nl < 0) return nl;
  double vdom = 8.0 * l[0] * l[1] * l[2];
  int ns = 0;
  for (int k = 0; k < nl; k++) {
    const int32_t* q = m->leaf + 4 * lv[k];
    int s = 1 << (m->c.lvl_max - q[3]);
    double h = s * m->hmin;
    double Iv[3][2], Dv[3][2];
    for (int a = 0; a < 3; a++) {
      double lo = m->c.lo[a] + q[a] * m->hmin;
      double t0 = box[6 * k + 2 * a] - lo, t1 = box[6 * k + 2 * a + 1] - lo;
      double len = box[6 * k + 2 * a + 1] - box[6 * k + 2 * a];
      Iv[a][1] = (t1 * t1 - t0 * t0) / (2.0 * h); /* int t/h */
      Iv[a][0] = len - Iv[a][1];                   /* int (1 - t/h) */
      Dv[a][0] = -len / h;                        /* int d/dx (1 - t/h) */
      Dv[a][1] = len / h;
    }
    const double* C = m->ik_c + (int64_t)lv[k] * 8 * ORC_MAXI;
    const int32_t* ids = m->ik_node + (int64_t)lv[k] * ORC_MAXI;
    for (int z = 0; z < m->ik_n[lv[k]]; z++) {
      int pos = -1;
      for (int t = 0; t < ns; t++) if (node[t] == ids[z]) pos = t;
      if (pos < 0) {
        if (ns >= ORC_MAXS) return ORC_ESTENCIL;
        pos = ns++;
        node[pos] = ids[z];
        S[pos] = 0; dS[3 * pos] = dS[3 * pos + 1] = dS[3 * pos + 2] = 0;
      }
      for (int v = 0; v < 8; v++) {
        double c = C[v * ORC_MAXI + z];
        if (c == 0.0) continue;
        int b0 = v & 1, b1 = (v >> 1) & 1, b2 = (v >> 2) & 1;
        S[pos] += c * Iv[0][b0] * Iv[1][b1] * Iv[2][b2] / vdom;
        dS[3 * pos + 0] += c * Dv[0][b0] * Iv[1][b1] * Iv[2][b2] / vdom;
        dS[3 * pos + 1] += c * Iv[0][b0] * Dv[1][b1] * Iv[2][b2] / vdom;
        dS[3 * pos + 2] += c * Iv[0][b0] * Iv[1][b1] * Dv[2][b2] / vdom;
      }
    }
  }
  return ns;
}

/* ---------------------------------------------------------------- small linear algebra */

static double det3(const double A[3][3]) {
  return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
         A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

static void inv3(const double A[3][3], double R[3][3]) {
  double d = det3(A);
  R[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / d;
  R[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / d;
  R[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / d;
  R[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / d;
  R[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / d;
  R[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / d;
  R[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / d;
  R[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / d;
  R[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / d;
}

static void matmul3(const double A[3][3], const double B[3][3], double C[3][3]) {
  double T[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      T[i][j] = 0;
      for (int k = 0; k < 3; k++) T[i][j] += A[i][k] * B[k][j];
    }
  memcpy(C, T, sizeof(T));
}

static void transpose3(const double A[3][3], double T[3][3]) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) T[i][j] = A[j][i];
}

/* cyclic Jacobi for a symmetric 3x3 matrix: rotations J(p,q) from the 2x2 symmetric Schur
 * decomposition until the off-diagonal norm is below 1e-15 of the matrix norm.
 * Eigenvalues in w, eigenvectors in the columns of V. */
static void jacobi3(const double A0[3][3], double w[3], double V[3][3]) {
  double A[3][3];
  memcpy(A, A0, sizeof(A));
  double nrm = 0;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) { nrm += A[i][j] * A[i][j]; V[i][j] = i == j; }
  nrm = sqrt(nrm);
  static const int P[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  for (int sweep = 0; sweep < 64; sweep++) {
    double off = sqrt(A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2]);
    if (off <= 1e-15 * nrm) break;
    for (int r = 0; r < 3; r++) {
      int p = P[r][0], q = P[r][1];
      if (A[p][q] == 0.0) continue;
      double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
      double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
      double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
      double Jr[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, Jt[3][3];
      Jr[p][p] = c; Jr[p][q] = s; Jr[q][p] = -s; Jr[q][q] = c;
      transpose3(Jr, Jt);
      matmul3(Jt, A, A);
      matmul3(A, Jr, A);
      A[p][q] = A[q][p] = 0.0;
      matmul3(V, Jr, V);
    }
  }
  for (int i = 0; i < 3; i++) w[i] = A[i][i];
}

static void sym_from6(const double v[6], double A[3][3]) {
  A[0][0] = v[0]; A[1][1] = v[1]; A[2][2] = v[2];
  A[0][1] = A[1][0] = v[3]; A[1][2] = A[2][1] = v[4]; A[0][2] = A[2][0] = v[5];
}
static void sym_to6(const double A[3][3], double v[6]) {
  v[0] = A[0][0]; v[1] = A[1][1]; v[2] = A[2][2]; v[3] = A[0][1]; v[4] = A[1][2]; v[5] = A[0][2];
}

/* ---------------------------------------------------------------- constitutive
 * Hencky elasticity (Kirchhoff stress linear in the elastic logarithmic strain) bounded by
 * a von Mises perfect-plasticity surface, returned in principal logarithmic strain space
 * with the small-strain radial return (Section 2.2 and the references it cites). The yield
 * function is sqrt(3 J2) - sigma_y. */
typedef struct {
  double x[3];          /* eigenvalues of the trial b */
  double N[3][3];       /* eigenvectors (columns) */
  double eps[3], eps_e[3], tau_p[3], shat[3];
  double lam, G, Kb, r, qtr;
  int plastic;
} orc_princ;

static int principal_update(const double btr[3][3], double E, double nu, double sy, orc_princ* P) {
  jacobi3(btr, P->x, P->N);
  for (int a = 0; a < 3; a++) if (!(P->x[a] > 0)) return ORC_EDET;
  P->lam = E * nu / ((1 + nu) * (1 - 2 * nu));
  P->G = E / (2 * (1 + nu));
  P->Kb = P->lam + 2.0 * P->G / 3.0;
  double tr = 0;
  for (int a = 0; a < 3; a++) { P->eps[a] = 0.5 * log(P->x[a]); tr += P->eps[a]; }
  double t[3], p = 0, s[3], ns = 0;
  for (int a = 0; a < 3; a++) { t[a] = P->lam * tr + 2 * P->G * P->eps[a]; p += t[a] / 3.0; }
  for (int a = 0; a < 3; a++) { s[a] = t[a] - p; ns += s[a] * s[a]; }
  ns = sqrt(ns);
  P->qtr = sqrt(1.5) * ns;
  P->plastic = isfinite(sy) && (P->qtr - sy > 0);
  P->r = 1.0;
  for (int a = 0; a < 3; a++) { P->shat[a] = ns > 0 ? s[a] / ns : 0.0; P->tau_p[a] = t[a]; P->eps_e[a] = P->eps[a]; }
  if (P->plastic) {
    P->r = sqrt(2.0 / 3.0) * sy / ns;
    for (int a = 0; a < 3; a++) {
      P->tau_p[a] = p + P->r * s[a];
      P->eps_e[a] = P->eps[a] - (1.0 - P->r) * s[a] / (2.0 * P->G);
    }
  }
  return ORC_OK;
}

static double theta_ab(double xa, double xb) {
  if (xa == xb) return 1.0 / xb;
  double d = (xa - xb) / xb;
  return log1p(d) / (d * xb);
}

int32_t orc_material_point(const double dF9[9], const double bn6[6], double Jn, double E, double nu, double sy,
                           double sigma6[6], double tau6[6], double a81[81], double be6[6], double info[3]) {
  double F[3][3], Ft[3][3], bn[3][3], btr[3][3];
  memcpy(F, dF9, sizeof(F));
  double Jd = det3(F);
  if (!(Jd > 0)) return ORC_EDET;
  sym_from6(bn6, bn);
  transpose3(F, Ft);
  matmul3(F, bn, btr);
  matmul3(btr, Ft, btr);
  for (int i = 0; i < 3; i++) for (int j = i + 1; j < 3; j++) btr[i][j] = btr[j][i] = 0.5 * (btr[i][j] + btr[j][i]);
  orc_princ P;
  int st = principal_update(btr, E, nu, sy, &P);
  if (st) return st;
  double J = Jd * Jn;
  double tau[3][3] = {{0}}, sig[3][3], be[3][3] = {{0}}, Nh[3][3] = {{0}};
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      for (int a = 0; a < 3; a++) {
        double mm = P.N[i][a] * P.N[j][a];
        tau[i][j] += P.tau_p[a] * mm;
        be[i][j] += exp(2.0 * P.eps_e[a]) * mm;
        Nh[i][j] += P.shat[a] * mm;
      }
  for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) sig[i][j] = tau[i][j] / J;
  if (sigma6) sym_to6(sig, sigma6);
  if (tau6) sym_to6(tau, tau6);
  if (be6) sym_to6(be, be6);
  if (info) { info[0] = P.plastic; info[1] = P.qtr; info[2] = J; }
  if (!a81) return ORC_OK;

  /* consistent spatial tangent a_ijkl = (1/2J) (D:L:B)_ijkl - sigma_il delta_jk with
   * D = dtau/deps (algorithmic, closed form), L = d ln b / d b (spectral), B = d b/d(grad u) */
  double D[3][3][3][3], L[3][3][3][3], B[3][3][3][3], DL[3][3][3][3];
  double th[3][3];
  for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++) th[a][b] = a == b ? 1.0 / P.x[a] : theta_ab(P.x[a], P.x[b]);
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      for (int k = 0; k < 3; k++)
        for (int l = 0; l < 3; l++) {
          double dij = i == j, dkl = k == l, dik = i == k, djl = j == l, dil = i == l, djk = j == k;
          double Is = 0.5 * (dik * djl + dil * djk);
          if (P.plastic)
            D[i][j][k][l] = P.Kb * dij * dkl + 2.0 * P.G * P.r * (Is - dij * dkl / 3.0 - Nh[i][j] * Nh[k][l]);
          else
            D[i][j][k][l] = P.lam * dij * dkl + 2.0 * P.G * Is;
          double Lv = 0;
          for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Lv += th[a][b] * P.N[i][a] * P.N[j][b] * P.N[k][a] * P.N[l][b];
          L[i][j][k][l] = Lv;
          B[i][j][k][l] = dik * btr[j][l] + djk * btr[i][l];
        }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      for (int r = 0; r < 3; r++)
        for (int s = 0; s < 3; s++) {
          double v = 0;
          for (int p = 0; p < 3; p++) for (int q = 0; q < 3; q++) v += D[i][j][p][q] * L[p][q][r][s];
          DL[i][j][r][s] = v;
        }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      for (int k = 0; k < 3; k++)
        for (int l = 0; l < 3; l++) {
          double v = 0;
          for (int r = 0; r < 3; r++) for (int s = 0; s < 3; s++) v += DL[i][j][r][s] * B[r][s][k][l];
          a81[((i * 3 + j) * 3 + k) * 3 + l] = v / (2.0 * J) - sig[i][l] * (j == k);
        }
  return ORC_OK;
}

/* ---------------------------------------------------------------- per-point kinematics */

typedef struct {
  int ns;
  int32_t node[ORC_MAXS];
  double S[ORC_MAXS], dS[3 * ORC_MAXS];
  double dF[3][3], Finv[3][3], Jd;
  double g[3 * ORC_MAXS]; /* grad_x S = dF^{-T} grad_n S */
} orc_kin;

static int kinematics(const orc_mesh* m, const orc_state* s, int64_t p, const double* u, orc_kin* k) {
  int64_t n = m->np;
  double x[3] = {s->x[p], s->x[n + p], s->x[2 * n + p]}, l[3] = {s->l[p], s->l[n + p], s->l[2 * n + p]};
  int ns = orc_point_basis(m, x, l, k->node, k->S, k->dS);
  if (ns < 0) return ns;
  k->ns = ns;
  for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) k->dF[i][j] = i == j;
  for (int v = 0; v < ns; v++)
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) k->dF[i][j] += u[3 * k->node[v] + i] * k->dS[3 * v + j];
  k->Jd = det3(k->dF);
  if (!(k->Jd > 0)) return ORC_EDET;
  inv3(k->dF, k->Finv);
  for (int v = 0; v < ns; v++)
    for (int j = 0; j < 3; j++) {
      double t = 0;
      for (int mm = 0; mm < 3; mm++) t += k->Finv[mm][j] * k->dS[3 * v + mm];
      k->g[3 * v + j] = t;
    }
  return ORC_OK;
}

static int64_t csr_find(const orc_mesh* m, int64_t row, int32_t colv) {
  int64_t lo = m->row_ptr[row], hi = m->row_ptr[row + 1] - 1;
  while (lo <= hi) {
    int64_t mid = (lo + hi) / 2;
    if (m->col[mid] == colv) return mid;
    if (m->col[mid] < colv) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

/* Updated-Lagrangian weak form (Section 2.1): f_v = sum_p V_p sigma_p grad_x S_vp with
 * V_p = det(dF) V_n, and K = d f_int / d u with the basis frozen over the step. One point's
 * share, added into f_int and K; the per-point outputs are written when their arrays are given. */
static int32_t assemble_point(const orc_mesh* m, const orc_state* s, const double* u, int64_t p, orc_kin* k,
                              double* f_int, double* K, double* sigma6, double* Fnew9, double* be6,
                              uint8_t* plastic, double* qtrial) {
  int64_t n = m->np;
  double a[81];
  int st = kinematics(m, s, p, u, k);
  if (st) return st;
  double bn[6], sig[6], tau[6], be[6], info[3];
  for (int c = 0; c < 6; c++) bn[c] = s->bn[c * n + p];
  st = orc_material_point((const double*)k->dF, bn, s->Jn[p], s->E[p], s->nu[p], s->sy[p], sig, tau, K ? a : NULL, be,
                          info);
  if (st) return st;
  if (sigma6) for (int c = 0; c < 6; c++) sigma6[c * n + p] = sig[c];
  if (be6) for (int c = 0; c < 6; c++) be6[c * n + p] = be[c];
  if (plastic) plastic[p] = (uint8_t)info[0];
  if (qtrial) qtrial[p] = info[1];
  if (Fnew9 && s->Fn) {
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) {
        double t = 0;
        for (int mm = 0; mm < 3; mm++) t += k->dF[i][mm] * s->Fn[(3 * mm + j) * n + p];
        Fnew9[(3 * i + j) * n + p] = t;
      }
  }
  double S3[3][3];
  sym_from6(sig, S3);
  double V = k->Jd * s->vol[p];
  for (int v = 0; v < k->ns; v++)
    for (int i = 0; i < 3; i++) {
      double t = 0;
      for (int j = 0; j < 3; j++) t += S3[i][j] * k->g[3 * v + j];
      f_int[3 * k->node[v] + i] += V * t;
    }
  if (!K) return ORC_OK;
  for (int va = 0; va < k->ns; va++)
    for (int vb = 0; vb < k->ns; vb++)
      for (int i = 0; i < 3; i++)
        for (int kk = 0; kk < 3; kk++) {
          double t = 0;
          for (int j = 0; j < 3; j++)
            for (int l = 0; l < 3; l++) t += k->g[3 * va + j] * a[((i * 3 + j) * 3 + kk) * 3 + l] * k->g[3 * vb + l];
          int64_t pos = csr_find(m, 3 * (int64_t)k->node[va] + i, 3 * k->node[vb] + kk);
          if (pos < 0) return ORC_ESTENCIL;
          K[pos] += V * t;
        }
  return ORC_OK;
}

int32_t orc_assemble(const orc_mesh* m, const orc_state* s, const double* u, double* f_int, double* K,
                     double* sigma6, double* Fnew9, double* be6, uint8_t* plastic, double* qtrial, int64_t* bad) {
  *bad = -1;
  memset(f_int, 0, (size_t)(3 * m->nindep) * sizeof(double));
  if (K) memset(K, 0, (size_t)m->nnz * sizeof(double));
  static orc_kin k;
  for (int64_t p = 0; p < m->np; p++) {
    int st = assemble_point(m, s, u, p, &k, f_int, K, sigma6, Fnew9, be6, plastic, qtrial);
    if (st) { *bad = p; return st; }
  }
  return ORC_OK;
}

/* The same assembly timed on several host threads (no other use): the points are cut into
 * nthreads contiguous ranges, each thread adds its points into its own f_int and K, and the
 * thread copies are added in thread order, so the result depends only on nthreads and equals
 * orc_assemble's up to the order of the sums. */
int32_t orc_assemble_threads(const orc_mesh* m, const orc_state* s, const double* u, double* f_int, double* K,
                             double* sigma6, int32_t nthreads, int64_t* bad) {
  *bad = -1;
  if (nthreads < 1) nthreads = 1;
  const int64_t nf = 3 * m->nindep, nk = K ? m->nnz : 0, n = m->np;
  double** fp = (double**)calloc((size_t)nthreads, sizeof(double*));
  double** kp = (double**)calloc((size_t)nthreads, sizeof(double*));
  int64_t* badt = (int64_t*)malloc((size_t)nthreads * sizeof(int64_t));
  int32_t* stt = (int32_t*)calloc((size_t)nthreads, sizeof(int32_t));
  int oom = !fp || !kp || !badt || !stt;
  for (int t = 0; t < nthreads && !oom; t++) {
    fp[t] = (double*)calloc((size_t)(nf > 0 ? nf : 1), sizeof(double));
    kp[t] = (double*)calloc((size_t)(nk > 0 ? nk : 1), sizeof(double));
    badt[t] = -1;
    if (!fp[t] || !kp[t]) oom = 1;
  }
  int32_t rc = ORC_OK;
  if (oom) {
    rc = ORC_EARG;
  } else {
#pragma omp parallel num_threads(nthreads)
    {
#ifdef _OPENMP
      const int t = omp_get_thread_num(), nt = omp_get_num_threads();
#else
      const int t = 0, nt = 1;
#endif
      orc_kin k;
      for (int tt = t; tt < nthreads; tt += nt) {  /* every range is taken, whatever team size */
        const int64_t p0 = n * tt / nthreads, p1 = n * (tt + 1) / nthreads;
        for (int64_t p = p0; p < p1; p++) {
          int st = assemble_point(m, s, u, p, &k, fp[tt], K ? kp[tt] : NULL, sigma6, NULL, NULL, NULL, NULL);
          if (st) { stt[tt] = st; badt[tt] = p; break; }
        }
      }
#pragma omp barrier
#pragma omp for schedule(static)
      for (int64_t i = 0; i < nf; i++) {
        double acc = 0;
        for (int tt = 0; tt < nthreads; tt++) acc += fp[tt][i];
        f_int[i] = acc;
      }
#pragma omp for schedule(static)
      for (int64_t i = 0; i < nk; i++) {
        double acc = 0;
        for (int tt = 0; tt < nthreads; tt++) acc += kp[tt][i];
        K[i] = acc;
      }
    }
    for (int t = 0; t < nthreads; t++)
      if (stt[t]) { rc = stt[t]; *bad = badt[t]; break; }
  }
  for (int t = 0; t < nthreads && fp && kp; t++) { free(fp[t]); free(kp[t]); }
  free(fp); free(kp); free(badt); free(stt);
  return rc;
}

/* body force term of the weak form: f_ext,v = sum_p S_vp m_p g */
int32_t orc_external_force(const orc_mesh* m, const orc_state* s, double* f_ext) {
  int64_t n = m->np;
  memset(f_ext, 0, (size_t)(3 * m->nindep) * sizeof(double));
  static int32_t node[ORC_MAXS];
  static double S[ORC_MAXS], dS[3 * ORC_MAXS];
  for (int64_t p = 0; p < n; p++) {
    double x[3] = {s->x[p], s->x[n + p], s->x[2 * n + p]}, l[3] = {s->l[p], s->l[n + p], s->l[2 * n + p]};
    int ns = orc_point_basis(m, x, l, node, S, dS);
    if (ns < 0) return ns;
    for (int v = 0; v < ns; v++)
      for (int i = 0; i < 3; i++) f_ext[3 * node[v] + i] += S[v] * s->mass[p] * s->g[i];
  }
  return ORC_OK;
}

/* Inertia term of the weak form (Section 2.1, eq. MPMweak: sum_p S_vp m_p a_p) with Newmark's
 * method at gamma = 1, beta = 1/2 (Section 2.4). Over a step with nodal displacement u the
 * point displacement is du_p = sum_v S_vp u_v (basis frozen at the start of the step); the
 * Newmark relations du = dt v_n + dt^2 ((1/2 - beta) a_n + beta a_{n+1}) and
 * v_{n+1} = v_n + dt ((1 - gamma) a_n + gamma a_{n+1}) give, at these parameters,
 *   a_p = 2 (du_p - dt v_p) / dt^2   and   v_p,new = v_p + dt a_p.
 * f_iner,v = sum_p S_vp m_p a_p; its derivative with respect to u is (2/dt^2) M with the
 * consistent mass M_vw = sum_p m_p S_vp S_wp (times the 3x3 identity), added into K when K is
 * given. vel, a_new, v_new are [3][n] in original point order. */
int32_t orc_inertia(const orc_mesh* m, const orc_state* s, const double* u, const double* vel, double dt,
                    double* f_iner, double* K, double* a_new, double* v_new, int64_t* bad) {
  *bad = -1;
  int64_t n = m->np;
  memset(f_iner, 0, (size_t)(3 * m->nindep) * sizeof(double));
  static int32_t node[ORC_MAXS];
  static double S[ORC_MAXS], dS[3 * ORC_MAXS];
  const double c2 = 2.0 / (dt * dt);
  for (int64_t p = 0; p < n; p++) {
    double x[3] = {s->x[p], s->x[n + p], s->x[2 * n + p]}, l[3] = {s->l[p], s->l[n + p], s->l[2 * n + p]};
    int ns = orc_point_basis(m, x, l, node, S, dS);
    if (ns < 0) { *bad = p; return ns; }
    double acc[3];
    for (int i = 0; i < 3; i++) {
      double du = 0;
      for (int v = 0; v < ns; v++) du += S[v] * u[3 * node[v] + i];
      acc[i] = c2 * (du - dt * vel[i * n + p]);
      if (a_new) a_new[i * n + p] = acc[i];
      if (v_new) v_new[i * n + p] = vel[i * n + p] + dt * acc[i];
    }
    for (int v = 0; v < ns; v++)
      for (int i = 0; i < 3; i++) f_iner[3 * node[v] + i] += S[v] * s->mass[p] * acc[i];
    if (!K) continue;
    for (int va = 0; va < ns; va++)
      for (int vb = 0; vb < ns; vb++)
        for (int i = 0; i < 3; i++) {
          int64_t pos = csr_find(m, 3 * (int64_t)node[va] + i, 3 * node[vb] + i);
          if (pos < 0) { *bad = p; return ORC_ESTENCIL; }
          K[pos] += c2 * s->mass[p] * S[va] * S[vb];
        }
  }
  return ORC_OK;
}

void orc_residual(int64_t ndof, const double* f_int, const double* f_ext, const uint8_t* dir, double* r,
                  double* rnorm) {
  double acc = 0;
  for (int64_t i = 0; i < ndof; i++) {
    r[i] = (dir && dir[i]) ? 0.0 : f_int[i] - (f_ext ? f_ext[i] : 0.0);
    acc += r[i] * r[i];
  }
  *rnorm = sqrt(acc);
}

/* principal Kirchhoff stresses for complex material parameters (used for the complex-step
 * derivative); the elastic/plastic branch is taken from the real parts. */
static void tau_principal_c(const double eps[3], double complex E, double complex nu, double complex sy, int sy_finite,
                            double complex t_out[3]) {
  double complex lam = E * nu / ((1 + nu) * (1 - 2 * nu)), G = E / (2 * (1 + nu));
  double tr = eps[0] + eps[1] + eps[2];
  double complex t[3], p = 0, s[3], ns2 = 0;
  for (int a = 0; a < 3; a++) { t[a] = lam * tr + 2 * G * eps[a]; p += t[a] / 3.0; }
  for (int a = 0; a < 3; a++) { s[a] = t[a] - p; ns2 += s[a] * s[a]; }
  double complex ns = csqrt(ns2);
  int plastic = sy_finite && (creal(csqrt(1.5 * ns2)) - creal(sy) > 0);
  for (int a = 0; a < 3; a++) t_out[a] = plastic ? p + csqrt(2.0 / 3.0) * sy / ns * s[a] : t[a];
}

/* Adjoint of L = lambda . f_int: with G = sum_v lambda_v (x) grad_x S_v, the point's share
 * is L_p = (V_n/J_n) tau : G, so dL/dVn = tau:G / J_n and dL/dtheta = (V_n/J_n) dtau/dtheta : G
 * (eigenvectors of the trial b do not depend on the material parameters). The parameter
 * derivatives of the principal stresses are taken by complex step. */
int32_t orc_adjoint(const orc_mesh* m, const orc_state* s, const double* u, const double* lambda, double* dE,
                    double* dnu, double* dsy, double* dV, int64_t* bad) {
  *bad = -1;
  int64_t n = m->np;
  static orc_kin k;
  for (int64_t p = 0; p < n; p++) {
    int st = kinematics(m, s, p, u, &k);
    if (st) { *bad = p; return st; }
    double G3[3][3] = {{0}};
    for (int v = 0; v < k.ns; v++)
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) G3[i][j] += lambda[3 * k.node[v] + i] * k.g[3 * v + j];
    double bn[3][3], Ft[3][3], btr[3][3];
    double bn6[6];
    for (int c = 0; c < 6; c++) bn6[c] = s->bn[c * n + p];
    sym_from6(bn6, bn);
    transpose3(k.dF, Ft);
    matmul3(k.dF, bn, btr);
    matmul3(btr, Ft, btr);
    for (int i = 0; i < 3; i++) for (int j = i + 1; j < 3; j++) btr[i][j] = btr[j][i] = 0.5 * (btr[i][j] + btr[j][i]);
    orc_princ P;
    st = principal_update(btr, s->E[p], s->nu[p], s->sy[p], &P);
    if (st) { *bad = p; return st; }
    double Ga[3];
    for (int a = 0; a < 3; a++) {
      Ga[a] = 0;
      for (int i = 0; i < 3; i++) for (int j = 0; j < 3; j++) Ga[a] += P.N[i][a] * G3[i][j] * P.N[j][a];
    }
    double tauG = 0;
    for (int a = 0; a < 3; a++) tauG += P.tau_p[a] * Ga[a];
    double Jn = s->Jn[p], Vn = s->vol[p];
    dV[p] = tauG / Jn;
    double E = s->E[p], nu = s->nu[p], sy = s->sy[p];
    int syf = isfinite(sy);
    double complex t[3];
    const double h = 1e-30;
    double d;
    tau_principal_c(P.eps, E + I * h * E, nu, syf ? sy : 0, syf, t);
    d = 0;
    for (int a = 0; a < 3; a++) d += cimag(t[a]) / (h * E) * Ga[a];
    dE[p] = Vn / Jn * d;
    tau_principal_c(P.eps, E, nu + I * h, syf ? sy : 0, syf, t);
    d = 0;
    for (int a = 0; a < 3; a++) d += cimag(t[a]) / h * Ga[a];
    dnu[p] = Vn / Jn * d;
    if (syf) {
      tau_principal_c(P.eps, E, nu, sy + I * h * sy, syf, t);
      d = 0;
      for (int a = 0; a < 3; a++) d += cimag(t[a]) / (h * sy) * Ga[a];
      dsy[p] = Vn / Jn * d;
    } else {
      dsy[p] = 0.0;
    }
  }
  return ORC_OK;
}
