/*
 * Oracle: ghost stabilisation of the stiffness (Section 4, eq. ghost). TEST INFRASTRUCTURE ONLY.
 *
 * Populated leaves: overlapped with positive volume by at least one material point domain.
 * Boundary leaves: populated leaves that share a face with an unpopulated leaf. Ghost faces:
 * the faces shared by a boundary leaf K+ and a populated leaf K- (each geometric face once; on
 * an octree face the shared region is the smaller of the two leaf faces). On each ghost face F
 *   j_F(u, v) = (h_F beta_F / kappa) int_F [d_n u] . [d_n v] dA,   kappa = 10,
 * [d_n u] = (grad u^+ - grad u^-) n (first normal derivative, read with k = 1), h_F the larger
 * side of the two leaves, beta_F the larger of the two leaves' maxima of the Young's moduli of
 * the points overlapping them. u on each leaf is the constrained trilinear field
 * sum_slot u_slot phi~_slot (Section 3.1, hanging node basis). The integrand is a product of
 * two functions bilinear on F, integrated here with a 3 x 3 Gauss rule (exact).
 *
 * The bilinear form adds (h beta / kappa) G_F[a][b] to the diagonal of the 3x3 block (a, b)
 * of K for every pair of nodes a, b of I(K+) u I(K-), and K_G u to the internal force (the
 * penalty acts on the displacement of the step).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "orc_internal.h"

static const double GHOST_KAPPA = 10.0;

/* the leaves across one face of leaf e: face on axis a, side sg (+1: the face at q_a + s) */
static int face_neighbours(const orc_mesh* m, int64_t e, int a, int sg, int32_t* out, int cap) {
  const int32_t* q = m->leaf + 4 * e;
  int s = 1 << (m->c.lvl_max - q[3]);
  int lim[3] = {m->nx, m->ny, m->nz};
  int pa = sg > 0 ? q[a] + s : q[a] - 1;
  if (pa < 0 || pa >= lim[a]) return 0;
  int b = (a + 1) % 3, c = (a + 2) % 3;
  int n = 0;
  for (int i = 0; i < s; i++)
    for (int j = 0; j < s; j++) {
      int cell[3];
      cell[a] = pa;
      cell[b] = q[b] + i;
      cell[c] = q[c] + j;
      int32_t k = m->leafmap[((int64_t)cell[2] * m->ny + cell[1]) * m->nx + cell[0]];
      int seen = 0;
      for (int t = 0; t < n; t++) seen |= out[t] == k;
      if (!seen && n < cap) out[n++] = k;
    }
  return n;
}

static int cmp_face(const void* x, const void* y) {
  const int32_t *p = (const int32_t*)x, *q = (const int32_t*)y;
  if (p[0] != q[0]) return p[0] < q[0] ? -1 : 1;
  return p[1] < q[1] ? -1 : (p[1] > q[1]);
}

/* ghost faces from the populated flags: rows (lo leaf, hi leaf, axis, plane, b0, b1, c0, c1)
 * in lattice units, sorted by (lo, hi); returns the count */
int64_t orc_ghost_build_faces(orc_mesh* m, const uint8_t* pop) {
  free(m->gface);
  m->gface = NULL;
  m->ngface = 0;
  uint8_t* bnd = (uint8_t*)calloc((size_t)m->nleaf + 1, 1);
  int32_t nb[4096];
  for (int64_t e = 0; e < m->nleaf; e++) {
    if (!pop[e]) continue;
    int s = 1 << (m->c.lvl_max - m->leaf[4 * e + 3]);
    int cap = s * s < 4096 ? s * s : 4096;
    for (int a = 0; a < 3 && !bnd[e]; a++)
      for (int sg = -1; sg <= 1; sg += 2) {
        int k = face_neighbours(m, e, a, sg, nb, cap);
        for (int t = 0; t < k; t++) bnd[e] |= !pop[nb[t]];
      }
  }
  int64_t cap = 1024, n = 0;
  int32_t* f = (int32_t*)malloc((size_t)cap * 8 * sizeof(int32_t));
  for (int64_t e = 0; e < m->nleaf; e++) {
    if (!bnd[e]) continue;
    const int32_t* q = m->leaf + 4 * e;
    int s = 1 << (m->c.lvl_max - q[3]);
    int ncap = s * s < 4096 ? s * s : 4096;
    for (int a = 0; a < 3; a++)
      for (int sg = -1; sg <= 1; sg += 2) {
        int k = face_neighbours(m, e, a, sg, nb, ncap);
        for (int t = 0; t < k; t++) {
          int32_t o = nb[t];
          if (!pop[o]) continue;
          const int32_t* r = m->leaf + 4 * o;
          int so = 1 << (m->c.lvl_max - r[3]);
          int b = (a + 1) % 3, c = (a + 2) % 3;
          int b0 = q[b] > r[b] ? q[b] : r[b], b1 = (q[b] + s) < (r[b] + so) ? q[b] + s : r[b] + so;
          int c0 = q[c] > r[c] ? q[c] : r[c], c1 = (q[c] + s) < (r[c] + so) ? q[c] + s : r[c] + so;
          if (n == cap) { cap *= 2; f = (int32_t*)realloc(f, (size_t)cap * 8 * sizeof(int32_t)); }
          int32_t* w = f + 8 * n++;
          w[0] = (int32_t)(e < o ? e : o);
          w[1] = (int32_t)(e < o ? o : e);
          w[2] = a;
          w[3] = sg > 0 ? q[a] + s : q[a];
          w[4] = b0; w[5] = b1; w[6] = c0; w[7] = c1;
        }
      }
  }
  free(bnd);
  qsort(f, (size_t)n, 8 * sizeof(int32_t), cmp_face);
  int64_t u = 0;  /* a face seen from both of its (boundary) leaves appears twice */
  for (int64_t i = 0; i < n; i++)
    if (u == 0 || f[8 * i] != f[8 * (u - 1)] || f[8 * i + 1] != f[8 * (u - 1) + 1]) {
      memmove(f + 8 * u, f + 8 * i, 8 * sizeof(int32_t));
      u++;
    }
  m->gface = f;
  m->ngface = u;
  return u;
}

/* node pairs of the ghost faces appended to pairs (independent ids a << 32 | b) */
int64_t orc_ghost_pairs(const orc_mesh* m, uint64_t** pairs, int64_t npair, int64_t* cap) {
  for (int64_t i = 0; i < m->ngface; i++) {
    int32_t ids[2 * ORC_MAXI];
    int ni = 0;
    for (int side = 0; side < 2; side++) {
      int32_t e = m->gface[8 * i + side];
      for (int z = 0; z < m->ik_n[e]; z++) {
        int32_t id = m->ik_node[(int64_t)e * ORC_MAXI + z];
        int seen = 0;
        for (int t = 0; t < ni; t++) seen |= ids[t] == id;
        if (!seen) ids[ni++] = id;
      }
    }
    for (int x = 0; x < ni; x++)
      for (int y = 0; y < ni; y++) {
        if (npair == *cap) { *cap *= 2; *pairs = (uint64_t*)realloc(*pairs, (size_t)*cap * sizeof(uint64_t)); }
        (*pairs)[npair++] = ((uint64_t)(uint32_t)ids[x] << 32) | (uint32_t)ids[y];
      }
  }
  return npair;
}

/* d phi~_slot / dx_a of leaf e at the point p (physical), for every slot */
static void slot_normal_derivative(const orc_mesh* m, int32_t e, const double p[3], int a, double* out) {
  const int32_t* q = m->leaf + 4 * e;
  int s = 1 << (m->c.lvl_max - q[3]);
  double h = s * m->hmin;
  double xi[3];
  for (int t = 0; t < 3; t++) xi[t] = (p[t] - (m->c.lo[t] + q[t] * m->hmin)) / h;
  double dphi[8];
  for (int v = 0; v < 8; v++) {
    double g = 1.0;
    for (int t = 0; t < 3; t++) {
      int bit = (v >> t) & 1;
      if (t == a) g *= (bit ? 1.0 : -1.0) / h;
      else g *= bit ? xi[t] : 1.0 - xi[t];
    }
    dphi[v] = g;
  }
  const double* C = m->ik_c + (int64_t)e * 8 * ORC_MAXI;
  for (int z = 0; z < m->ik_n[e]; z++) {
    double d = 0.0;
    for (int v = 0; v < 8; v++) d += C[v * ORC_MAXI + z] * dphi[v];
    out[z] = d;
  }
}

int32_t orc_ghost_assemble(const orc_mesh* m, const orc_state* s, const double* u, double* K, double* f,
                           double* beta_leaf) {
  if (!m->gface && m->ngface) return ORC_EARG;
  int64_t n = m->np;
  double* beta = (double*)calloc((size_t)m->nleaf + 1, sizeof(double));
  int32_t lv[ORC_MAXL];
  double box[6 * ORC_MAXL];
  for (int64_t p = 0; p < n; p++) {
    double x[3] = {s->x[p], s->x[n + p], s->x[2 * n + p]}, l[3] = {s->l[p], s->l[n + p], s->l[2 * n + p]};
    int nl = orc_point_leaves(m, x, l, lv, box);
    if (nl < 0) { free(beta); return nl; }
    for (int k = 0; k < nl; k++)
      if (s->E[p] > beta[lv[k]]) beta[lv[k]] = s->E[p];
  }
  if (beta_leaf) memcpy(beta_leaf, beta, (size_t)m->nleaf * sizeof(double));
  const double gx[3] = {0.5 - 0.5 * sqrt(0.6), 0.5, 0.5 + 0.5 * sqrt(0.6)};
  const double gw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  for (int64_t i = 0; i < m->ngface; i++) {
    const int32_t* F = m->gface + 8 * i;
    int32_t ep = F[0], em = F[1];
    int a = F[2], b = (a + 1) % 3, c = (a + 2) % 3;
    int32_t ids[2 * ORC_MAXI];
    int ni = 0, map[2][ORC_MAXI];
    for (int side = 0; side < 2; side++) {
      int32_t e = F[side];
      for (int z = 0; z < m->ik_n[e]; z++) {
        int32_t id = m->ik_node[(int64_t)e * ORC_MAXI + z];
        int pos = -1;
        for (int t = 0; t < ni; t++) if (ids[t] == id) pos = t;
        if (pos < 0) { pos = ni; ids[ni++] = id; }
        map[side][z] = pos;
      }
    }
    double G[2 * ORC_MAXI][2 * ORC_MAXI];
    memset(G, 0, sizeof(G));
    double fb = (F[5] - F[4]) * m->hmin, fc = (F[7] - F[6]) * m->hmin;
    for (int gi = 0; gi < 3; gi++)
      for (int gj = 0; gj < 3; gj++) {
        double p[3];
        p[a] = m->c.lo[a] + F[3] * m->hmin;
        p[b] = m->c.lo[b] + F[4] * m->hmin + gx[gi] * fb;
        p[c] = m->c.lo[c] + F[6] * m->hmin + gx[gj] * fc;
        double J[2 * ORC_MAXI];
        memset(J, 0, sizeof(J));
        double d[ORC_MAXI];
        slot_normal_derivative(m, ep, p, a, d);
        for (int z = 0; z < m->ik_n[ep]; z++) J[map[0][z]] += d[z];
        slot_normal_derivative(m, em, p, a, d);
        for (int z = 0; z < m->ik_n[em]; z++) J[map[1][z]] -= d[z];
        double w = gw[gi] * gw[gj] * fb * fc;
        for (int x = 0; x < ni; x++)
          for (int y = 0; y < ni; y++) G[x][y] += w * J[x] * J[y];
      }
    int sp = 1 << (m->c.lvl_max - m->leaf[4 * ep + 3]), sm = 1 << (m->c.lvl_max - m->leaf[4 * em + 3]);
    double hF = (sp > sm ? sp : sm) * m->hmin;
    double bF = beta[ep] > beta[em] ? beta[ep] : beta[em];
    double sc = hF * bF / GHOST_KAPPA;
    for (int x = 0; x < ni; x++)
      for (int y = 0; y < ni; y++) {
        double v = sc * G[x][y];
        for (int r = 0; r < 3; r++) {
          if (f) f[3 * (int64_t)ids[x] + r] += v * u[3 * (int64_t)ids[y] + r];
          if (K) {
            int64_t row = 3 * (int64_t)ids[x] + r, lo = m->row_ptr[row], hi = m->row_ptr[row + 1] - 1;
            int32_t cv = 3 * ids[y] + r;
            int64_t pos = -1;
            while (lo <= hi) {
              int64_t mid = (lo + hi) / 2;
              if (m->col[mid] == cv) { pos = mid; break; }
              if (m->col[mid] < cv) lo = mid + 1;
              else hi = mid - 1;
            }
            if (pos < 0) { free(beta); return ORC_ESTENCIL; }
            K[pos] += v;
          }
        }
      }
  }
  free(beta);
  return ORC_OK;
}

int64_t orc_ghost_nfaces(const orc_mesh* m) { return m->ngface; }

void orc_ghost_faces(const orc_mesh* m, int32_t* out) {
  if (m->ngface) memcpy(out, m->gface, (size_t)m->ngface * 8 * sizeof(int32_t));
}

void orc_mesh_set_ghost(orc_mesh* m, int32_t enable) { m->ghost = enable; }
