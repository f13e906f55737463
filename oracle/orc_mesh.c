/*
 * Oracle: octree mesh, hanging nodes, constraints, numbering, point order and the CSR
 * pattern. TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Everything here is done on dense arrays over the finest lattice, by direct application
 * of the definitions:
 *   - refinement Steps 1-3 of Section 5, repeated until no element is marked, each round
 *     followed by 2:1 face/edge balance to a fixpoint ("no more than one hanging node on
 *     an edge or face", Section 5);
 *   - hanging node: a node lying on the boundary of an element without being one of its
 *     vertices (Section 3.1, hanging node equation); K_n is the coarsest such element;
 *   - constraint weights phi_{i K_n}(x_n) (Section 3.1, constraint equation, reduced form);
 *   - independent set I(K) and modified basis coefficients (Section 3.1, hanging node basis).
 */
#include "orc_internal.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define TIE 1e-12   /* relative slack that makes ties on the refinement predicates inclusive */

uint64_t orc_morton3(uint64_t x, uint64_t y, uint64_t z) {
  uint64_t r = 0;
  for (int b = 0; b < 21; b++) {
    r |= ((x >> b) & 1ull) << (3 * b);
    r |= ((y >> b) & 1ull) << (3 * b + 1);
    r |= ((z >> b) & 1ull) << (3 * b + 2);
  }
  return r;
}

/* ---------------------------------------------------------------- body geometry */

/* distance^2 from (rho, z) to the segment (r0,z0)-(r1,z1) in the meridian half-plane */
static double seg_d2(double r, double z, double r0, double z0, double r1, double z1) {
  double dr = r1 - r0, dz = z1 - z0;
  double L2 = dr * dr + dz * dz;
  double t = L2 > 0 ? ((r - r0) * dr + (z - z0) * dz) / L2 : 0.0;
  if (t < 0) t = 0;
  if (t > 1) t = 1;
  double er = r - (r0 + t * dr), ez = z - (z0 + t * dz);
  return er * er + ez * ez;
}

/* Step 2: is point p within distance dx of the closed body (distance 0 inside)? */
static int body_near(const orc_crit* c, const double p[3], double dx) {
  const double* b = c->body;
  switch (c->body_kind) {
    case 1: {
      double d2 = (p[0] - b[0]) * (p[0] - b[0]) + (p[1] - b[1]) * (p[1] - b[1]) + (p[2] - b[2]) * (p[2] - b[2]);
      double R = b[3] + dx;
      return d2 <= R * R * (1.0 + TIE);
    }
    case 2: {
      double rho = sqrt((p[0] - b[0]) * (p[0] - b[0]) + (p[1] - b[1]) * (p[1] - b[1]));
      double z = p[2], za = b[2], R = b[3], t = b[4], zt = b[5];
      double zc = za + R / t;
      double rad = (z - za) * t;
      if (rad > R) rad = R;
      if (z >= za && z <= zt && rho <= rad) return 1;
      double d2 = seg_d2(rho, z, 0.0, za, R, zc);
      double d = seg_d2(rho, z, R, zc, R, zt);
      if (d < d2) d2 = d;
      d = seg_d2(rho, z, R, zt, 0.0, zt);
      if (d < d2) d2 = d;
      return d2 <= dx * dx * (1.0 + TIE);
    }
    case 3: {
      double d2 = 0;
      for (int a = 0; a < 3; a++) {
        double lo = b[2 * a], hi = b[2 * a + 1], e = 0;
        if (p[a] < lo) e = lo - p[a];
        else if (p[a] > hi) e = p[a] - hi;
        d2 += e * e;
      }
      return d2 <= dx * dx * (1.0 + TIE);
    }
    default:
      return 0;
  }
}

/* Step 1: does the closed box [lo,hi] meet the closed body? */
static int body_meets(const orc_crit* c, const double lo[3], const double hi[3]) {
  const double* b = c->body;
  switch (c->body_kind) {
    case 1: {
      double d2 = 0;
      for (int a = 0; a < 3; a++) {
        double e = 0;
        if (b[a] < lo[a]) e = lo[a] - b[a];
        else if (b[a] > hi[a]) e = b[a] - hi[a];
        d2 += e * e;
      }
      return d2 <= b[3] * b[3] * (1.0 + TIE);
    }
    case 2: {
      /* the solid's radius grows with z, so the box meets it iff at the highest common z
       * the radial distance of the box footprint to the axis is within the radius */
      double za = b[2], R = b[3], t = b[4], zt = b[5];
      double z0 = lo[2] > za ? lo[2] : za;
      double z1 = hi[2] < zt ? hi[2] : zt;
      if (z0 > z1) return 0;
      double rad = (z1 - za) * t;
      if (rad > R) rad = R;
      double d2 = 0;
      for (int a = 0; a < 2; a++) {
        double e = 0;
        if (b[a] < lo[a]) e = lo[a] - b[a];
        else if (b[a] > hi[a]) e = b[a] - hi[a];
        d2 += e * e;
      }
      return d2 <= rad * rad * (1.0 + TIE);
    }
    case 3: {
      for (int a = 0; a < 3; a++)
        if (hi[a] < b[2 * a] || lo[a] > b[2 * a + 1]) return 0;
      return 1;
    }
    default:
      return 0;
  }
}

/* ---------------------------------------------------------------- tree */

typedef struct {
  int32_t* v; /* x,y,z,level */
  int64_t n, cap;
} leafvec;

static void lv_push(leafvec* L, int x, int y, int z, int lev) {
  if (L->n == L->cap) {
    L->cap = L->cap ? 2 * L->cap : 1024;
    L->v = (int32_t*)realloc(L->v, (size_t)L->cap * 4 * sizeof(int32_t));
  }
  int32_t* q = L->v + 4 * L->n++;
  q[0] = x; q[1] = y; q[2] = z; q[3] = lev;
}

static int lsize(const orc_mesh* m, int lev) { return 1 << (m->c.lvl_max - lev); }

static void leaf_box(const orc_mesh* m, const int32_t* q, double lo[3], double hi[3]) {
  int s = lsize(m, q[3]);
  for (int a = 0; a < 3; a++) {
    lo[a] = m->c.lo[a] + q[a] * m->hmin;
    hi[a] = m->c.lo[a] + (q[a] + s) * m->hmin;
  }
}

static int64_t cidx(const orc_mesh* m, int i, int j, int k) { return ((int64_t)k * m->ny + j) * m->nx + i; }
static int64_t nidx(const orc_mesh* m, int i, int j, int k) {
  return ((int64_t)k * (m->ny + 1) + j) * (m->nx + 1) + i;
}

static void fill_leafmap(orc_mesh* m, const leafvec* L) {
  for (int64_t e = 0; e < L->n; e++) {
    const int32_t* q = L->v + 4 * e;
    int s = lsize(m, q[3]);
    for (int k = q[2]; k < q[2] + s; k++)
      for (int j = q[1]; j < q[1] + s; j++)
        for (int i = q[0]; i < q[0] + s; i++) m->leafmap[cidx(m, i, j, k)] = (int32_t)e;
  }
}

static void split_marked(leafvec* L, const uint8_t* mark, const orc_mesh* m) {
  leafvec N = {0, 0, 0};
  for (int64_t e = 0; e < L->n; e++) {
    const int32_t* q = L->v + 4 * e;
    if (!mark[e]) {
      lv_push(&N, q[0], q[1], q[2], q[3]);
      continue;
    }
    int h = lsize(m, q[3]) / 2;
    for (int c = 0; c < 8; c++)
      lv_push(&N, q[0] + (c & 1) * h, q[1] + ((c >> 1) & 1) * h, q[2] + ((c >> 2) & 1) * h, q[3] + 1);
  }
  free(L->v);
  *L = N;
}

/* highest level among the leaves sharing a face or an edge segment with leaf q */
static int max_neighbour_level(const orc_mesh* m, const int32_t* q) {
  int s = lsize(m, q[3]);
  int best = -1;
  for (int dz = -1; dz <= 1; dz++)
    for (int dy = -1; dy <= 1; dy++)
      for (int dx = -1; dx <= 1; dx++) {
        int nz = (dx != 0) + (dy != 0) + (dz != 0);
        if (nz == 0 || nz == 3) continue; /* faces and edges only */
        int d[3] = {dx, dy, dz}, r0[3], r1[3];
        int ok = 1;
        for (int a = 0; a < 3; a++) {
          int lim = a == 0 ? m->nx : (a == 1 ? m->ny : m->nz);
          if (d[a] < 0) { r0[a] = q[a] - 1; r1[a] = q[a] - 1; }
          else if (d[a] > 0) { r0[a] = q[a] + s; r1[a] = q[a] + s; }
          else { r0[a] = q[a]; r1[a] = q[a] + s - 1; }
          if (r0[a] < 0 || r1[a] >= lim) ok = 0;
        }
        if (!ok) continue;
        /* levels are looked up through m->leaf, the vector the leaf map indexes */
        for (int k = r0[2]; k <= r1[2]; k++)
          for (int j = r0[1]; j <= r1[1]; j++)
            for (int i = r0[0]; i <= r1[0]; i++) {
              int lvl = m->leaf[4 * m->leafmap[cidx(m, i, j, k)] + 3];
              if (lvl > best) best = lvl;
            }
      }
  return best;
}

static void balance(orc_mesh* m, leafvec* L) {
  for (;;) {
    fill_leafmap(m, L);
    m->leaf = L->v; /* max_neighbour_level reads levels through m->leaf */
    uint8_t* mark = (uint8_t*)calloc((size_t)L->n, 1);
    int64_t nm = 0;
    for (int64_t e = 0; e < L->n; e++) {
      const int32_t* q = L->v + 4 * e;
      if (max_neighbour_level(m, q) > q[3] + 1) { mark[e] = 1; nm++; }
    }
    if (nm) split_marked(L, mark, m);
    free(mark);
    if (!nm) break;
  }
  m->leaf = NULL;
}

typedef struct { uint64_t key; int64_t idx; } keyidx;
static int cmp_keyidx(const void* a, const void* b) {
  const keyidx *p = (const keyidx*)a, *q = (const keyidx*)b;
  if (p->key != q->key) return p->key < q->key ? -1 : 1;
  return p->idx < q->idx ? -1 : (p->idx > q->idx);
}

orc_mesh* orc_mesh_build(const orc_crit* c, int32_t* status) {
  *status = ORC_OK;
  if (c->lvl_max < c->lvl_base || c->lvl_max - c->lvl_base > 12 || c->h0 <= 0) { *status = ORC_EARG; return NULL; }
  orc_mesh* m = (orc_mesh*)calloc(1, sizeof(orc_mesh));
  m->c = *c;
  m->s0 = 1 << (c->lvl_max - c->lvl_base);
  m->nx = c->base[0] * m->s0;
  m->ny = c->base[1] * m->s0;
  m->nz = c->base[2] * m->s0;
  m->hmin = c->h0 / (double)m->s0;
  m->leafmap = (int32_t*)malloc((size_t)m->nx * m->ny * m->nz * sizeof(int32_t));

  leafvec L = {0, 0, 0};
  for (int k = 0; k < c->base[2]; k++)
    for (int j = 0; j < c->base[1]; j++)
      for (int i = 0; i < c->base[0]; i++) lv_push(&L, i * m->s0, j * m->s0, k * m->s0, c->lvl_base);

  /* Steps 1-3 repeated until no element is marked */
  for (;;) {
    uint8_t* mark = (uint8_t*)calloc((size_t)L.n, 1);
    int64_t nm = 0;
    for (int64_t e = 0; e < L.n; e++) {
      const int32_t* q = L.v + 4 * e;
      if (q[3] >= c->lvl_max || c->body_kind == 0) continue;
      double lo[3], hi[3];
      leaf_box(m, q, lo, hi);
      int hit = body_meets(c, lo, hi); /* Step 1 */
      for (int v = 0; v < 8 && !hit; v++) { /* Step 2 */
        double p[3] = {(v & 1) ? hi[0] : lo[0], (v & 2) ? hi[1] : lo[1], (v & 4) ? hi[2] : lo[2]};
        hit = body_near(c, p, c->dx_region);
      }
      if (hit) { mark[e] = 1; nm++; }
    }
    if (nm) split_marked(&L, mark, m); /* Step 3 */
    free(mark);
    if (!nm) break;
    balance(m, &L);
  }
  balance(m, &L);

  /* Morton order of leaves */
  m->nleaf = L.n;
  keyidx* ki = (keyidx*)malloc((size_t)L.n * sizeof(keyidx));
  for (int64_t e = 0; e < L.n; e++) {
    ki[e].key = orc_morton3(L.v[4 * e], L.v[4 * e + 1], L.v[4 * e + 2]);
    ki[e].idx = e;
  }
  qsort(ki, (size_t)L.n, sizeof(keyidx), cmp_keyidx);
  m->leaf = (int32_t*)malloc((size_t)L.n * 4 * sizeof(int32_t));
  for (int64_t e = 0; e < L.n; e++) memcpy(m->leaf + 4 * e, L.v + 4 * ki[e].idx, 4 * sizeof(int32_t));
  free(ki);
  free(L.v);
  {
    leafvec S = {m->leaf, m->nleaf, m->nleaf};
    fill_leafmap(m, &S);
  }

  /* nodes = union of leaf vertices, numbered in Morton order */
  int64_t nlat = (int64_t)(m->nx + 1) * (m->ny + 1) * (m->nz + 1);
  m->nodemap = (int32_t*)malloc((size_t)nlat * sizeof(int32_t));
  for (int64_t i = 0; i < nlat; i++) m->nodemap[i] = -1;
  int64_t nn = 0;
  for (int64_t e = 0; e < m->nleaf; e++) {
    const int32_t* q = m->leaf + 4 * e;
    int s = lsize(m, q[3]);
    for (int v = 0; v < 8; v++) {
      int64_t id = nidx(m, q[0] + (v & 1) * s, q[1] + ((v >> 1) & 1) * s, q[2] + ((v >> 2) & 1) * s);
      if (m->nodemap[id] < 0) { m->nodemap[id] = 0; nn++; }
    }
  }
  ki = (keyidx*)malloc((size_t)nn * sizeof(keyidx));
  int64_t t = 0;
  for (int k = 0; k <= m->nz; k++)
    for (int j = 0; j <= m->ny; j++)
      for (int i = 0; i <= m->nx; i++)
        if (m->nodemap[nidx(m, i, j, k)] >= 0) {
          ki[t].key = orc_morton3(i, j, k);
          ki[t].idx = nidx(m, i, j, k);
          t++;
        }
  qsort(ki, (size_t)nn, sizeof(keyidx), cmp_keyidx);
  m->nnode = nn;
  m->node_ijk = (int32_t*)malloc((size_t)nn * 3 * sizeof(int32_t));
  for (int64_t n = 0; n < nn; n++) {
    int64_t id = ki[n].idx;
    m->nodemap[id] = (int32_t)n;
    m->node_ijk[3 * n] = (int32_t)(id % (m->nx + 1));
    m->node_ijk[3 * n + 1] = (int32_t)((id / (m->nx + 1)) % (m->ny + 1));
    m->node_ijk[3 * n + 2] = (int32_t)(id / ((int64_t)(m->nx + 1) * (m->ny + 1)));
  }
  free(ki);

  /* hanging nodes: on the boundary of an element without being one of its vertices */
  m->hang = (uint8_t*)calloc((size_t)nn, 1);
  m->hang_owner = (int32_t*)malloc((size_t)nn * sizeof(int32_t));
  for (int64_t n = 0; n < nn; n++) m->hang_owner[n] = -1;
  for (int64_t e = 0; e < m->nleaf; e++) {
    const int32_t* q = m->leaf + 4 * e;
    int s = lsize(m, q[3]);
    if (s < 2) continue;
    for (int a = 0; a < 3; a++)
      for (int side = 0; side < 2; side++) {
        int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
        for (int u = 0; u <= s; u++)
          for (int w = 0; w <= s; w++) {
            int p[3];
            p[a] = q[a] + side * s;
            p[b1] = q[b1] + u;
            p[b2] = q[b2] + w;
            int corner = (u == 0 || u == s) && (w == 0 || w == s);
            if (corner) continue;
            int32_t n = m->nodemap[nidx(m, p[0], p[1], p[2])];
            if (n < 0) continue;
            m->hang[n] = 1;
            int32_t o = m->hang_owner[n];
            if (o < 0 || m->leaf[4 * o + 3] > q[3]) m->hang_owner[n] = (int32_t)e; /* coarsest */
          }
      }
  }

  /* independent numbering and constraint weights */
  m->indep = (int32_t*)malloc((size_t)nn * sizeof(int32_t));
  m->indep_node = (int32_t*)malloc((size_t)nn * sizeof(int32_t));
  m->nindep = 0;
  for (int64_t n = 0; n < nn; n++) {
    if (m->hang[n]) m->indep[n] = -1;
    else { m->indep_node[m->nindep] = (int32_t)n; m->indep[n] = (int32_t)m->nindep++; }
  }
  m->hang_nsup = (int8_t*)calloc((size_t)nn, 1);
  m->hang_sup = (int32_t*)malloc((size_t)nn * 4 * sizeof(int32_t));
  m->hang_w = (double*)calloc((size_t)nn * 4, sizeof(double));
  for (int64_t i = 0; i < nn * 4; i++) m->hang_sup[i] = -1;
  for (int64_t n = 0; n < nn; n++) {
    if (!m->hang[n]) continue;
    const int32_t* q = m->leaf + 4 * m->hang_owner[n];
    int s = lsize(m, q[3]);
    double xi[3];
    for (int a = 0; a < 3; a++) xi[a] = (double)(m->node_ijk[3 * n + a] - q[a]) / (double)s;
    for (int v = 0; v < 8; v++) {
      double phi = 1.0;
      for (int a = 0; a < 3; a++) phi *= ((v >> a) & 1) ? xi[a] : 1.0 - xi[a];
      if (phi == 0.0) continue;
      int32_t vn = m->nodemap[nidx(m, q[0] + (v & 1) * s, q[1] + ((v >> 1) & 1) * s, q[2] + ((v >> 2) & 1) * s)];
      if (m->hang[vn] || m->hang_nsup[n] >= 4) { *status = ORC_ETREE; orc_mesh_free(m); return NULL; }
      m->hang_sup[4 * n + m->hang_nsup[n]] = m->indep[vn];
      m->hang_w[4 * n + m->hang_nsup[n]] = phi;
      m->hang_nsup[n]++;
    }
  }

  /* I(K) and C_K */
  m->ik_n = (int32_t*)calloc((size_t)m->nleaf, sizeof(int32_t));
  m->ik_node = (int32_t*)malloc((size_t)m->nleaf * ORC_MAXI * sizeof(int32_t));
  m->ik_c = (double*)calloc((size_t)m->nleaf * 8 * ORC_MAXI, sizeof(double));
  for (int64_t e = 0; e < m->nleaf; e++) {
    const int32_t* q = m->leaf + 4 * e;
    int s = lsize(m, q[3]);
    int32_t* ids = m->ik_node + e * ORC_MAXI;
    int cnt = 0;
    int32_t vn[8];
    for (int v = 0; v < 8; v++) vn[v] = m->nodemap[nidx(m, q[0] + (v & 1) * s, q[1] + ((v >> 1) & 1) * s, q[2] + ((v >> 2) & 1) * s)];
    /* union of independent vertices and supports of hanging vertices */
    for (int v = 0; v < 8; v++) {
      int32_t cand[4];
      int nc = 0;
      if (!m->hang[vn[v]]) cand[nc++] = m->indep[vn[v]];
      else for (int r = 0; r < m->hang_nsup[vn[v]]; r++) cand[nc++] = m->hang_sup[4 * vn[v] + r];
      for (int r = 0; r < nc; r++) {
        int found = 0;
        for (int z = 0; z < cnt; z++) found |= ids[z] == cand[r];
        if (!found) {
          if (cnt >= ORC_MAXI) { *status = ORC_ETREE; orc_mesh_free(m); return NULL; }
          ids[cnt++] = cand[r];
        }
      }
    }
    for (int a = 1; a < cnt; a++) /* insertion sort ascending */
      for (int b = a; b > 0 && ids[b - 1] > ids[b]; b--) { int32_t tmp = ids[b]; ids[b] = ids[b - 1]; ids[b - 1] = tmp; }
    m->ik_n[e] = cnt;
    double* C = m->ik_c + e * 8 * ORC_MAXI;
    for (int v = 0; v < 8; v++) {
      if (!m->hang[vn[v]]) {
        for (int z = 0; z < cnt; z++) if (ids[z] == m->indep[vn[v]]) C[v * ORC_MAXI + z] += 1.0;
      } else {
        for (int r = 0; r < m->hang_nsup[vn[v]]; r++)
          for (int z = 0; z < cnt; z++)
            if (ids[z] == m->hang_sup[4 * vn[v] + r]) C[v * ORC_MAXI + z] += m->hang_w[4 * vn[v] + r];
      }
    }
  }
  return m;
}

void orc_mesh_free(orc_mesh* m) {
  if (!m) return;
  free(m->leaf); free(m->leafmap); free(m->node_ijk); free(m->nodemap); free(m->hang); free(m->indep);
  free(m->indep_node); free(m->hang_owner); free(m->hang_nsup); free(m->hang_sup); free(m->hang_w);
  free(m->ik_n); free(m->ik_node); free(m->ik_c); free(m->px); free(m->pl); free(m->perm); free(m->pleaf);
  free(m->pnleaf); free(m->sup_off); free(m->sup_node); free(m->row_ptr); free(m->col); free(m->gface);
  free(m);
}

void orc_mesh_counts(const orc_mesh* m, int64_t out[9]) {
  int64_t nh = 0;
  for (int64_t n = 0; n < m->nnode; n++) nh += m->hang[n];
  out[0] = m->nleaf; out[1] = m->nnode; out[2] = m->nindep; out[3] = nh; out[4] = m->np;
  out[5] = m->nnz; out[6] = m->nstraddle; out[7] = m->maxsup;
  int64_t act = 0;
  if (m->row_ptr)
    for (int64_t r = 0; r < 3 * m->nindep; r++) act += m->row_ptr[r + 1] > m->row_ptr[r];
  out[8] = act;
}

void orc_mesh_leaves(const orc_mesh* m, int32_t* al) { memcpy(al, m->leaf, (size_t)m->nleaf * 4 * sizeof(int32_t)); }

void orc_mesh_nodes(const orc_mesh* m, int32_t* ijk) {
  for (int64_t i = 0; i < m->nindep; i++) memcpy(ijk + 3 * i, m->node_ijk + 3 * m->indep_node[i], 3 * sizeof(int32_t));
}

void orc_mesh_hanging(const orc_mesh* m, int32_t* ijk, int32_t* sup, double* w, int32_t* owner) {
  int64_t h = 0;
  for (int64_t n = 0; n < m->nnode; n++) {
    if (!m->hang[n]) continue;
    memcpy(ijk + 3 * h, m->node_ijk + 3 * n, 3 * sizeof(int32_t));
    for (int r = 0; r < 4; r++) { sup[4 * h + r] = m->hang_sup[4 * n + r]; w[4 * h + r] = m->hang_w[4 * n + r]; }
    owner[h] = m->hang_owner[n];
    h++;
  }
}

void orc_mesh_cells(const orc_mesh* m, int32_t* n, int32_t* inodes, double* cmat) {
  memcpy(n, m->ik_n, (size_t)m->nleaf * sizeof(int32_t));
  memcpy(inodes, m->ik_node, (size_t)m->nleaf * ORC_MAXI * sizeof(int32_t));
  memcpy(cmat, m->ik_c, (size_t)m->nleaf * 8 * ORC_MAXI * sizeof(double));
}

/* ---------------------------------------------------------------- points */

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Every leaf meeting the domain with positive volume: each axis overlap must exceed
 * 1e-12 of the domain's side (zero-volume contacts do not count). */
int orc_point_leaves(const orc_mesh* m, const double x[3], const double l[3], int32_t* lv, double* box) {
  int lim[3] = {m->nx, m->ny, m->nz};
  int r0[3], r1[3];
  for (int a = 0; a < 3; a++) {
    r0[a] = clampi((int)floor((x[a] - l[a] - m->c.lo[a]) / m->hmin), 0, lim[a] - 1);
    r1[a] = clampi((int)floor((x[a] + l[a] - m->c.lo[a]) / m->hmin), 0, lim[a] - 1);
  }
  int cnt = 0;
  double vsum = 0, vdom = (2.0 * l[0]) * (2.0 * l[1]) * (2.0 * l[2]);
  for (int k = r0[2]; k <= r1[2]; k++)
    for (int j = r0[1]; j <= r1[1]; j++)
      for (int i = r0[0]; i <= r1[0]; i++) {
        int32_t e = m->leafmap[cidx(m, i, j, k)];
        int seen = 0;
        for (int z = 0; z < cnt; z++) seen |= lv[z] == e;
        if (seen) continue;
        double lo[3], hi[3], b[6];
        leaf_box(m, m->leaf + 4 * e, lo, hi);
        int pos = 1;
        double vol = 1.0;
        for (int a = 0; a < 3; a++) {
          double a0 = x[a] - l[a] > lo[a] ? x[a] - l[a] : lo[a];
          double a1 = x[a] + l[a] < hi[a] ? x[a] + l[a] : hi[a];
          double o = a1 - a0;
          if (!(o > 1e-12 * (2.0 * l[a]))) pos = 0;
          b[2 * a] = a0; b[2 * a + 1] = a1;
          vol *= o;
        }
        if (!pos) continue;
        if (cnt >= ORC_MAXL) return ORC_ESTENCIL;
        lv[cnt] = e;
        for (int z = 0; z < 6; z++) box[6 * cnt + z] = b[z];
        vsum += vol;
        cnt++;
      }
  if (!(fabs(vsum - vdom) <= 1e-12 * vdom)) return ORC_EOUTSIDE;
  return cnt;
}

typedef struct { int32_t leaf; int64_t idx; } ptkey;
static int cmp_ptkey(const void* a, const void* b) {
  const ptkey *p = (const ptkey*)a, *q = (const ptkey*)b;
  if (p->leaf != q->leaf) return p->leaf < q->leaf ? -1 : 1;
  return p->idx < q->idx ? -1 : (p->idx > q->idx);
}
static int cmp_u64(const void* a, const void* b) {
  uint64_t p = *(const uint64_t*)a, q = *(const uint64_t*)b;
  return p < q ? -1 : (p > q);
}

int32_t orc_mesh_set_points(orc_mesh* m, const double* x, const double* l, int64_t n, int64_t* bad) {
  *bad = -1;
  free(m->px); free(m->pl); free(m->perm); free(m->pleaf); free(m->pnleaf); free(m->sup_off); free(m->sup_node);
  free(m->row_ptr); free(m->col);
  m->row_ptr = NULL; m->col = NULL; m->nnz = 0;
  m->np = n;
  m->px = (double*)malloc((size_t)(3 * n + 1) * sizeof(double));
  m->pl = (double*)malloc((size_t)(3 * n + 1) * sizeof(double));
  memcpy(m->px, x, (size_t)3 * n * sizeof(double));
  memcpy(m->pl, l, (size_t)3 * n * sizeof(double));
  m->perm = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
  m->pleaf = (int32_t*)malloc((size_t)(n + 1) * sizeof(int32_t));
  m->pnleaf = (uint8_t*)malloc((size_t)(n + 1));
  m->sup_off = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));

  /* point order: (leaf containing the centre, original index) */
  int lim[3] = {m->nx, m->ny, m->nz};
  ptkey* pk = (ptkey*)malloc((size_t)(n + 1) * sizeof(ptkey));
  for (int64_t p = 0; p < n; p++) {
    int q[3];
    for (int a = 0; a < 3; a++) {
      double xa = x[a * n + p];
      if (!isfinite(xa) || !isfinite(l[a * n + p]) || !(l[a * n + p] > 0)) { *bad = p; free(pk); return ORC_ENONFINITE; }
      q[a] = clampi((int)floor((xa - m->c.lo[a]) / m->hmin), 0, lim[a] - 1);
    }
    pk[p].leaf = m->leafmap[cidx(m, q[0], q[1], q[2])];
    pk[p].idx = p;
    m->pleaf[p] = pk[p].leaf;
  }
  qsort(pk, (size_t)n, sizeof(ptkey), cmp_ptkey);
  for (int64_t s = 0; s < n; s++) m->perm[s] = pk[s].idx;
  free(pk);

  /* supports: union of I(K) over the overlapped leaves */
  int64_t cap = 8 * n + 64, used = 0;
  m->sup_node = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
  m->nstraddle = 0;
  m->maxsup = 0;
  uint8_t* leaf_pop = (uint8_t*)calloc((size_t)m->nleaf, 1);
  uint8_t* any_pop = (uint8_t*)calloc((size_t)m->nleaf + 1, 1);  /* overlapped by any point */
  int32_t lv[ORC_MAXL];
  double box[6 * ORC_MAXL];
  int64_t npair_cap = 1 << 20, npair = 0;
  uint64_t* pairs = (uint64_t*)malloc((size_t)npair_cap * sizeof(uint64_t));
  for (int64_t p = 0; p < n; p++) {
    double xp[3] = {x[p], x[n + p], x[2 * n + p]}, lp[3] = {l[p], l[n + p], l[2 * n + p]};
    int nl = orc_point_leaves(m, xp, lp, lv, box);
    if (nl < 0) { *bad = p; free(leaf_pop); free(any_pop); free(pairs); return nl; }
    m->pnleaf[p] = (uint8_t)nl;
    int32_t sup[ORC_MAXS];
    int ns = 0;
    for (int k = 0; k < nl; k++)
      for (int z = 0; z < m->ik_n[lv[k]]; z++) {
        int32_t id = m->ik_node[lv[k] * ORC_MAXI + z];
        int f = 0;
        for (int t = 0; t < ns; t++) f |= sup[t] == id;
        if (!f) {
          if (ns >= ORC_MAXS) { *bad = p; free(leaf_pop); free(any_pop); free(pairs); return ORC_ESTENCIL; }
          sup[ns++] = id;
        }
      }
    for (int a = 1; a < ns; a++)
      for (int b = a; b > 0 && sup[b - 1] > sup[b]; b--) { int32_t tmp = sup[b]; sup[b] = sup[b - 1]; sup[b - 1] = tmp; }
    if (used + ns > cap) { cap = 2 * cap + ns; m->sup_node = (int32_t*)realloc(m->sup_node, (size_t)cap * sizeof(int32_t)); }
    m->sup_off[p] = used;
    memcpy(m->sup_node + used, sup, (size_t)ns * sizeof(int32_t));
    used += ns;
    if (ns > m->maxsup) m->maxsup = ns;
    for (int k = 0; k < nl; k++) any_pop[lv[k]] = 1;
    if (nl == 1) leaf_pop[lv[0]] = 1;
    else {
      m->nstraddle++;
      for (int a = 0; a < ns; a++)
        for (int b = 0; b < ns; b++) {
          if (npair == npair_cap) { npair_cap *= 2; pairs = (uint64_t*)realloc(pairs, (size_t)npair_cap * sizeof(uint64_t)); }
          pairs[npair++] = ((uint64_t)(uint32_t)sup[a] << 32) | (uint32_t)sup[b];
        }
    }
  }
  m->sup_off[n] = used;
  /* points lying in one leaf couple exactly the pairs of I(K) x I(K) of that leaf */
  for (int64_t e = 0; e < m->nleaf; e++) {
    if (!leaf_pop[e]) continue;
    const int32_t* ids = m->ik_node + e * ORC_MAXI;
    for (int a = 0; a < m->ik_n[e]; a++)
      for (int b = 0; b < m->ik_n[e]; b++) {
        if (npair == npair_cap) { npair_cap *= 2; pairs = (uint64_t*)realloc(pairs, (size_t)npair_cap * sizeof(uint64_t)); }
        pairs[npair++] = ((uint64_t)(uint32_t)ids[a] << 32) | (uint32_t)ids[b];
      }
  }
  free(leaf_pop);
  free(m->gface);
  m->gface = NULL;
  m->ngface = 0;
  if (m->ghost) {
    orc_ghost_build_faces(m, any_pop);
    npair = orc_ghost_pairs(m, &pairs, npair, &npair_cap);
  }
  free(any_pop);
  qsort(pairs, (size_t)npair, sizeof(uint64_t), cmp_u64);
  int64_t nu = 0;
  for (int64_t i = 0; i < npair; i++)
    if (i == 0 || pairs[i] != pairs[i - 1]) pairs[nu++] = pairs[i];

  /* CSR over all 3*n_indep DOF rows, dense 3x3 blocks per coupled node pair */
  int64_t nrow = 3 * m->nindep;
  int64_t* deg = (int64_t*)calloc((size_t)m->nindep + 1, sizeof(int64_t));
  for (int64_t i = 0; i < nu; i++) deg[pairs[i] >> 32]++;
  m->row_ptr = (int64_t*)malloc((size_t)(nrow + 1) * sizeof(int64_t));
  m->row_ptr[0] = 0;
  for (int64_t a = 0; a < m->nindep; a++)
    for (int c = 0; c < 3; c++) m->row_ptr[3 * a + c + 1] = m->row_ptr[3 * a + c] + 3 * deg[a];
  m->nnz = m->row_ptr[nrow];
  m->col = (int32_t*)malloc((size_t)(m->nnz + 1) * sizeof(int32_t));
  int64_t i0 = 0;
  for (int64_t a = 0; a < m->nindep; a++) {
    for (int c = 0; c < 3; c++) {
      int64_t w = m->row_ptr[3 * a + c];
      for (int64_t i = i0; i < i0 + deg[a]; i++) {
        int32_t b = (int32_t)(pairs[i] & 0xffffffffu);
        for (int k = 0; k < 3; k++) m->col[w++] = 3 * b + k;
      }
    }
    i0 += deg[a];
  }
  free(deg);
  free(pairs);
  return ORC_OK;
}

void orc_mesh_perm(const orc_mesh* m, int64_t* perm, int32_t* point_leaf, uint8_t* nleaf) {
  memcpy(perm, m->perm, (size_t)m->np * sizeof(int64_t));
  memcpy(point_leaf, m->pleaf, (size_t)m->np * sizeof(int32_t));
  memcpy(nleaf, m->pnleaf, (size_t)m->np);
}

void orc_mesh_csr(const orc_mesh* m, int64_t* row_ptr, int32_t* col) {
  memcpy(row_ptr, m->row_ptr, (size_t)(3 * m->nindep + 1) * sizeof(int64_t));
  memcpy(col, m->col, (size_t)m->nnz * sizeof(int32_t));
}
