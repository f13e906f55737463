// Ghost stabilisation of the stiffness (Section 4, eq. ghost), host part: the ghost faces of
// the octree and, per face, the matrix of jump integrals
//   G_F[a][b] = int_F [d_n phi~_a] [d_n phi~_b] dA
// over the up to 16 slot nodes of the face's two leaves. A boundary leaf is a populated leaf
// (one that some point domain overlaps) with an unpopulated face neighbour; the ghost faces
// are the faces it shares with populated leaves (the smaller leaf's face where the two sizes
// differ). [.] is the jump across F of the normal derivative of the constrained trilinear
// basis of each leaf; the integrand is a product of two functions bilinear on F, so a 2 x 2
// Gauss rule on F is exact. h_F is the larger side of the two leaves, kappa = 10.
#include <algorithm>
#include <cmath>
#include <vector>

#include "geom.h"

namespace mpm {

constexpr double kGhostKappa = 10.0;

// leaves across one face of leaf e (axis a, side sg = +1 for the face at q_a + s). 2:1
// balance leaves one neighbour at least as large, or four of half size.
static int face_neighbours(const LeafGeo& G, const HostTree& T, int64_t e, int a, int sg, int32_t out[4]) {
  const int32_t* q = &T.leaf[4 * e];
  const int s = 1 << (G.lmax - q[3]);
  const int pa = sg > 0 ? q[a] + s : q[a] - 1;
  if (pa < 0 || pa >= G.lat[a]) return 0;
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  auto leaf_at = [&](int ob, int oc) {
    double p[3];
    int cell[3];
    cell[a] = pa;
    cell[b] = q[b] + ob;
    cell[c] = q[c] + oc;
    for (int t = 0; t < 3; ++t) p[t] = G.lo[t] + (cell[t] + 0.5) * G.hmin;
    return int32_t(leaf_of_point(G, p[0], p[1], p[2]));
  };
  const int32_t k0 = leaf_at(0, 0);
  const int s0 = 1 << (G.lmax - T.leaf[4 * k0 + 3]);
  if (s0 >= s || s == 1) {
    out[0] = k0;
    return 1;
  }
  const int hs = s / 2;
  out[0] = k0;
  out[1] = leaf_at(hs, 0);
  out[2] = leaf_at(0, hs);
  out[3] = leaf_at(hs, hs);
  return 4;
}

// normal derivative along axis a of the 8 slot functions of leaf e at the physical point p
static void slot_dn(const LeafGeo& G, const HostTree& T, int32_t e, const double p[3], int a, double out[8]) {
  const int32_t* q = &T.leaf[4 * e];
  const double h = double(1 << (G.lmax - q[3])) * G.hmin;
  double xi[3];
  for (int t = 0; t < 3; ++t) xi[t] = (p[t] - (G.lo[t] + q[t] * G.hmin)) / h;
  double dv[8];
  for (int v = 0; v < 8; ++v) {
    double g = 1.0;
    for (int t = 0; t < 3; ++t) {
      const int bit = (v >> t) & 1;
      g *= t == a ? (bit ? 1.0 : -1.0) / h : (bit ? xi[t] : 1.0 - xi[t]);
    }
    dv[v] = g;
  }
  const double* C = &T.cell_cmat[64 * int64_t(e)];
  for (int z = 0; z < 8; ++z) {
    double d = 0.0;
    for (int v = 0; v < 8; ++v) d += C[8 * v + z] * dv[v];
    out[z] = d;
  }
}

int64_t ghost_faces_host(const HostTree& T, const LeafGeo& G, const std::vector<uint8_t>& pop, GhostHost* out) {
  const int64_t nl = int64_t(T.leaf.size() / 4);
  std::vector<uint8_t> bnd(nl, 0);
  int32_t nb[4];
  for (int64_t e = 0; e < nl; ++e) {
    if (!pop[e]) continue;
    for (int a = 0; a < 3 && !bnd[e]; ++a)
      for (int sg = -1; sg <= 1; sg += 2) {
        const int k = face_neighbours(G, T, e, a, sg, nb);
        for (int t = 0; t < k; ++t) bnd[e] |= !pop[nb[t]];
      }
  }
  struct Face {
    int32_t lo, hi, axis, plane, b0, b1, c0, c1;
  };
  std::vector<Face> faces;
  for (int64_t e = 0; e < nl; ++e) {
    if (!bnd[e]) continue;
    const int32_t* q = &T.leaf[4 * e];
    const int s = 1 << (G.lmax - q[3]);
    for (int a = 0; a < 3; ++a)
      for (int sg = -1; sg <= 1; sg += 2) {
        const int k = face_neighbours(G, T, e, a, sg, nb);
        for (int t = 0; t < k; ++t) {
          const int32_t o = nb[t];
          if (!pop[o]) continue;
          const int32_t* r = &T.leaf[4 * o];
          const int so = 1 << (G.lmax - r[3]);
          const int b = (a + 1) % 3, c = (a + 2) % 3;
          Face f;
          f.lo = int32_t(std::min<int64_t>(e, o));
          f.hi = int32_t(std::max<int64_t>(e, o));
          f.axis = a;
          f.plane = sg > 0 ? q[a] + s : q[a];
          f.b0 = std::max(q[b], r[b]);
          f.b1 = std::min(q[b] + s, r[b] + so);
          f.c0 = std::max(q[c], r[c]);
          f.c1 = std::min(q[c] + s, r[c] + so);
          faces.push_back(f);
        }
      }
  }
  std::sort(faces.begin(), faces.end(),
            [](const Face& x, const Face& y) { return x.lo != y.lo ? x.lo < y.lo : x.hi < y.hi; });
  faces.erase(std::unique(faces.begin(), faces.end(),
                          [](const Face& x, const Face& y) { return x.lo == y.lo && x.hi == y.hi; }),
              faces.end());
  const int64_t nf = int64_t(faces.size());
  out->nf = nf;
  out->leaf2.assign(2 * nf, 0);
  out->nodes.assign(16 * nf, -1);
  out->G.assign(256 * nf, 0.0);
  out->h.assign(nf, 0.0);
  out->face.assign(8 * nf, 0);
  const double gx[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  for (int64_t i = 0; i < nf; ++i) {
    const Face& f = faces[i];
    int32_t* ids = &out->nodes[16 * i];
    int ni = 0, map[2][8];
    const int32_t lv[2] = {f.lo, f.hi};
    for (int side = 0; side < 2; ++side)
      for (int z = 0; z < 8; ++z) {
        const int32_t id = T.cell_nodes[8 * int64_t(lv[side]) + z];
        int pos = -1;
        for (int t = 0; t < ni; ++t)
          if (ids[t] == id) pos = t;
        if (pos < 0) {
          pos = ni;
          ids[ni++] = id;
        }
        map[side][z] = pos;
      }
    const int a = f.axis, b = (a + 1) % 3, c = (a + 2) % 3;
    const double fb = (f.b1 - f.b0) * G.hmin, fc = (f.c1 - f.c0) * G.hmin;
    double* Gm = &out->G[256 * i];
    for (int gi = 0; gi < 2; ++gi)
      for (int gj = 0; gj < 2; ++gj) {
        double p[3];
        p[a] = G.lo[a] + f.plane * G.hmin;
        p[b] = G.lo[b] + f.b0 * G.hmin + gx[gi] * fb;
        p[c] = G.lo[c] + f.c0 * G.hmin + gx[gj] * fc;
        double J[16] = {0.0};
        double d[8];
        slot_dn(G, T, lv[0], p, a, d);
        for (int z = 0; z < 8; ++z) J[map[0][z]] += d[z];
        slot_dn(G, T, lv[1], p, a, d);
        for (int z = 0; z < 8; ++z) J[map[1][z]] -= d[z];
        const double w = 0.25 * fb * fc;
        for (int x = 0; x < ni; ++x)
          for (int y = 0; y < ni; ++y) Gm[16 * x + y] += w * J[x] * J[y];
      }
    const int s_lo = 1 << (G.lmax - T.leaf[4 * int64_t(f.lo) + 3]);
    const int s_hi = 1 << (G.lmax - T.leaf[4 * int64_t(f.hi) + 3]);
    out->h[i] = double(std::max(s_lo, s_hi)) * G.hmin / kGhostKappa;  // h_F / kappa
    out->leaf2[2 * i] = f.lo;
    out->leaf2[2 * i + 1] = f.hi;
    int32_t* fr = &out->face[8 * i];
    fr[0] = f.lo;
    fr[1] = f.hi;
    fr[2] = f.axis;
    fr[3] = f.plane;
    fr[4] = f.b0;
    fr[5] = f.b1;
    fr[6] = f.c0;
    fr[7] = f.c1;
  }
  return nf;
}

}  // namespace mpm
