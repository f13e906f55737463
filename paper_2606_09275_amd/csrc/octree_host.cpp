// Host construction of the 2:1-balanced octree, its nodes, hanging-node constraints and the
// per-element independent sets I(K) (Sections 3.1 and 5 of the paper).
//
// Leaves live in a hash set keyed by (Morton key of the anchor, level); balance is a ripple
// work-list: every leaf checks the 18 face/edge neighbour positions of its own size and
// splits any leaf there that is more than one level coarser, pushing the children back.
// Hanging nodes are found from the parent lattice: a vertex of a leaf that sits at an edge
// midpoint (face centre) of its parent hangs iff a leaf of the parent's level shares that
// edge (face); its supports are the parent's edge end points (face corners).
#include <algorithm>
#include <array>
#include <cmath>
#include <unordered_set>

#include "internal.h"

namespace mpm {

namespace {

constexpr double kTie = 1e-12;  // relative slack: ties of distance predicates count as inside

// squared distance from (r, z) in the meridian half-plane to segment p0-p1
double seg_dist2(double r, double z, double r0, double z0, double r1, double z1) {
  const double er = r1 - r0, ez = z1 - z0;
  const double len2 = er * er + ez * ez;
  double t = 0.0;
  if (len2 > 0.0) t = std::min(1.0, std::max(0.0, ((r - r0) * er + (z - z0) * ez) / len2));
  const double dr = r0 + t * er - r, dz = z0 + t * ez - z;
  return dr * dr + dz * dz;
}

struct Body {
  const mpm_refine_t& c;
  // Step 2: point within distance dx of the closed solid (distance 0 inside)
  bool near(const double p[3], double dx) const {
    const double* b = c.body;
    if (c.body_kind == MPM_BODY_SPHERE) {
      const double ex = p[0] - b[0], ey = p[1] - b[1], ez = p[2] - b[2];
      const double reach = b[3] + dx;
      return ex * ex + ey * ey + ez * ez <= reach * reach * (1.0 + kTie);
    }
    if (c.body_kind == MPM_BODY_CONE) {
      const double ax = p[0] - b[0], ay = p[1] - b[1];
      const double r = std::sqrt(ax * ax + ay * ay), z = p[2];
      const double zap = b[2], R = b[3], tn = b[4], ztop = b[5];
      const double zsh = zap + R / tn;  // where the cone reaches the shaft radius
      if (z >= zap && z <= ztop && r <= std::min(R, (z - zap) * tn)) return true;
      double d2 = seg_dist2(r, z, 0.0, zap, R, zsh);
      d2 = std::min(d2, seg_dist2(r, z, R, zsh, R, ztop));
      d2 = std::min(d2, seg_dist2(r, z, R, ztop, 0.0, ztop));
      return d2 <= dx * dx * (1.0 + kTie);
    }
    if (c.body_kind == MPM_BODY_BOX) {
      double d2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        const double e = std::max(0.0, std::max(b[2 * a] - p[a], p[a] - b[2 * a + 1]));
        d2 += e * e;
      }
      return d2 <= dx * dx * (1.0 + kTie);
    }
    return false;
  }
  // Step 1: closed box [lo, hi] meets the closed solid
  bool meets(const double lo[3], const double hi[3]) const {
    const double* b = c.body;
    auto gap = [](double v, double l, double h) { return v < l ? l - v : (v > h ? v - h : 0.0); };
    if (c.body_kind == MPM_BODY_SPHERE) {
      double d2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        const double e = gap(b[a], lo[a], hi[a]);
        d2 += e * e;
      }
      return d2 <= b[3] * b[3] * (1.0 + kTie);
    }
    if (c.body_kind == MPM_BODY_CONE) {
      // radius is non-decreasing in z: test the highest z the box and the solid share
      const double zl = std::max(lo[2], b[2]), zh = std::min(hi[2], b[5]);
      if (zl > zh) return false;
      const double rad = std::min(b[3], (zh - b[2]) * b[4]);
      const double ex = gap(b[0], lo[0], hi[0]), ey = gap(b[1], lo[1], hi[1]);
      return ex * ex + ey * ey <= rad * rad * (1.0 + kTie);
    }
    if (c.body_kind == MPM_BODY_BOX) {
      for (int a = 0; a < 3; ++a)
        if (hi[a] < b[2 * a] || lo[a] > b[2 * a + 1]) return false;
      return true;
    }
    return false;
  }
};

struct Forest {
  const mpm_refine_t& c;
  int lbase, lmax, lat[3];
  double hmin;
  std::unordered_set<uint64_t> S;

  static uint64_t pack(uint64_t x, uint64_t y, uint64_t z, int lev) { return (morton(x, y, z) << 5) | uint64_t(lev); }
  static void unpack(uint64_t k, int q[4]) {
    q[3] = int(k & 31);
    const uint64_t m = k >> 5;
    q[0] = int(compact3(m));
    q[1] = int(compact3(m >> 1));
    q[2] = int(compact3(m >> 2));
  }
  int size(int lev) const { return 1 << (lmax - lev); }
  bool has(int x, int y, int z, int lev) const { return S.count(pack(x, y, z, lev)) != 0; }
  // level of the leaf holding finest cell (x,y,z) if that level is <= maxlev, else -1
  int coarse_leaf(int x, int y, int z, int maxlev, int anc[3]) const {
    for (int lev = lbase; lev <= maxlev; ++lev) {
      const int s = size(lev);
      const int ax = x / s * s, ay = y / s * s, az = z / s * s;
      if (has(ax, ay, az, lev)) {
        anc[0] = ax; anc[1] = ay; anc[2] = az;
        return lev;
      }
    }
    return -1;
  }
  void split(const int q[4], std::vector<uint64_t>* pushed) {
    S.erase(pack(q[0], q[1], q[2], q[3]));
    const int h = size(q[3]) / 2;
    for (int ch = 0; ch < 8; ++ch) {
      const uint64_t k = pack(q[0] + (ch & 1) * h, q[1] + ((ch >> 1) & 1) * h, q[2] + ((ch >> 2) & 1) * h, q[3] + 1);
      S.insert(k);
      if (pushed) pushed->push_back(k);
    }
  }
  void balance() {
    std::vector<uint64_t> work(S.begin(), S.end());
    while (!work.empty()) {
      const uint64_t k = work.back();
      work.pop_back();
      if (!S.count(k)) continue;
      int q[4];
      unpack(k, q);
      if (q[3] - lbase < 2) continue;  // nothing can be two levels coarser
      const int s = size(q[3]);
      for (int d = 0; d < 27; ++d) {
        const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
        const int nzc = (dx != 0) + (dy != 0) + (dz != 0);
        if (nzc == 0 || nzc == 3) continue;  // faces and edges
        const int p[3] = {q[0] + dx * s, q[1] + dy * s, q[2] + dz * s};
        if (p[0] < 0 || p[1] < 0 || p[2] < 0 || p[0] >= lat[0] || p[1] >= lat[1] || p[2] >= lat[2]) continue;
        for (;;) {
          int anc[3];
          const int lev = coarse_leaf(p[0], p[1], p[2], q[3] - 2, anc);
          if (lev < 0) break;
          const int nq[4] = {anc[0], anc[1], anc[2], lev};
          split(nq, &work);
        }
      }
    }
  }
};

}  // namespace

int32_t build_tree(const mpm_refine_t& c, HostTree& T, int lat_out[3], double* hmin_out) {
  if (c.lvl_max < c.lvl_base || c.lvl_max - c.lvl_base > 13 || !(c.h0 > 0) || c.base[0] <= 0 || c.base[1] <= 0 ||
      c.base[2] <= 0) {
    set_error(MPM_EARG, "octree_build: bad refinement levels, base grid or h0");
    return MPM_EARG;
  }
  Forest F{c, c.lvl_base, c.lvl_max, {0, 0, 0}, 0.0, {}};
  const int s0 = 1 << (c.lvl_max - c.lvl_base);
  for (int a = 0; a < 3; ++a) F.lat[a] = c.base[a] * s0;
  if (std::max({F.lat[0], F.lat[1], F.lat[2]}) >= (1 << 13)) {
    set_error(MPM_ESTENCIL, "octree_build: finest lattice exceeds 8191 cells per axis");
    return MPM_ESTENCIL;
  }
  F.hmin = c.h0 / double(s0);
  for (int k = 0; k < c.base[2]; ++k)
    for (int j = 0; j < c.base[1]; ++j)
      for (int i = 0; i < c.base[0]; ++i) F.S.insert(Forest::pack(i * s0, j * s0, k * s0, c.lvl_base));

  Body body{c};
  if (c.body_kind != MPM_BODY_NONE) {
    for (;;) {  // Steps 1-3 until nothing is marked, then balance
      std::vector<std::array<int, 4>> marked;
      for (uint64_t k : F.S) {
        int q[4];
        Forest::unpack(k, q);
        if (q[3] >= c.lvl_max) continue;
        const int s = F.size(q[3]);
        double lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
          lo[a] = c.lo[a] + q[a] * F.hmin;
          hi[a] = c.lo[a] + (q[a] + s) * F.hmin;
        }
        bool hit = body.meets(lo, hi);
        for (int v = 0; v < 8 && !hit; ++v) {
          const double p[3] = {(v & 1) ? hi[0] : lo[0], (v & 2) ? hi[1] : lo[1], (v & 4) ? hi[2] : lo[2]};
          hit = body.near(p, c.dx_region);
        }
        if (hit) marked.push_back({q[0], q[1], q[2], q[3]});
      }
      if (marked.empty()) break;
      for (auto& q : marked) F.split(q.data(), nullptr);
      F.balance();
    }
  }

  // leaves in Morton order
  std::vector<uint64_t> keys(F.S.begin(), F.S.end());
  std::sort(keys.begin(), keys.end());
  const int64_t nl = int64_t(keys.size());
  T.leaf.resize(nl * 4);
  T.leaf_key.resize(nl);
  for (int64_t e = 0; e < nl; ++e) {
    Forest::unpack(keys[e], &T.leaf[4 * e]);
    T.leaf_key[e] = keys[e] >> 5;
  }
  auto leaf_rank = [&](int x, int y, int z) -> int64_t {
    const uint64_t m = morton(x, y, z);
    auto it = std::lower_bound(T.leaf_key.begin(), T.leaf_key.end(), m);
    return (it != T.leaf_key.end() && *it == m) ? int64_t(it - T.leaf_key.begin()) : -1;
  };

  // all nodes (leaf vertices), Morton order
  std::vector<uint64_t> nkey;
  nkey.reserve(nl * 8);
  for (int64_t e = 0; e < nl; ++e) {
    const int32_t* q = &T.leaf[4 * e];
    const int s = F.size(q[3]);
    for (int v = 0; v < 8; ++v) nkey.push_back(morton(q[0] + (v & 1) * s, q[1] + ((v >> 1) & 1) * s, q[2] + ((v >> 2) & 1) * s));
  }
  std::sort(nkey.begin(), nkey.end());
  nkey.erase(std::unique(nkey.begin(), nkey.end()), nkey.end());
  const int64_t nn = int64_t(nkey.size());
  auto node_of = [&](int x, int y, int z) -> int64_t {
    const uint64_t m = morton(x, y, z);
    auto it = std::lower_bound(nkey.begin(), nkey.end(), m);
    return (it != nkey.end() && *it == m) ? int64_t(it - nkey.begin()) : -1;
  };

  // hanging vertices from the parent lattice
  std::vector<int64_t> owner(nn, -1);
  std::vector<uint8_t> hmask(nl, 0), child(nl, 0);
  for (int64_t e = 0; e < nl; ++e) {
    const int32_t* q = &T.leaf[4 * e];
    if (q[3] == c.lvl_base) continue;
    const int s = F.size(q[3]), ps = 2 * s;
    const int P[3] = {q[0] / ps * ps, q[1] / ps * ps, q[2] / ps * ps};
    const int cc[3] = {(q[0] - P[0]) / s, (q[1] - P[1]) / s, (q[2] - P[2]) / s};
    child[e] = uint8_t(cc[0] | (cc[1] << 1) | (cc[2] << 2));
    for (int v = 0; v < 8; ++v) {
      int pos[3], mids = 0;
      for (int a = 0; a < 3; ++a) {
        pos[a] = cc[a] + ((v >> a) & 1);
        mids += pos[a] == 1;
      }
      if (mids == 0 || mids == 3) continue;
      // parent-level cells sharing the parent's edge / face through this vertex
      int64_t best = -1;
      for (int sh = 1; sh < 8; ++sh) {
        int off[3];
        bool ok = true;
        for (int a = 0; a < 3; ++a) {
          off[a] = 0;
          if ((sh >> a) & 1) {
            if (pos[a] == 1) { ok = false; break; }  // only step across the boundary planes
            off[a] = pos[a] == 0 ? -1 : 1;
          }
        }
        if (!ok) continue;
        const int nb[3] = {P[0] + off[0] * ps, P[1] + off[1] * ps, P[2] + off[2] * ps};
        if (nb[0] < 0 || nb[1] < 0 || nb[2] < 0 || nb[0] >= F.lat[0] || nb[1] >= F.lat[1] || nb[2] >= F.lat[2]) continue;
        if (!F.has(nb[0], nb[1], nb[2], q[3] - 1)) continue;
        const int64_t r = leaf_rank(nb[0], nb[1], nb[2]);
        if (best < 0 || r < best) best = r;
      }
      if (best < 0) continue;
      hmask[e] |= uint8_t(1u << v);
      const int64_t n = node_of(q[0] + ((v & 1) ? s : 0), q[1] + (((v >> 1) & 1) ? s : 0), q[2] + (((v >> 2) & 1) ? s : 0));
      if (owner[n] < 0 || best < owner[n]) owner[n] = best;
    }
  }
  // a vertex flagged hanging by one leaf must be flagged by every leaf that has it
  for (int64_t e = 0; e < nl; ++e) {
    const int32_t* q = &T.leaf[4 * e];
    const int s = F.size(q[3]);
    for (int v = 0; v < 8; ++v) {
      const int64_t n = node_of(q[0] + (v & 1) * s, q[1] + ((v >> 1) & 1) * s, q[2] + ((v >> 2) & 1) * s);
      if ((owner[n] >= 0) != bool((hmask[e] >> v) & 1)) {
        set_error(MPM_ETREE, "octree_build: inconsistent hanging-node classification (tree not 2:1 balanced)", n);
        return MPM_ETREE;
      }
    }
  }

  // independent numbering
  std::vector<int32_t> indep(nn, -1);
  int64_t ni = 0, nh = 0;
  for (int64_t n = 0; n < nn; ++n) {
    if (owner[n] < 0) indep[n] = int32_t(ni++);
    else ++nh;
  }
  T.node_ijk.resize(ni * 3);
  T.hang_ijk.resize(nh * 3);
  T.hang_sup.assign(nh * 4, -1);
  T.hang_w.assign(nh * 4, 0.0);
  T.hang_owner.resize(nh);
  for (int64_t n = 0, h = 0; n < nn; ++n) {
    const int x = int(compact3(nkey[n])), y = int(compact3(nkey[n] >> 1)), z = int(compact3(nkey[n] >> 2));
    if (owner[n] < 0) {
      int32_t* d = &T.node_ijk[3 * indep[n]];
      d[0] = x; d[1] = y; d[2] = z;
      continue;
    }
    T.hang_ijk[3 * h] = x; T.hang_ijk[3 * h + 1] = y; T.hang_ijk[3 * h + 2] = z;
    T.hang_owner[h] = int32_t(owner[n]);
    const int32_t* K = &T.leaf[4 * owner[n]];
    const int sK = F.size(K[3]);
    int r = 0;
    for (int v = 0; v < 8; ++v) {  // vertices of K_n with non-zero trilinear weight at x_n
      const int vx = K[0] + (v & 1) * sK, vy = K[1] + ((v >> 1) & 1) * sK, vz = K[2] + ((v >> 2) & 1) * sK;
      const int dd[3] = {std::abs(x - vx), std::abs(y - vy), std::abs(z - vz)};
      double w = 1.0;
      for (int a = 0; a < 3; ++a) w *= dd[a] == 0 ? 1.0 : (2 * dd[a] == sK ? 0.5 : 0.0);
      if (w == 0.0) continue;
      const int64_t sn = node_of(vx, vy, vz);
      if (sn < 0 || indep[sn] < 0 || r >= 4) {
        set_error(MPM_ETREE, "octree_build: constraint support is not an independent node", n);
        return MPM_ETREE;
      }
      T.hang_sup[4 * h + r] = indep[sn];
      T.hang_w[4 * h + r] = w;
      ++r;
    }
    ++h;
  }

  // I(K) slots and constraint codes
  T.cell_nodes.resize(nl * 8);
  T.cell_code.resize(nl);
  T.cell_cmat.assign(nl * 64, 0.0);
  for (int64_t e = 0; e < nl; ++e) {
    const int32_t* q = &T.leaf[4 * e];
    const int s = F.size(q[3]);
    const int cc = child[e];
    T.cell_code[e] = int32_t(hmask[e]) | (cc << 8);
    // C_K[j][k]: an independent vertex keeps its own slot; a hanging vertex j, mid-edge of
    // the parent on the axes M_j, spreads phi_j with weight 2^-|M_j| over the slots that agree
    // with j off M_j (the parent corners of its edge or face)
    for (int j = 0; j < 8; ++j) {
      const int M = (j ^ cc) & 7, nm = (M & 1) + ((M >> 1) & 1) + ((M >> 2) & 1);
      for (int k = 0; k < 8; ++k) {
        double v;
        if (!((hmask[e] >> j) & 1)) v = j == k ? 1.0 : 0.0;
        else v = (((j ^ k) & ~M & 7) == 0) ? (nm == 1 ? 0.5 : 0.25) : 0.0;
        T.cell_cmat[64 * e + 8 * j + k] = v;
      }
    }
    int32_t* slots = &T.cell_nodes[8 * e];
    for (int v = 0; v < 8; ++v) {
      int p[3];
      for (int a = 0; a < 3; ++a) {
        const int va = (v >> a) & 1, ca = (cc >> a) & 1;
        // a hanging vertex is replaced by the parent corner on the far side of each axis on
        // which it sits mid-edge (parent-lattice coordinate 1)
        const int pa = ((hmask[e] >> v) & 1) && va != ca ? (1 - ca) * 2 * s : (ca + va) * s;
        p[a] = q[a] - ca * s + pa;
      }
      const int64_t n = node_of(p[0], p[1], p[2]);
      if (n < 0 || indep[n] < 0) {
        set_error(MPM_ETREE, "octree_build: element slot is not an independent node", e);
        return MPM_ETREE;
      }
      slots[v] = indep[n];
    }
    for (int a = 0; a < 8; ++a)
      for (int b = a + 1; b < 8; ++b)
        if (slots[a] == slots[b]) {
          set_error(MPM_ETREE, "octree_build: |I(K)| < 8 (constraint chain or unbalanced tree)", e);
          return MPM_ETREE;
        }
  }
  lat_out[0] = F.lat[0]; lat_out[1] = F.lat[1]; lat_out[2] = F.lat[2];
  *hmin_out = F.hmin;
  return MPM_OK;
}

}  // namespace mpm
