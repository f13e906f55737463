// Octree construction on the GPU: refinement Steps 1-3 with 2:1 balance across faces and
// edges (Section 5), nodes, hanging nodes and their constraints, and the slot nodes and
// constraint matrices of every leaf (Section 3.1).
//
// Leaves are 64-bit keys (Morton key of the anchor << 5 | level), kept sorted: splitting a
// leaf into its 8 children in child order keeps the Morton order, so a round is a marking
// kernel and an order-keeping expansion (scan of 1 or 8 outputs per leaf). Balance ripples:
// every leaf at least two levels finer than the base looks at the 18 face and edge neighbour
// cells of its own size and flags the leaf holding each of them when that leaf is more than
// one level coarser; the flagged leaves are split and the check repeats until nothing is
// flagged. Each split is forced by a leaf that no balanced refinement can avoid, so the result
// is the unique coarsest balanced refinement, whatever the order of the splits.
//
// Nodes are the leaf vertices (sorted Morton keys of their lattice coordinates, duplicates
// removed). A vertex that sits mid-edge or mid-face of its leaf's parent hangs when a leaf of
// the parent's level shares that edge or face; its owner is the lowest-ranked such leaf, and
// its supports are the owner's vertices with non-zero trilinear weight there (1/2 on an edge,
// 1/4 on a face).
#include <algorithm>

#include "internal.h"

namespace mpm {

namespace {

constexpr double kTie = 1e-12;  // relative slack: ties of distance predicates count as inside
constexpr int kLevBits = 5;

struct TreeParams {
  double lo[3];
  double hmin;
  int lbase, lmax;
  int lat[3];
  int body_kind;
  double body[8];
  double dx;
};

__host__ __device__ inline uint64_t pack_leaf(int x, int y, int z, int lev) {
  return (morton(uint64_t(x), uint64_t(y), uint64_t(z)) << kLevBits) | uint64_t(lev);
}
__device__ inline void unpack_leaf(uint64_t k, int q[4]) {
  q[3] = int(k & 31u);
  const uint64_t m = k >> kLevBits;
  q[0] = int(compact3(m));
  q[1] = int(compact3(m >> 1));
  q[2] = int(compact3(m >> 2));
}

// squared distance from (r, z) in the meridian half-plane to the segment p0-p1
__device__ double seg_dist2(double r, double z, double r0, double z0, double r1, double z1) {
#pragma clang fp contract(off)
  const double er = r1 - r0, ez = z1 - z0;
  const double len2 = er * er + ez * ez;
  double t = 0.0;
  if (len2 > 0.0) t = fmin(1.0, fmax(0.0, ((r - r0) * er + (z - z0) * ez) / len2));
  const double dr = r0 + t * er - r, dz = z0 + t * ez - z;
  return dr * dr + dz * dz;
}

// Step 2: point within distance dx of the closed solid (distance 0 inside)
__device__ bool body_near(const TreeParams& c, const double p[3], double dx) {
#pragma clang fp contract(off)
  const double* b = c.body;
  if (c.body_kind == MPM_BODY_SPHERE) {
    const double ex = p[0] - b[0], ey = p[1] - b[1], ez = p[2] - b[2];
    const double reach = b[3] + dx;
    return ex * ex + ey * ey + ez * ez <= reach * reach * (1.0 + kTie);
  }
  if (c.body_kind == MPM_BODY_CONE) {
    const double ax = p[0] - b[0], ay = p[1] - b[1];
    const double r = sqrt(ax * ax + ay * ay), z = p[2];
    const double zap = b[2], R = b[3], tn = b[4], ztop = b[5];
    const double zsh = zap + R / tn;  // where the cone reaches the shaft radius
    if (z >= zap && z <= ztop && r <= fmin(R, (z - zap) * tn)) return true;
    double d2 = seg_dist2(r, z, 0.0, zap, R, zsh);
    d2 = fmin(d2, seg_dist2(r, z, R, zsh, R, ztop));
    d2 = fmin(d2, seg_dist2(r, z, R, ztop, 0.0, ztop));
    return d2 <= dx * dx * (1.0 + kTie);
  }
  if (c.body_kind == MPM_BODY_BOX) {
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double e = fmax(0.0, fmax(b[2 * a] - p[a], p[a] - b[2 * a + 1]));
      d2 += e * e;
    }
    return d2 <= dx * dx * (1.0 + kTie);
  }
  return false;
}

__device__ inline double gap(double v, double l, double h) { return v < l ? l - v : (v > h ? v - h : 0.0); }

// Step 1: the closed box [lo, hi] meets the closed solid
__device__ bool body_meets(const TreeParams& c, const double lo[3], const double hi[3]) {
#pragma clang fp contract(off)
  const double* b = c.body;
  if (c.body_kind == MPM_BODY_SPHERE) {
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double e = gap(b[a], lo[a], hi[a]);
      d2 += e * e;
    }
    return d2 <= b[3] * b[3] * (1.0 + kTie);
  }
  if (c.body_kind == MPM_BODY_CONE) {
    // the radius does not decrease with z: test the highest z the box and the solid share
    const double zl = fmax(lo[2], b[2]), zh = fmin(hi[2], b[5]);
    if (zl > zh) return false;
    const double rad = fmin(b[3], (zh - b[2]) * b[4]);
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

// rank of the leaf holding finest cell (x, y, z): the last key whose anchor does not exceed
// the cell's Morton key
__device__ int64_t leaf_at(const uint64_t* __restrict__ keys, int64_t nl, int x, int y, int z) {
  const uint64_t m = morton(uint64_t(x), uint64_t(y), uint64_t(z));
  int64_t lo = 0, hi = nl;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((keys[mid] >> kLevBits) <= m) lo = mid + 1;
    else hi = mid;
  }
  return lo - 1;
}

// rank of the leaf with exactly this anchor and level, or -1
__device__ int64_t leaf_exact(const uint64_t* __restrict__ keys, int64_t nl, int x, int y, int z, int lev) {
  const int64_t r = leaf_at(keys, nl, x, y, z);
  if (r < 0) return -1;
  return keys[r] == pack_leaf(x, y, z, lev) ? r : -1;
}

// rank of the node with these lattice coordinates, or -1
__device__ int64_t node_at(const uint64_t* __restrict__ nkey, int64_t nn, int x, int y, int z) {
  const uint64_t m = morton(uint64_t(x), uint64_t(y), uint64_t(z));
  int64_t lo = 0, hi = nn;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (nkey[mid] < m) lo = mid + 1;
    else hi = mid;
  }
  return (lo < nn && nkey[lo] == m) ? lo : -1;
}

__device__ inline void flag_error(DevErr* err, int32_t code, int64_t index) {
  if (atomicCAS(&err->code, 0, code) == 0) err->index = (unsigned long long)index;
}

// base cells in Morton order: candidate Morton indices of a 2^B cube, kept when inside
__global__ void k_base_count(int64_t ncand, int bx, int by, int bz, int32_t* __restrict__ cnt) {
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m >= ncand) return;
  const int x = int(compact3(uint64_t(m))), y = int(compact3(uint64_t(m) >> 1)), z = int(compact3(uint64_t(m) >> 2));
  cnt[m] = (x < bx && y < by && z < bz) ? 1 : 0;
}
__global__ void k_base_emit(int64_t ncand, const int32_t* __restrict__ cnt, const int64_t* __restrict__ off, int s0,
                            int lbase, uint64_t* __restrict__ keys) {
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m >= ncand || !cnt[m]) return;
  const int x = int(compact3(uint64_t(m))), y = int(compact3(uint64_t(m) >> 1)), z = int(compact3(uint64_t(m) >> 2));
  keys[off[m]] = pack_leaf(x * s0, y * s0, z * s0, lbase);
}

// Steps 1-2: 8 outputs for a marked leaf, 1 otherwise
__global__ void k_tree_mark(const uint64_t* __restrict__ keys, int64_t nl, TreeParams c, int32_t* __restrict__ cnt) {
#pragma clang fp contract(off)
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nl) return;
  int q[4];
  unpack_leaf(keys[e], q);
  if (q[3] >= c.lmax) {
    cnt[e] = 1;
    return;
  }
  const int s = 1 << (c.lmax - q[3]);
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    lo[a] = c.lo[a] + double(q[a]) * c.hmin;
    hi[a] = c.lo[a] + double(q[a] + s) * c.hmin;
  }
  bool hit = body_meets(c, lo, hi);
  for (int v = 0; v < 8 && !hit; ++v) {
    const double p[3] = {(v & 1) ? hi[0] : lo[0], (v & 2) ? hi[1] : lo[1], (v & 4) ? hi[2] : lo[2]};
    hit = body_near(c, p, c.dx);
  }
  cnt[e] = hit ? 8 : 1;
}

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t n, int32_t v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// balance: flag (8 outputs) every leaf more than one level coarser than a face or edge
// neighbour cell of a leaf's own size
__global__ void k_tree_balance(const uint64_t* __restrict__ keys, int64_t nl, TreeParams c,
                               int32_t* __restrict__ cnt) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nl) return;
  int q[4];
  unpack_leaf(keys[e], q);
  if (q[3] - c.lbase < 2) return;  // nothing can be two levels coarser
  const int s = 1 << (c.lmax - q[3]);
  for (int d = 0; d < 27; ++d) {
    const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
    const int nzc = (dx != 0) + (dy != 0) + (dz != 0);
    if (nzc == 0 || nzc == 3) continue;  // faces and edges
    const int p[3] = {q[0] + dx * s, q[1] + dy * s, q[2] + dz * s};
    if (p[0] < 0 || p[1] < 0 || p[2] < 0 || p[0] >= c.lat[0] || p[1] >= c.lat[1] || p[2] >= c.lat[2]) continue;
    const int64_t j = leaf_at(keys, nl, p[0], p[1], p[2]);
    if (j >= 0 && int(keys[j] & 31u) <= q[3] - 2) cnt[j] = 8;
  }
}

// order-keeping expansion: a leaf with 8 outputs is replaced by its children in child order
__global__ void k_tree_expand(const uint64_t* __restrict__ kin, const int32_t* __restrict__ cnt,
                              const int64_t* __restrict__ off, int64_t nl, int lmax, uint64_t* __restrict__ kout) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nl) return;
  const int64_t o = off[e];
  if (cnt[e] == 1) {
    kout[o] = kin[e];
    return;
  }
  int q[4];
  unpack_leaf(kin[e], q);
  const int h = (1 << (lmax - q[3])) / 2;
  for (int ch = 0; ch < 8; ++ch)
    kout[o + ch] = pack_leaf(q[0] + (ch & 1) * h, q[1] + ((ch >> 1) & 1) * h, q[2] + ((ch >> 2) & 1) * h, q[3] + 1);
}

__global__ void k_tree_leaves(const uint64_t* __restrict__ keys, int64_t nl, int32_t* __restrict__ leaf,
                              uint64_t* __restrict__ leaf_key) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nl) return;
  int q[4];
  unpack_leaf(keys[e], q);
  for (int a = 0; a < 4; ++a) leaf[4 * e + a] = q[a];
  leaf_key[e] = keys[e] >> kLevBits;
}

__global__ void k_vertex_keys(const int32_t* __restrict__ leaf, int64_t nl, int lmax, uint64_t* __restrict__ vk) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= 8 * nl) return;
  const int64_t e = t >> 3;
  const int v = int(t & 7);
  const int32_t* q = leaf + 4 * e;
  const int s = 1 << (lmax - q[3]);
  vk[t] = morton(uint64_t(q[0] + (v & 1) * s), uint64_t(q[1] + ((v >> 1) & 1) * s), uint64_t(q[2] + ((v >> 2) & 1) * s));
}

__global__ void k_unique_flags(const uint64_t* __restrict__ k, int64_t n, int32_t* __restrict__ cnt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = (i == 0 || k[i] != k[i - 1]) ? 1 : 0;
}
__global__ void k_compact_u64(const uint64_t* __restrict__ k, const int32_t* __restrict__ cnt,
                              const int64_t* __restrict__ off, int64_t n, uint64_t* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n && cnt[i]) out[off[i]] = k[i];
}

constexpr unsigned long long kNoOwner = 0x7fffffffffffffffull;

__global__ void k_fill_u64(unsigned long long* __restrict__ a, int64_t n, unsigned long long v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// hanging vertices from the parent lattice; owner[n] = lowest rank of a parent-level leaf
// sharing the parent edge or face through the vertex
__global__ void k_hanging(const int32_t* __restrict__ leaf, const uint64_t* __restrict__ keys, int64_t nl,
                          const uint64_t* __restrict__ nkey, int64_t nn, TreeParams c, uint8_t* __restrict__ hmask,
                          uint8_t* __restrict__ child, unsigned long long* __restrict__ owner, DevErr* err) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nl) return;
  const int32_t* q = leaf + 4 * e;
  if (q[3] == c.lbase) {
    hmask[e] = 0;
    child[e] = 0;
    return;
  }
  const int s = 1 << (c.lmax - q[3]), ps = 2 * s;
  const int P[3] = {q[0] / ps * ps, q[1] / ps * ps, q[2] / ps * ps};
  const int cc[3] = {(q[0] - P[0]) / s, (q[1] - P[1]) / s, (q[2] - P[2]) / s};
  child[e] = uint8_t(cc[0] | (cc[1] << 1) | (cc[2] << 2));
  uint8_t hm = 0;
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
          if (pos[a] == 1) {
            ok = false;  // only step across the boundary planes
            break;
          }
          off[a] = pos[a] == 0 ? -1 : 1;
        }
      }
      if (!ok) continue;
      const int nb[3] = {P[0] + off[0] * ps, P[1] + off[1] * ps, P[2] + off[2] * ps};
      if (nb[0] < 0 || nb[1] < 0 || nb[2] < 0 || nb[0] >= c.lat[0] || nb[1] >= c.lat[1] || nb[2] >= c.lat[2]) continue;
      const int64_t r = leaf_exact(keys, nl, nb[0], nb[1], nb[2], q[3] - 1);
      if (r >= 0 && (best < 0 || r < best)) best = r;
    }
    if (best < 0) continue;
    hm |= uint8_t(1u << v);
    const int64_t n = node_at(nkey, nn, q[0] + ((v & 1) ? s : 0), q[1] + (((v >> 1) & 1) ? s : 0),
                              q[2] + (((v >> 2) & 1) ? s : 0));
    if (n < 0) {
      flag_error(err, MPM_ETREE, e);
      continue;
    }
    atomicMin(owner + n, (unsigned long long)best);
  }
  hmask[e] = hm;
}

// a vertex flagged hanging by one leaf must be flagged by every leaf that has it
__global__ void k_hang_check(const int32_t* __restrict__ leaf, int64_t nl, const uint64_t* __restrict__ nkey,
                             int64_t nn, int lmax, const uint8_t* __restrict__ hmask,
                             const unsigned long long* __restrict__ owner, DevErr* err) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= 8 * nl) return;
  const int64_t e = t >> 3;
  const int v = int(t & 7);
  const int32_t* q = leaf + 4 * e;
  const int s = 1 << (lmax - q[3]);
  const int64_t n = node_at(nkey, nn, q[0] + (v & 1) * s, q[1] + ((v >> 1) & 1) * s, q[2] + ((v >> 2) & 1) * s);
  if (n < 0 || (owner[n] != kNoOwner) != bool((hmask[e] >> v) & 1)) flag_error(err, MPM_ETREE, n);
}

__global__ void k_indep_flags(const unsigned long long* __restrict__ owner, int64_t nn, int32_t* __restrict__ cnt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < nn) cnt[i] = owner[i] == kNoOwner ? 1 : 0;
}

// independent nodes, hanging nodes and their constraint supports and weights
__global__ void k_nodes_out(const uint64_t* __restrict__ nkey, int64_t nn, const unsigned long long* __restrict__ owner,
                            const int64_t* __restrict__ ind, const int32_t* __restrict__ leaf, int lmax,
                            int32_t* __restrict__ node_ijk, int32_t* __restrict__ hang_ijk,
                            int32_t* __restrict__ hang_sup, double* __restrict__ hang_w,
                            int32_t* __restrict__ hang_owner, DevErr* err) {
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  const int x = int(compact3(nkey[n])), y = int(compact3(nkey[n] >> 1)), z = int(compact3(nkey[n] >> 2));
  if (owner[n] == kNoOwner) {
    int32_t* d = node_ijk + 3 * ind[n];
    d[0] = x;
    d[1] = y;
    d[2] = z;
    return;
  }
  const int64_t h = n - ind[n];
  hang_ijk[3 * h] = x;
  hang_ijk[3 * h + 1] = y;
  hang_ijk[3 * h + 2] = z;
  hang_owner[h] = int32_t(owner[n]);
  const int32_t* K = leaf + 4 * int64_t(owner[n]);
  const int sK = 1 << (lmax - K[3]);
  int r = 0;
  for (int k = 0; k < 4; ++k) {
    hang_sup[4 * h + k] = -1;
    hang_w[4 * h + k] = 0.0;
  }
  for (int v = 0; v < 8; ++v) {  // vertices of K_n with non-zero trilinear weight at x_n
    const int vx = K[0] + (v & 1) * sK, vy = K[1] + ((v >> 1) & 1) * sK, vz = K[2] + ((v >> 2) & 1) * sK;
    const int dd[3] = {abs(x - vx), abs(y - vy), abs(z - vz)};
    double w = 1.0;
    for (int a = 0; a < 3; ++a) w *= dd[a] == 0 ? 1.0 : (2 * dd[a] == sK ? 0.5 : 0.0);
    if (w == 0.0) continue;
    const int64_t sn = node_at(nkey, nn, vx, vy, vz);
    if (sn < 0 || owner[sn] != kNoOwner || r >= 4) {
      flag_error(err, MPM_ETREE, n);
      return;
    }
    hang_sup[4 * h + r] = int32_t(ind[sn]);
    hang_w[4 * h + r] = w;
    ++r;
  }
}

// slot nodes I(K), constraint codes and C_K of every leaf
__global__ void k_cells(const int32_t* __restrict__ leaf, int64_t nl, const uint64_t* __restrict__ nkey, int64_t nn,
                        const unsigned long long* __restrict__ owner, const int64_t* __restrict__ ind, int lmax,
                        const uint8_t* __restrict__ hmask, const uint8_t* __restrict__ child,
                        int32_t* __restrict__ cell_nodes, int32_t* __restrict__ cell_code,
                        double* __restrict__ cell_cmat, DevErr* err) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nl) return;
  const int32_t* q = leaf + 4 * e;
  const int s = 1 << (lmax - q[3]);
  const int cc = child[e], hm = hmask[e];
  cell_code[e] = hm | (cc << 8);
  // C_K[j][k]: an independent vertex keeps its own slot; a hanging vertex j, mid-edge of the
  // parent on the axes M_j, spreads phi_j with weight 2^-|M_j| over the slots that agree with
  // j off M_j (the parent corners of its edge or face)
  for (int j = 0; j < 8; ++j) {
    const int M = (j ^ cc) & 7, nm = (M & 1) + ((M >> 1) & 1) + ((M >> 2) & 1);
    for (int k = 0; k < 8; ++k) {
      double v;
      if (!((hm >> j) & 1)) v = j == k ? 1.0 : 0.0;
      else v = (((j ^ k) & ~M & 7) == 0) ? (nm == 1 ? 0.5 : 0.25) : 0.0;
      cell_cmat[64 * e + 8 * j + k] = v;
    }
  }
  int32_t slots[8];
  for (int v = 0; v < 8; ++v) {
    int p[3];
    for (int a = 0; a < 3; ++a) {
      const int va = (v >> a) & 1, ca = (cc >> a) & 1;
      // a hanging vertex is replaced by the parent corner on the far side of each axis on
      // which it sits mid-edge (parent-lattice coordinate 1)
      const int pa = ((hm >> v) & 1) && va != ca ? (1 - ca) * 2 * s : (ca + va) * s;
      p[a] = q[a] - ca * s + pa;
    }
    const int64_t n = node_at(nkey, nn, p[0], p[1], p[2]);
    if (n < 0 || owner[n] != kNoOwner) {
      flag_error(err, MPM_ETREE, e);
      slots[v] = 0;
    } else {
      slots[v] = int32_t(ind[n]);
    }
    cell_nodes[8 * e + v] = slots[v];
  }
  for (int a = 0; a < 8; ++a)
    for (int b = a + 1; b < 8; ++b)
      if (slots[a] == slots[b]) flag_error(err, MPM_ETREE, e);
}

int32_t read_i64(const int64_t* d, int64_t* out) {
  MPM_HIP(hipMemcpy(out, d, 8, hipMemcpyDeviceToHost));
  return MPM_OK;
}

inline dim3 grid_of(int64_t n, int threads = 256) { return dim3(unsigned((n + threads - 1) / threads)); }

}  // namespace

// Builds the tree of crit on the device into the mesh's leaf, node, hanging-node and cell
// arrays and counts (n_leaf, n_node, n_hang, nx, ny, nz, hmin).
int32_t gpu_build_tree(mpm_mesh* m, const mpm_refine_t& c, hipStream_t st) {
  if (c.lvl_max < c.lvl_base || c.lvl_max - c.lvl_base > 13 || !(c.h0 > 0) || c.base[0] <= 0 || c.base[1] <= 0 ||
      c.base[2] <= 0 || c.lvl_base < 0 || c.lvl_max > 31) {
    set_error(MPM_EARG, "octree_build: bad refinement levels, base grid or h0");
    return MPM_EARG;
  }
  const int s0 = 1 << (c.lvl_max - c.lvl_base);
  TreeParams P;
  for (int a = 0; a < 3; ++a) {
    P.lo[a] = c.lo[a];
    P.lat[a] = c.base[a] * s0;
  }
  if (std::max({P.lat[0], P.lat[1], P.lat[2]}) >= (1 << 13)) {
    set_error(MPM_ESTENCIL, "octree_build: finest lattice exceeds 8191 cells per axis");
    return MPM_ESTENCIL;
  }
  P.hmin = c.h0 / double(s0);
  P.lbase = c.lvl_base;
  P.lmax = c.lvl_max;
  P.body_kind = c.body_kind;
  for (int k = 0; k < 8; ++k) P.body[k] = c.body[k];
  P.dx = c.dx_region;
  m->nx = P.lat[0];
  m->ny = P.lat[1];
  m->nz = P.lat[2];
  m->hmin = P.hmin;

  // base cells in Morton order
  int B = 0;
  while ((1 << B) < std::max({c.base[0], c.base[1], c.base[2]})) ++B;
  const int64_t ncand = int64_t(1) << (3 * B);
  DevBuf keys, work, cnt, off;
  int32_t rc = cnt.alloc(size_t(ncand) * 4, "octree_build: base flags");
  if (!rc) rc = off.alloc(size_t(ncand + 1) * 8, "octree_build: base offsets");
  if (rc) return rc;
  hipLaunchKernelGGL(k_base_count, grid_of(ncand), dim3(256), 0, st, ncand, c.base[0], c.base[1], c.base[2],
                     cnt.as<int32_t>());
  if ((rc = scan_counts(cnt.as<int32_t>(), ncand, off.as<int64_t>(), st))) return rc;
  int64_t nl = int64_t(c.base[0]) * c.base[1] * c.base[2];
  if ((rc = keys.alloc(size_t(nl) * 8, "octree_build: leaves"))) return rc;
  hipLaunchKernelGGL(k_base_emit, grid_of(ncand), dim3(256), 0, st, ncand, cnt.as<int32_t>(), off.as<int64_t>(), s0,
                     c.lvl_base, keys.as<uint64_t>());

  // one expansion of the leaves by the counts in cnt; returns whether anything was split
  auto expand = [&](bool* changed) -> int32_t {
    int32_t r = scan_counts(cnt.as<int32_t>(), nl, off.as<int64_t>(), st);
    int64_t total = 0;
    if (!r) r = read_i64(off.as<int64_t>() + nl, &total);
    if (r) return r;
    *changed = total != nl;
    if (!*changed) return MPM_OK;
    if (total >= (int64_t(1) << 31)) {
      set_error(MPM_ESTENCIL, "octree_build: too many leaves");
      return MPM_ESTENCIL;
    }
    if ((r = work.alloc(size_t(total) * 8, "octree_build: leaves"))) return r;
    hipLaunchKernelGGL(k_tree_expand, grid_of(nl), dim3(256), 0, st, keys.as<uint64_t>(), cnt.as<int32_t>(),
                       off.as<int64_t>(), nl, c.lvl_max, work.as<uint64_t>());
    MPM_HIP(hipGetLastError());
    std::swap(keys.p, work.p);
    nl = total;
    if ((r = cnt.alloc(size_t(nl) * 4, "octree_build: leaf flags"))) return r;
    return off.alloc(size_t(nl + 1) * 8, "octree_build: leaf offsets");
  };
  if ((rc = cnt.alloc(size_t(nl) * 4, "octree_build: leaf flags"))) return rc;
  if ((rc = off.alloc(size_t(nl + 1) * 8, "octree_build: leaf offsets"))) return rc;
  if (c.body_kind != MPM_BODY_NONE) {
    for (;;) {  // Steps 1-3 until nothing is marked, each round followed by balance
      hipLaunchKernelGGL(k_tree_mark, grid_of(nl), dim3(256), 0, st, keys.as<uint64_t>(), nl, P, cnt.as<int32_t>());
      bool changed = false;
      if ((rc = expand(&changed))) return rc;
      if (!changed) break;
      for (;;) {
        hipLaunchKernelGGL(k_fill_i32, grid_of(nl), dim3(256), 0, st, cnt.as<int32_t>(), nl, 1);
        hipLaunchKernelGGL(k_tree_balance, grid_of(nl), dim3(256), 0, st, keys.as<uint64_t>(), nl, P,
                           cnt.as<int32_t>());
        bool split = false;
        if ((rc = expand(&split))) return rc;
        if (!split) break;
      }
    }
  }
  m->n_leaf = nl;

  // leaves
  DevBuf dleaf, dkey;
  if ((rc = dleaf.alloc(size_t(nl) * 16, "octree_build: leaf anchors")) ||
      (rc = dkey.alloc(size_t(nl) * 8, "octree_build: leaf keys")))
    return rc;
  hipLaunchKernelGGL(k_tree_leaves, grid_of(nl), dim3(256), 0, st, keys.as<uint64_t>(), nl, dleaf.as<int32_t>(),
                     dkey.as<uint64_t>());
  // nodes: sorted unique vertex keys
  const int64_t nv = 8 * nl;
  DevBuf vk, vcnt, voff, nkey;
  if ((rc = vk.alloc(size_t(nv) * 8, "octree_build: vertex keys")) ||
      (rc = vcnt.alloc(size_t(nv) * 4, "octree_build: vertex flags")) ||
      (rc = voff.alloc(size_t(nv + 1) * 8, "octree_build: vertex offsets")))
    return rc;
  hipLaunchKernelGGL(k_vertex_keys, grid_of(nv), dim3(256), 0, st, dleaf.as<int32_t>(), nl, c.lvl_max,
                     vk.as<uint64_t>());
  if ((rc = sort_u64(vk.as<uint64_t>(), nv, 42, st))) return rc;
  hipLaunchKernelGGL(k_unique_flags, grid_of(nv), dim3(256), 0, st, vk.as<uint64_t>(), nv, vcnt.as<int32_t>());
  if ((rc = scan_counts(vcnt.as<int32_t>(), nv, voff.as<int64_t>(), st))) return rc;
  int64_t nn = 0;
  if ((rc = read_i64(voff.as<int64_t>() + nv, &nn))) return rc;
  if ((rc = nkey.alloc(size_t(nn) * 8, "octree_build: node keys"))) return rc;
  hipLaunchKernelGGL(k_compact_u64, grid_of(nv), dim3(256), 0, st, vk.as<uint64_t>(), vcnt.as<int32_t>(),
                     voff.as<int64_t>(), nv, nkey.as<uint64_t>());

  // hanging nodes
  DevBuf hmask, child, owner, icnt, ind;
  if ((rc = hmask.alloc(size_t(nl), "octree_build: hanging masks")) ||
      (rc = child.alloc(size_t(nl), "octree_build: child indices")) ||
      (rc = owner.alloc(size_t(nn) * 8, "octree_build: owners")) ||
      (rc = icnt.alloc(size_t(nn) * 4, "octree_build: node flags")) ||
      (rc = ind.alloc(size_t(nn + 1) * 8, "octree_build: node ranks")))
    return rc;
  hipLaunchKernelGGL(k_fill_u64, grid_of(nn), dim3(256), 0, st, owner.as<unsigned long long>(), nn, kNoOwner);
  hipLaunchKernelGGL(k_hanging, grid_of(nl), dim3(256), 0, st, dleaf.as<int32_t>(), keys.as<uint64_t>(), nl,
                     nkey.as<uint64_t>(), nn, P, hmask.as<uint8_t>(), child.as<uint8_t>(),
                     owner.as<unsigned long long>(), m->d_err);
  hipLaunchKernelGGL(k_hang_check, grid_of(nv), dim3(256), 0, st, dleaf.as<int32_t>(), nl, nkey.as<uint64_t>(), nn,
                     c.lvl_max, hmask.as<uint8_t>(), owner.as<unsigned long long>(), m->d_err);
  if ((rc = read_error(m, st, "octree_build (hanging nodes)"))) return rc;
  hipLaunchKernelGGL(k_indep_flags, grid_of(nn), dim3(256), 0, st, owner.as<unsigned long long>(), nn,
                     icnt.as<int32_t>());
  if ((rc = scan_counts(icnt.as<int32_t>(), nn, ind.as<int64_t>(), st))) return rc;
  int64_t ni = 0;
  if ((rc = read_i64(ind.as<int64_t>() + nn, &ni))) return rc;
  const int64_t nh = nn - ni;
  m->n_node = ni;
  m->n_hang = nh;
  DevBuf b_node, b_hijk, b_hsup, b_hw, b_hown, b_cn, b_cc, b_cm;
  if ((rc = b_node.alloc(size_t(ni) * 12, "octree_build: nodes")) ||
      (rc = b_hijk.alloc(size_t(nh) * 12, "octree_build: hanging nodes")) ||
      (rc = b_hsup.alloc(size_t(nh) * 16, "octree_build: constraint supports")) ||
      (rc = b_hw.alloc(size_t(nh) * 32, "octree_build: constraint weights")) ||
      (rc = b_hown.alloc(size_t(nh) * 4, "octree_build: constraint owners")) ||
      (rc = b_cn.alloc(size_t(nl) * 32, "octree_build: slot nodes")) ||
      (rc = b_cc.alloc(size_t(nl) * 4, "octree_build: constraint codes")) ||
      (rc = b_cm.alloc(size_t(nl) * 512, "octree_build: constraint matrices")))
    return rc;
  hipLaunchKernelGGL(k_nodes_out, grid_of(nn), dim3(256), 0, st, nkey.as<uint64_t>(), nn,
                     owner.as<unsigned long long>(), ind.as<int64_t>(), dleaf.as<int32_t>(), c.lvl_max,
                     b_node.as<int32_t>(), b_hijk.as<int32_t>(), b_hsup.as<int32_t>(), b_hw.as<double>(),
                     b_hown.as<int32_t>(), m->d_err);
  hipLaunchKernelGGL(k_cells, grid_of(nl), dim3(256), 0, st, dleaf.as<int32_t>(), nl, nkey.as<uint64_t>(), nn,
                     owner.as<unsigned long long>(), ind.as<int64_t>(), c.lvl_max, hmask.as<uint8_t>(),
                     child.as<uint8_t>(), b_cn.as<int32_t>(), b_cc.as<int32_t>(), b_cm.as<double>(), m->d_err);
  MPM_HIP(hipGetLastError());
  if ((rc = read_error(m, st, "octree_build (constraints)"))) return rc;
  auto release = [](DevBuf& b) {
    void* p = b.p;
    b.p = nullptr;
    return p;
  };
  m->d_leaf = static_cast<int32_t*>(release(dleaf));
  m->d_leaf_key = static_cast<uint64_t*>(release(dkey));
  m->d_node_ijk = static_cast<int32_t*>(release(b_node));
  m->d_hang_ijk = static_cast<int32_t*>(release(b_hijk));
  m->d_hang_sup = static_cast<int32_t*>(release(b_hsup));
  m->d_hang_w = static_cast<double*>(release(b_hw));
  m->d_hang_owner = static_cast<int32_t*>(release(b_hown));
  m->d_cell_nodes = static_cast<int32_t*>(release(b_cn));
  m->d_cell_code = static_cast<int32_t*>(release(b_cc));
  m->d_cell_cmat = static_cast<double*>(release(b_cm));
  return MPM_OK;
}

}  // namespace mpm
