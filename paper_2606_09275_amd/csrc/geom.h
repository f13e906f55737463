// Device/host geometry of leaves and GIMP domains: which leaves a point domain overlaps.
#pragma once
#include "internal.h"

namespace mpm {

struct LeafGeo {
  const int32_t* leaf;      // n_leaf x 4
  const uint64_t* leaf_key; // n_leaf, ascending
  const int32_t* cellmap;   // leaf of every finest lattice cell, x fastest (or null: search the keys)
  int64_t n_leaf;
  double lo[3];
  double hmin;
  int lmax;
  int lat[3];
};

// Leaf containing the finest lattice cell of point p: the last leaf whose anchor key does
// not exceed the cell's Morton key (leaves tile the box as contiguous Morton ranges).
__host__ __device__ inline int64_t leaf_of_point(const LeafGeo& G, double px, double py, double pz) {
#pragma clang fp contract(off)
  const double p[3] = {px, py, pz};
  int q[3];
  for (int a = 0; a < 3; ++a) {
    double t = floor((p[a] - G.lo[a]) / G.hmin);
    int v = t < 0.0 ? 0 : (t > double(G.lat[a] - 1) ? G.lat[a] - 1 : int(t));
    q[a] = v;
  }
  if (G.cellmap) return G.cellmap[(int64_t(q[2]) * G.lat[1] + q[1]) * G.lat[0] + q[0]];
  const uint64_t m = morton(uint64_t(q[0]), uint64_t(q[1]), uint64_t(q[2]));
  int64_t lo = 0, hi = G.n_leaf;  // first key > m
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (G.leaf_key[mid] <= m) lo = mid + 1;
    else hi = mid;
  }
  return lo - 1;
}

__host__ __device__ inline void leaf_bounds(const LeafGeo& G, int64_t e, double lo[3], double hi[3], double* h) {
#pragma clang fp contract(off)
  const int32_t* q = G.leaf + 4 * e;
  const int s = 1 << (G.lmax - q[3]);
  for (int a = 0; a < 3; ++a) {
    lo[a] = G.lo[a] + double(q[a]) * G.hmin;
    hi[a] = G.lo[a] + double(q[a] + s) * G.hmin;
  }
  *h = double(s) * G.hmin;
}

// Leaves overlapped with positive volume by the domain [x-l, x+l] (an axis overlap must
// exceed 1e-12 of the domain side). Leaf boundaries crossing the domain are collected per
// axis; at most one distinct plane per axis is supported, which holds whenever every
// overlapped leaf is at least as wide as the domain. Returns the number of leaves (<= 8)
// or MPM_EOUTSIDE / MPM_ESTENCIL.
__host__ __device__ inline int domain_leaves(const LeafGeo& G, int64_t k0, const double x[3], const double l[3],
                                             int32_t out[kMaxPointLeaves]) {
#pragma clang fp contract(off)
  double a0[3], a1[3], thr[3];
  for (int a = 0; a < 3; ++a) {
    a0[a] = x[a] - l[a];
    a1[a] = x[a] + l[a];
    thr[a] = 1e-12 * (2.0 * l[a]);
    const double mlo = G.lo[a], mhi = G.lo[a] + double(G.lat[a]) * G.hmin;
    if (mlo - a0[a] > thr[a] || a1[a] - mhi > thr[a]) return MPM_EOUTSIDE;
  }
  double plane[3] = {0, 0, 0};
  bool has[3] = {false, false, false};
  auto add_faces = [&](int64_t e) -> bool {
    double lo[3], hi[3], h;
    leaf_bounds(G, e, lo, hi, &h);
    for (int a = 0; a < 3; ++a) {
      const double f[2] = {lo[a], hi[a]};
      for (int s = 0; s < 2; ++s) {
        if (!(a0[a] < f[s] && f[s] < a1[a])) continue;
        if (has[a] && plane[a] != f[s]) return false;
        has[a] = true;
        plane[a] = f[s];
      }
    }
    return true;
  };
  if (!add_faces(k0)) return MPM_ESTENCIL;
  int nout = 0;
  for (int iter = 0; iter < 4; ++iter) {
    bool h0[3] = {has[0], has[1], has[2]};
    nout = 0;
    for (int c = 0; c < 8; ++c) {
      double ctr[3];
      bool skip = false;
      for (int a = 0; a < 3; ++a) {
        const int side = (c >> a) & 1;
        if (!has[a]) {
          if (side) skip = true;
          ctr[a] = 0.5 * (a0[a] + a1[a]);
        } else {
          ctr[a] = side ? 0.5 * (plane[a] + a1[a]) : 0.5 * (a0[a] + plane[a]);
        }
      }
      if (skip) continue;
      const int64_t e = leaf_of_point(G, ctr[0], ctr[1], ctr[2]);
      if (!add_faces(e)) return MPM_ESTENCIL;
      bool seen = false;
      for (int t = 0; t < nout; ++t) seen |= out[t] == int32_t(e);
      if (!seen) out[nout++] = int32_t(e);
    }
    if (h0[0] == has[0] && h0[1] == has[1] && h0[2] == has[2]) break;
  }
  // keep leaves with a positive-volume overlap
  int nk = 0;
  for (int t = 0; t < nout; ++t) {
    double lo[3], hi[3], h;
    leaf_bounds(G, out[t], lo, hi, &h);
    bool pos = true;
    for (int a = 0; a < 3; ++a) {
      const double o = (a1[a] < hi[a] ? a1[a] : hi[a]) - (a0[a] > lo[a] ? a0[a] : lo[a]);
      pos = pos && (o > thr[a]);
    }
    if (pos) out[nk++] = out[t];
  }
  return nk;
}

}  // namespace mpm
