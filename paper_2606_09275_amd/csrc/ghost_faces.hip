// Ghost faces of the octree on the GPU (Section 4, eq. ghost) and, per face, the matrix of jump
// integrals
//   G_F[a][b] = int_F [d_n phi~_a] [d_n phi~_b] dA
// over the up to 16 slot nodes of the face's two leaves. A boundary leaf is a populated leaf
// (one that some point domain overlaps) with an unpopulated face neighbour; the ghost faces
// are the faces it shares with populated leaves (the smaller leaf's face where the two sizes
// differ). [.] is the jump across F of the normal derivative of the constrained trilinear
// basis of each leaf; the integrand is a product of two functions bilinear on F, so a 2 x 2
// Gauss rule on F is exact. h_F is the larger side of the two leaves, kappa = 10.
//
// Every boundary leaf emits the (lower rank, higher rank) key of each of its ghost faces; the
// keys are sorted and deduplicated (a face between two boundary leaves is emitted twice), so
// faces come in ascending leaf-pair order. One workgroup per face then builds its node union
// and G_F, and a stable sort of the (node, face * 16 + local index) incidences gives every
// node's contributions in ascending face order.
#include <algorithm>
#include <cmath>

#include "geom.h"

namespace mpm {

namespace {

constexpr double kGhostKappa = 10.0;

inline dim3 grid_of(int64_t n, int threads = 256) {
  return dim3(unsigned(std::max<int64_t>(1, (n + threads - 1) / threads)));
}

// leaves across one face of leaf e (axis a, side sg = +1 for the face at q_a + s). 2:1
// balance leaves one neighbour at least as large, or four of half size.
__device__ int face_neighbours(const LeafGeo& G, int64_t e, int a, int sg, int32_t out[4]) {
  const int32_t* q = G.leaf + 4 * e;
  const int s = 1 << (G.lmax - q[3]);
  const int pa = sg > 0 ? q[a] + s : q[a] - 1;
  if (pa < 0 || pa >= G.lat[a]) return 0;
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  auto at = [&](int ob, int oc) {
    int cell[3];
    cell[a] = pa;
    cell[b] = q[b] + ob;
    cell[c] = q[c] + oc;
    double p[3];
    for (int t = 0; t < 3; ++t) p[t] = G.lo[t] + (double(cell[t]) + 0.5) * G.hmin;
    return int32_t(leaf_of_point(G, p[0], p[1], p[2]));
  };
  const int32_t k0 = at(0, 0);
  const int s0 = 1 << (G.lmax - G.leaf[4 * int64_t(k0) + 3]);
  out[0] = k0;
  if (s0 >= s || s == 1) return 1;
  const int hs = s / 2;
  out[1] = at(hs, 0);
  out[2] = at(0, hs);
  out[3] = at(hs, hs);
  return 4;
}

// number of ghost faces a leaf emits (0 unless it is a boundary leaf), or the keys themselves
template <bool EMIT>
__global__ void k_ghost_leaf(LeafGeo G, const int32_t* __restrict__ pop, int32_t* __restrict__ cnt,
                             const int64_t* __restrict__ off, uint64_t* __restrict__ keys) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= G.n_leaf) return;
  if (EMIT && !cnt[e]) return;
  int32_t nb[4];
  if (!EMIT) {
    bool bnd = false;
    if (pop[e])
      for (int d = 0; d < 6 && !bnd; ++d) {
        const int k = face_neighbours(G, e, d >> 1, (d & 1) ? 1 : -1, nb);
        for (int t = 0; t < k; ++t) bnd |= !pop[nb[t]];
      }
    if (!bnd) {
      cnt[e] = 0;
      return;
    }
  }
  int64_t o = EMIT ? off[e] : 0;
  int c = 0;
  for (int d = 0; d < 6; ++d) {
    const int k = face_neighbours(G, e, d >> 1, (d & 1) ? 1 : -1, nb);
    for (int t = 0; t < k; ++t) {
      if (!pop[nb[t]]) continue;
      if (EMIT) {
        const uint64_t lo = uint64_t(e < nb[t] ? e : nb[t]), hi = uint64_t(e < nb[t] ? nb[t] : e);
        keys[o++] = (lo << 32) | hi;
      }
      ++c;
    }
  }
  if (!EMIT) cnt[e] = c;
}

__global__ void k_unique_keys(const uint64_t* __restrict__ k, int64_t n, int32_t* __restrict__ cnt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = (i == 0 || k[i] != k[i - 1]) ? 1 : 0;
}
__global__ void k_compact_keys(const uint64_t* __restrict__ k, const int32_t* __restrict__ cnt,
                               const int64_t* __restrict__ off, int64_t n, uint64_t* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n && cnt[i]) out[off[i]] = k[i];
}

// normal derivative along axis a of the 8 slot functions of leaf e at the physical point p
__device__ void slot_dn(const LeafGeo& G, const double* __restrict__ cmat, int64_t e, const double p[3], int a,
                        double out[8]) {
#pragma clang fp contract(off)
  const int32_t* q = G.leaf + 4 * e;
  const double h = double(1 << (G.lmax - q[3])) * G.hmin;
  double xi[3];
  for (int t = 0; t < 3; ++t) xi[t] = (p[t] - (G.lo[t] + double(q[t]) * G.hmin)) / h;
  double dv[8];
  for (int v = 0; v < 8; ++v) {
    double g = 1.0;
    for (int t = 0; t < 3; ++t) {
      const int bit = (v >> t) & 1;
      g *= t == a ? (bit ? 1.0 : -1.0) / h : (bit ? xi[t] : 1.0 - xi[t]);
    }
    dv[v] = g;
  }
  const double* C = cmat + 64 * e;
  for (int z = 0; z < 8; ++z) {
    double d = 0.0;
    for (int v = 0; v < 8; ++v) d += C[8 * v + z] * dv[v];
    out[z] = d;
  }
}

// One workgroup (one wavefront) per face: lane 0 forms the face record and the node union;
// lanes (Gauss point g, node x) form the jumps J_g[x]; each lane then sums four entries of G_F
// over the Gauss points in order.
__global__ __launch_bounds__(64) void k_ghost_face(LeafGeo G, const uint64_t* __restrict__ fkeys,
                                                   const int32_t* __restrict__ cell_nodes,
                                                   const double* __restrict__ cmat, int32_t* __restrict__ face,
                                                   int32_t* __restrict__ leaf2, int32_t* __restrict__ nodes,
                                                   double* __restrict__ Gm, double* __restrict__ hF) {
#pragma clang fp contract(off)
  __shared__ int32_t rec[8];
  __shared__ int32_t ids[16];
  __shared__ int8_t map[2][8];
  __shared__ double J[4][16];
  const int64_t f = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t lv[2] = {int64_t(fkeys[f] >> 32), int64_t(fkeys[f] & 0xffffffffu)};
  if (lane == 0) {
    const int32_t* q = G.leaf + 4 * lv[0];
    const int32_t* r = G.leaf + 4 * lv[1];
    const int s = 1 << (G.lmax - q[3]), so = 1 << (G.lmax - r[3]);
    int a = 0, plane = 0;
    for (int t = 0; t < 3; ++t) {
      if (q[t] + s == r[t]) {
        a = t;
        plane = r[t];
      } else if (r[t] + so == q[t]) {
        a = t;
        plane = q[t];
      }
    }
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    rec[0] = int32_t(lv[0]);
    rec[1] = int32_t(lv[1]);
    rec[2] = a;
    rec[3] = plane;
    rec[4] = q[b] > r[b] ? q[b] : r[b];
    rec[5] = q[b] + s < r[b] + so ? q[b] + s : r[b] + so;
    rec[6] = q[c] > r[c] ? q[c] : r[c];
    rec[7] = q[c] + s < r[c] + so ? q[c] + s : r[c] + so;
    int ni = 0;
    for (int side = 0; side < 2; ++side)
      for (int z = 0; z < 8; ++z) {
        const int32_t id = cell_nodes[8 * lv[side] + z];
        int pos = -1;
        for (int t = 0; t < ni; ++t)
          if (ids[t] == id) pos = t;
        if (pos < 0) {
          pos = ni;
          ids[ni++] = id;
        }
        map[side][z] = int8_t(pos);
      }
    for (int t = ni; t < 16; ++t) ids[t] = -1;
    hF[f] = double(s > so ? s : so) * G.hmin / kGhostKappa;  // h_F / kappa
  }
  __syncthreads();
  const int a = rec[2], b = (a + 1) % 3, c = (a + 2) % 3;
  const double fb = double(rec[5] - rec[4]) * G.hmin, fc = double(rec[7] - rec[6]) * G.hmin;
  {
    const double gx[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
    const int g = lane >> 4, x = lane & 15;
    double p[3];
    p[a] = G.lo[a] + double(rec[3]) * G.hmin;
    p[b] = G.lo[b] + double(rec[4]) * G.hmin + gx[g >> 1] * fb;
    p[c] = G.lo[c] + double(rec[6]) * G.hmin + gx[g & 1] * fc;
    double d[8], jx = 0.0;
    slot_dn(G, cmat, lv[0], p, a, d);
    for (int z = 0; z < 8; ++z)
      if (map[0][z] == x) jx += d[z];
    slot_dn(G, cmat, lv[1], p, a, d);
    for (int z = 0; z < 8; ++z)
      if (map[1][z] == x) jx -= d[z];
    J[g][x] = jx;
  }
  __syncthreads();
  const double w = 0.25 * fb * fc;
  for (int t = lane; t < 256; t += 64) {
    const int x = t >> 4, y = t & 15;
    double v = 0.0;
    for (int g = 0; g < 4; ++g) v += w * J[g][x] * J[g][y];
    Gm[256 * f + t] = (ids[x] >= 0 && ids[y] >= 0) ? v : 0.0;
  }
  if (lane < 8) face[8 * f + lane] = rec[lane];
  if (lane < 2) leaf2[2 * f + lane] = rec[lane];
  if (lane < 16) nodes[16 * f + lane] = ids[lane];
}

// (node, face * 16 + local index) incidences; padding slots get a key past every node
__global__ void k_ghost_incidences(const int32_t* __restrict__ nodes, int64_t nf, uint32_t* __restrict__ key,
                                   uint32_t* __restrict__ val) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= 16 * nf) return;
  const int32_t id = nodes[t];
  key[t] = id >= 0 ? uint32_t(id) : 0xffffffffu;
  val[t] = uint32_t(t);
}
__global__ void k_run_flags(const uint32_t* __restrict__ key, int64_t n, int32_t* __restrict__ cnt) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}
__global__ void k_run_lists(const uint32_t* __restrict__ key, const int32_t* __restrict__ cnt,
                            const int64_t* __restrict__ off, int64_t n, int32_t* __restrict__ gnode,
                            int32_t* __restrict__ gcon_off) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (cnt[i]) {
    gnode[off[i]] = int32_t(key[i]);
    gcon_off[off[i]] = int32_t(i);
  }
  if (i == n - 1) gcon_off[off[n]] = int32_t(n);
}
__global__ void k_copy_u32(const uint32_t* __restrict__ a, int64_t n, int32_t* __restrict__ b) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = int32_t(a[i]);
}

int32_t read_i64_h(const int64_t* d, int64_t* out) {
  MPM_HIP(hipMemcpy(out, d, 8, hipMemcpyDeviceToHost));
  return MPM_OK;
}
int bits_of(int64_t v) {
  int b = 1;
  while ((int64_t(1) << b) <= v) ++b;
  return b;
}

}  // namespace

// Ghost faces of the mesh for the overlapped-leaf flags pop (device, n_leaf): fills the mesh's
// face arrays (d_gf_*, d_gnode, d_gcon_off, d_gcon, h_gface, n_gface, n_gnode).
int32_t gpu_ghost_faces(mpm_mesh* m, const int32_t* pop, hipStream_t st) {
  const int64_t nl = m->n_leaf;
  const LeafGeo G = make_geo(m);
  DevBuf cnt, off, keys, ucnt, uoff, fkeys;
  int32_t rc = MPM_OK;
  if ((rc = cnt.alloc(size_t(nl) * 4, "ghost faces: counts")) ||
      (rc = off.alloc(size_t(nl + 1) * 8, "ghost faces: offsets")))
    return rc;
  hipLaunchKernelGGL(k_ghost_leaf<false>, grid_of(nl), dim3(256), 0, st, G, pop, cnt.as<int32_t>(), nullptr, nullptr);
  if ((rc = scan_counts(cnt.as<int32_t>(), nl, off.as<int64_t>(), st))) return rc;
  int64_t nk = 0;
  if ((rc = read_i64_h(off.as<int64_t>() + nl, &nk))) return rc;
  m->n_gface = 0;
  m->n_gnode = 0;
  if (!nk) return MPM_OK;
  if ((rc = keys.alloc(size_t(nk) * 8, "ghost faces: keys"))) return rc;
  hipLaunchKernelGGL(k_ghost_leaf<true>, grid_of(nl), dim3(256), 0, st, G, pop, cnt.as<int32_t>(), off.as<int64_t>(),
                     keys.as<uint64_t>());
  if ((rc = sort_u64(keys.as<uint64_t>(), nk, 32 + bits_of(nl), st))) return rc;
  if ((rc = ucnt.alloc(size_t(nk) * 4, "ghost faces: flags")) ||
      (rc = uoff.alloc(size_t(nk + 1) * 8, "ghost faces: offsets")))
    return rc;
  hipLaunchKernelGGL(k_unique_keys, grid_of(nk), dim3(256), 0, st, keys.as<uint64_t>(), nk, ucnt.as<int32_t>());
  if ((rc = scan_counts(ucnt.as<int32_t>(), nk, uoff.as<int64_t>(), st))) return rc;
  int64_t nf = 0;
  if ((rc = read_i64_h(uoff.as<int64_t>() + nk, &nf))) return rc;
  if (nf >= (int64_t(1) << 27)) {
    set_error(MPM_EARG, "octree_build: too many ghost faces");
    return MPM_EARG;
  }
  if ((rc = fkeys.alloc(size_t(nf) * 8, "ghost faces: faces"))) return rc;
  hipLaunchKernelGGL(k_compact_keys, grid_of(nk), dim3(256), 0, st, keys.as<uint64_t>(), ucnt.as<int32_t>(),
                     uoff.as<int64_t>(), nk, fkeys.as<uint64_t>());
  DevBuf face;
  if ((rc = face.alloc(size_t(nf) * 32, "ghost faces: records"))) return rc;
  MPM_HIP(hipMalloc(&m->d_gf_leaf, size_t(nf) * 8));
  MPM_HIP(hipMalloc(&m->d_gf_nodes, size_t(nf) * 64));
  MPM_HIP(hipMalloc(&m->d_gf_G, size_t(nf) * 256 * 8));
  MPM_HIP(hipMalloc(&m->d_gf_h, size_t(nf) * 8));
  hipLaunchKernelGGL(k_ghost_face, dim3(unsigned(nf)), dim3(64), 0, st, G, fkeys.as<uint64_t>(), m->d_cell_nodes,
                     m->d_cell_cmat, face.as<int32_t>(), m->d_gf_leaf, m->d_gf_nodes, m->d_gf_G, m->d_gf_h);
  MPM_HIP(hipGetLastError());
  m->n_gface = nf;
  // per-node contributions in ascending face order
  const int64_t ni = 16 * nf;
  const int64_t nblk = (ni + kRsTile - 1) / kRsTile;
  DevBuf ik, iv, ikt, ivt, hist, rcnt, roff;
  if ((rc = ik.alloc(size_t(ni) * 4, "ghost faces: incidences")) ||
      (rc = iv.alloc(size_t(ni) * 4, "ghost faces: incidences")) ||
      (rc = ikt.alloc(size_t(ni) * 4, "ghost faces: incidences")) ||
      (rc = ivt.alloc(size_t(ni) * 4, "ghost faces: incidences")) ||
      (rc = hist.alloc(size_t(nblk) * 1024 + 1024, "ghost faces: incidence counts")) ||
      (rc = rcnt.alloc(size_t(ni) * 4, "ghost faces: runs")) ||
      (rc = roff.alloc(size_t(ni + 1) * 8, "ghost faces: runs")))
    return rc;
  hipLaunchKernelGGL(k_ghost_incidences, grid_of(ni), dim3(256), 0, st, m->d_gf_nodes, nf, ik.as<uint32_t>(),
                     iv.as<uint32_t>());
  uint32_t *ks = ik.as<uint32_t>(), *vs = iv.as<uint32_t>();
  if ((rc = radix_sort(ik.as<uint32_t>(), iv.as<uint32_t>(), ni, 32, ikt.as<uint32_t>(), ivt.as<uint32_t>(),
                       hist.as<uint32_t>(), hist.as<uint32_t>() + size_t(nblk) * 256, st, &ks, &vs)))
    return rc;
  // valid incidences are those before the first padding key
  int64_t nvalid = 0;
  {
    std::vector<int32_t> hn(size_t(nf) * 16);
    MPM_HIP(hipStreamSynchronize(st));
    MPM_HIP(hipMemcpy(hn.data(), m->d_gf_nodes, hn.size() * 4, hipMemcpyDeviceToHost));
    for (int32_t id : hn) nvalid += id >= 0;
  }
  hipLaunchKernelGGL(k_run_flags, grid_of(nvalid), dim3(256), 0, st, ks, nvalid, rcnt.as<int32_t>());
  if ((rc = scan_counts(rcnt.as<int32_t>(), nvalid, roff.as<int64_t>(), st))) return rc;
  if ((rc = read_i64_h(roff.as<int64_t>() + nvalid, &m->n_gnode))) return rc;
  MPM_HIP(hipMalloc(&m->d_gnode, size_t(std::max<int64_t>(1, m->n_gnode)) * 4));
  MPM_HIP(hipMalloc(&m->d_gcon_off, size_t(m->n_gnode + 1) * 4));
  MPM_HIP(hipMalloc(&m->d_gcon, size_t(std::max<int64_t>(1, nvalid)) * 4));
  hipLaunchKernelGGL(k_run_lists, grid_of(nvalid), dim3(256), 0, st, ks, rcnt.as<int32_t>(), roff.as<int64_t>(),
                     nvalid, m->d_gnode, m->d_gcon_off);
  hipLaunchKernelGGL(k_copy_u32, grid_of(nvalid), dim3(256), 0, st, vs, nvalid, m->d_gcon);
  MPM_HIP(hipGetLastError());
  // host copy of the face records
  m->h_gface.resize(size_t(nf) * 8);
  MPM_HIP(hipStreamSynchronize(st));
  MPM_HIP(hipMemcpy(m->h_gface.data(), face.p, size_t(nf) * 32, hipMemcpyDeviceToHost));
  return MPM_OK;
}

}  // namespace mpm
