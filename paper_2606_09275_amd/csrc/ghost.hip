// Ghost stabilisation of the stiffness (Section 4, eq. ghost), device part: the largest
// Young's modulus of the points overlapping each leaf, and one workgroup per node adding
// (h_F beta_F / kappa) G_F to the diagonals of its 3x3 blocks and K_G u to its forces, with
// beta_F the larger leaf maximum of the face's two leaves. The faces, G_F and h_F / kappa are
// built once per mesh (ghost_faces.hip).
#include "geom.h"

namespace mpm {

// ------------------------------------------------------------------ device
// beta[e] = largest Young's modulus of the points overlapping leaf e (0 if none). Points are
// sorted by leaf: one wavefront per 64 points takes the maximum of each of its segments (runs
// of one leaf), then per leaf the maximum over the leaf's segments (one thread per leaf, the
// whole wavefront for a leaf with many segments), so a leaf holding many points needs no
// atomics. Points overlapping several leaves count in
// k_leaf_beta_strad (E > 0, so the integer order of the IEEE bit patterns is the order of the
// values there).
__global__ __launch_bounds__(64) void k_seg_beta(const double* __restrict__ E, const int32_t* __restrict__ pleaf,
                                                 const uint8_t* __restrict__ pnleaf, const int64_t* __restrict__ fidx,
                                                 int64_t nf, const int32_t* __restrict__ wave_seg,
                                                 double* __restrict__ segmax) {
  // lane j of the list of points whose domain lies in one leaf (the segments' order)
  const int64_t j = int64_t(blockIdx.x) * 64 + threadIdx.x;
  const int lane = threadIdx.x;
  int32_t leaf = -1;
  double v = 0.0;
  const bool inr = j < nf;
  if (inr) {
    const int64_t i = fidx ? fidx[j] : j;
    leaf = pleaf[i];
    if (pnleaf[i] == 1 && E[i] > 0.0) v = E[i];
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double ov = __shfl_down(v, off);
    const int32_t ol = __shfl_down(leaf, off);
    if (lane + off < 64 && ol == leaf) v = fmax(v, ov);
  }
  const int32_t prev = __shfl_up(leaf, 1);
  const bool head = inr && (lane == 0 || prev != leaf);
  const uint64_t hm = __ballot(head);
  if (head) segmax[wave_seg[blockIdx.x] + __popcll(hm & ((1ull << lane) - 1ull))] = v;
}

// One thread per leaf; a leaf with more than kLightSeg segments (coarse leaves holding many
// points) is taken by the whole wavefront in turn: strided loads, then a shuffle reduction.
constexpr int kLightSeg = 8;
__global__ __launch_bounds__(256) void k_leaf_beta(const double* __restrict__ segmax, const int32_t* __restrict__ seg0,
                                                   const int32_t* __restrict__ nseg, int64_t n_leaf,
                                                   double* __restrict__ beta) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int32_t s0 = 0, ns = 0;
  if (e < n_leaf) {
    s0 = seg0[e];
    ns = nseg[e];
  }
  double v = 0.0;
  const bool heavy = ns > kLightSeg;
  if (!heavy)
    for (int j = 0; j < ns; ++j) v = fmax(v, segmax[s0 + j]);
  uint64_t hm = __ballot(heavy);  // every lane takes part (no early exit before this loop)
  while (hm) {
    const int src = __ffsll((unsigned long long)hm) - 1;
    hm &= hm - 1;
    const int32_t hs0 = __shfl(s0, src), hns = __shfl(ns, src);
    double w = 0.0;
    for (int j = lane; j < hns; j += 64) w = fmax(w, segmax[hs0 + j]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) w = fmax(w, __shfl_xor(w, off));
    if (lane == src) v = w;
  }
  if (e < n_leaf) beta[e] = v;
}

__global__ void k_leaf_beta_strad(const double* __restrict__ E, const int64_t* __restrict__ strad,
                                  const int32_t* __restrict__ strad_leaf, int64_t ns, double* beta) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= ns) return;
  const double e = E[strad[t]];
  if (!(e > 0.0)) return;
  for (int k = 0; k < kMaxPointLeaves; ++k) {
    const int32_t l = strad_leaf[t * kMaxPointLeaves + k];
    if (l < 0) break;
    atomicMax(reinterpret_cast<unsigned long long*>(beta + l), (unsigned long long)__double_as_longlong(e));
  }
}

// scale of each face: (h_F / kappa) * beta_F, beta_F the larger leaf maximum of its two leaves
__global__ void k_face_scale(const double* __restrict__ gh, const int32_t* __restrict__ gleaf,
                             const double* __restrict__ beta, int64_t nf, double* __restrict__ sc) {
  const int64_t fc = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (fc < nf) sc[fc] = gh[fc] * fmax(beta[gleaf[2 * fc]], beta[gleaf[2 * fc + 1]]);
}

// One workgroup (one wavefront) per node with ghost contributions (face F, local index ia of
// the node), taken four at a time: 16-lane group g holds contribution g of the batch, its lane
// ib the face's node ib, with weight w = scale_F G_F[ia][ib]. The weights are added to an LDS
// accumulator indexed by the block column of node ib in the node's rows, group after group
// (ascending face order, no atomics), and w u_ib to the force, summed per group and then over
// the groups in order. The accumulated weights finally go to the diagonal entries of the
// three rows' 3x3 blocks (the form couples equal displacement components only). Every K
// entry and force belongs to one node's rows, so the result is reproducible.
constexpr int kGhostMaxDeg = 1024;  // equals the widest node row the mesh accepts

template <typename T>
__global__ __launch_bounds__(64) void k_ghost_gather(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ gnode,
                                                     const int32_t* __restrict__ gcon_off,
                                                     const int32_t* __restrict__ gcon, const int32_t* __restrict__ gnodes,
                                                     const double* __restrict__ gG, const double* __restrict__ gsc,
                                                     const int16_t* __restrict__ gbpos, const double* __restrict__ u,
                                                     T* K, double* f) {
  __shared__ double acc[kGhostMaxDeg];
  const int64_t nd = gnode[blockIdx.x];
  const int lane = threadIdx.x, grp = lane >> 4, ib = lane & 15;
  const int c0 = gcon_off[blockIdx.x], c1 = gcon_off[blockIdx.x + 1];
  const int64_t r0 = row_ptr[3 * nd], len3 = row_ptr[3 * nd + 1] - r0;
  const int deg = int(len3 / 3);
  if (K) {
    for (int t = lane; t < deg; t += 64) acc[t] = 0.0;
    __syncthreads();
  }
  double fs0 = 0.0, fs1 = 0.0, fs2 = 0.0;
  for (int cb = c0; cb < c1; cb += 4) {
    const int cc = cb + grp;
    double w = 0.0, a0 = 0.0, a1 = 0.0, a2 = 0.0;
    int pos = -1;
    if (cc < c1) {
      const int32_t code = gcon[cc];  // face * 16 + ia
      const int64_t fc = code >> 4;
      const int ia = code & 15;
      const int32_t nb = gnodes[16 * fc + ib];
      if (nb >= 0) {
        w = gsc[fc] * gG[256 * fc + 16 * ia + ib];
        pos = gbpos[256 * fc + 16 * ia + ib];
        a0 = w * u[3 * int64_t(nb)];
        a1 = w * u[3 * int64_t(nb) + 1];
        a2 = w * u[3 * int64_t(nb) + 2];
      }
    }
    if (K)
      for (int g = 0; g < 4; ++g) {
        if (grp == g && pos >= 0) acc[pos] += w;  // distinct columns within one face
        __syncthreads();
      }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) {
      a0 += __shfl_xor(a0, off);
      a1 += __shfl_xor(a1, off);
      a2 += __shfl_xor(a2, off);
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      fs0 += __shfl(a0, 16 * g);
      fs1 += __shfl(a1, 16 * g);
      fs2 += __shfl(a2, 16 * g);
    }
  }
  if (K)
    for (int t = lane; t < deg; t += 64) {
      const double w = acc[t];
      if (w != 0.0)
        for (int r = 0; r < 3; ++r) {
          T* e = K + r0 + r * len3 + 3 * t + r;
          *e = T(double(*e) + w);
        }
    }
  if (lane == 0) {
    f[3 * nd] += fs0;
    f[3 * nd + 1] += fs1;
    f[3 * nd + 2] += fs2;
  }
}

int32_t ghost_apply(const mpm_mesh* m, const mpm_state_t* s, const double* u, int32_t precision, void* K, double* f,
                    hipStream_t st) {
  if (!m->n_gface) return MPM_OK;
  if (m->n_fast)
    hipLaunchKernelGGL(k_seg_beta, dim3(unsigned(m->n_wave)), dim3(64), 0, st, s->E, m->d_pleaf, m->d_pnleaf,
                       m->d_fidx, m->n_fast, m->d_wave_seg, m->d_gsegmax);
  hipLaunchKernelGGL(k_leaf_beta, dim3(unsigned((m->n_leaf + 255) / 256)), dim3(256), 0, st, m->d_gsegmax,
                     m->d_leaf_seg0, m->d_leaf_nseg, m->n_leaf, m->d_gbeta);
  if (m->n_straddle)
    hipLaunchKernelGGL(k_leaf_beta_strad, dim3(unsigned((m->n_straddle + 255) / 256)), dim3(256), 0, st, s->E,
                       m->d_strad, m->d_strad_leaf, m->n_straddle, m->d_gbeta);
  hipLaunchKernelGGL(k_face_scale, dim3(unsigned((m->n_gface + 255) / 256)), dim3(256), 0, st, m->d_gf_h,
                     m->d_gf_leaf, m->d_gbeta, m->n_gface, m->d_gf_sc);
  if (m->n_gnode) {
    if (precision == MPM_F64)
      hipLaunchKernelGGL(k_ghost_gather<double>, dim3(unsigned(m->n_gnode)), dim3(64), 0, st, m->d_row_ptr,
                         m->d_gnode, m->d_gcon_off, m->d_gcon, m->d_gf_nodes, m->d_gf_G, m->d_gf_sc, m->d_gf_bpos, u,
                         static_cast<double*>(K), f);
    else
      hipLaunchKernelGGL(k_ghost_gather<float>, dim3(unsigned(m->n_gnode)), dim3(64), 0, st, m->d_row_ptr, m->d_gnode,
                         m->d_gcon_off, m->d_gcon, m->d_gf_nodes, m->d_gf_G, m->d_gf_sc, m->d_gf_bpos, u,
                         static_cast<float*>(K), f);
  }
  MPM_HIP(hipGetLastError());
  return MPM_OK;
}

}  // namespace mpm
