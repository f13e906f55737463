// Ghost stabilisation of the stiffness (Section 4, eq. ghost), device part: the largest
// Young's modulus of the points overlapping each leaf, and one workgroup per node adding
// (h_F beta_F / kappa) G_F to the diagonals of its 3x3 blocks and K_G u to its forces, with
// beta_F the larger leaf maximum of the face's two leaves. The faces, G_F and h_F / kappa come
// from the host part at mesh construction.
#include "geom.h"

namespace mpm {

// ------------------------------------------------------------------ device
// beta[e] = largest Young's modulus of the points overlapping leaf e (0 if none); E > 0, so
// the integer order of the IEEE bit patterns is the order of the values.
__global__ void k_zero_beta(double* beta, int64_t nl) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < nl) beta[e] = 0.0;
}

__global__ void k_leaf_beta(const double* __restrict__ E, const int32_t* __restrict__ pleaf,
                            const uint8_t* __restrict__ pnleaf, int64_t n, const int64_t* __restrict__ strad,
                            const int32_t* __restrict__ strad_leaf, int64_t ns, double* beta) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    if (pnleaf[i] == 1) {
      const double v = E[i] > 0.0 ? E[i] : 0.0;
      atomicMax(reinterpret_cast<unsigned long long*>(beta + pleaf[i]), (unsigned long long)__double_as_longlong(v));
    }
  } else if (i < n + ns) {
    const int64_t t = i - n;
    const double v = E[strad[t]] > 0.0 ? E[strad[t]] : 0.0;
    for (int k = 0; k < kMaxPointLeaves; ++k) {
      const int32_t e = strad_leaf[t * kMaxPointLeaves + k];
      if (e < 0) break;
      atomicMax(reinterpret_cast<unsigned long long*>(beta + e), (unsigned long long)__double_as_longlong(v));
    }
  }
}

// One workgroup (one wavefront) per node with ghost contributions. For each contribution
// (face F, local index ia of the node), in ascending face order, lanes 0..15 take the face's
// nodes ib: w = (h_F / kappa) beta_F G_F[ia][ib] is added to the LDS accumulator of the block
// column of node ib in the node's rows, and w u_ib to the force. The accumulated weights are
// then added to the diagonal entries of the three rows' 3x3 blocks (the form couples equal
// displacement components only). Each K entry and force belongs to one node's rows: no
// atomics, and the summation order is fixed.
constexpr int kGhostMaxDeg = 1024;  // equals the widest node row the mesh accepts

template <typename T>
__global__ __launch_bounds__(64) void k_ghost_gather(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ gnode,
                                                     const int32_t* __restrict__ gcon_off,
                                                     const int32_t* __restrict__ gcon, const int32_t* __restrict__ gnodes,
                                                     const double* __restrict__ gG, const double* __restrict__ gh,
                                                     const int32_t* __restrict__ gleaf,
                                                     const int16_t* __restrict__ gbpos, const double* __restrict__ beta,
                                                     const double* __restrict__ u, T* K, double* f) {
  __shared__ double acc[kGhostMaxDeg];
  const int64_t nd = gnode[blockIdx.x];
  const int lane = threadIdx.x;
  const int c0 = gcon_off[blockIdx.x], c1 = gcon_off[blockIdx.x + 1];
  const int64_t r0 = row_ptr[3 * nd], len3 = row_ptr[3 * nd + 1] - r0;
  const int deg = int(len3 / 3);
  if (K) {
    for (int t = lane; t < deg; t += 64) acc[t] = 0.0;
    __syncthreads();
  }
  double fs0 = 0.0, fs1 = 0.0, fs2 = 0.0;
  for (int cc = c0; cc < c1; ++cc) {
    const int32_t code = gcon[cc];  // face * 16 + ia
    const int64_t fc = code >> 4;
    const int ia = code & 15;
    const double sc = gh[fc] * fmax(beta[gleaf[2 * fc]], beta[gleaf[2 * fc + 1]]);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    if (lane < 16) {
      const int32_t nb = gnodes[16 * fc + lane];
      if (nb >= 0) {
        const double w = sc * gG[256 * fc + 16 * ia + lane];
        if (K) acc[gbpos[256 * fc + 16 * ia + lane]] += w;  // distinct columns within one face
        a0 = w * u[3 * int64_t(nb)];
        a1 = w * u[3 * int64_t(nb) + 1];
        a2 = w * u[3 * int64_t(nb) + 2];
      }
    }
    if (K) __syncthreads();
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) {
      a0 += __shfl_xor(a0, off);
      a1 += __shfl_xor(a1, off);
      a2 += __shfl_xor(a2, off);
    }
    fs0 += a0;
    fs1 += a1;
    fs2 += a2;
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
  hipLaunchKernelGGL(k_zero_beta, dim3(unsigned((m->n_leaf + 255) / 256)), dim3(256), 0, st, m->d_gbeta, m->n_leaf);
  const int64_t tot = m->n_point + m->n_straddle;
  if (tot)
    hipLaunchKernelGGL(k_leaf_beta, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st, s->E, m->d_pleaf,
                       m->d_pnleaf, m->n_point, m->d_strad, m->d_strad_leaf, m->n_straddle, m->d_gbeta);
  if (m->n_gnode) {
    if (precision == MPM_F64)
      hipLaunchKernelGGL(k_ghost_gather<double>, dim3(unsigned(m->n_gnode)), dim3(64), 0, st, m->d_row_ptr,
                         m->d_gnode, m->d_gcon_off, m->d_gcon, m->d_gf_nodes, m->d_gf_G, m->d_gf_h, m->d_gf_leaf,
                         m->d_gf_bpos, m->d_gbeta, u, static_cast<double*>(K), f);
    else
      hipLaunchKernelGGL(k_ghost_gather<float>, dim3(unsigned(m->n_gnode)), dim3(64), 0, st, m->d_row_ptr, m->d_gnode,
                         m->d_gcon_off, m->d_gcon, m->d_gf_nodes, m->d_gf_G, m->d_gf_h, m->d_gf_leaf, m->d_gf_bpos,
                         m->d_gbeta, u, static_cast<float*>(K), f);
  }
  MPM_HIP(hipGetLastError());
  return MPM_OK;
}

}  // namespace mpm
