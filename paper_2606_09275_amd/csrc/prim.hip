// Device primitives of the mesh construction: exclusive scan of counts and a 64-bit key sort
// built from the 32-bit radix sort.
#include "internal.h"

namespace mpm {

constexpr int kScanThreads = 256, kScanItems = 4, kScanBlock = kScanThreads * kScanItems;

// per block of kScanBlock counts: local exclusive offsets and the block total
__global__ __launch_bounds__(kScanThreads) void k_scan_local(const int32_t* __restrict__ in, int64_t n,
                                                             int64_t* __restrict__ out, int64_t* __restrict__ tot) {
  __shared__ int64_t wt[kScanThreads / 64];
  const int64_t base = int64_t(blockIdx.x) * kScanBlock + int64_t(threadIdx.x) * kScanItems;
  int64_t v[kScanItems], t = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? int64_t(in[base + k]) : 0;
    t += v[k];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int64_t inc = t;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t o = __shfl_up(inc, off);
    if (lane >= off) inc += o;
  }
  if (lane == 63) wt[wv] = inc;
  __syncthreads();
  int64_t pre = inc - t;
  for (int w = 0; w < wv; ++w) pre += wt[w];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = pre;
    pre += v[k];
  }
  if (threadIdx.x == kScanThreads - 1) tot[blockIdx.x] = pre;
}

// exclusive scan of nb block totals in place (one workgroup); tot[nb] = grand total
__global__ __launch_bounds__(1024) void k_scan_totals(int64_t* tot, int64_t nb) {
  __shared__ int64_t wt[16];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t base = 0; base < nb; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = i < nb ? tot[i] : 0;
    int64_t inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t o = __shfl_up(inc, off);
      if (lane >= off) inc += o;
    }
    if (lane == 63) wt[wv] = inc;
    __syncthreads();
    int64_t pre = carry;
    for (int w = 0; w < wv; ++w) pre += wt[w];
    if (i < nb) tot[i] = pre + inc - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry = pre + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) tot[nb] = carry;
}

__global__ void k_scan_add(int64_t* __restrict__ out, int64_t n, const int64_t* __restrict__ tot, int64_t nb) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] += tot[i / kScanBlock];
  if (i == 0) out[n] = tot[nb];
}

int32_t scan_counts(const int32_t* in, int64_t n, int64_t* out, hipStream_t st) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  DevBuf tot;
  if (const int32_t rc = tot.alloc(size_t(nb + 1) * 8, "scan: block totals")) return rc;
  if (nb) hipLaunchKernelGGL(k_scan_local, dim3(unsigned(nb)), dim3(kScanThreads), 0, st, in, n, out, tot.as<int64_t>());
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(1024), 0, st, tot.as<int64_t>(), nb);
  hipLaunchKernelGGL(k_scan_add, dim3(unsigned(n / 256 + 1)), dim3(256), 0, st, out, n, tot.as<int64_t>(), nb);
  MPM_HIP(hipGetLastError());
  // the totals buffer is freed at scope exit: wait for the kernels that read it
  MPM_HIP(hipStreamSynchronize(st));
  return MPM_OK;
}

__global__ void k_u64_split(const uint64_t* __restrict__ keys, int64_t n, uint32_t* __restrict__ lo,
                            uint32_t* __restrict__ idx) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    lo[i] = uint32_t(keys[i]);
    idx[i] = uint32_t(i);
  }
}
__global__ void k_u64_hi(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ idx, int64_t n,
                         uint32_t* __restrict__ hi) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) hi[i] = uint32_t(keys[idx[i]] >> 32);
}
__global__ void k_u64_gather(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ idx, int64_t n,
                             uint64_t* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = keys[idx[i]];
}

int32_t sort_u64(uint64_t* keys, int64_t n, int bits, hipStream_t st) {
  if (n <= 1) return MPM_OK;
  if (n > int64_t(UINT32_MAX)) {
    set_error(MPM_EARG, "sort: more than 2^32 - 1 keys");
    return MPM_EARG;
  }
  const int64_t nblk = (n + kRsTile - 1) / kRsTile;
  DevBuf a, b, c, d, h, g;
  int32_t rc = a.alloc(size_t(n) * 4, "sort: keys");
  if (!rc) rc = b.alloc(size_t(n) * 4, "sort: values");
  if (!rc) rc = c.alloc(size_t(n) * 4, "sort: key work");
  if (!rc) rc = d.alloc(size_t(n) * 4, "sort: value work");
  if (!rc) rc = h.alloc(size_t(nblk) * 256 * 4 + 256 * 4, "sort: counts");
  if (!rc) rc = g.alloc(size_t(n) * 8, "sort: gathered keys");
  if (rc) return rc;
  uint32_t* hist = h.as<uint32_t>();
  uint32_t* tot = hist + size_t(nblk) * 256;
  const dim3 grid(unsigned((n + 255) / 256));
  hipLaunchKernelGGL(k_u64_split, grid, dim3(256), 0, st, keys, n, a.as<uint32_t>(), b.as<uint32_t>());
  uint32_t *ks = nullptr, *vs = nullptr;
  rc = radix_sort(a.as<uint32_t>(), b.as<uint32_t>(), n, bits < 32 ? bits : 32, c.as<uint32_t>(), d.as<uint32_t>(),
                  hist, tot, st, &ks, &vs);
  if (rc) return rc;
  if (bits > 32) {
    // second stage: the high halves in the order of the first, sorted stably
    uint32_t* hi = ks;  // the low halves are no longer needed
    uint32_t* kt = ks == a.as<uint32_t>() ? c.as<uint32_t>() : a.as<uint32_t>();
    uint32_t* vt = vs == b.as<uint32_t>() ? d.as<uint32_t>() : b.as<uint32_t>();
    hipLaunchKernelGGL(k_u64_hi, grid, dim3(256), 0, st, keys, vs, n, hi);
    uint32_t *ks2 = nullptr, *vs2 = nullptr;
    rc = radix_sort(hi, vs, n, bits - 32, kt, vt, hist, tot, st, &ks2, &vs2);
    if (rc) return rc;
    vs = vs2;
  }
  hipLaunchKernelGGL(k_u64_gather, grid, dim3(256), 0, st, keys, vs, n, g.as<uint64_t>());
  MPM_HIP(hipMemcpyAsync(keys, g.p, size_t(n) * 8, hipMemcpyDeviceToDevice, st));
  MPM_HIP(hipGetLastError());
  MPM_HIP(hipStreamSynchronize(st));
  return MPM_OK;
}

}  // namespace mpm
