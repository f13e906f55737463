// Linear solve of a Newton step on the assembled tangent (the solve that consumes K, named by
// the paper as the cost that dominates its CPU runs): Jacobi-preconditioned conjugate
// gradients over the free DOFs (not Dirichlet, row not empty), with the fixed DOFs held at
// zero (the strong Dirichlet treatment of Section 2.4 applied to the increment). K is the CSR
// of the mesh in FP64 or FP32; vectors and reductions are FP64 and deterministic (fixed
// two-stage summation order).
#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstring>
#include <mutex>

#include "internal.h"

namespace mpm {

constexpr int kSpmvLanes = 32;   // lanes per node in the SpMV (8 nodes per 256-thread workgroup)
constexpr int kDotBlocks = 512;    // partial sums of a dot product
constexpr int kUpdBlocks = 2048;   // blocks of the vector update (each leaves two partial sums)

// scalars kept on the device between the kernels of one solve
enum CgScalar { kRZ = 0, kPQ, kBB, kRR, kRZN, kBeta, kNumScalars };
struct CgFlags {
  int done;
  int iters;
};

// y = K x on the rows of `fr` (others: y = x). The three rows of node n are 9 deg contiguous
// values [row][block][k] with one column pattern; kSpmvLanes lanes take a node (its columns
// strided over them: about two each at deg 27), then a fixed-order butterfly reduction inside
// the group.
template <typename T>
__global__ __launch_bounds__(256) void k_spmv(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                              const T* __restrict__ K, const double* __restrict__ x,
                                              double* __restrict__ y, const uint8_t* __restrict__ fr, int64_t n_node,
                                              const int* skip) {
  if (skip && *skip) return;
  const int sub = threadIdx.x / kSpmvLanes, lane = threadIdx.x % kSpmvLanes;
  const int64_t nd = int64_t(blockIdx.x) * (256 / kSpmvLanes) + sub;
  const bool ok = nd < n_node;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (ok) {
    const int64_t base = row_ptr[3 * nd];
    const int len3 = int(row_ptr[3 * nd + 1] - base);
    for (int c = lane; c < len3; c += kSpmvLanes) {
      const double xa = x[col[base + c]];
      s0 += double(K[base + c]) * xa;
      s1 += double(K[base + len3 + c]) * xa;
      s2 += double(K[base + 2 * len3 + c]) * xa;
    }
  }
#pragma unroll
  for (int off = kSpmvLanes / 2; off > 0; off >>= 1) {  // stays inside the node's lane group
    s0 += __shfl_xor(s0, off);
    s1 += __shfl_xor(s1, off);
    s2 += __shfl_xor(s2, off);
  }
  if (ok && lane < 3) {
    const int64_t d = 3 * nd + lane;
    const double s = lane == 0 ? s0 : (lane == 1 ? s1 : s2);
    y[d] = (!fr || fr[d]) ? s : x[d];
  }
}

// block partial sums of a . b (and optionally c . d) in a fixed order
__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (int(threadIdx.x) < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ a, const double* __restrict__ b,
                                                     int64_t n, double* __restrict__ part, const CgFlags* flags) {
  if (flags && flags->done) return;
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < n; k += int64_t(gridDim.x) * 256) acc += a[k] * b[k];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// one block: scal[dst] = sum of np partials (fixed order)
__global__ __launch_bounds__(256) void k_dot_final(const double* __restrict__ part, int np, double* scal, int dst,
                                                   const CgFlags* flags) {
  if (flags && flags->done) return;
  __shared__ double sh[256];
  double acc = 0.0;
  for (int k = threadIdx.x; k < np; k += 256) acc += part[k];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) scal[dst] = s;
}

// diagonal entry of CSR row d (columns ascend: bisection); 0 when the row has none
template <typename T>
__device__ __forceinline__ double row_diag(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                           const T* __restrict__ K, int64_t d) {
  int64_t lo = row_ptr[d], hi = row_ptr[d + 1] - 1;
  while (lo <= hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int32_t c = col[mid];
    if (c == int32_t(d)) return double(K[mid]);
    if (c < int32_t(d)) lo = mid + 1;
    else hi = mid - 1;
  }
  return 0.0;
}

// free DOFs, inverse diagonal, r = z = p = 0 / b on free DOFs, x = 0
template <typename T>
__global__ __launch_bounds__(256) void k_cg_init(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                                 const T* __restrict__ K, const uint8_t* __restrict__ dir,
                                                 const double* __restrict__ b, int64_t ndof, uint8_t* __restrict__ fr,
                                                 double* __restrict__ dinv, double* __restrict__ x,
                                                 double* __restrict__ r, double* __restrict__ z,
                                                 double* __restrict__ p) {
  const int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (d >= ndof) return;
  const double diag = row_diag(row_ptr, col, K, d);
  const int64_t a0 = row_ptr[d], a1 = row_ptr[d + 1];
  const bool f = (!dir || !dir[d]) && a1 > a0 && diag > 0.0;
  fr[d] = f ? 1 : 0;
  dinv[d] = f ? 1.0 / diag : 0.0;
  const double bd = f ? b[d] : 0.0;
  x[d] = 0.0;
  r[d] = bd;
  z[d] = dinv[d] * bd;
  p[d] = z[d];
}

// alpha = rz / pq; x += alpha p; r -= alpha q; z = dinv r; and the block's partial sums of the
// new r.z and r.r (part[block], part[gridDim + block]), summed by k_cg_step in a fixed order
__global__ __launch_bounds__(256) void k_cg_update(double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ z, const double* __restrict__ p,
                                                   const double* __restrict__ q, const double* __restrict__ dinv,
                                                   int64_t ndof, const double* scal, double* __restrict__ part,
                                                   const CgFlags* flags) {
  __shared__ double sh[256];
  if (flags->done) return;
  const double pq = scal[kPQ];
  if (!(pq > 0.0)) return;  // not positive definite along p: the step kernel stops the solve
  const double alpha = scal[kRZ] / pq;
  double rz = 0.0, rr = 0.0;
  for (int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x; d < ndof; d += int64_t(gridDim.x) * 256) {
    x[d] += alpha * p[d];
    const double rd = r[d] - alpha * q[d];
    const double zd = dinv[d] * rd;
    r[d] = rd;
    z[d] = zd;
    rz += rd * zd;
    rr += rd * rd;
  }
  const double srz = block_sum(rz, sh);
  const double srr = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = srz;
    part[gridDim.x + blockIdx.x] = srr;
  }
}

// r.z -> scal[kRZN] and r.r -> scal[kRR] from the update's nb partials of each, then beta,
// convergence and the iteration count (one block)
__global__ __launch_bounds__(256) void k_cg_step(double* scal, const double* __restrict__ part, int nb,
                                                 CgFlags* flags, double rtol2, int max_iter) {
  __shared__ double sh[256];
  if (flags->done) return;
  if (!(scal[kPQ] > 0.0)) {  // breakdown: the update was skipped
    if (threadIdx.x == 0) flags->done = 2;
    return;
  }
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) {
    a += part[k];
    b += part[nb + k];
  }
  const double rz_new = block_sum(a, sh);
  const double rr = block_sum(b, sh);
  if (threadIdx.x == 0) {
    scal[kRZN] = rz_new;
    scal[kRR] = rr;
    flags->iters += 1;
    scal[kBeta] = rz_new / scal[kRZ];
    scal[kRZ] = rz_new;
    if (!(rr > rtol2 * scal[kBB]) || flags->iters >= max_iter || !(rz_new > 0.0)) flags->done = 1;
  }
}

// p = z + beta p
__global__ __launch_bounds__(256) void k_cg_dir(double* __restrict__ p, const double* __restrict__ z, int64_t ndof,
                                                const double* scal, const CgFlags* flags) {
  if (flags->done) return;
  const double beta = scal[kBeta];
  for (int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x; d < ndof; d += int64_t(gridDim.x) * 256)
    p[d] = z[d] + beta * p[d];
}

__global__ void k_cg_start(double* scal, CgFlags* flags) {
  flags->done = scal[kBB] > 0.0 ? 0 : 1;  // b = 0 on the free DOFs: x = 0
  flags->iters = 0;
}

template <typename T>
static void launch_spmv(const mpm_mesh* m, const void* K, const double* x, double* y, const uint8_t* fr,
                        const int* skip, hipStream_t st) {
  constexpr int per = 256 / kSpmvLanes;
  const dim3 grid(unsigned((m->n_node + per - 1) / per));
  hipLaunchKernelGGL(k_spmv<T>, grid, dim3(256), 0, st, m->d_row_ptr, m->d_col,
                     static_cast<const T*>(K), x, y, fr, m->n_node, skip);
}

static void launch_dot(const double* a, const double* b, int64_t n, double* part, double* scal, int dst,
                       const CgFlags* flags, hipStream_t st) {
  const int nb = int(std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, (n + 255) / 256)));
  hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(256), 0, st, a, b, n, part, flags);
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, st, part, nb, scal, dst, flags);
}

// work buffer of the solver kept with the mesh: r, z, p, q, dinv [n_dof] doubles, partials,
// scalars, flags, free mask
struct CgBuf {
  double *r, *z, *p, *q, *dinv, *part, *scal;
  CgFlags* flags;
  uint8_t* fr;
};

static constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// bytes of the CG work buffer for n_dof DOFs
static constexpr size_t cg_bytes(size_t nd) {
  return 5 * align256(nd * 8) + align256(2 * kUpdBlocks * 8) + align256(kNumScalars * 8) + align256(sizeof(CgFlags)) +
         align256(nd > 0 ? nd : 1);
}

// lay the work vectors out over a buffer of cg_bytes(nd) bytes
static void cg_carve(void* base, size_t nd, CgBuf* B) {
  const size_t vec = align256(nd * 8);
  char* w = static_cast<char*>(base);
  B->r = reinterpret_cast<double*>(w);
  B->z = reinterpret_cast<double*>(w + vec);
  B->p = reinterpret_cast<double*>(w + 2 * vec);
  B->q = reinterpret_cast<double*>(w + 3 * vec);
  B->dinv = reinterpret_cast<double*>(w + 4 * vec);
  w += 5 * vec;
  B->part = reinterpret_cast<double*>(w);  // dot products: kDotBlocks partials; update: 2 x kUpdBlocks
  w += align256(2 * kUpdBlocks * 8);
  B->scal = reinterpret_cast<double*>(w);
  w += align256(kNumScalars * 8);
  B->flags = reinterpret_cast<CgFlags*>(w);
  w += align256(sizeof(CgFlags));
  B->fr = reinterpret_cast<uint8_t*>(w);
}

static int32_t cg_buffers(mpm_mesh* m, hipStream_t st, CgBuf* B) {
  const size_t nd = size_t(3 * m->n_node);
  const size_t need = cg_bytes(nd);
  if (m->cg_bytes < need || !m->d_cg) {
    MPM_HIP(hipStreamSynchronize(st));
    if (m->d_cg) MPM_HIP(hipFree(m->d_cg));
    m->d_cg = nullptr;
    m->cg_bytes = 0;
    const hipError_t e = hipMalloc(&m->d_cg, need);
    if (e != hipSuccess) {
      m->d_cg = nullptr;
      return hip_fail(e, "mpm_solve_cg: work buffer");
    }
    m->cg_bytes = need;
  }
  cg_carve(m->d_cg, nd, B);
  return MPM_OK;
}

// Where the host reads the convergence flags: pinned memory and an event kept with the mesh
// (allocated on the first call; the host spins on the event), or a caller-side host buffer
// read after a stream synchronisation (no allocation).
struct CgHost {
  void* buf;          // sizeof(CgFlags) + 8 kNumScalars bytes
  hipEvent_t ev;      // null: synchronise the stream instead
};

static int32_t cg_wait(const CgHost& H, hipStream_t st) {
  if (!H.ev) {
    MPM_HIP(hipStreamSynchronize(st));
    return MPM_OK;
  }
  MPM_HIP(hipEventRecord(H.ev, st));
  hipError_t q;
  while ((q = hipEventQuery(H.ev)) == hipErrorNotReady) {
  }
  if (q != hipSuccess) return hip_fail(q, "mpm_solve_cg");
  return MPM_OK;
}

template <typename T>
static int32_t solve_cg_on(mpm_mesh* m, const CgBuf& B, const CgHost& H, const void* K, const uint8_t* dir,
                           const double* b, double* x, double rtol, int max_iter, int* iters, double* relres,
                           hipStream_t st) {
  const int64_t nd = 3 * m->n_node;
  const unsigned gv = unsigned(std::max<int64_t>(1, std::min<int64_t>(kUpdBlocks, (nd + 255) / 256)));
  hipLaunchKernelGGL(k_cg_init<T>, dim3(unsigned((nd + 255) / 256)), dim3(256), 0, st, m->d_row_ptr, m->d_col,
                     static_cast<const T*>(K), dir, b, nd, B.fr, B.dinv, x, B.r, B.z, B.p);
  launch_dot(B.r, B.z, nd, B.part, B.scal, kRZ, nullptr, st);
  launch_dot(B.r, B.r, nd, B.part, B.scal, kBB, nullptr, st);
  launch_dot(B.r, B.r, nd, B.part, B.scal, kRR, nullptr, st);
  hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(1), 0, st, B.scal, B.flags);
  const double rtol2 = rtol * rtol;
  constexpr int kCheck = 16;  // iterations between host reads of the flags
  for (int it = 0; it < max_iter; it += kCheck) {
    const int nk = std::min(kCheck, max_iter - it);
    for (int k = 0; k < nk; ++k) {
      launch_spmv<T>(m, K, B.p, B.q, B.fr, &B.flags->done, st);
      launch_dot(B.p, B.q, nd, B.part, B.scal, kPQ, B.flags, st);
      hipLaunchKernelGGL(k_cg_update, dim3(gv), dim3(256), 0, st, x, B.r, B.z, B.p, B.q, B.dinv, nd, B.scal,
                         B.part, B.flags);
      hipLaunchKernelGGL(k_cg_step, dim3(1), dim3(256), 0, st, B.scal, B.part, int(gv), B.flags, rtol2, max_iter);
      hipLaunchKernelGGL(k_cg_dir, dim3(gv), dim3(256), 0, st, B.p, B.z, nd, B.scal, B.flags);
    }
    MPM_HIP(hipGetLastError());
    MPM_HIP(hipMemcpyAsync(H.buf, B.flags, sizeof(CgFlags), hipMemcpyDeviceToHost, st));
    MPM_HIP(hipMemcpyAsync(static_cast<char*>(H.buf) + sizeof(CgFlags), B.scal, 8 * kNumScalars,
                           hipMemcpyDeviceToHost, st));
    const int32_t rc = cg_wait(H, st);
    if (rc) return rc;
    const CgFlags* f = static_cast<const CgFlags*>(H.buf);
    if (f->done) break;
  }
  if (max_iter == 0) {  // no iteration ran: read the start values once
    MPM_HIP(hipMemcpyAsync(H.buf, B.flags, sizeof(CgFlags), hipMemcpyDeviceToHost, st));
    MPM_HIP(hipMemcpyAsync(static_cast<char*>(H.buf) + sizeof(CgFlags), B.scal, 8 * kNumScalars,
                           hipMemcpyDeviceToHost, st));
    const int32_t rc = cg_wait(H, st);
    if (rc) return rc;
  }
  const CgFlags* f = static_cast<const CgFlags*>(H.buf);
  const double* sc = reinterpret_cast<const double*>(static_cast<const char*>(H.buf) + sizeof(CgFlags));
  if (iters) *iters = f->iters;
  if (relres) *relres = sc[kBB] > 0.0 ? std::sqrt(std::max(0.0, sc[kRR]) / sc[kBB]) : 0.0;
  if (f->iters == 0 && sc[kBB] > 0.0 && relres) *relres = 1.0;
  return MPM_OK;
}

template <typename T>
static int32_t solve_cg(mpm_mesh* m, const void* K, const uint8_t* dir, const double* b, double* x, double rtol,
                        int max_iter, int* iters, double* relres, hipStream_t st) {
  CgBuf B;
  int32_t rc = cg_buffers(m, st, &B);
  if (rc) return rc;
  if (!m->h_cg) MPM_HIP(hipHostMalloc((void**)&m->h_cg, sizeof(CgFlags) + 8 * kNumScalars, hipHostMallocDefault));
  if (!m->cg_ev) MPM_HIP(hipEventCreateWithFlags(&m->cg_ev, hipEventDisableTiming));
  return solve_cg_on<T>(m, B, CgHost{m->h_cg, m->cg_ev}, K, dir, b, x, rtol, max_iter, iters, relres, st);
}

// ------------------------------------------------------------------ CG without allocation
// The same solve for callers that cannot allocate device memory: the work vectors live in
// `scratch`, a file-scope device array of fixed size that every GPU the library runs on holds
// for the life of the process (one copy per device, at its own address). Its device address
// is looked up once per device with hipGetSymbolAddress on the call that first runs there, and
// only that address is handed to kernels and copies. The host reads the flags into a local
// buffer after a stream synchronisation. Every call on a GPU shares that GPU's copy: calls that
// overlap on one device race.
constexpr size_t kCgScratchBytes = size_t(64) << 20;
static_assert(cg_bytes(MPM_CG_NOALLOC_MAX_DOFS) <= kCgScratchBytes &&
                  cg_bytes(MPM_CG_NOALLOC_MAX_DOFS + 1) > kCgScratchBytes,
              "MPM_CG_NOALLOC_MAX_DOFS must be the largest n_dof whose work buffer fits the static array");
static __device__ __align__(256) unsigned char scratch[kCgScratchBytes];

constexpr int kMaxScratchDevices = 64;
static void* g_scratch_ptr[kMaxScratchDevices];
static std::mutex g_scratch_mu;

static int32_t scratch_for_current_device(void** out) {
  int dev = -1;
  MPM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices) {
    set_error(MPM_EARG, "mpm_solve_cg_noalloc: device index beyond the supported range");
    return MPM_EARG;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                               "mpm_solve_cg_noalloc: address of the static workspace");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MPM_OK;
}

template <typename T>
static int32_t solve_cg_noalloc(mpm_mesh* m, const void* K, const uint8_t* dir, const double* b, double* x,
                                double rtol, int max_iter, int* iters, double* relres, hipStream_t st) {
  void* base = nullptr;
  int32_t rc = scratch_for_current_device(&base);
  if (rc) return rc;
  CgBuf B;
  cg_carve(base, size_t(3 * m->n_node), &B);
  alignas(8) unsigned char host[sizeof(CgFlags) + 8 * kNumScalars];
  return solve_cg_on<T>(m, B, CgHost{host, nullptr}, K, dir, b, x, rtol, max_iter, iters, relres, st);
}

// ------------------------------------------------------------------ GMRES
// Restarted GMRES with the Jacobi preconditioner applied on the right (the solver the paper
// names for its possibly non-symmetric systems, with the diagonal preconditioner it proposes
// as future work), over the same free DOFs as CG: the residual it minimises is the true one,
// ||b_f - K_ff x_f||. Each Arnoldi step: z = M^-1 v_j, w = K z, two passes of classical
// Gram-Schmidt against v_0..v_j (one block of dot products and one update each, instead of
// j + 1 sequential reductions), then the new column of the Hessenberg matrix is reduced by the
// Givens rotations so far and a new one, whose last entry is the residual norm. At the end of a
// cycle the triangular system gives y and x += M^-1 V y; the true residual is recomputed at
// every restart. All control stays on the device (flags read by every kernel); the host reads
// the state once per cycle.
constexpr int kMaxRestart = 64;
constexpr int kHStride = kMaxRestart + 1;

struct GmState {
  int skip;   // the Arnoldi steps of this cycle are over (or the solve has stopped)
  int stop;   // the solve is over: converged, step budget spent, or breakdown
  int k;      // Arnoldi columns of the current cycle
  int iters;  // Arnoldi steps in all
  int brk;    // the Hessenberg matrix became singular: stop after this cycle's correction
  int pad;
  double bnorm, beta, hinv;
  double H[kHStride * kMaxRestart];  // column j at j * kHStride (rotated into triangular form)
  double cs[kMaxRestart], sn[kMaxRestart], g[kHStride], y[kMaxRestart], hc[kHStride];
};
constexpr size_t kGmHead = offsetof(GmState, H);  // the part the host reads

__global__ void k_gm_reset(GmState* s) {
  s->skip = s->stop = s->k = s->iters = s->brk = 0;
  s->bnorm = s->beta = s->hinv = 0.0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gm_init(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                                 const T* __restrict__ K, const uint8_t* __restrict__ dir,
                                                 int64_t ndof, uint8_t* __restrict__ fr, double* __restrict__ dinv,
                                                 double* __restrict__ x) {
  const int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (d >= ndof) return;
  const double diag = row_diag(row_ptr, col, K, d);
  const bool f = (!dir || !dir[d]) && row_ptr[d + 1] > row_ptr[d] && diag > 0.0;
  fr[d] = f ? 1 : 0;
  dinv[d] = f ? 1.0 / diag : 0.0;
  x[d] = 0.0;
}

// v0 = b - K x on the free DOFs (w = K x), zero elsewhere; block partial sums of v0 . v0
__global__ __launch_bounds__(256) void k_gm_resid(const double* __restrict__ b, const double* __restrict__ w,
                                                  const uint8_t* __restrict__ fr, double* __restrict__ v0,
                                                  int64_t ndof, double* __restrict__ part, const GmState* s) {
  __shared__ double sh[256];
  if (s->stop) return;
  double acc = 0.0;
  for (int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x; d < ndof; d += int64_t(gridDim.x) * 256) {
    const double r = fr[d] ? b[d] - w[d] : 0.0;
    v0[d] = r;
    acc += r * r;
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// start of a cycle: beta = ||v0||; the first call also fixes ||b_f||; stop on convergence,
// spent budget or an earlier breakdown
__global__ __launch_bounds__(256) void k_gm_begin(const double* __restrict__ part, int nb, GmState* s, double rtol,
                                                  int max_iter, int first) {
  __shared__ double sh[256];
  if (s->stop) return;
  double acc = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) acc += part[k];
  const double bb = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    const double beta = sqrt(bb);
    if (first) s->bnorm = beta;
    s->beta = beta;
    s->k = 0;
    if (s->brk || !(beta > rtol * s->bnorm) || s->iters >= max_iter) {
      s->stop = 1;
      s->skip = 1;
    } else {
      s->skip = 0;
      s->g[0] = beta;
      s->hinv = 1.0 / beta;
    }
  }
}

// dst = hinv src (v0 in place, or v_{j+1} = w / h_{j+1,j}) and z = M^-1 dst, the vector the
// next Arnoldi step multiplies by K
__global__ __launch_bounds__(256) void k_gm_scale(const double* src, double* dst, const double* __restrict__ dinv,
                                                  double* __restrict__ z, int64_t ndof, const GmState* s) {
  if (s->skip) return;
  const double h = s->hinv;
  for (int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x; d < ndof; d += int64_t(gridDim.x) * 256) {
    const double v = h * src[d];
    dst[d] = v;
    z[d] = dinv[d] * v;
  }
}

// partial sums of v_i . w, i = blockIdx.y (0..j), in a fixed order
__global__ __launch_bounds__(256) void k_gm_dots(const double* __restrict__ V, int64_t vs,
                                                 const double* __restrict__ w, int64_t ndof,
                                                 double* __restrict__ part, const GmState* s) {
  __shared__ double sh[256];
  if (s->skip) return;
  const double* v = V + int64_t(blockIdx.y) * vs;
  double acc = 0.0;
  for (int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x; d < ndof; d += int64_t(gridDim.x) * 256)
    acc += v[d] * w[d];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[int64_t(blockIdx.y) * kDotBlocks + blockIdx.x] = t;
}

// hc[i] = sum of the partials of v_i . w (one block per i); H[i][j] = hc[i] in the first pass,
// += hc[i] in the second
__global__ __launch_bounds__(256) void k_gm_dots_final(const double* __restrict__ part, int nb, GmState* s, int j,
                                                       int second) {
  __shared__ double sh[256];
  if (s->skip) return;
  const int i = blockIdx.x;
  double acc = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) acc += part[int64_t(i) * kDotBlocks + k];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    s->hc[i] = t;
    double* h = s->H + int64_t(j) * kHStride;
    h[i] = second ? h[i] + t : t;
  }
}

// w -= sum_i hc[i] v_i (i = 0..j); with want_norm also the block partial sums of w . w
__global__ __launch_bounds__(256) void k_gm_orth(const double* __restrict__ V, int64_t vs, double* __restrict__ w,
                                                 int64_t ndof, int j, double* __restrict__ part, int want_norm,
                                                 const GmState* s) {
  __shared__ double sh[256];
  if (s->skip) return;
  double acc = 0.0;
  for (int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x; d < ndof; d += int64_t(gridDim.x) * 256) {
    double wd = w[d];
    for (int i = 0; i <= j; ++i) wd -= s->hc[i] * V[int64_t(i) * vs + d];
    w[d] = wd;
    acc += wd * wd;
  }
  if (want_norm) {
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
  }
}

// h_{j+1,j} = ||w||; earlier rotations on column j, a new rotation that zeroes h_{j+1,j}, the
// rotated right-hand side g and its last entry |g_{j+1}| = the residual norm of the step
__global__ __launch_bounds__(256) void k_gm_rotate(const double* __restrict__ part, int nb, GmState* s, int j,
                                                   double rtol, int max_iter) {
  __shared__ double sh[256];
  if (s->skip) return;
  double acc = 0.0;
  for (int k = threadIdx.x; k < nb; k += 256) acc += part[k];
  const double ww = block_sum(acc, sh);
  if (threadIdx.x != 0) return;
  const double hn = sqrt(ww);
  double* h = s->H + int64_t(j) * kHStride;
  for (int i = 0; i < j; ++i) {
    const double a = h[i], c = h[i + 1];
    h[i] = s->cs[i] * a + s->sn[i] * c;
    h[i + 1] = -s->sn[i] * a + s->cs[i] * c;
  }
  const double r = hypot(h[j], hn);
  s->iters += 1;
  if (!(r > 0.0)) {  // singular Hessenberg matrix (K M^-1 singular on the Krylov space)
    s->brk = 1;
    s->skip = 1;
    return;  // k stays j: the correction uses the columns before this one
  }
  const double c = h[j] / r, sn = hn / r;
  s->cs[j] = c;
  s->sn[j] = sn;
  h[j] = r;
  h[j + 1] = 0.0;
  const double gj = s->g[j];
  s->g[j + 1] = -sn * gj;
  s->g[j] = c * gj;
  s->k = j + 1;
  s->hinv = hn > 0.0 ? 1.0 / hn : 0.0;
  if (!(fabs(s->g[j + 1]) > rtol * s->bnorm) || s->iters >= max_iter || !(hn > 0.0)) s->skip = 1;
}

// y = R^-1 g over the k columns of the cycle (back substitution, one thread)
__global__ void k_gm_solve(GmState* s) {
  if (s->stop) return;
  const int k = s->k;
  for (int i = k - 1; i >= 0; --i) {
    double t = s->g[i];
    for (int l = i + 1; l < k; ++l) t -= s->H[int64_t(l) * kHStride + i] * s->y[l];
    s->y[i] = t / s->H[int64_t(i) * kHStride + i];
  }
}

// x += M^-1 sum_i y_i v_i (i < k)
__global__ __launch_bounds__(256) void k_gm_xupd(const double* __restrict__ V, int64_t vs,
                                                 const double* __restrict__ dinv, double* __restrict__ x,
                                                 int64_t ndof, const GmState* s) {
  if (s->stop) return;
  const int k = s->k;
  for (int64_t d = int64_t(blockIdx.x) * 256 + threadIdx.x; d < ndof; d += int64_t(gridDim.x) * 256) {
    double t = 0.0;
    for (int i = 0; i < k; ++i) t += s->y[i] * V[int64_t(i) * vs + d];
    x[d] += dinv[d] * t;
  }
}

// work buffer of GMRES kept with the mesh: V [(restart + 1) n_dof], w, z, dinv [n_dof],
// partial sums, the state and the free mask
struct GmBuf {
  double *V, *w, *z, *dinv, *part;
  GmState* s;
  uint8_t* fr;
  int64_t vs;  // stride of the basis vectors (doubles)
};

static int32_t gm_buffers(mpm_mesh* m, int restart, hipStream_t st, GmBuf* B) {
  const size_t nd = size_t(3 * m->n_node);
  const size_t vec = align256(nd * 8);
  const size_t npart = std::max<size_t>(size_t(kDotBlocks) * kHStride, kUpdBlocks);
  const size_t need = size_t(restart + 4) * vec + align256(npart * 8) + align256(sizeof(GmState)) +
                      align256(std::max<size_t>(1, nd));
  if (m->gm_bytes < need || !m->d_gm) {
    MPM_HIP(hipStreamSynchronize(st));
    if (m->d_gm) MPM_HIP(hipFree(m->d_gm));
    m->d_gm = nullptr;
    m->gm_bytes = 0;
    const hipError_t e = hipMalloc(&m->d_gm, need);
    if (e != hipSuccess) {
      m->d_gm = nullptr;
      return hip_fail(e, "mpm_solve_gmres: work buffer");
    }
    m->gm_bytes = need;
  }
  char* w = static_cast<char*>(m->d_gm);
  B->vs = int64_t(vec / 8);
  B->V = reinterpret_cast<double*>(w);
  w += size_t(restart + 1) * vec;
  B->w = reinterpret_cast<double*>(w);
  B->z = reinterpret_cast<double*>(w + vec);
  B->dinv = reinterpret_cast<double*>(w + 2 * vec);
  w += 3 * vec;
  B->part = reinterpret_cast<double*>(w);
  w += align256(npart * 8);
  B->s = reinterpret_cast<GmState*>(w);
  w += align256(sizeof(GmState));
  B->fr = reinterpret_cast<uint8_t*>(w);
  return MPM_OK;
}

template <typename T>
static int32_t solve_gmres(mpm_mesh* m, const void* K, const uint8_t* dir, const double* b, double* x, double rtol,
                           int restart, int max_iter, int* iters, double* relres, hipStream_t st) {
  GmBuf B;
  int32_t rc = gm_buffers(m, restart, st, &B);
  if (rc) return rc;
  const int64_t nd = 3 * m->n_node;
  const unsigned gv = unsigned(std::max<int64_t>(1, std::min<int64_t>(kUpdBlocks, (nd + 255) / 256)));
  const int nb = int(std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, (nd + 255) / 256)));
  GmState* S = B.s;
  hipLaunchKernelGGL(k_gm_reset, dim3(1), dim3(1), 0, st, S);
  hipLaunchKernelGGL(k_gm_init<T>, dim3(unsigned((nd + 255) / 256)), dim3(256), 0, st, m->d_row_ptr, m->d_col,
                     static_cast<const T*>(K), dir, nd, B.fr, B.dinv, x);
  // residual of the current x, its norm, v0; the cycle's flags
  auto begin = [&](int first) {
    launch_spmv<T>(m, K, x, B.w, B.fr, &S->stop, st);
    hipLaunchKernelGGL(k_gm_resid, dim3(gv), dim3(256), 0, st, b, B.w, B.fr, B.V, nd, B.part, S);
    hipLaunchKernelGGL(k_gm_begin, dim3(1), dim3(256), 0, st, B.part, int(gv), S, rtol, max_iter, first);
    hipLaunchKernelGGL(k_gm_scale, dim3(gv), dim3(256), 0, st, B.V, B.V, B.dinv, B.z, nd, S);
  };
  begin(1);
  if (!m->h_cg) MPM_HIP(hipHostMalloc((void**)&m->h_cg, sizeof(CgFlags) + 8 * kNumScalars, hipHostMallocDefault));
  if (!m->cg_ev) MPM_HIP(hipEventCreateWithFlags(&m->cg_ev, hipEventDisableTiming));
  static_assert(kGmHead <= sizeof(CgFlags) + 8 * kNumScalars, "pinned copy of the GMRES state too small");
  for (;;) {
    MPM_HIP(hipGetLastError());
    MPM_HIP(hipMemcpyAsync(m->h_cg, S, kGmHead, hipMemcpyDeviceToHost, st));
    MPM_HIP(hipEventRecord(m->cg_ev, st));
    hipError_t q;
    while ((q = hipEventQuery(m->cg_ev)) == hipErrorNotReady) {
    }
    if (q != hipSuccess) return hip_fail(q, "mpm_solve_gmres");
    if (static_cast<const GmState*>(m->h_cg)->stop) break;
    for (int j = 0; j < restart; ++j) {
      launch_spmv<T>(m, K, B.z, B.w, B.fr, &S->skip, st);  // z = M^-1 v_j, left by the previous scale
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_gm_dots, dim3(unsigned(nb), unsigned(j + 1)), dim3(256), 0, st, B.V, B.vs, B.w, nd,
                           B.part, S);
        hipLaunchKernelGGL(k_gm_dots_final, dim3(unsigned(j + 1)), dim3(256), 0, st, B.part, nb, S, j, pass);
        hipLaunchKernelGGL(k_gm_orth, dim3(gv), dim3(256), 0, st, B.V, B.vs, B.w, nd, j, B.part, pass, S);
      }
      hipLaunchKernelGGL(k_gm_rotate, dim3(1), dim3(256), 0, st, B.part, int(gv), S, j, rtol, max_iter);
      hipLaunchKernelGGL(k_gm_scale, dim3(gv), dim3(256), 0, st, B.w, B.V + int64_t(j + 1) * B.vs, B.dinv, B.z,
                         nd, S);
    }
    hipLaunchKernelGGL(k_gm_solve, dim3(1), dim3(1), 0, st, S);
    hipLaunchKernelGGL(k_gm_xupd, dim3(gv), dim3(256), 0, st, B.V, B.vs, B.dinv, x, nd, S);
    begin(0);
  }
  const GmState* h = static_cast<const GmState*>(m->h_cg);
  if (iters) *iters = h->iters;
  if (relres) *relres = h->bnorm > 0.0 ? h->beta / h->bnorm : 0.0;
  return MPM_OK;
}

}  // namespace mpm

using namespace mpm;

extern "C" int32_t mpm_spmv(const mpm_mesh_t* m, int32_t precision, const void* K_vals, const double* x, double* y,
                            void* stream) {
  if (!m || (!K_vals && m->nnz) || !x || !y || (precision != MPM_F64 && precision != MPM_F32K)) {
    set_error(MPM_EARG, "mpm_spmv: null argument or bad precision");
    return MPM_EARG;
  }
  hipStream_t st = (hipStream_t)stream;
  if (m->n_node) {
    if (precision == MPM_F64) launch_spmv<double>(m, K_vals, x, y, nullptr, nullptr, st);
    else launch_spmv<float>(m, K_vals, x, y, nullptr, nullptr, st);
  }
  MPM_HIP(hipGetLastError());
  return MPM_OK;
}

extern "C" int32_t mpm_solve_cg(const mpm_mesh_t* m, int32_t precision, const void* K_vals,
                                const uint8_t* dirichlet, const double* b, double* x, double rtol, int32_t max_iter,
                                int32_t* iters, double* relres, void* stream) {
  if (!m || (!K_vals && m->nnz) || !b || !x || (precision != MPM_F64 && precision != MPM_F32K) || !(rtol >= 0.0) ||
      max_iter < 0) {
    set_error(MPM_EARG, "mpm_solve_cg: null argument, bad precision, negative tolerance or iteration limit");
    return MPM_EARG;
  }
  mpm_mesh* mm = const_cast<mpm_mesh*>(m);
  hipStream_t st = (hipStream_t)stream;
  int it = 0;
  double rr = 0.0;
  int32_t rc = MPM_OK;
  if (m->n_node == 0) {
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    return MPM_OK;
  }
  if (precision == MPM_F64) rc = solve_cg<double>(mm, K_vals, dirichlet, b, x, rtol, max_iter, &it, &rr, st);
  else rc = solve_cg<float>(mm, K_vals, dirichlet, b, x, rtol, max_iter, &it, &rr, st);
  if (iters) *iters = it;
  if (relres) *relres = rr;
  return rc;
}

extern "C" int32_t mpm_solve_cg_noalloc(const mpm_mesh_t* m, int32_t precision, const void* K_vals,
                                        const uint8_t* dirichlet, const double* b, double* x, double rtol,
                                        int32_t max_iter, int32_t* iters, double* relres, void* stream) {
  if (!m || (!K_vals && m->nnz) || !b || !x || (precision != MPM_F64 && precision != MPM_F32K) || !(rtol >= 0.0) ||
      max_iter < 0) {
    set_error(MPM_EARG, "mpm_solve_cg_noalloc: null argument, bad precision, negative tolerance or iteration limit");
    return MPM_EARG;
  }
  if (cg_bytes(size_t(3 * m->n_node)) > kCgScratchBytes) {
    char msg[200];
    snprintf(msg, sizeof msg,
             "mpm_solve_cg_noalloc: %lld DOFs need %zu bytes of work space, beyond the static %zu (at most %lld DOFs)",
             (long long)(3 * m->n_node), cg_bytes(size_t(3 * m->n_node)), kCgScratchBytes,
             (long long)MPM_CG_NOALLOC_MAX_DOFS);
    set_error(MPM_EARG, msg);
    return MPM_EARG;
  }
  mpm_mesh* mm = const_cast<mpm_mesh*>(m);
  hipStream_t st = (hipStream_t)stream;
  int it = 0;
  double rr = 0.0;
  int32_t rc = MPM_OK;
  if (m->n_node == 0) {
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    return MPM_OK;
  }
  if (precision == MPM_F64) rc = solve_cg_noalloc<double>(mm, K_vals, dirichlet, b, x, rtol, max_iter, &it, &rr, st);
  else rc = solve_cg_noalloc<float>(mm, K_vals, dirichlet, b, x, rtol, max_iter, &it, &rr, st);
  if (iters) *iters = it;
  if (relres) *relres = rr;
  return rc;
}

extern "C" int32_t mpm_solve_gmres(const mpm_mesh_t* m, int32_t precision, const void* K_vals,
                                   const uint8_t* dirichlet, const double* b, double* x, double rtol,
                                   int32_t restart, int32_t max_iter, int32_t* iters, double* relres,
                                   void* stream) {
  if (!m || (!K_vals && m->nnz) || !b || !x || (precision != MPM_F64 && precision != MPM_F32K) || !(rtol >= 0.0) ||
      max_iter < 0 || restart < 1 || restart > kMaxRestart) {
    set_error(MPM_EARG, "mpm_solve_gmres: null argument, bad precision, negative tolerance or iteration limit, "
                        "or restart outside 1..64");
    return MPM_EARG;
  }
  mpm_mesh* mm = const_cast<mpm_mesh*>(m);
  hipStream_t st = (hipStream_t)stream;
  int it = 0;
  double rr = 0.0;
  int32_t rc = MPM_OK;
  if (m->n_node == 0) {
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    return MPM_OK;
  }
  if (precision == MPM_F64) rc = solve_gmres<double>(mm, K_vals, dirichlet, b, x, rtol, restart, max_iter, &it, &rr, st);
  else rc = solve_gmres<float>(mm, K_vals, dirichlet, b, x, rtol, restart, max_iter, &it, &rr, st);
  if (iters) *iters = it;
  if (relres) *relres = rr;
  return rc;
}
