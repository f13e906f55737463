// Internal definitions of the gfx950 octree GIMP assembly library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mpm_gimp.h"

namespace mpm {

// ------------------------------------------------------------------ errors
void set_error(int32_t code, const std::string& msg, int64_t index = -1);
int32_t hip_fail(hipError_t e, const char* what);

#define MPM_HIP(call)                                       \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return ::mpm::hip_fail(e_, #call); \
  } while (0)

// device error word: [0] first error code (0 none), [1..2] first offending index (int64)
struct DevErr {
  int32_t code;
  int32_t pad;
  unsigned long long index;
};

// ------------------------------------------------------------------ Morton keys
// bits b of x, y, z go to bits 3b, 3b+1, 3b+2 (21 bits per axis)
__host__ __device__ inline uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}
__host__ __device__ inline uint64_t morton(uint64_t x, uint64_t y, uint64_t z) {
  return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}
// inverse of spread3: bits 3b of v back to bit b
__host__ __device__ inline uint64_t compact3(uint64_t v) {
  v &= 0x1249249249249249ull;
  v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
  v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
  v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
  v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
  v = (v ^ (v >> 32)) & 0x1fffffull;
  return v;
}

constexpr int kMaxPointLeaves = 8; // leaves a point domain may overlap (one boundary per axis)
constexpr int kGenRec = 74;        // doubles per straddling point: the general path's tangent record
constexpr int kNarrowRow = 128;    // rows of at most this many block columns run with less LDS
constexpr int kGatherNarrow = 64;  // the row gather's split: rows of at most this many block columns

// per-leaf constraint code: bits 0..7 hanging vertices, bits 8..10 child index in the parent
__host__ __device__ inline int code_hmask(int32_t code) { return code & 0xff; }
__host__ __device__ inline int code_child(int32_t code) { return (code >> 8) & 7; }

// ------------------------------------------------------------------ mesh handle
}  // namespace mpm

struct mpm_mesh {
  mpm_refine_t crit;
  int nx, ny, nz;
  double hmin;
  int64_t n_leaf = 0, n_node = 0, n_hang = 0, n_point = 0, nnz = 0, n_straddle = 0, n_active_rows = 0;
  int32_t max_support = 0;
  int leaf_bits = 1;            // bits needed for a leaf rank
  int32_t* d_cellmap = nullptr; // nx*ny*nz leaf ranks of the finest cells (x fastest), if not too large
  // device arrays (owned)
  int32_t* d_leaf = nullptr;        // n_leaf x 4
  uint64_t* d_leaf_key = nullptr;   // n_leaf
  int32_t* d_cell_nodes = nullptr;  // n_leaf x 8
  int32_t* d_cell_code = nullptr;   // n_leaf
  double* d_cell_cmat = nullptr;    // n_leaf x 64
  int32_t* d_node_ijk = nullptr;
  int32_t* d_hang_ijk = nullptr;
  int32_t* d_hang_sup = nullptr;
  double* d_hang_w = nullptr;
  int32_t* d_hang_owner = nullptr;
  int64_t* d_perm = nullptr;        // n_point
  int32_t* d_pleaf = nullptr;       // n_point (sorted)
  uint8_t* d_pnleaf = nullptr;      // n_point (sorted)
  int64_t* d_row_ptr = nullptr;
  int32_t* d_col = nullptr;
  // segments: maximal runs of one leaf inside a 64-point wavefront of the sorted points
  int64_t n_wave = 0, n_seg = 0, n_con = 0;
  int32_t max_deg = 0;              // largest number of coupled nodes of one node row
  int32_t* d_wave_seg = nullptr;    // n_wave + 1: first segment of each wavefront
  int32_t* d_leaf_seg0 = nullptr;   // n_leaf: first segment of the leaf
  int32_t* d_leaf_nseg = nullptr;   // n_leaf: number of segments of the leaf
  // node -> contributions (segment, slot) of its (populated leaf, slot) incidences, in
  // ascending leaf then segment order
  int32_t* d_con_off = nullptr;     // n_node + 1
  int32_t* d_con_seg = nullptr;     // segment * 8 + slot
  int32_t* d_con_bp = nullptr;      // offset of the slot's 8 block columns in d_bpos
  int16_t* d_bpos = nullptr;        // n_leaf x 64: block column of slot b's node in the row of slot a's node
  // records 0..n_seg-1 are wavefront segments; after them one record per heavily populated
  // leaf (its segments summed) and the partial sums of those leaves' chunks
  int64_t n_rec = 0;
  void* d_segK = nullptr;           // n_rec x 36 upper-triangle 3x3 slot blocks (a <= b; b outer, a inner), double or float
  double* d_segF = nullptr;         // n_rec x 24 reduced nodal forces
  void* d_segM = nullptr;           // n_rec x 36 inertia coefficients sum (2 m / dt^2) S_a S_b (a <= b), double or float
  // record reductions (first record, count, output record), run in two stages
  int64_t n_red1 = 0, n_red2 = 0;
  int32_t* d_red1 = nullptr;        // n_red1 x 3: chunks of a heavy leaf's segments
  int32_t* d_red2 = nullptr;        // n_red2 x 3: chunk records of a heavy leaf
  int64_t* d_strad = nullptr;       // n_straddle sorted positions
  int32_t* d_strad_leaf = nullptr;  // n_straddle x 8 overlapped leaves (-1 pad)
  double* d_grec = nullptr;         // n_straddle x kGenRec: per-point tangent records of the general path
  // rows that straddling points reach: the nodes in their supports and, per node, the
  // straddling points (indices into d_strad) whose support holds it, in ascending order
  int64_t n_snode = 0;
  int32_t* d_snode = nullptr;       // n_snode
  // the same rows in launch order: those of at most kNarrowRow block columns first (their
  // kernel takes less LDS), then the rest; n_snode_narrow of the first kind
  int32_t* d_srow = nullptr;        // n_snode indices into d_snode
  int64_t n_snode_narrow = 0;
  // when some row has more than kGatherNarrow block columns: the nodes in the row gather's launch
  // order, those of at most kGatherNarrow columns first (their launch takes less LDS), each part
  // ascending; n_gnarrow of the first kind (null when every row is narrow)
  int32_t* d_gorder = nullptr;
  int64_t n_gnarrow = 0;
  // the straddling points are grouped by their number of leaves: 2, 3-4 and 5-8 (each group
  // in point order); group g holds the indices strad_grp[g] .. strad_grp[g + 1]
  int64_t strad_grp[4] = {0, 0, 0, 0};
  // the points whose domain lies in one leaf, in sorted order (n_fast of them): the fast path's
  // wavefronts and segments run over this list; null when every point is such a point
  int64_t* d_fidx = nullptr;
  int64_t n_fast = 0;
  // a second stream (default priority) on which the straddling points' kernels run beside the
  // fast path, and the events that fork it from and join it to the caller's stream; created
  // with the mesh when some domain straddles
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  int64_t* d_sinc_off = nullptr;    // n_snode + 1
  int32_t* d_sinc = nullptr;
  // support of each straddling point in slot order (the union of its leaves' slot nodes in
  // ascending node order): slots d_sup_off[t] .. d_sup_off[t + 1] of the arrays below
  int64_t* d_sup_off = nullptr;     // n_straddle + 1
  int32_t* d_sup_id = nullptr;      // node of each slot
  uint32_t* d_sup_src = nullptr;    // per slot: bit q (0..7) = leaf q of the point holds the node,
                                    // bits 8 + 3q .. 10 + 3q = its vertex in that leaf
  double* d_sup_g = nullptr;        // per slot, written by each assembly: S and the spatial gradient
  // per CSR block (index row_ptr[3 a] / 9 + j) of a row a reached by straddling points whose
  // column node c is above a: the block column of a in the row of c
  int32_t* d_tpos = nullptr;
  mpm::DevErr* d_err = nullptr;
  mpm::DevErr* h_err = nullptr;     // pinned host copy of the error word
  hipEvent_t err_ev = nullptr;      // marks the error-word copy (polled, no blocking sync)
  double* d_partial = nullptr;      // residual partial sums
  // work buffers of the point sort and of the state permutation, kept between calls (grown
  // on demand) so that the per-step calls allocate nothing
  void* d_scratch = nullptr;        // radix sort keys, values, per-tile counts
  size_t scratch_bytes = 0;
  void* d_stage = nullptr;          // record-major staging copy of permuted arrays
  size_t stage_bytes = 0;
  void* d_cg = nullptr;             // conjugate-gradient vectors, partial sums, scalars
  size_t cg_bytes = 0;
  void* d_gm = nullptr;             // GMRES basis, work vectors, partial sums, state
  size_t gm_bytes = 0;
  void* h_cg = nullptr;             // pinned host copy of the solver flags and scalars
  hipEvent_t cg_ev = nullptr;
  void* d_split = nullptr;          // GIMP split: per-block counts and their scan
  size_t split_bytes = 0;
  int64_t* h_word = nullptr;        // pinned host copy of one device word (counts)
  // ghost stabilisation (enabled by mpm_refine_t.ghost): faces, their node unions and jump
  // matrices; the nodes with ghost couplings and, per node, its (face * 16 + local index)
  // contributions in ascending face order; the block column of every face node pair in the
  // row of the first node; the per-leaf maximum Young's modulus (recomputed per call)
  int64_t n_gface = 0, n_gnode = 0;
  std::vector<int32_t> h_gface;     // n_gface x 8 face records (host copy)
  int32_t* d_gf_leaf = nullptr;     // n_gface x 2
  int32_t* d_gf_nodes = nullptr;    // n_gface x 16
  double* d_gf_G = nullptr;         // n_gface x 256
  double* d_gf_h = nullptr;         // n_gface: h_F / kappa
  double* d_gf_sc = nullptr;        // n_gface: (h_F / kappa) beta_F of the current call
  int16_t* d_gf_bpos = nullptr;     // n_gface x 256
  int32_t* d_gnode = nullptr;       // n_gnode
  int32_t* d_gcon_off = nullptr;    // n_gnode + 1
  int32_t* d_gcon = nullptr;
  double* d_gbeta = nullptr;        // n_leaf
  double* d_gsegmax = nullptr;      // n_seg: largest modulus of each point segment
  // kernel timing (measurement)
  bool timing = false;
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  double t_asm = 0, t_adj = 0, t_gat = 0;
  int64_t n_asm = 0, n_adj = 0, n_gat = 0;
};

namespace mpm {
struct LeafGeo;
LeafGeo make_geo(const mpm_mesh* m);
// ghost faces of the leaves flagged in pop (device, n_leaf): the mesh's face arrays
int32_t gpu_ghost_faces(mpm_mesh* m, const int32_t* pop, hipStream_t st);
// copies the device error word to the host; sets the message and returns its code
int32_t read_error(mpm_mesh* m, hipStream_t st, const char* what);
// grows a work buffer of the mesh to at least `bytes` (old contents dropped)
int32_t ensure_buffer(void** buf, size_t* have, size_t bytes, hipStream_t st, const char* what);
// leaves overlapped by each straddling point's domain (m->d_strad_leaf from m->d_strad)
int32_t strad_leaves(mpm_mesh* m, const double* dx, const double* dl, hipStream_t st);
// copies one device int64 to the host (ordered on st, waits for it)
int32_t read_word(mpm_mesh* m, const int64_t* d, int64_t* out, hipStream_t st, const char* what);

// Stable LSD radix sort of (keys, vals) by the low `bits` bits of the 32-bit keys, 8-bit
// digits over tiles of kRsTile elements; ktmp/vtmp: n-element work arrays, hist: 256 x
// (tiles) counts, tot: 256 totals. The result ends in whichever buffer the last pass wrote.
constexpr int kRsThreads = 256;
constexpr int kRsRounds = 16;
constexpr int kRsTile = kRsThreads * kRsRounds;
int32_t radix_sort(uint32_t* keys, uint32_t* vals, int64_t n, int bits, uint32_t* ktmp, uint32_t* vtmp, uint32_t* hist,
                   uint32_t* tot, hipStream_t st, uint32_t** kres, uint32_t** vres);

// Device work buffer owned by one construction step (freed on scope exit).
struct DevBuf {
  void* p = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  int32_t alloc(size_t bytes, const char* what) {
    if (p) (void)hipFree(p);
    p = nullptr;
    const hipError_t e = hipMalloc(&p, bytes ? bytes : 8);
    if (e != hipSuccess) {
      p = nullptr;
      return hip_fail(e, what);
    }
    return MPM_OK;
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// exclusive scan of n int32 counts into int64 offsets: out[i] = sum of in[0..i), out[n] =
// the total (out: n + 1 entries)
int32_t scan_counts(const int32_t* in, int64_t n, int64_t* out, hipStream_t st);
// sorts n 64-bit keys in place by their low `bits` bits (stable two-stage LSD radix)
int32_t sort_u64(uint64_t* keys, int64_t n, int bits, hipStream_t st);
// adds the ghost form's stiffness to K (precision's type) and K_G u to f on stream st
int32_t ghost_apply(const mpm_mesh* m, const mpm_state_t* s, const double* u, int32_t precision, void* K, double* f,
                    hipStream_t st);
}  // namespace mpm
