/*
 * mpm_gimp.h — C ABI of the MI355X (gfx950) octree GIMP material point assembly library.
 *
 * The library builds a 2:1-balanced octree around a rigid body, resolves hanging nodes by
 * constraints, orders material points by Morton key, and assembles — per Newton iteration —
 * the internal force vector f_int and the tangent K (fixed-pattern CSR) of the implicit
 * updated-Lagrangian GIMP material point method, plus the adjoint of f_int with respect to
 * the per-point material parameters. Paper references are to "An implicit octree-based
 * adaptive Material Point Method" (Bird, Coombs, Augarde, Pretti, O'Hare).
 *
 * Conventions
 *   - Every call returns an int32 status: MPM_OK (0) or a negative MPM_E* code. On error no
 *     output is guaranteed; mpm_last_error() gives a message and mpm_last_error_index() the
 *     first offending point (sorted position) or node, or -1.
 *   - Per-point arrays are structure-of-arrays, component-major: a[c * n + p].
 *   - Symmetric 3x3 tensors are stored as 6 components (xx, yy, zz, xy, yz, xz); general 3x3
 *     tensors as 9 components, row-major (xx, xy, xz, yx, ...).
 *   - DOF numbering: dof = 3 * node + c (c = 0,1,2 for x,y,z) over independent nodes in
 *     ascending Morton key of their integer lattice coordinates.
 *   - "device" pointers are HIP device memory (e.g. torch tensors on the GPU); they stay
 *     owned by the caller unless stated. All device work is ordered on the caller's
 *     hipStream_t `stream` (NULL = default stream). A mesh handle must not be used
 *     concurrently from two streams. On a mesh where some point domains overlap several
 *     leaves, the assembly and adjoint calls also run the kernels of those points on a
 *     second stream that the mesh owns (default priority), forked from `stream` by an event at
 *     the start of the call and joined to it by another before the call's work that needs
 *     them: seen from `stream` the call stays ordered.
 *   - No exception crosses this interface. The library is not re-entrant for one handle.
 */
#ifndef MPM_GIMP_H
#define MPM_GIMP_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MPM_OK 0
#define MPM_EARG -1        /* bad argument (null pointer, size mismatch, bad precision ...) */
#define MPM_EDET -2        /* det(dF) <= 0 or a non-positive eigenvalue of the trial b */
#define MPM_ESTENCIL -3    /* point domain needs more than one leaf boundary per axis, or
                              lattice/leaf counts exceed the key widths */
#define MPM_EOUTSIDE -4    /* point domain not inside the mesh box */
#define MPM_ETREE -5       /* octree inconsistency (unbalanced, constraint chain) */
#define MPM_EHIP -6        /* HIP runtime error */
#define MPM_ENONFINITE -7  /* non-finite input */

/* arithmetic of mpm_assemble / mpm_assemble_adjoint */
#define MPM_F64 0          /* everything in FP64 */
#define MPM_F32K 1         /* basis, stress, tangent and K values in FP32; f_int, residual and
                              its norm accumulated in FP64 (adjoint: FP32 point arithmetic,
                              FP64 outputs) */

/* body kinds for the refinement criterion */
#define MPM_BODY_NONE 0    /* no refinement */
#define MPM_BODY_SPHERE 1  /* body = {cx, cy, cz, R} */
#define MPM_BODY_CONE 2    /* cone tip + cylindrical shaft on a vertical axis:
                              body = {axis_x, axis_y, z_apex, R, tan(half apex angle), z_top} */
#define MPM_BODY_BOX 3     /* axis-aligned box: body = {x0, x1, y0, y1, z0, z1} */

/* Refinement criterion (Section 5, Steps 1-3): leaves coarser than lvl_max that meet the
 * closed body (Step 1) or have a vertex within dx_region of it (Step 2) are split (Step 3);
 * rounds repeat until nothing is marked, each followed by 2:1 balance across faces and
 * edges (at most one hanging node per edge or face). The mesh box is lo + [0, base*h0];
 * base cells have level lvl_base; a level-l leaf has side h0 * 2^(lvl_base - l).
 * Ties of the distance predicates are inclusive up to a relative 1e-12 slack.
 * ghost != 0 adds the ghost stabilisation of Section 4 (eq. ghost) to every assembly on the
 * mesh; see octree_build and mpm_assemble. */
typedef struct {
  double lo[3];
  int32_t base[3];
  double h0;
  int32_t lvl_base, lvl_max;
  int32_t body_kind;
  double body[8];
  double dx_region;
  int32_t ghost;
} mpm_refine_t;

typedef struct mpm_mesh mpm_mesh_t;

typedef struct {
  int64_t n_leaf;        /* leaves (elements) */
  int64_t n_node;        /* independent nodes */
  int64_t n_hang;        /* hanging (constrained) nodes */
  int64_t n_dof;         /* 3 * n_node */
  int64_t nnz;           /* CSR entries */
  int64_t n_point;       /* material points */
  int64_t n_straddle;    /* points whose domain overlaps more than one leaf */
  int64_t n_active_rows; /* DOF rows with at least one entry */
  int32_t max_support;   /* largest point support (nodes) */
  int32_t lattice[3];    /* finest-lattice cells per axis */
  double h_min;          /* finest cell size */
  int64_t n_ghost_face;  /* ghost faces (0 unless mpm_refine_t.ghost) */
} mpm_mesh_info_t;

/* Library-owned device arrays, valid until mpm_mesh_free (read only). */
typedef struct {
  const int32_t* leaf;          /* [n_leaf][4] anchor (finest-lattice units) x,y,z, level;
                                   ascending Morton key of the anchor */
  const int32_t* node_ijk;      /* [n_node][3] lattice coordinates of independent nodes */
  const int32_t* hang_ijk;      /* [n_hang][3] hanging nodes, ascending Morton key */
  const int32_t* hang_support;  /* [n_hang][4] independent node ids of S(n), -1 padded */
  const double* hang_weight;    /* [n_hang][4] phi_{i K_n}(x_n): 1/2 (edge) or 1/4 (face) */
  const int32_t* hang_owner;    /* [n_hang] K_n (coarsest element the node hangs on; ties:
                                   lowest Morton rank) */
  const int32_t* cell_nodes;    /* [n_leaf][8] I(K): slot k = vertex k if independent, else
                                   the parent corner that replaces it */
  const double* cell_cmat;      /* [n_leaf][8][8] C_K[vertex][slot]: phi~_slot = sum_vertex
                                   C_K[vertex][slot] phi_vertex (Section 3.1, hanging node basis) */
  const int64_t* perm;          /* [n_point] sorted position -> original index */
  const int32_t* point_leaf;    /* [n_point] sorted position -> leaf containing the centre */
  const uint8_t* point_nleaf;   /* [n_point] sorted position -> leaves overlapped */
  const int64_t* row_ptr;       /* [n_dof + 1] */
  const int32_t* col;           /* [nnz], ascending within each row */
} mpm_mesh_arrays_t;

/* Material point state, SoA device arrays in SORTED point order (see mpm_permute).
 * Updated-Lagrangian: the step starts from F_n (J_n = det F_n) and the elastic left
 * Cauchy-Green tensor b_n; V_n is the point volume at the start of the step and also
 * (generated configs) 8 l1 l2 l3 of the GIMP domain. Elastic points: sy = +inf.
 * On a mesh built without points every per-point array of every entry point (state fields,
 * per-point outputs, point order) may be NULL, and so may K values when nnz = 0. */
typedef struct {
  const double* x;    /* [3][n] domain centres */
  const double* l;    /* [3][n] domain half side lengths */
  const double* vol;  /* [n] V_n */
  const double* mass; /* [n] m_p */
  const double* Jn;   /* [n] det F_n */
  const double* bn;   /* [6][n] elastic left Cauchy-Green b_n */
  const double* Fn;   /* [9][n] F_n, only read when F_new is requested (may be NULL) */
  const double* E;    /* [n] Young's modulus */
  const double* nu;   /* [n] Poisson's ratio */
  const double* sy;   /* [n] uniaxial yield stress (von Mises, perfect plasticity) */
  double g[3];        /* body acceleration */
} mpm_state_t;

/* Build the octree from the criterion, enumerate nodes, hanging nodes and constraints
 * (Section 3.1), sort the points by (leaf containing the centre, original index), find the leaves each GIMP domain overlaps with positive volume
 * (Section 3.2; overlaps thinner than 1e-12 of the domain side do not count), and build the
 * CSR pattern: a node pair is coupled iff some point's support holds both; each coupled
 * pair is a dense 3x3 block; rows of unsupported nodes are empty.
 *   x, l: [3][n] host OR device arrays (detected), caller-owned; n may be 0 (mesh only).
 *   *out_mesh: new library-owned handle (free with mpm_mesh_free).
 * With crit->ghost != 0 (Section 4): a leaf is populated when some point domain overlaps it;
 * a boundary leaf is a populated leaf with an unpopulated face neighbour; the ghost faces are
 * the faces shared by a boundary leaf and a populated leaf (each once; between leaves of two
 * sizes the face is the smaller leaf's face). The nodes of the two leaves of a ghost face are
 * coupled in the pattern too, and per face the library keeps the 16 x 16 matrix
 * G_F[a][b] = int_F [d_n phi~_a] [d_n phi~_b] dA of the jumps across F of the normal
 * derivatives of the two leaves' constrained trilinear basis functions (2 x 2 Gauss rule,
 * exact for the biquadratic integrand).
 * Every construction step runs on the device (refinement, balance, numbering, constraints,
 * point order, overlap classification, CSR pattern, ghost faces); the host only reads counts
 * between the steps and keeps the ghost face records. Besides the pattern and the segment
 * records, the mesh keeps, per point whose domain overlaps several leaves, 592 bytes of device
 * memory (that point's tangent record, rewritten by every assembly) and 40 bytes per node of
 * its support (the node, the leaves holding it, and the slot's basis value and spatial
 * gradient, rewritten by every assembly), plus 4 bytes per (node, such point) incidence, 4
 * bytes per CSR block of the node rows those points reach, 8 bytes per point whose domain
 * lies in one leaf (their list), and a second stream with two events.
 * Errors: MPM_EARG (bad criterion or null argument, 2^32 points or more when some domains
 * straddle), MPM_ESTENCIL (lattice or leaf counts beyond the key widths, a domain over more
 * than one leaf boundary per axis, or more than 2^26 domains over several leaves),
 * MPM_EOUTSIDE, MPM_ENONFINITE, MPM_EHIP. */
int32_t octree_build(const mpm_refine_t* crit, const double* x, const double* l, int64_t n, void* stream,
                     mpm_mesh_t** out_mesh);
int32_t mpm_mesh_info(const mpm_mesh_t* mesh, mpm_mesh_info_t* out);
int32_t mpm_mesh_arrays(const mpm_mesh_t* mesh, mpm_mesh_arrays_t* out);
/* Ghost faces of the mesh (host out [n_ghost_face][8], caller-owned): lower leaf rank, higher
 * leaf rank, normal axis, plane, then the face's extent [b0, b1) x [c0, c1) along the axes
 * (axis + 1) % 3 and (axis + 2) % 3, all in finest-lattice units; sorted by leaf pair. */
int32_t mpm_ghost_faces(const mpm_mesh_t* mesh, int32_t* out);
void mpm_mesh_free(mpm_mesh_t* mesh);

/* Re-order points of an existing mesh (device only): leaf search and a stable radix sort by
 * leaf rank for n device points x [3][n] (must equal the mesh's point count). Writes
 * perm_out [n] (sorted position -> original index) and leaf_out [n] (sorted position ->
 * leaf); the mesh's own perm is not changed. The work buffers (about 16 n bytes) are kept
 * with the mesh: the first call allocates them, later calls allocate nothing. */
int32_t mpm_point_sort(const mpm_mesh_t* mesh, const double* x, int64_t n, int64_t* perm_out, int32_t* leaf_out,
                       void* stream);

/* dst[c][p] = src[c][perm[p]] for c < ncomp (device, double): brings original-order state
 * into sorted order. perm = the mesh's perm when NULL. For 2 <= ncomp <= 32 the device counts
 * the breaks of consecutive runs in perm: with at most one per 64 points (points that moved
 * little since the last sort) the arrays are gathered directly, else they pass through a
 * record-major staging copy (8 ncomp n + 256 bytes, kept with the mesh and grown when a call
 * needs more). src and dst must not overlap. */
int32_t mpm_permute(const mpm_mesh_t* mesh, const int64_t* perm, const double* src, double* dst, int32_t ncomp,
                    void* stream);

/* Body force of the weak form (Section 2.1, eq. MPMweak): f_ext[v] = sum_p S_vp m_p g,
 * FP64 device output [n_dof] (overwritten). */
int32_t mpm_external_force(const mpm_mesh_t* mesh, const mpm_state_t* s, double* f_ext, void* stream);

/* One Newton-iteration assembly (Section 2.1 weak form, discrete GIMP basis of Section 3.2
 * eq. GIMP numerical, hanging node basis of Section 3.1, Hencky / von Mises of Section 2.2):
 * per point, with u the nodal displacement of the step (device [n_dof]):
 *   S_vp, grad S_vp (one-point rule per domain/leaf overlap); H = sum_v u_v (x) grad S_v;
 *   dF = I + H; b_tr = dF b_n dF^T; principal logarithmic strains; radial return onto
 *   sqrt(3 J2) = sy; tau; sigma = tau / (det dF J_n); consistent tangent.
 *   f_int[v] += V sigma grad_x S_v,  K[(a,i),(b,k)] += V grad_x S_a . a_i.k. . grad_x S_b,
 *   V = det(dF) V_n, grad_x S = dF^-T grad S. K is the exact Jacobian d f_int / d u.
 * Outputs (device, caller-owned, overwritten):
 *   f_int [n_dof] FP64; K_vals [nnz] FP64 (MPM_F64) or FP32 (MPM_F32K), may be NULL;
 *   sigma6 [6][n] FP64 Cauchy stress, may be NULL;
 *   r [n_dof] = f_int - f_ext with DOFs where dirichlet[dof] != 0 zeroed (f_ext, dirichlet
 *   may be NULL = zero / none), and rnorm (device, 1 double) = ||r||_2 in FP64; both may be
 *   NULL; F_new [9][n] = dF F_n and be_new [6][n] the elastic left Cauchy-Green tensor of
 *   the returned strains, sum_a exp(2 eps_e,a) n_a n_a^T (Section 2.2), may be NULL (commit
 *   state; both are formed from their increments, F_n + H F_n and I + sum expm1(2 eps_e,a)
 *   n_a n_a^T, so that MPM_F32K keeps the relative accuracy of the strain).
 * On a mesh built with ghost stabilisation (Section 4, eq. ghost) the penalty
 *   j(u, v) = sum_F (h_F beta_F / kappa) int_F [d_n u] . [d_n v] dA,  kappa = 10,
 * h_F the larger side of the face's two leaves and beta_F the larger of their maxima of the
 * Young's moduli of the points overlapping them, adds K_G (the same scalar form on each
 * displacement component) to K and K_G u to f_int.
 * Synchronises `stream` once at the end to read the device error flag. */
int32_t mpm_assemble(const mpm_mesh_t* mesh, const mpm_state_t* s, const double* u, int32_t precision,
                     const double* f_ext, const uint8_t* dirichlet, double* f_int, void* K_vals, double* sigma6,
                     double* r, double* rnorm, double* F_new, double* be_new, void* stream);

/* Dynamic Newton-iteration assembly: mpm_assemble plus the inertia term of the weak form
 * (Section 2.1, eq. MPMweak: sum_p S_vp m_p a_p) under Newmark's method with gamma = 1,
 * beta = 1/2 (Section 2.4). With du_p = sum_v S_vp u_v (basis frozen at the start of the
 * step) the point acceleration is a_p = 2 (du_p - dt v_n,p) / dt^2 and the updated velocity
 * v_n,p + dt a_p; the inertia force adds sum_p S_vp m_p a_p to f_int and its derivative
 * (2 / dt^2) M, M_vw = sum_p m_p S_vp S_wp (consistent mass, times the 3x3 identity), to K.
 *   v_n: [3][n] device point velocities at the start of the step (sorted order, FP64);
 *   dt > 0: step size; s->mass must be set.
 *   f_int receives f_int + f_inertia; r = that - f_ext (Dirichlet DOFs zeroed);
 *   a_new, v_new: [3][n] device, may be NULL. Other arguments and errors as mpm_assemble;
 *   MPM_EARG also for dt <= 0 or non-finite, or a missing v_n or mass. */
int32_t mpm_assemble_dynamic(const mpm_mesh_t* mesh, const mpm_state_t* s, const double* u, const double* v_n,
                             double dt, int32_t precision, const double* f_ext, const uint8_t* dirichlet,
                             double* f_int, void* K_vals, double* sigma6, double* r, double* rnorm, double* a_new,
                             double* v_new, void* stream);

/* Adjoint of the assembly for L = lambda . f_int(u) (lambda: device [n_dof]): per point
 * dL/dE, dL/dnu, dL/dsy, dL/dV_n (device [n] FP64 each, caller-owned). Gather only (no
 * atomics); the return map is recomputed, nothing is stored by the forward pass.
 * The ghost penalty depends on E only through per-leaf maxima (not differentiable where two
 * points tie); a mesh built with ghost stabilisation returns MPM_EARG. */
int32_t mpm_assemble_adjoint(const mpm_mesh_t* mesh, const mpm_state_t* s, const double* u, const double* lambda,
                             int32_t precision, double* dL_dE, double* dL_dnu, double* dL_dsy, double* dL_dV,
                             void* stream);

/* y = K x for the assembled CSR of the mesh (K_vals [nnz] FP64 for MPM_F64 or FP32 for
 * MPM_F32K; x, y [n_dof] FP64 device, y overwritten; products and sums in FP64). The three
 * rows of a node share one column pattern; each node's rows are summed by one wavefront in a
 * fixed order, so y is reproducible. */
int32_t mpm_spmv(const mpm_mesh_t* mesh, int32_t precision, const void* K_vals, const double* x, double* y,
                 void* stream);

/* Linear solve of a Newton step on the assembled tangent: Jacobi-preconditioned conjugate
 * gradients for K_ff x_f = b_f over the free DOFs (dirichlet[dof] == 0 when dirichlet is not
 * NULL, row not empty, positive diagonal); x is zero on the other DOFs (the strong Dirichlet
 * treatment of Section 2.4 applied to the increment) and b there is ignored. Stops when
 * ||b_f - K_ff x_f|| <= rtol ||b_f|| (recursively updated residual), after max_iter
 * iterations, or when p.Kp <= 0 (K_ff not positive definite along the search direction).
 *   K_vals: [nnz] FP64 (MPM_F64) or FP32 (MPM_F32K); b, x: [n_dof] FP64 device (x written);
 *   iters, relres: host outputs (may be NULL): iterations taken, final ||r|| / ||b_f||.
 * Vectors, dot products and the preconditioner are FP64; reductions have a fixed order, so
 * the iterates are reproducible. Work vectors (5 n_dof doubles) are kept with the mesh. The
 * host reads the convergence flag every 16 iterations (one stream synchronisation each). */
int32_t mpm_solve_cg(const mpm_mesh_t* mesh, int32_t precision, const void* K_vals, const uint8_t* dirichlet,
                     const double* b, double* x, double rtol, int32_t max_iter, int32_t* iters, double* relres,
                     void* stream);

/* Allocation-free variant of mpm_solve_cg, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * same arguments, kernels, iterates and outputs as mpm_solve_cg, but it calls no hipMalloc,
 * hipFree or other allocating routine. Its work vectors live in a static device array of
 * 64 MiB that every GPU the library runs on holds for the life of the process, which limits
 * n_dof to MPM_CG_NOALLOC_MAX_DOFS (about 41 bytes per DOF); a larger mesh is refused with
 * MPM_EARG and a message that gives both sizes. The first call on a device looks up that
 * device's copy of the array. All calls on one GPU share its array and everything in it is
 * rewritten before it is read, but calls that overlap on one device (two streams or two
 * threads at once) race and must be serialised by the caller. The host reads the convergence
 * flag after a stream synchronisation every 16 iterations, so the call itself cannot be
 * captured into a graph as a whole. */
#define MPM_CG_NOALLOC_MAX_DOFS 1635968
int32_t mpm_solve_cg_noalloc(const mpm_mesh_t* mesh, int32_t precision, const void* K_vals,
                             const uint8_t* dirichlet, const double* b, double* x, double rtol, int32_t max_iter,
                             int32_t* iters, double* relres, void* stream);

/* Linear solve of a Newton step with restarted GMRES, the Krylov solver the paper names for its
 * possibly non-symmetric systems (Section 1), with the diagonal Jacobi preconditioner it
 * proposes (Section 6), applied on the right so that the minimised residual is the true one.
 * Same free DOFs, Dirichlet treatment, precisions and output as mpm_solve_cg; needs no
 * symmetry or definiteness of K_ff, only a positive diagonal on the free DOFs.
 *   restart: Arnoldi steps per cycle, 1..64; max_iter: Arnoldi steps in all.
 * A cycle ends when the residual norm given by the Givens rotations falls to rtol ||b_f||, at
 * max_iter steps, or when the Krylov space is invariant; the correction x += M^-1 V y is then
 * applied and the true residual ||b_f - K_ff x_f|| recomputed, which decides whether to stop.
 * relres is that recomputed residual over ||b_f|| (0 when b_f = 0). If the Hessenberg matrix
 * becomes singular (K_ff M^-1 singular on the Krylov space) the solve ends after that cycle's
 * correction with the residual reached. Orthogonalisation: two passes of classical
 * Gram-Schmidt per step; reductions in a fixed order (reproducible iterates). Work memory
 * ((restart + 4) n_dof doubles) is kept with the mesh; the host reads the state once per
 * cycle. Errors: MPM_EARG (null argument, bad precision, negative tolerance or iteration limit,
 * restart outside 1..64), MPM_EHIP. */
int32_t mpm_solve_gmres(const mpm_mesh_t* mesh, int32_t precision, const void* K_vals, const uint8_t* dirichlet,
                        const double* b, double* x, double rtol, int32_t restart, int32_t max_iter, int32_t* iters,
                        double* relres, void* stream);

/* GIMP refinement criterion of the adaptive strategy (Section 5): split[p] = 1 when a leaf that
 * point p's domain overlaps with positive volume has half side l_K < beta l_p, l_p the largest
 * of the domain's three half sides (the paper uses beta = 2). The mesh gives the leaves only
 * (it may have been built without points); x, l: [3][n] device, any order; split: [n] device
 * uint8, written; *n_split (host): number of points flagged. Errors: MPM_EARG (null argument,
 * beta not positive and finite), MPM_ENONFINITE, MPM_EOUTSIDE, MPM_ESTENCIL (a domain over more
 * than 4096 lattice cells of the finest level whose leaves do not trigger the split; only
 * possible for beta well below 2), with the first such point. */
int32_t mpm_split_mark(const mpm_mesh_t* mesh, const double* x, const double* l, int64_t n, double beta,
                       uint8_t* split, int64_t* n_split, void* stream);

/* Output state of mpm_split_apply: device [c][n_out] arrays, same fields as mpm_state_t. */
typedef struct {
  double* x;
  double* l;
  double* vol;
  double* mass;
  double* Jn;
  double* bn;
  double* Fn;
  double* E;
  double* nu;
  double* sy;
} mpm_state_out_t;

/* Splits the flagged GIMPs (Section 5, transfer of GIMP data). Point p with split[p] != 0
 * becomes 8 GIMPs tiling its domain: child c (bit a of c for axis a) is centred at
 * x_a - l_a / 2 (bit clear) or x_a + l_a / 2 (bit set), with half sides l / 2 and volume and
 * mass / 8; J_n, b_n, F_n, velocity and material parameters are copied. With the reference
 * positions X (X_in/X_out), each child gets X + F_n^{-1} (x_c - x), and a material parameter
 * selected by prop_mask (bit 0 E, bit 1 nu, bit 2 sy) is evaluated there as
 * props[4r] + props[4r+1] X_1 + props[4r+2] X_2 + props[4r+3] X_3 (props: host [3][4]) rather
 * than copied. Unflagged points are copied. The output keeps the input order: a point, or its
 * 8 children in child order.
 *   in: x, l, vol, mass required; Jn, bn, Fn, E, nu, sy optional, each paired with the same
 *   field of out (both NULL or both set); X_in/X_out and v_in/v_out optional pairs [3][n]
 *   (X_in needs Fn);
 *   n_out must equal n + 7 * (number of flagged points). Inputs and outputs must not overlap.
 * A work buffer (8 bytes per 256 points for block counts, 8 (n + 1) bytes of output offsets
 * and 8 n_out bytes of parent indices) is kept with the mesh and grown when a call needs more. */
int32_t mpm_split_apply(const mpm_mesh_t* mesh, int64_t n, const uint8_t* split, const mpm_state_t* in,
                        const double* X_in, const double* v_in, const double* props, int32_t prop_mask,
                        const mpm_state_out_t* out, double* X_out, double* v_out, int64_t n_out, void* stream);

/* Kernel timing for measurement tools. enable = 1: from now on HIP events bracket the fused
 * assembly kernel (single-leaf points), the row-gather kernel that writes f_int and K, and
 * the adjoint kernel (single-leaf points) on the caller's stream, and their elapsed times
 * accumulate in the handle (read at the synchronisation that ends each call; kernels on the
 * mesh's second stream may run inside these spans); enable = 0: stop; enable = -1: only read.
 * ms_out (host, 6 doubles, may be NULL): [0] assembly-kernel ms summed, [1] its launches,
 * [2] adjoint-kernel ms, [3] adjoint launches, [4] gather-kernel ms, [5] gather launches;
 * reading resets the sums. */
int32_t mpm_kernel_timing(mpm_mesh_t* mesh, int32_t enable, double* ms_out);

/* last error of the calling thread */
int32_t mpm_last_error(char* buf, size_t n);
int64_t mpm_last_error_index(void);

#ifdef __cplusplus
}
#endif
#endif
