/*
 * CPU reference ("oracle") for the octree GIMP MPM assembly.
 *
 * TEST INFRASTRUCTURE ONLY. This code exists to check the HIP library; nothing in the
 * product path may link, load or call it. It shares no code with the library: its own
 * octree (dense finest-lattice maps), its own hanging-node search (scan of element
 * boundaries, paper Section 3.1 definition of a hanging node), exact GIMP integrals
 * (antiderivatives of the trilinear basis over each domain/element overlap, the convolution
 * of Section 3.2 "GIMP basis"), a literal 4th-order-tensor consistent tangent and a
 * complex-step parameter derivative for the adjoint. Everything is FP64, single thread.
 *
 * Where the paper leaves a choice open this file takes the same readings as the library: a
 * von Mises surface sqrt(3 J2) = sigma_y on the Kirchhoff stress with a radial return in
 * principal logarithmic strains; K as the exact Jacobian of f_int with the basis frozen; a
 * leaf counts in a support only if every axis overlap exceeds 1e-12 of the domain side;
 * 2:1 balance across faces and edges; edge-hanging ties to the lowest Morton rank; points
 * ordered by (leaf containing the centre, original index); Newmark gamma = 1, beta = 1/2.
 */
#ifndef MPM_ORACLE_H
#define MPM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double lo[3];
  int32_t base[3];
  double h0;
  int32_t lvl_base, lvl_max;
  int32_t body_kind;      /* 0 none, 1 sphere, 2 cone+shaft, 3 box */
  double body[8];
  double dx_region;
} orc_crit;

typedef struct orc_mesh orc_mesh;

/* status codes (same meaning as the library's) */
#define ORC_OK 0
#define ORC_EARG -1
#define ORC_EDET -2
#define ORC_ESTENCIL -3
#define ORC_EOUTSIDE -4
#define ORC_ETREE -5
#define ORC_ENONFINITE -7

#define ORC_MAXI 27     /* max |I(K)| accepted */
#define ORC_MAXS 128    /* max support size of one point */
#define ORC_MAXL 1024   /* max leaves overlapped by one point domain */

orc_mesh* orc_mesh_build(const orc_crit* c, int32_t* status);
void orc_mesh_free(orc_mesh* m);
/* counts: [0] n_leaf [1] n_node_all [2] n_indep [3] n_hang [4] n_point [5] nnz
 *         [6] n_straddle [7] max support size [8] n_rows_active(dof rows) */
void orc_mesh_counts(const orc_mesh* m, int64_t out[9]);
void orc_mesh_leaves(const orc_mesh* m, int32_t* anchor_level /* n_leaf x 4 */);
void orc_mesh_nodes(const orc_mesh* m, int32_t* ijk /* n_indep x 3 */);
void orc_mesh_hanging(const orc_mesh* m, int32_t* ijk /* n_hang x 3 */, int32_t* sup /* x4, -1 pad */,
                      double* w /* x4 */, int32_t* owner_leaf);
/* I(K) sorted ascending by independent node id (count per leaf in n), and C_K with
 * cmat[leaf][vertex j][slot] (8 x ORC_MAXI) */
void orc_mesh_cells(const orc_mesh* m, int32_t* n, int32_t* inodes /* n_leaf x ORC_MAXI */,
                    double* cmat /* n_leaf x 8 x ORC_MAXI */);

/* Ghost stabilisation (Section 4): enable before orc_mesh_set_points to add the couplings of
 * the ghost faces to the CSR pattern; faces: n x 8 (lo leaf, hi leaf, axis, plane, b0, b1,
 * c0, c1 in lattice units) */
void orc_mesh_set_ghost(orc_mesh* m, int32_t enable);
int64_t orc_ghost_nfaces(const orc_mesh* m);
void orc_ghost_faces(const orc_mesh* m, int32_t* out);

/* points: SoA x[3][n], l[3][n] */
int32_t orc_mesh_set_points(orc_mesh* m, const double* x, const double* l, int64_t n, int64_t* bad_index);
void orc_mesh_perm(const orc_mesh* m, int64_t* perm /* sorted position -> original index */,
                   int32_t* point_leaf /* original index -> leaf */, uint8_t* nleaf /* original index */);
void orc_mesh_csr(const orc_mesh* m, int64_t* row_ptr /* 3*n_indep+1 */, int32_t* col /* nnz */);

/* basis of one point (any position): returns support size, or negative status */
int32_t orc_point_basis(const orc_mesh* m, const double x[3], const double l[3], int32_t* node,
                        double* S, double* dS /* 3 per node */);

/* single material point update:
 * dF row-major 3x3; bn = (xx,yy,zz,xy,yz,xz); outputs sigma6, tau6 (same order),
 * a81[i][j][k][l] = spatial tangent, be6 = updated elastic left Cauchy-Green.
 * info[0] = plastic flag, info[1] = trial von Mises stress q_tr, info[2] = J */
int32_t orc_material_point(const double dF[9], const double bn[6], double Jn, double E, double nu,
                           double sy, double sigma6[6], double tau6[6], double a81[81], double be6[6],
                           double info[3]);

/* state arrays in ORIGINAL point order (SoA), u and outputs over 3*n_indep DOFs.
 * K is over the CSR pattern from orc_mesh_csr. sigma6 is [6][n]. */
typedef struct {
  const double *x, *l, *vol, *mass, *Jn, *bn, *E, *nu, *sy, *Fn;
  double g[3];
} orc_state;

/* plastic[p]: 1 where the trial stress lies outside the yield surface; qtrial[p]: the trial
 * von Mises stress sqrt(3 J2) of the Kirchhoff stress (both may be NULL). */
int32_t orc_assemble(const orc_mesh* m, const orc_state* s, const double* u, double* f_int, double* K,
                     double* sigma6, double* Fnew9, double* be6, uint8_t* plastic, double* qtrial,
                     int64_t* bad_index);
/* orc_assemble on nthreads host threads (timing of the oracle on all cores): per-thread f_int and
 * K added in thread order; sigma6 as orc_assemble (may be NULL). */
int32_t orc_assemble_threads(const orc_mesh* m, const orc_state* s, const double* u, double* f_int, double* K,
                             double* sigma6, int32_t nthreads, int64_t* bad_index);
int32_t orc_external_force(const orc_mesh* m, const orc_state* s, double* f_ext);
/* Newmark (gamma = 1, beta = 1/2) inertia term: f_iner over 3*n_indep DOFs, (2/dt^2) x the
 * consistent mass added into K (CSR pattern; may be NULL), point acceleration and updated
 * velocity [3][n] (may be NULL); vel = point velocities at the start of the step [3][n]. */
int32_t orc_inertia(const orc_mesh* m, const orc_state* s, const double* u, const double* vel, double dt,
                    double* f_iner, double* K, double* a_new, double* v_new, int64_t* bad_index);
/* ghost term: K += K_G (may be NULL), f += K_G u (may be NULL), beta_leaf [n_leaf] = max E of
 * the points overlapping each leaf (may be NULL) */
/* GIMP refinement criterion (Section 5): split[p] = 1 when a leaf overlapped by point p's domain
 * has half side < beta * (largest half side of the domain); bad = first failing point */
int32_t orc_split_mark(const orc_mesh* m, const double* x, const double* l, int64_t n, double beta, uint8_t* split,
                       int64_t* bad);
int32_t orc_ghost_assemble(const orc_mesh* m, const orc_state* s, const double* u, double* K, double* f,
                           double* beta_leaf);
/* r = f_int - f_ext with dirichlet DOFs zeroed; returns ||r||_2 in *rnorm */
void orc_residual(int64_t ndof, const double* f_int, const double* f_ext, const uint8_t* dirichlet,
                  double* r, double* rnorm);
/* L = lambda . f_int(u): per point dL/dE, dL/dnu, dL/dsy, dL/dVn (original order) */
int32_t orc_adjoint(const orc_mesh* m, const orc_state* s, const double* u, const double* lambda,
                    double* dE, double* dnu, double* dsy, double* dV, int64_t* bad_index);

#ifdef __cplusplus
}
#endif
#endif
