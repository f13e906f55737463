/* Internal definitions shared by the oracle's translation units (test infrastructure only). */
#ifndef MPM_ORC_INTERNAL_H
#define MPM_ORC_INTERNAL_H
#include "oracle.h"
#include <stddef.h>

struct orc_mesh {
  orc_crit c;
  int nx, ny, nz;            /* finest-lattice cells per axis */
  int s0;                    /* base cell size in finest-lattice units */
  double hmin;               /* finest cell size */
  int64_t nleaf;
  int32_t* leaf;             /* nleaf x 4: anchor x,y,z (lattice units), level; ascending Morton key */
  int32_t* leafmap;          /* finest cell -> leaf index */
  int64_t nnode;             /* all nodes (vertices of leaves), ascending Morton key */
  int32_t* node_ijk;         /* nnode x 3 */
  int32_t* nodemap;          /* node lattice point -> node index, -1 if not a node */
  uint8_t* hang;             /* per node */
  int32_t* indep;            /* per node: independent id, -1 for hanging nodes */
  int64_t nindep;
  int32_t* indep_node;       /* independent id -> node index */
  int32_t* hang_owner;       /* per node: owning coarse leaf K_n (-1 if independent) */
  int8_t* hang_nsup;
  int32_t* hang_sup;         /* per node x 4: independent ids of S(n) */
  double* hang_w;            /* per node x 4: phi_{i K_n}(x_n) */
  int32_t* ik_n;             /* per leaf: |I(K)| */
  int32_t* ik_node;          /* per leaf x ORC_MAXI: independent ids, ascending */
  double* ik_c;              /* per leaf x 8 x ORC_MAXI: C_K[vertex][slot] */
  /* points */
  int64_t np;
  double* px;                /* 3 x np (copy) */
  double* pl;
  int64_t* perm;             /* sorted position -> original index */
  int32_t* pleaf;            /* original index -> leaf containing the centre */
  uint8_t* pnleaf;           /* original index -> number of overlapped leaves */
  int64_t* sup_off;          /* np+1 */
  int32_t* sup_node;
  int64_t nstraddle;
  int maxsup;
  int64_t nnz;
  int64_t* row_ptr;          /* 3*nindep + 1 */
  int32_t* col;
  /* ghost stabilisation */
  int32_t ghost;             /* add ghost-face couplings to the CSR pattern at set_points */
  int64_t ngface;
  int32_t* gface;            /* ngface x 8: lo leaf, hi leaf, axis, plane, b0, b1, c0, c1 */
};

int64_t orc_ghost_build_faces(orc_mesh* m, const uint8_t* pop);
int64_t orc_ghost_pairs(const orc_mesh* m, uint64_t** pairs, int64_t npair, int64_t* cap);

uint64_t orc_morton3(uint64_t x, uint64_t y, uint64_t z);
/* overlapped leaves of a domain (centre x, half-lengths l): returns count or negative status.
 * lv[k] leaf ids, box[k*6..] = overlap intervals (lo0,hi0,lo1,hi1,lo2,hi2) */
int orc_point_leaves(const orc_mesh* m, const double x[3], const double l[3], int32_t* lv, double* box);

#endif
