/*
 * Oracle: which GIMPs the adaptive strategy refines (Section 5, GIMP refinement criterion).
 * TEST INFRASTRUCTURE ONLY.
 *
 * A GIMP p is split when a leaf K that its domain overlaps with positive volume has half side
 * l_K < beta l_p (beta >= 2, user defined). GIMP domains here are boxes with three half sides;
 * l_p is read as the largest of them, so that after the split every axis of the children
 * meets the criterion the paper states for a cube.
 */
#include <math.h>

#include "orc_internal.h"

int32_t orc_split_mark(const orc_mesh* m, const double* x, const double* l, int64_t n, double beta, uint8_t* split,
                       int64_t* bad) {
  int32_t lv[ORC_MAXL];
  double box[6 * ORC_MAXL];
  for (int64_t p = 0; p < n; p++) {
    double xp[3] = {x[p], x[n + p], x[2 * n + p]}, lp[3] = {l[p], l[n + p], l[2 * n + p]};
    int nl = orc_point_leaves(m, xp, lp, lv, box);
    if (nl < 0) {
      *bad = p;
      return nl;
    }
    double lmax = lp[0] > lp[1] ? lp[0] : lp[1];
    lmax = lmax > lp[2] ? lmax : lp[2];
    split[p] = 0;
    for (int k = 0; k < nl; k++) {
      int s = 1 << (m->c.lvl_max - m->leaf[4 * lv[k] + 3]);
      double lK = 0.5 * s * m->hmin;
      if (lK < beta * lmax) split[p] = 1;
    }
  }
  return ORC_OK;
}
