/* The per-system stopping decision of one update, shared by the device-side
 * decision kernel (k_decide) and its CPU test.  Plain C: no HIP types, so a
 * host compiler can build it; the kernel's header defines TC2_HD as
 * __host__ __device__ before including it.
 *
 * The rule (readings of Sec. 2.3's tolerance and of the recursion's precision
 * floor), for update k = 1, 2, ... of a system:
 *  - a non-finite product value (bad) stops the system with TC2_ENAN;
 *  - k >= 2 and every change of E0 = Tr(X0 H), Tr(X1_d H) and Tr(X1_d H1_d)
 *    since the previous iterate strictly below tol: TC2_OK;
 *  - k >= 3, |iota_k| < 1 and |iota_k| >= |iota_{k-2}|, with
 *    iota = Tr X0 - ||X0||_F^2: TC2_FLOOR_REACHED (the stall guard);
 *  - k >= max_iter: TC2_NOT_CONVERGED.
 * The tests are taken in this order.  Arithmetic in FP64, with the host
 * rule's operations, so that both take the same decisions. */
#ifndef TC2_DECIDE_RULE_H
#define TC2_DECIDE_RULE_H

#include <math.h>

#include "../../include/tc2.h"

#ifndef TC2_HD
#define TC2_HD
#endif

/* e: the new iterate's values, e[0] = E0, e[1 + d] = Tr(X1_d H),
 *    e[1 + D + d] = Tr(X1_d H1_d), d < D (1 + 2D values);
 * prev: the previous iterate's values, replaced by e;
 * iota1, iota2: iota of the last two updates, shifted (iota1 becomes iota);
 * k: updates run, incremented.
 * Returns 1 and sets *status when the system stops, else 0. */
static inline TC2_HD int tc2_decide_rule(int D, const double *e, double iota, int bad,
                                         double tol, int max_iter, double *prev,
                                         double *iota1, double *iota2, int *k,
                                         int *status) {
  const int kk = ++*k;
  double dmax = 0.0;
  for (int m = 0; m < 1 + 2 * D; ++m) {
    const double v = fabs(e[m] - prev[m]);
    dmax = dmax < v ? v : dmax;
    prev[m] = e[m];
  }
  const double iota_km2 = *iota2; /* iota two updates back (k >= 3) */
  *iota2 = *iota1;
  *iota1 = iota;
  if (bad) {
    *status = TC2_ENAN;
    return 1;
  }
  if (kk >= 2 && dmax < tol) {
    *status = TC2_OK;
    return 1;
  }
  if (kk >= 3 && fabs(iota) < 1.0 && fabs(iota) >= fabs(iota_km2)) {
    *status = TC2_FLOOR_REACHED;
    return 1;
  }
  if (kk >= max_iter) {
    *status = TC2_NOT_CONVERGED;
    return 1;
  }
  return 0;
}

#endif
