/* ctypes shim over the library's per-system stopping rule
 * (paper_2009_03551_amd/csrc/tc2_decide_rule.h, the rule that the device-side
 * decision kernel applies), built with gcc for its CPU test. */
#include <stddef.h>

#include "../../paper_2009_03551_amd/csrc/tc2_decide_rule.h"

/* Replays updates 1..n of one system through the rule.  e holds n + 1 rows of
 * 1 + 2D values: row 0 the initial iterate's (E0, Tr(X1_d H), Tr(X1_d H1_d)),
 * row u those after update u; iota[u - 1] and bad[u - 1] belong to update u
 * (bad may be NULL).  Returns the update at which the rule stops (0 when it
 * does not within n updates) and sets *status. */
int decide_replay(int D, int n, const double *e, const double *iota, const int *bad,
                  double tol, int max_iter, int *status) {
  double prev[1 + 2 * 3];
  double iota1 = 0.0, iota2 = 0.0;
  int k = 0;
  if (D < 0 || D > 3) return -1;
  for (int m = 0; m < 1 + 2 * D; ++m) prev[m] = e[m];
  for (int u = 1; u <= n; ++u)
    if (tc2_decide_rule(D, e + (size_t)u * (1 + 2 * D), iota[u - 1], bad ? bad[u - 1] : 0, tol,
                        max_iter, prev, &iota1, &iota2, &k, status))
      return u;
  return 0;
}
