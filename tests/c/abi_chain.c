/*
 * A plain C caller of the library's C ABI (include/tc2.h), with no Python and
 * no torch: one FP64 TC2 + response solve (Sec. 2.2) of a chain of NA atoms
 * with two orbitals each (one occupied), nearest-neighbour couplings, and the
 * atom position as the perturbation H1.  Prints one line:
 *     <status> <iters> <branches> <Tr(X1 H1)> <Tr X0>
 * and exits 0 when the solve converged or reached its precision floor.
 */
#include <stdio.h>

#include "tc2.h"

#define NA 32
#define B 2

/* entry (r, c) of the coupling block between atoms i and i + 1 */
static double coupling(int i, int r, int c) {
  static const double base[2][2] = {{-0.30, 0.10}, {0.05, 0.20}};
  return base[r][c] * (1.0 + 0.1 * (double)(i % 3));
}

int main(void) {
  static int64_t rp[NA + 1], rp1[NA + 1];
  static int32_t ci[3 * NA], ci1[NA];
  static double hv[3 * NA * B * B], h1v[NA * B * B];
  int nnz = 0;
  for (int i = 0; i < NA; ++i) {
    rp[i] = nnz;
    if (i > 0) { /* H_{i,i-1} = H_{i-1,i}^T */
      ci[nnz] = i - 1;
      for (int r = 0; r < B; ++r)
        for (int c = 0; c < B; ++c) hv[(nnz * B + r) * B + c] = coupling(i - 1, c, r);
      ++nnz;
    }
    ci[nnz] = i; /* onsite: occupied orbital at -1, virtual at +1 */
    for (int r = 0; r < B; ++r)
      for (int c = 0; c < B; ++c) hv[(nnz * B + r) * B + c] = r == c ? (r == 0 ? -1.0 : 1.0) : 0.0;
    ++nnz;
    if (i + 1 < NA) {
      ci[nnz] = i + 1;
      for (int r = 0; r < B; ++r)
        for (int c = 0; c < B; ++c) hv[(nnz * B + r) * B + c] = coupling(i, r, c);
      ++nnz;
    }
  }
  rp[NA] = nnz;
  for (int i = 0; i < NA; ++i) {
    const double x = (double)i - 0.5 * (double)(NA - 1);
    rp1[i] = i;
    ci1[i] = i;
    for (int r = 0; r < B; ++r)
      for (int c = 0; c < B; ++c) h1v[(i * B + r) * B + c] = r == c ? x : 0.0;
  }
  rp1[NA] = NA;

  tc2_problem p = {0};
  p.H.nb = NA;
  p.H.b = B;
  p.H.row_ptr = rp;
  p.H.col = ci;
  p.H.val = hv;
  p.n_dir = 1;
  p.H1[0].nb = NA;
  p.H1[0].b = B;
  p.H1[0].row_ptr = rp1;
  p.H1[0].col = ci1;
  p.H1[0].val = h1v;
  p.n_occ = NA;
  p.eps_drop = 1e-10;
  p.tol = 1e-10;
  p.max_iter = 100;

  tc2_options o = {0};
  o.precision = TC2_FP64;
  o.skip = 1;  /* exact norm-bound screen */
  o.graph = 1; /* each update as one captured graph */

  tc2_ctx *ctx = NULL;
  tc2_status st = tc2_setup(&p, 1, &o, &ctx);
  if (st != TC2_OK) {
    fprintf(stderr, "tc2_setup: %s\n", tc2_strerror(st));
    return 2;
  }
  tc2_result res = {0};
  st = tc2_run(ctx, NULL, &res);
  printf("%d %d %s %.17g %.17g\n", (int)st, res.iters, res.branches, res.trace_x1h1[0],
         res.tr_x0);
  tc2_free(ctx);
  return (st == TC2_OK || st == TC2_FLOOR_REACHED) ? 0 : 3;
}
