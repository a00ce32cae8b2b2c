// Branch and stopping decisions on the device (device_loop option).
//
// After each captured update a one-workgroup kernel reads the per-system
// scalars the update reduced and applies, per active system:
//  - the branch rule of Eq. TC2 (SQUARE when Tr X0 >= Nocc, else DOUBLE) for
//    the next update, written to the flag array the next update's kernels
//    read;
//  - the stopping rule: after k >= 2 updates, stop when the band energies
//    Tr(X0 H), Tr(X1_d H) and the traces Tr(X1_d H1_d) all changed by less
//    than tol (Sec. 2.3); after k >= 3, stop at the precision floor when
//    |iota_k| >= |iota_{k-2}| with |iota_k| < 1 (iota = Tr X0 - ||X0||_F^2);
//    stop at max_iter; a non-finite product value stops the system with
//    TC2_ENAN.
// The arithmetic is the host rule's, in FP64, so both take the same
// decisions.  The per-system record also keeps the branch string and the
// counters that the host reports at the end of the solve.
#pragma once

#include "tc2_internal.h"
#include "../../include/tc2.h"

#define TC2_HD __host__ __device__
#include "tc2_decide_rule.h"

namespace tc2 {

struct DecideSys {
  double prev[1 + 2 * MAXD];     // E0, E1_d, alpha_d of the last iterate
  double iota1, iota2;           // iota of the last two updates (k, k - 1)
  double trip;                   // union-pattern block triples, summed
  unsigned long long nominal;    // full-product block triples, summed
  int k;                         // updates run
  int status;                    // tc2_status of the system
  char branches[TC2_MAX_ITER + 8];  // 'S' / 'D' per update, NUL-terminated
};

struct DecideParam {
  double n_occ;                  // Nocc as a double (the host compares the same)
  double tol;
  int max_iter;
  int pad;
};

// The word the host polls: any system still active after the last update,
// updates that ran with an active system, a stage overflow seen, and the
// per-update device counters summed.
struct DecideWord {
  int any_active;
  int updates;
  int overflow;
  int pad;
  unsigned long long exec_pairs;
  unsigned long long screened[2];
};

struct DecideArgs {
  int nsys, D;
  int init;                      // 1: before the first update (branch, prev only)
  const double* scal;            // nsys x NQ scalars of the new iterate
  const int* bad;                // per system: a non-finite value was produced
  const unsigned long long* nominal;  // per system: this update's full triples
  const unsigned long long* exec_pairs;  // this update's executed pairs
  const unsigned long long* screened;    // this update's skip counters, or null
  const int* overflow;           // this update's stage overflow flag
  const DecideParam* param;
  DecideSys* state;
  int* active;                   // per system, read by the next update
  int* branch;                   // per system, read by the next update
  DecideWord* word;
};

void launch_decide(hipStream_t st, const DecideArgs& a);

}  // namespace tc2
