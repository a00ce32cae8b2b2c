// Branch and stopping decisions on the device (see tc2_decide.h): one
// workgroup, one thread per system, launched at the end of each captured
// update so that the host need not read the scalars between updates.
#include "tc2_decide.h"

namespace tc2 {

__global__ void __launch_bounds__(256) k_decide(DecideArgs a) {
  __shared__ int any, ran;
  if (threadIdx.x == 0) {
    any = 0;
    ran = 0;
  }
  __syncthreads();
  const int D = a.D;
  for (int s = threadIdx.x; s < a.nsys; s += blockDim.x) {
    if (!a.active[s]) continue;
    DecideSys& S = a.state[s];
    const DecideParam& P = a.param[s];
    const double* q = a.scal + (size_t)s * NQ;
    double cur[1 + 2 * MAXD];
    cur[0] = q[Q_E0];
    for (int d = 0; d < D; ++d) {
      cur[1 + d] = q[Q_E1 + d];
      cur[1 + D + d] = q[Q_AL + d];
    }
    if (a.init) {
      // before the first update: the energies to compare with, and the
      // branch of the first update from the initial trace
      for (int k = 0; k < 1 + 2 * D; ++k) S.prev[k] = cur[k];
      a.branch[s] = q[Q_TR0] >= P.n_occ ? 1 : 0;
      atomicOr(&any, 1);
      continue;
    }
    atomicOr(&ran, 1);
    // the update just run took a.branch[s]
    if (S.k < TC2_MAX_ITER + 4) {
      S.branches[S.k] = a.branch[s] ? 'S' : 'D';
      S.branches[S.k + 1] = 0;
    }
    S.trip += q[Q_TRIP];
    S.nominal += a.nominal[s];
    const int bad = a.bad[s];
    const int stop = tc2_decide_rule(D, cur, q[Q_TR0] - q[Q_FRO0], bad, P.tol, P.max_iter, S.prev,
                                     &S.iota1, &S.iota2, &S.k, &S.status);
    if (!bad) a.branch[s] = q[Q_TR0] >= P.n_occ ? 1 : 0;
    if (stop) a.active[s] = 0;
    else atomicOr(&any, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    DecideWord& w = *a.word;
    w.any_active = any;
    if (!a.init && ran) {
      w.updates += 1;
      w.exec_pairs += *a.exec_pairs;
      if (a.screened) {
        w.screened[0] += a.screened[0];
        w.screened[1] += a.screened[1];
      }
      if (*a.overflow) w.overflow = 1;
    }
  }
  if (!a.init && *a.overflow) {
    // never with the dense-bound stage; the host reports it and the updates
    // already queued find no active system
    __syncthreads();
    for (int s = threadIdx.x; s < a.nsys; s += blockDim.x) a.active[s] = 0;
    if (threadIdx.x == 0) a.word->any_active = 0;
  }
}

void launch_decide(hipStream_t st, const DecideArgs& a) {
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(256), 0, st, a);
}

}  // namespace tc2
