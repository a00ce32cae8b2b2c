// Dense O(N^3) density matrix and first-order response (Sec. 2.1, the O(N^3)
// method): the reference of the crossover experiment of Sec. 4, in which the
// linear-scaling TC2 / TC2-CPSCF path is timed against diagonalisation.
//
// Steps on the device:
//   H (BSR)  -> dense, column-major  (k_densify)
//   H = C E C^T                      (rocSOLVER dsyevd, ascending e)
//   P0 = C_occ C_occ^T               (rocBLAS dsyrk, upper; k_mirror_upper)
//   per direction d (Eq. cpscf-LCAO with U_pp = 0, and Eq. DM1):
//     T = H1_d C_occ                 (rocBLAS dgemm)
//     G = C_virt^T T                 (dgemm)
//     M_ai = G_ai / (e_i - e_a)      (k_gap_scale)
//     Y = C_virt M                   (dgemm)
//     P1_d = Y C_occ^T + C_occ Y^T   (rocBLAS dsyr2k, upper; k_mirror_upper)
//   traces over the stored blocks of H and H1_d (k_trace_bsr; partial sums per
//   workgroup added on the host in a fixed order)
#include "tc2_host.h"
#include "tc2_internal.h"
#include "../../include/tc2.h"

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cstring>
#include <new>
#include <vector>

namespace {

constexpr int TR_BLOCKS = 512;  // workgroups of the trace kernel
constexpr int TR_THREADS = 256;

// Element k of the values of a BSR matrix (entry e = k / b^2, row-major inside
// the block) to its place in a column-major N x N matrix that is zero.
__global__ void k_densify(long long nval, int b, const int* row_of, const int* col,
                          const double* val, long long N, double* A) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < nval; k += stride) {
    const long long e = k / (b * b);
    const int rc = (int)(k - e * b * b), r = rc / b, c = rc - r * b;
    const long long i = (long long)row_of[e] * b + r, j = (long long)col[e] * b + c;
    A[i + j * N] = val[k];
  }
}

// G (nv x no, column-major) divided element-wise by the gap e_i - e_a between
// occupied state i (< no) and virtual state a (index no + a in e).
__global__ void k_gap_scale(long long nv, long long no, const double* e, double* G) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < nv * no; k += stride) {
    const long long i = k / nv, a = k - i * nv;
    G[k] /= e[i] - e[no + a];
  }
}

// The N x N identity (column-major).
__global__ void k_identity(long long N, double* A) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < N * N; k += stride)
    A[k] = (k % (N + 1)) == 0 ? 1.0 : 0.0;
}

// Copy the upper triangle of a column-major N x N matrix onto the lower one.
__global__ void k_mirror_upper(long long N, double* A) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < N * N; k += stride) {
    const long long c = k / N, r = k - c * N;
    if (r > c) A[k] = A[c + r * N];
  }
}

// Tr(A B) = sum_ij A_ij B_ji over the stored values of the BSR matrix B (A
// dense, column-major; both symmetric): one partial sum per workgroup.
__global__ __launch_bounds__(TR_THREADS) void k_trace_bsr(long long nval, int b, const int* row_of,
                                                          const int* col, const double* val,
                                                          long long N, const double* A,
                                                          double* partial) {
  __shared__ double red[TR_THREADS];
  double s = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < nval; k += stride) {
    const long long e = k / (b * b);
    const int rc = (int)(k - e * b * b), r = rc / b, c = rc - r * b;
    const long long i = (long long)row_of[e] * b + r, j = (long long)col[e] * b + c;
    s += A[j + i * N] * val[k];  // A_ji B_ij
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = TR_THREADS / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

unsigned grid_for(long long n) {
  const long long g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

struct Dev {  // device allocation released with its owner
  void* p = nullptr;
  ~Dev() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t bytes) { return tc2::dev_malloc(&p, bytes ? bytes : 8); }
  double* d() const { return (double*)p; }
  int* i() const { return (int*)p; }
};

struct DenseBsr {  // a BSR matrix on the device, with the row of every entry
  Dev row_of, col, val;
  long long nnz = 0, nval = 0;
};

struct Call {  // resources of one call
  hipStream_t own = nullptr;
  rocblas_handle h = nullptr;
  hipEvent_t ev[5] = {};
  ~Call() {
    for (hipEvent_t& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (h) (void)rocblas_destroy_handle(h);
    if (own) (void)hipStreamDestroy(own);
  }
};

#define DCHK(x)                                                    \
  do {                                                             \
    hipError_t e_ = (x);                                           \
    if (e_ != hipSuccess) return e_ == hipErrorOutOfMemory ? TC2_ENOMEM : TC2_EDEVICE; \
  } while (0)
#define BCHK(x)                                                    \
  do {                                                             \
    rocblas_status s_ = (x);                                       \
    if (s_ != rocblas_status_success)                              \
      return s_ == rocblas_status_memory_error ? TC2_ENOMEM : TC2_EDEVICE; \
  } while (0)

tc2_status upload_bsr(const tc2_bsr& m, hipStream_t st, DenseBsr& d) {
  const int nb = m.nb, b = m.b;
  d.nnz = m.row_ptr[nb];
  d.nval = d.nnz * b * b;
  std::vector<int> row_of((size_t)d.nnz);
  for (int i = 0; i < nb; ++i)
    for (int64_t p = m.row_ptr[i]; p < m.row_ptr[i + 1]; ++p) row_of[(size_t)p] = i;
  DCHK(d.row_of.alloc((size_t)d.nnz * sizeof(int)));
  DCHK(d.col.alloc((size_t)d.nnz * sizeof(int)));
  DCHK(d.val.alloc((size_t)d.nval * sizeof(double)));
  if (d.nnz > 0) {
    DCHK(hipMemcpyAsync(d.row_of.p, row_of.data(), (size_t)d.nnz * sizeof(int),
                        hipMemcpyHostToDevice, st));
    DCHK(hipMemcpyAsync(d.col.p, m.col, (size_t)d.nnz * sizeof(int), hipMemcpyHostToDevice, st));
    DCHK(hipMemcpyAsync(d.val.p, m.val, (size_t)d.nval * sizeof(double), hipMemcpyHostToDevice,
                        st));
  }
  // the host vector must outlive the copy
  DCHK(hipStreamSynchronize(st));
  return TC2_OK;
}

tc2_status densify(const DenseBsr& m, int b, long long N, hipStream_t st, double* A) {
  DCHK(hipMemsetAsync(A, 0, (size_t)N * N * sizeof(double), st));
  if (m.nval > 0)
    hipLaunchKernelGGL(k_densify, dim3(grid_for(m.nval)), dim3(256), 0, st, m.nval, b,
                       m.row_of.i(), m.col.i(), m.val.d(), N, A);
  DCHK(hipGetLastError());
  return TC2_OK;
}

// Tr(A B) over the stored values of B, summed on the host in a fixed order
tc2_status trace(const DenseBsr& m, int b, long long N, const double* A, double* part,
                 hipStream_t st, double* out) {
  *out = 0.0;
  if (m.nval == 0) return TC2_OK;
  hipLaunchKernelGGL(k_trace_bsr, dim3(TR_BLOCKS), dim3(TR_THREADS), 0, st, m.nval, b,
                     m.row_of.i(), m.col.i(), m.val.d(), N, A, part);
  DCHK(hipGetLastError());
  double h[TR_BLOCKS];
  DCHK(hipMemcpyAsync(h, part, sizeof(h), hipMemcpyDeviceToHost, st));
  DCHK(hipStreamSynchronize(st));
  double s = 0.0;
  for (int k = 0; k < TR_BLOCKS; ++k) s += h[k];
  *out = s;
  return TC2_OK;
}

tc2_status mirror(long long N, double* A, hipStream_t st) {
  hipLaunchKernelGGL(k_mirror_upper, dim3(grid_for(N * N)), dim3(256), 0, st, N, A);
  DCHK(hipGetLastError());
  return TC2_OK;
}

tc2_status to_host(double* host, const double* dev, size_t n, hipStream_t st) {
  if (!host) return TC2_OK;
  DCHK(hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, st));
  DCHK(hipStreamSynchronize(st));
  return TC2_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  return hipEventElapsedTime(&ms, a, b) == hipSuccess ? ms : 0.f;
}

tc2_status dense_impl(const tc2_problem* p, const tc2_dense_options* o, tc2_dense_result* r) {
  const int b = p->H.b, nb = p->H.nb, D = p->n_dir;
  if (b < 1 || b > 16 || nb < 1 || D < 0 || D > 3) return TC2_EINVAL;
  const long long N = (long long)nb * b;
  if (N > TC2_DENSE_MAX_N) return TC2_EINVAL;
  if (p->n_occ < 0 || p->n_occ > N) return TC2_EINVAL;
  if (tc2_status st = tc2::validate_bsr(p->H, nb, b); st != TC2_OK) return st;
  if (!tc2::has_diag(p->H, nb)) return TC2_ENONSYM;
  for (int d = 0; d < D; ++d)
    if (tc2_status st = tc2::validate_bsr(p->H1[d], nb, b); st != TC2_OK) return st;
  if (tc2_status st = tc2::select_gfx950(o->device, nullptr); st != TC2_OK) return st;

  Call call;
  hipStream_t st = (hipStream_t)o->hip_stream;
  if (!st) {
    DCHK(hipStreamCreateWithFlags(&call.own, hipStreamNonBlocking));
    st = call.own;
  }
  for (hipEvent_t& e : call.ev) DCHK(hipEventCreate(&e));
  BCHK(rocblas_create_handle(&call.h));
  BCHK(rocblas_set_stream(call.h, st));

  const long long no = p->n_occ, nv = N - no;
  DenseBsr H, H1[3];
  if (tc2_status s = upload_bsr(p->H, st, H); s != TC2_OK) return s;
  for (int d = 0; d < D; ++d)
    if (tc2_status s = upload_bsr(p->H1[d], st, H1[d]); s != TC2_OK) return s;
  Dev A, P, part, e;
  DCHK(A.alloc((size_t)N * N * sizeof(double)));
  DCHK(P.alloc((size_t)N * N * sizeof(double)));
  DCHK(part.alloc(TR_BLOCKS * sizeof(double)));
  DCHK(e.alloc((size_t)N * sizeof(double)));

  DCHK(hipEventRecord(call.ev[0], st));
  std::vector<double> eh((size_t)N, 0.0);
  const bool trivial = no == 0 || no == N;
  if (!trivial) {
    // ---- eigenpairs: A <- C (columns), e ascending
    Dev work, info;
    DCHK(work.alloc((size_t)N * sizeof(double)));
    DCHK(info.alloc(sizeof(int)));
    if (tc2_status s = densify(H, b, N, st, A.d()); s != TC2_OK) return s;
    BCHK(rocsolver_dsyevd(call.h, rocblas_evect_original, rocblas_fill_upper, (rocblas_int)N,
                          A.d(), (rocblas_int)N, e.d(), work.d(), info.i()));
    int hinfo = 0;
    DCHK(hipMemcpyAsync(&hinfo, info.p, sizeof(int), hipMemcpyDeviceToHost, st));
    DCHK(hipMemcpyAsync(eh.data(), e.p, (size_t)N * sizeof(double), hipMemcpyDeviceToHost, st));
    DCHK(hipStreamSynchronize(st));
    if (hinfo != 0) return TC2_EDEVICE;
    r->gap = eh[(size_t)no] - eh[(size_t)no - 1];
    if (!(r->gap > 0.0)) return TC2_EDEGENERATE;
  }
  DCHK(hipEventRecord(call.ev[1], st));

  // ---- P0
  if (no == 0) {
    DCHK(hipMemsetAsync(P.p, 0, (size_t)N * N * sizeof(double), st));
  } else if (no == N) {
    hipLaunchKernelGGL(k_identity, dim3(grid_for(N * N)), dim3(256), 0, st, N, P.d());
    DCHK(hipGetLastError());
  } else {
    const double one = 1.0, zero = 0.0;
    BCHK(rocblas_dsyrk(call.h, rocblas_fill_upper, rocblas_operation_none, (rocblas_int)N,
                       (rocblas_int)no, &one, A.d(), (rocblas_int)N, &zero, P.d(), (rocblas_int)N));
    if (tc2_status s = mirror(N, P.d(), st); s != TC2_OK) return s;
  }
  if (tc2_status s = trace(H, b, N, P.d(), part.d(), st, &r->e0); s != TC2_OK) return s;
  {
    // Tr P0 from the diagonal: the trace of P0 against the identity pattern
    std::vector<double> diag((size_t)N);
    DCHK(hipMemcpy2DAsync(diag.data(), sizeof(double), P.p, (size_t)(N + 1) * sizeof(double),
                          sizeof(double), (size_t)N, hipMemcpyDeviceToHost, st));
    DCHK(hipStreamSynchronize(st));
    double t = 0.0;
    for (double v : diag) t += v;
    r->tr_p0 = t;
  }
  if (tc2_status s = to_host(o->p0, P.d(), (size_t)N * N, st); s != TC2_OK) return s;
  DCHK(hipEventRecord(call.ev[2], st));

  // ---- P1_d
  if (D > 0) {
    Dev H1d, T, G, Y;
    if (!trivial) {
      DCHK(H1d.alloc((size_t)N * N * sizeof(double)));
      DCHK(T.alloc((size_t)N * no * sizeof(double)));
      DCHK(G.alloc((size_t)nv * no * sizeof(double)));
      DCHK(Y.alloc((size_t)N * no * sizeof(double)));
    }
    for (int d = 0; d < D; ++d) {
      if (trivial) {
        DCHK(hipMemsetAsync(P.p, 0, (size_t)N * N * sizeof(double), st));
      } else {
        const double one = 1.0, zero = 0.0;
        const double* Cocc = A.d();
        const double* Cvirt = A.d() + no * N;
        if (tc2_status s = densify(H1[d], b, N, st, H1d.d()); s != TC2_OK) return s;
        BCHK(rocblas_dgemm(call.h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)N,
                           (rocblas_int)no, (rocblas_int)N, &one, H1d.d(), (rocblas_int)N, Cocc,
                           (rocblas_int)N, &zero, T.d(), (rocblas_int)N));
        BCHK(rocblas_dgemm(call.h, rocblas_operation_transpose, rocblas_operation_none,
                           (rocblas_int)nv, (rocblas_int)no, (rocblas_int)N, &one, Cvirt,
                           (rocblas_int)N, T.d(), (rocblas_int)N, &zero, G.d(), (rocblas_int)nv));
        hipLaunchKernelGGL(k_gap_scale, dim3(grid_for(nv * no)), dim3(256), 0, st, nv, no, e.d(),
                           G.d());
        DCHK(hipGetLastError());
        BCHK(rocblas_dgemm(call.h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)N,
                           (rocblas_int)no, (rocblas_int)nv, &one, Cvirt, (rocblas_int)N, G.d(),
                           (rocblas_int)nv, &zero, Y.d(), (rocblas_int)N));
        BCHK(rocblas_dsyr2k(call.h, rocblas_fill_upper, rocblas_operation_none, (rocblas_int)N,
                            (rocblas_int)no, &one, Y.d(), (rocblas_int)N, Cocc, (rocblas_int)N,
                            &zero, P.d(), (rocblas_int)N));
        if (tc2_status s = mirror(N, P.d(), st); s != TC2_OK) return s;
        // T = H1 C_occ (2 N^2 no), G (2 N nv no), Y (2 N nv no), P1 (2 N^2 no)
        r->flops_p1 += 4.0 * (double)N * N * no + 4.0 * (double)N * nv * no;
      }
      if (tc2_status s = trace(H, b, N, P.d(), part.d(), st, &r->e1[d]); s != TC2_OK) return s;
      if (tc2_status s = trace(H1[d], b, N, P.d(), part.d(), st, &r->trace_p1h1[d]); s != TC2_OK)
        return s;
      if (tc2_status s = to_host(o->p1[d], P.d(), (size_t)N * N, st); s != TC2_OK) return s;
    }
  }
  DCHK(hipEventRecord(call.ev[3], st));
  DCHK(hipEventSynchronize(call.ev[3]));
  r->ms_eigh = elapsed(call.ev[0], call.ev[1]);
  r->ms_p0 = elapsed(call.ev[1], call.ev[2]);
  r->ms_p1 = elapsed(call.ev[2], call.ev[3]);
  r->seconds = elapsed(call.ev[0], call.ev[3]) * 1e-3;
  if (o->eigenvalues && !trivial) std::memcpy(o->eigenvalues, eh.data(), (size_t)N * sizeof(double));
  return TC2_OK;
}

}  // namespace

extern "C" TC2_API tc2_status tc2_dense_response(const tc2_problem* problem,
                                                 const tc2_dense_options* opts,
                                                 tc2_dense_result* res) {
  if (!problem || !opts || !res) return TC2_EINVAL;
  std::memset(res, 0, sizeof(*res));
  tc2_status s;
  try {
    s = dense_impl(problem, opts, res);
  } catch (...) {
    s = TC2_ENOMEM;
  }
  res->status = s;
  return s;
}
