// Loewdin orthogonalisation for a non-orthogonal basis (Sec. 2.2): the
// orthogonal forms H_orth = S^-1/2 H S^-1/2 and H1_orth = S^-1/2 H1 S^-1/2
// that the TC2 cycles take, with S^-1/2 from a Newton-Schulz iteration of
// block-sparse products, and the back-transform P = S^-1/2 P_orth S^-1/2 of
// the converged density matrices.
//
// Every product C = A B is an atom-block-sparse product with the block filter
// of Sec. 2.3 (an off-diagonal block whose Frobenius norm is below eps is
// dropped).  B is always symmetric, so B_KJ is read as the transpose of the
// stored B_JK, and C_IJ sums A_IK B_JK^T over the columns K common to row I of
// A and row J of B (the MFMA operand layout of the TC2 kernels).  A product
// whose exact value is symmetric is computed on the upper blocks only and
// mirrored, so that it is exactly symmetric.
//
// Per product, on the device: symbolic pattern (union of rows, an LDS bitmap
// per output row), numeric blocks (one wave per candidate output block, FP64
// MFMA), then a gather into the kept (and, for symmetric products, mirrored)
// pattern.  The host assembles the kept pattern from the keep flags.
#include "tc2_device.h"
#include "tc2_host.h"
#include "../../include/tc2.h"

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

using namespace tc2;

namespace {

constexpr int GT = 256;               // threads of the symbolic kernel
constexpr int MAX_NB = 1 << 18;       // block rows (LDS bitmap of 32 KiB)

// ------------------------------------------------------------------ kernels
// Row-major b x b blocks -> padded column-major 16 x 16 tiles, and back.
__global__ void k_pack(long long n, int b, const double* val, double* v) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n * BS; k += stride) {
    const long long e = k / BS;
    const int q = (int)(k - e * BS), c = q / BP, r = q - c * BP;
    v[k] = (r < b && c < b) ? val[e * b * b + r * b + c] : 0.0;
  }
}

__global__ void k_unpack(long long n, int b, const double* v, double* val) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n * b * b; k += stride) {
    const long long e = k / (b * b);
    const int q = (int)(k - e * b * b), r = q / b, c = q - r * b;
    val[k] = v[e * BS + c * BP + r];
  }
}

// Operands of C = A B (+ A2 B2): row pointers, columns and values of A and B,
// and of the optional second pair (np = 1 or 2).
struct Pairs {
  int np;
  const int* arp[2];
  const int* aci[2];
  const double* av[2];
  const int* brp[2];
  const int* bci[2];
  const double* bv[2];
};

// Pattern of C, one workgroup per row I: the union, over the pairs and over K
// in row I of A, of row K of B (only J >= I when `upper`).  Pass 0 counts the
// columns of each row; pass 1 writes them, ascending, from C_rp.
__global__ __launch_bounds__(GT) void k_gp_symbolic(int pass, int nb, Pairs g, int upper,
                                                    int* cnt, const int* Crp, int* Cci) {
  extern __shared__ unsigned bits[];
  __shared__ int ssum[GT];
  const int I = blockIdx.x, t = threadIdx.x;
  const int nwords = (nb + 31) >> 5;
  for (int w = t; w < nwords; w += GT) bits[w] = 0u;
  __syncthreads();
  for (int k = 0; k < g.np; ++k) {
    const int *Arp = g.arp[k], *Aci = g.aci[k], *Brp = g.brp[k], *Bci = g.bci[k];
    for (int p = Arp[I]; p < Arp[I + 1]; ++p) {
      const int K = Aci[p];
      for (int q = Brp[K] + t; q < Brp[K + 1]; q += GT) {
        const int J = Bci[q];
        if (!upper || J >= I) atomicOr(&bits[J >> 5], 1u << (J & 31));
      }
    }
  }
  __syncthreads();
  const int wpt = (nwords + GT - 1) / GT;
  const int w0 = min(nwords, t * wpt), w1 = min(nwords, w0 + wpt);
  int c = 0;
  for (int w = w0; w < w1; ++w) c += __popc(bits[w]);
  ssum[t] = c;
  __syncthreads();
  for (int o = 1; o < GT; o <<= 1) {  // inclusive scan
    const int u = t >= o ? ssum[t - o] : 0;
    __syncthreads();
    ssum[t] += u;
    __syncthreads();
  }
  if (pass == 0) {
    if (t == GT - 1) cnt[I] = ssum[t];
    return;
  }
  int pos = Crp[I] + ssum[t] - c;
  for (int w = w0; w < w1; ++w) {
    unsigned x = bits[w];
    while (x) {
      const int bit = __ffs(x) - 1;
      x &= x - 1;
      Cci[pos++] = (w << 5) + bit;
    }
  }
}

// Numeric blocks of the candidate entries of C (one wave per entry): the sum,
// over the pairs and the columns K common to row I of A and row J of B, of
// A_IK B_JK^T; then (sym) the upper scalar triangle of a diagonal block
// mirrored onto its lower one, the Frobenius norm and the keep flag (diagonal
// blocks are always kept).
__global__ __launch_bounds__(256) void k_gp_numeric(long long nnz, const int* Crow, const int* Cci,
                                                    Pairs g, int sym, double eps, double* Cv,
                                                    int* keep) {
  __shared__ double stage[4][BS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long nw = (long long)gridDim.x * 4;
  for (long long e = (long long)blockIdx.x * 4 + wave; e < nnz; e += nw) {
    const int I = Crow[e], J = Cci[e];
    Acc<double> acc;
    acc.v = d4{0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < g.np; ++k) {
      const int* Aci = g.aci[k];
      const int* Bci = g.bci[k];
      const double* Av = g.av[k];
      const double* Bv = g.bv[k];
      const int a0 = g.arp[k][I], a1 = g.arp[k][I + 1];
      const int b0 = g.brp[k][J], nbj = g.brp[k][J + 1] - b0;
      for (int c0 = a0; c0 < a1; c0 += 64) {
        const int p = c0 + lane;
        int q = -1;
        if (p < a1) {
          const int f = bsearch_eq(Bci + b0, nbj, Aci[p]);
          q = f >= 0 ? b0 + f : -1;
        }
        unsigned long long m = __ballot(q >= 0);
        while (m) {
          const int l = __ffsll((long long)m) - 1;
          m &= m - 1;
          const long long pp = __builtin_amdgcn_readlane(p, l);
          const long long qq = __builtin_amdgcn_readlane(q, l);
#pragma unroll
          for (int kk = 0; kk < 4; ++kk)
            mfma(acc, Av[pp * BS + lane + 64 * kk], Bv[qq * BS + lane + 64 * kk]);
        }
      }
    }
    double* st = stage[wave];
#pragma unroll
    for (int j = 0; j < 4; ++j) st[(lane & 15) * BP + Acc<double>::row(lane, j)] = acc.v[j];
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    double v[4], ss = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = lane + 64 * i, c = idx / BP, r = idx - c * BP;
      v[i] = (sym && I == J && r > c) ? st[r * BP + c] : st[idx];
      ss += v[i] * v[i];
    }
    ss = wave_sum(ss);
    const bool kept = I == J || sqrt(ss) >= eps;
#pragma unroll
    for (int i = 0; i < 4; ++i) Cv[e * BS + lane + 64 * i] = v[i];
    if (lane == 0) keep[e] = kept ? 1 : 0;
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // stage reads done before reuse
  }
}

// out[e] = in[src[e]], transposed where src[e] has bit 31 set.
__global__ __launch_bounds__(256) void k_gp_gather(long long n, const unsigned* src,
                                                   const double* in, double* out) {
  const int lane = threadIdx.x & 63;
  const long long nw = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long e = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; e < n; e += nw) {
    const unsigned s = src[e];
    const long long from = (long long)(s & 0x7fffffffu) * BS;
    const bool tr = (s >> 31) != 0u;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = lane + 64 * i, c = idx / BP, r = idx - c * BP;
      out[e * BS + idx] = in[from + (tr ? r * BP + c : idx)];
    }
  }
}

// v <- alpha v, plus beta on the scalar diagonal (r = c < b) of diagonal blocks.
__global__ void k_affine(long long n, int b, const int* row, const int* ci, double alpha,
                         double beta, double* v) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n * BS; k += stride) {
    const long long e = k / BS;
    const int q = (int)(k - e * BS), c = q / BP, r = q - c * BP;
    const double d = (row[e] == ci[e] && r == c && r < b) ? beta : 0.0;
    v[k] = alpha * v[k] + d;
  }
}

// Partial sums of (C - I)^2 over the stored elements, one per workgroup.
__global__ __launch_bounds__(256) void k_resid(long long n, int b, const int* row, const int* ci,
                                               const double* v, double* partial) {
  __shared__ double red[256];
  double s = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n * BS; k += stride) {
    const long long e = k / BS;
    const int q = (int)(k - e * BS), c = q / BP, r = q - c * BP;
    const double x = v[k] - ((row[e] == ci[e] && r == c && r < b) ? 1.0 : 0.0);
    s += x * x;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

unsigned grid_for(long long n, int per_block = 256) {
  const long long g = (n + per_block - 1) / per_block;
  return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

// ------------------------------------------------------------------ host side
#define LCHK(x)                                                                   \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) return e_ == hipErrorOutOfMemory ? TC2_ENOMEM : TC2_EDEVICE; \
  } while (0)

struct Buf {  // device allocation released with its owner
  void* p = nullptr;
  ~Buf() {
    if (p) (void)hipFree(p);
  }
  Buf() = default;
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  Buf(Buf&& o) noexcept : p(o.p) { o.p = nullptr; }
  Buf& operator=(Buf&& o) noexcept {
    if (this != &o) {
      if (p) (void)hipFree(p);
      p = o.p;
      o.p = nullptr;
    }
    return *this;
  }
  hipError_t alloc(size_t bytes) {
    if (p) (void)hipFree(p);
    p = nullptr;
    return tc2::dev_malloc(&p, bytes ? bytes : 8);
  }
  int* i() const { return (int*)p; }
  double* d() const { return (double*)p; }
};

// A block-sparse matrix on the device (full pattern, padded column-major
// values) with host copies of its pattern.
struct GMat {
  int nb = 0, b = 0;
  std::vector<int> rp, ci, row;  // host
  Buf drp, dci, drow, v;         // device
  long long nnz() const { return rp.empty() ? 0 : rp.back(); }
};

struct Ctx {
  hipStream_t st = nullptr;
  hipStream_t own = nullptr;
  Buf part, cnt, keep, src;
  std::vector<int> hcnt;
  ~Ctx() {
    if (own) (void)hipStreamDestroy(own);
  }
};

tc2_status upload_pattern(GMat& m, hipStream_t st) {
  const long long nnz = m.nnz();
  m.row.assign((size_t)nnz, 0);
  for (int i = 0; i < m.nb; ++i)
    for (int p = m.rp[i]; p < m.rp[i + 1]; ++p) m.row[(size_t)p] = i;
  LCHK(m.drp.alloc(m.rp.size() * sizeof(int)));
  LCHK(m.dci.alloc((size_t)nnz * sizeof(int)));
  LCHK(m.drow.alloc((size_t)nnz * sizeof(int)));
  LCHK(hipMemcpyAsync(m.drp.p, m.rp.data(), m.rp.size() * sizeof(int), hipMemcpyHostToDevice, st));
  if (nnz) {
    LCHK(hipMemcpyAsync(m.dci.p, m.ci.data(), (size_t)nnz * sizeof(int), hipMemcpyHostToDevice, st));
    LCHK(hipMemcpyAsync(m.drow.p, m.row.data(), (size_t)nnz * sizeof(int), hipMemcpyHostToDevice,
                        st));
  }
  LCHK(hipStreamSynchronize(st));  // the host vectors may change after return
  return TC2_OK;
}

tc2_status from_bsr(const tc2_bsr& a, hipStream_t st, GMat& m) {
  m.nb = a.nb;
  m.b = a.b;
  const long long nnz = a.row_ptr[a.nb];
  m.rp.resize((size_t)a.nb + 1);
  for (int i = 0; i <= a.nb; ++i) m.rp[(size_t)i] = (int)a.row_ptr[i];
  m.ci.assign(a.col, a.col + nnz);
  if (tc2_status s = upload_pattern(m, st); s != TC2_OK) return s;
  Buf raw;
  LCHK(raw.alloc((size_t)nnz * a.b * a.b * sizeof(double)));
  LCHK(m.v.alloc((size_t)nnz * BS * sizeof(double)));
  if (nnz) {
    LCHK(hipMemcpyAsync(raw.p, a.val, (size_t)nnz * a.b * a.b * sizeof(double),
                        hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_pack, dim3(grid_for(nnz * BS)), dim3(256), 0, st, nnz, a.b, raw.d(),
                       m.v.d());
    LCHK(hipGetLastError());
  }
  LCHK(hipStreamSynchronize(st));
  return TC2_OK;
}

tc2_status identity(int nb, int b, hipStream_t st, GMat& m) {
  m.nb = nb;
  m.b = b;
  m.rp.resize((size_t)nb + 1);
  m.ci.resize((size_t)nb);
  for (int i = 0; i <= nb; ++i) m.rp[(size_t)i] = i;
  for (int i = 0; i < nb; ++i) m.ci[(size_t)i] = i;
  if (tc2_status s = upload_pattern(m, st); s != TC2_OK) return s;
  LCHK(m.v.alloc((size_t)nb * BS * sizeof(double)));
  LCHK(hipMemsetAsync(m.v.p, 0, (size_t)nb * BS * sizeof(double), st));
  hipLaunchKernelGGL(k_affine, dim3(grid_for((long long)nb * BS)), dim3(256), 0, st,
                     (long long)nb, b, m.drow.i(), m.dci.i(), 1.0, 1.0, m.v.d());
  LCHK(hipGetLastError());
  return TC2_OK;
}

tc2_status copy_scaled(const GMat& a, double s, hipStream_t st, GMat& m) {
  m.nb = a.nb;
  m.b = a.b;
  m.rp = a.rp;
  m.ci = a.ci;
  if (tc2_status r = upload_pattern(m, st); r != TC2_OK) return r;
  LCHK(m.v.alloc((size_t)a.nnz() * BS * sizeof(double)));
  if (a.nnz()) {
    LCHK(hipMemcpyAsync(m.v.p, a.v.p, (size_t)a.nnz() * BS * sizeof(double),
                        hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_affine, dim3(grid_for(a.nnz() * BS)), dim3(256), 0, st, a.nnz(), a.b,
                       m.drow.i(), m.dci.i(), s, 0.0, m.v.d());
    LCHK(hipGetLastError());
  }
  return TC2_OK;
}

// C = A B (+ A2 B2) with the block filter applied to the sum; sym: upper
// blocks computed and mirrored.
tc2_status product(Ctx& x, const GMat& A, const GMat& B, bool sym, double eps, GMat& C,
                   const GMat* A2 = nullptr, const GMat* B2 = nullptr) {
  hipStream_t st = x.st;
  const int nb = A.nb;
  Pairs g{};
  g.np = A2 ? 2 : 1;
  const GMat* as[2] = {&A, A2};
  const GMat* bs[2] = {&B, B2};
  for (int k = 0; k < g.np; ++k) {
    g.arp[k] = as[k]->drp.i();
    g.aci[k] = as[k]->dci.i();
    g.av[k] = as[k]->v.d();
    g.brp[k] = bs[k]->drp.i();
    g.bci[k] = bs[k]->dci.i();
    g.bv[k] = bs[k]->v.d();
  }
  const size_t shm = (size_t)((nb + 31) >> 5) * sizeof(unsigned);
  LCHK(x.cnt.alloc((size_t)nb * sizeof(int)));
  hipLaunchKernelGGL(k_gp_symbolic, dim3(nb), dim3(GT), shm, st, 0, nb, g, sym ? 1 : 0,
                     x.cnt.i(), nullptr, nullptr);
  LCHK(hipGetLastError());
  x.hcnt.resize((size_t)nb);
  LCHK(hipMemcpyAsync(x.hcnt.data(), x.cnt.p, (size_t)nb * sizeof(int), hipMemcpyDeviceToHost, st));
  LCHK(hipStreamSynchronize(st));
  GMat cand;
  cand.nb = nb;
  cand.b = A.b;
  cand.rp.assign((size_t)nb + 1, 0);
  long long tot = 0;
  for (int i = 0; i < nb; ++i) {
    tot += x.hcnt[(size_t)i];
    if (tot > 0x7ffffffeLL) return TC2_EOVERFLOW;
    cand.rp[(size_t)i + 1] = (int)tot;
  }
  LCHK(cand.drp.alloc(cand.rp.size() * sizeof(int)));
  LCHK(hipMemcpyAsync(cand.drp.p, cand.rp.data(), cand.rp.size() * sizeof(int),
                      hipMemcpyHostToDevice, st));
  LCHK(cand.dci.alloc((size_t)tot * sizeof(int)));
  hipLaunchKernelGGL(k_gp_symbolic, dim3(nb), dim3(GT), shm, st, 1, nb, g, sym ? 1 : 0, nullptr,
                     cand.drp.i(), cand.dci.i());
  LCHK(hipGetLastError());
  cand.ci.resize((size_t)tot);
  if (tot)
    LCHK(hipMemcpyAsync(cand.ci.data(), cand.dci.p, (size_t)tot * sizeof(int),
                        hipMemcpyDeviceToHost, st));
  LCHK(hipStreamSynchronize(st));
  cand.row.assign((size_t)tot, 0);
  for (int i = 0; i < nb; ++i)
    for (int p = cand.rp[(size_t)i]; p < cand.rp[(size_t)i + 1]; ++p) cand.row[(size_t)p] = i;
  LCHK(cand.drow.alloc((size_t)tot * sizeof(int)));
  if (tot)
    LCHK(hipMemcpyAsync(cand.drow.p, cand.row.data(), (size_t)tot * sizeof(int),
                        hipMemcpyHostToDevice, st));
  LCHK(cand.v.alloc((size_t)tot * BS * sizeof(double)));
  LCHK(x.keep.alloc((size_t)tot * sizeof(int)));
  if (tot) {
    hipLaunchKernelGGL(k_gp_numeric, dim3(grid_for(tot, 4)), dim3(256), 0, st, tot,
                       cand.drow.i(), cand.dci.i(), g, sym ? 1 : 0, eps, cand.v.d(),
                       x.keep.i());
    LCHK(hipGetLastError());
  }
  std::vector<int> keep((size_t)tot);
  if (tot)
    LCHK(hipMemcpyAsync(keep.data(), x.keep.p, (size_t)tot * sizeof(int), hipMemcpyDeviceToHost, st));
  LCHK(hipStreamSynchronize(st));

  // kept pattern: as is, or the kept upper blocks and their mirrors
  C.nb = nb;
  C.b = A.b;
  std::vector<unsigned> src;
  C.rp.assign((size_t)nb + 1, 0);
  C.ci.clear();
  if (!sym) {
    for (int i = 0; i < nb; ++i) {
      for (int p = cand.rp[(size_t)i]; p < cand.rp[(size_t)i + 1]; ++p)
        if (keep[(size_t)p]) {
          C.ci.push_back(cand.ci[(size_t)p]);
          src.push_back((unsigned)p);
        }
      C.rp[(size_t)i + 1] = (int)C.ci.size();
    }
  } else {
    // lower part of row J: kept upper blocks (I, J), I < J, in increasing I
    std::vector<std::vector<int>> low((size_t)nb);
    for (int i = 0; i < nb; ++i)
      for (int p = cand.rp[(size_t)i]; p < cand.rp[(size_t)i + 1]; ++p)
        if (keep[(size_t)p] && cand.ci[(size_t)p] > i) low[(size_t)cand.ci[(size_t)p]].push_back(p);
    for (int j = 0; j < nb; ++j) {
      for (int p : low[(size_t)j]) {
        C.ci.push_back(cand.row[(size_t)p]);
        src.push_back((unsigned)p | 0x80000000u);
      }
      for (int p = cand.rp[(size_t)j]; p < cand.rp[(size_t)j + 1]; ++p)
        if (keep[(size_t)p]) {
          C.ci.push_back(cand.ci[(size_t)p]);
          src.push_back((unsigned)p);
        }
      if (C.ci.size() > 0x7ffffffeULL) return TC2_EOVERFLOW;
      C.rp[(size_t)j + 1] = (int)C.ci.size();
    }
  }
  if (tc2_status s = upload_pattern(C, st); s != TC2_OK) return s;
  const long long n = C.nnz();
  LCHK(C.v.alloc((size_t)n * BS * sizeof(double)));
  LCHK(x.src.alloc((size_t)n * sizeof(unsigned)));
  if (n) {
    LCHK(hipMemcpyAsync(x.src.p, src.data(), (size_t)n * sizeof(unsigned), hipMemcpyHostToDevice,
                        st));
    hipLaunchKernelGGL(k_gp_gather, dim3(grid_for(n, 4)), dim3(256), 0, st, n,
                       (const unsigned*)x.src.p, cand.v.d(), C.v.d());
    LCHK(hipGetLastError());
  }
  LCHK(hipStreamSynchronize(st));  // src and cand are released on return
  return TC2_OK;
}

// ||C - I||_F
tc2_status resid_norm(Ctx& x, const GMat& C, double* out) {
  constexpr int NBLK = 256;
  LCHK(x.part.alloc(NBLK * sizeof(double)));
  double h[NBLK];
  if (C.nnz() == 0) {
    *out = std::sqrt((double)C.nb * C.b);
    return TC2_OK;
  }
  hipLaunchKernelGGL(k_resid, dim3(NBLK), dim3(256), 0, x.st, C.nnz(), C.b, C.drow.i(),
                     C.dci.i(), C.v.d(), x.part.d());
  LCHK(hipGetLastError());
  LCHK(hipMemcpyAsync(h, x.part.p, sizeof(h), hipMemcpyDeviceToHost, x.st));
  LCHK(hipStreamSynchronize(x.st));
  double s = 0.0;
  for (double v : h) s += v;
  *out = std::sqrt(s);
  return TC2_OK;
}

// Library-allocated host copy (row-major b x b blocks); tc2_bsr_release frees it.
tc2_status to_host(Ctx& x, const GMat& m, tc2_bsr* out) {
  const long long nnz = m.nnz();
  int64_t* rp = (int64_t*)malloc(sizeof(int64_t) * ((size_t)m.nb + 1));
  int32_t* ci = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
  double* val = (double*)malloc(sizeof(double) * (size_t)(nnz ? nnz * m.b * m.b : 1));
  if (!rp || !ci || !val) {
    free(rp);
    free(ci);
    free(val);
    return TC2_ENOMEM;
  }
  for (int i = 0; i <= m.nb; ++i) rp[i] = m.rp[(size_t)i];
  for (long long p = 0; p < nnz; ++p) ci[p] = m.ci[(size_t)p];
  Buf raw;
  hipError_t e = raw.alloc((size_t)nnz * m.b * m.b * sizeof(double));
  if (e == hipSuccess && nnz) {
    hipLaunchKernelGGL(k_unpack, dim3(grid_for(nnz * m.b * m.b)), dim3(256), 0, x.st, nnz, m.b,
                       m.v.d(), raw.d());
    e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(val, raw.p, (size_t)nnz * m.b * m.b * sizeof(double),
                         hipMemcpyDeviceToHost, x.st);
    if (e == hipSuccess) e = hipStreamSynchronize(x.st);
  }
  if (e != hipSuccess) {
    free(rp);
    free(ci);
    free(val);
    return e == hipErrorOutOfMemory ? TC2_ENOMEM : TC2_EDEVICE;
  }
  out->nb = m.nb;
  out->b = m.b;
  out->row_ptr = rp;
  out->col = ci;
  out->val = val;
  return TC2_OK;
}

tc2_status check_opts(const tc2_lowdin_options* o, bool need_tol) {
  if (!o) return TC2_EINVAL;
  if (!(o->eps >= 0.0) || !std::isfinite(o->eps)) return TC2_EINVAL;
  if (need_tol && (!(o->tol > 0.0) || o->max_iter < 1 || o->max_iter > TC2_MAX_ITER))
    return TC2_EINVAL;
  return TC2_OK;
}

tc2_status start(const tc2_lowdin_options* o, Ctx& x) {
  if (tc2_status s = select_gfx950(o->device, nullptr); s != TC2_OK) return s;
  x.st = (hipStream_t)o->hip_stream;
  if (!x.st) {
    LCHK(hipStreamCreateWithFlags(&x.own, hipStreamNonBlocking));
    x.st = x.own;
  }
  return TC2_OK;
}

void release(tc2_bsr* m) {
  if (!m) return;
  free((void*)m->row_ptr);
  free((void*)m->col);
  free((void*)m->val);
  std::memset(m, 0, sizeof(*m));
}

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// The zero matrix (empty pattern).
tc2_status zero(int nb, int b, hipStream_t st, GMat& m) {
  m.nb = nb;
  m.b = b;
  m.rp.assign((size_t)nb + 1, 0);
  m.ci.clear();
  if (tc2_status s = upload_pattern(m, st); s != TC2_OK) return s;
  LCHK(m.v.alloc(0));
  return TC2_OK;
}

tc2_status scale(GMat& m, double s, hipStream_t st) {
  if (m.nnz() == 0) return TC2_OK;
  hipLaunchKernelGGL(k_affine, dim3(grid_for(m.nnz() * BS)), dim3(256), 0, st, m.nnz(), m.b,
                     m.drow.i(), m.dci.i(), s, 0.0, m.v.d());
  LCHK(hipGetLastError());
  return TC2_OK;
}

// Where tc2_lowdin and tc2_lowdin_response put their outputs.
struct LowdinOut {
  int32_t* iters;
  double *resid, *lambda, *seconds;
  tc2_bsr *Z, *H, *H1, *Z1;  // Z1: NULL for a field perturbation
};

// S^-1/2 by the coupled Newton-Schulz iteration and, with S1, its derivative
// along each S1_d (the same updates differentiated: M1 = Z1 Y + Z Y1,
// T1 = -M1/2, Y1 <- Y1 T + Y T1, Z1 <- Z1 T + Z T1); then the orthogonal forms
// Z H Z and, per direction, Z H1_d Z or (with S1) Z1 H Z + Z H1_d Z + Z H Z1.
tc2_status lowdin_core(const tc2_bsr* S, const tc2_bsr* H, int32_t n_dir, const tc2_bsr* H1,
                       const tc2_bsr* S1, const tc2_lowdin_options* o, LowdinOut out) {
  if (!S || !H || (n_dir > 0 && !H1) || n_dir < 0 || n_dir > 3) return TC2_EINVAL;
  if (tc2_status s = check_opts(o, true); s != TC2_OK) return s;
  const int nb = S->nb, b = S->b;
  if (nb < 1 || b < 1 || b > BP || nb > MAX_NB) return TC2_EINVAL;
  if (tc2_status s = validate_bsr(*S, nb, b); s != TC2_OK) return s;
  if (!has_diag(*S, nb)) return TC2_ENONSYM;
  if (tc2_status s = validate_bsr(*H, nb, b); s != TC2_OK) return s;
  for (int d = 0; d < n_dir; ++d) {
    if (tc2_status s = validate_bsr(H1[d], nb, b); s != TC2_OK) return s;
    if (S1)
      if (tc2_status s = validate_bsr(S1[d], nb, b); s != TC2_OK) return s;
  }
  // Gershgorin upper bound of S over its scalar rows
  double lam = 0.0;
  for (int i = 0; i < nb; ++i)
    for (int rr = 0; rr < b; ++rr) {
      double c = 0.0, rad = 0.0;
      for (int64_t p = S->row_ptr[i]; p < S->row_ptr[i + 1]; ++p)
        for (int cc = 0; cc < b; ++cc) {
          const double v = S->val[(p * b + rr) * b + cc];
          if (S->col[p] == i && cc == rr) c = v; else rad += std::fabs(v);
        }
      lam = std::max(lam, c + rad);
    }
  if (!(lam > 0.0)) return TC2_EDEGENERATE;
  *out.lambda = lam;
  const int nd = S1 ? n_dir : 0;  // derivative directions

  Ctx x;
  if (tc2_status s = start(o, x); s != TC2_OK) return s;
  Events ev;
  LCHK(hipEventCreate(&ev.a));
  LCHK(hipEventCreate(&ev.b));
  GMat gS, gH, gS1[3];
  if (tc2_status s = from_bsr(*S, x.st, gS); s != TC2_OK) return s;
  if (tc2_status s = from_bsr(*H, x.st, gH); s != TC2_OK) return s;
  for (int d = 0; d < nd; ++d)
    if (tc2_status s = from_bsr(S1[d], x.st, gS1[d]); s != TC2_OK) return s;
  LCHK(hipEventRecord(ev.a, x.st));
  GMat Y, Z, Y1[3], Z1[3];
  if (tc2_status s = copy_scaled(gS, 1.0 / lam, x.st, Y); s != TC2_OK) return s;
  if (tc2_status s = identity(nb, b, x.st, Z); s != TC2_OK) return s;
  for (int d = 0; d < nd; ++d) {
    if (tc2_status s = copy_scaled(gS1[d], 1.0 / lam, x.st, Y1[d]); s != TC2_OK) return s;
    if (tc2_status s = zero(nb, b, x.st, Z1[d]); s != TC2_OK) return s;
  }
  const double sqN = std::sqrt((double)nb * b);
  tc2_status status = TC2_OK;
  int iters = 0;
  double prev = -1.0;
  for (;;) {
    GMat M;
    if (tc2_status s = product(x, Z, Y, true, o->eps, M); s != TC2_OK) return s;
    double res = 0.0;
    if (tc2_status s = resid_norm(x, M, &res); s != TC2_OK) return s;
    *out.resid = res / sqN;
    if (!std::isfinite(*out.resid)) return TC2_ENAN;
    if (*out.resid < o->tol) break;
    // stall guard: the last update did not halve the residual, so the filter
    // or rounding sets it now
    if (prev >= 0.0 && *out.resid > 0.5 * prev) {
      status = TC2_FLOOR_REACHED;
      break;
    }
    prev = *out.resid;
    if (iters == o->max_iter) {
      status = TC2_NOT_CONVERGED;
      break;
    }
    // T = (3 I - M) / 2, in place
    hipLaunchKernelGGL(k_affine, dim3(grid_for(M.nnz() * BS)), dim3(256), 0, x.st, M.nnz(), b,
                       M.drow.i(), M.dci.i(), -0.5, 1.5, M.v.d());
    LCHK(hipGetLastError());
    for (int d = 0; d < nd; ++d) {
      GMat T1, Y1n, Z1n;  // T1 = -(Z1 Y + Z Y1)/2 from the current iterates
      if (tc2_status s = product(x, Z1[d], Y, true, o->eps, T1, &Z, &Y1[d]); s != TC2_OK) return s;
      if (tc2_status s = scale(T1, -0.5, x.st); s != TC2_OK) return s;
      if (tc2_status s = product(x, Y1[d], M, true, o->eps, Y1n, &Y, &T1); s != TC2_OK) return s;
      if (tc2_status s = product(x, Z1[d], M, true, o->eps, Z1n, &Z, &T1); s != TC2_OK) return s;
      Y1[d] = std::move(Y1n);
      Z1[d] = std::move(Z1n);
    }
    GMat Y2, Z2;
    if (tc2_status s = product(x, Y, M, true, o->eps, Y2); s != TC2_OK) return s;
    if (tc2_status s = product(x, Z, M, true, o->eps, Z2); s != TC2_OK) return s;
    Y = std::move(Y2);
    Z = std::move(Z2);
    ++iters;
  }
  *out.iters = iters;
  // S^-1/2 = Z / sqrt(lam), and its derivatives
  const double r = 1.0 / std::sqrt(lam);
  if (tc2_status s = scale(Z, r, x.st); s != TC2_OK) return s;
  for (int d = 0; d < nd; ++d)
    if (tc2_status s = scale(Z1[d], r, x.st); s != TC2_OK) return s;
  // orthogonal forms
  GMat Q, Ho, H1o[3];
  if (tc2_status s = product(x, Z, gH, false, o->eps, Q); s != TC2_OK) return s;
  if (tc2_status s = product(x, Q, Z, true, o->eps, Ho); s != TC2_OK) return s;
  for (int d = 0; d < n_dir; ++d) {
    GMat g, Q1;
    if (tc2_status s = from_bsr(H1[d], x.st, g); s != TC2_OK) return s;
    if (!S1) {  // Z H1 Z
      if (tc2_status s = product(x, Z, g, false, o->eps, Q1); s != TC2_OK) return s;
      if (tc2_status s = product(x, Q1, Z, true, o->eps, H1o[d]); s != TC2_OK) return s;
    } else {  // (Z1 H + Z H1) Z + (Z H) Z1
      if (tc2_status s = product(x, Z1[d], gH, false, o->eps, Q1, &Z, &g); s != TC2_OK) return s;
      if (tc2_status s = product(x, Q1, Z, true, o->eps, H1o[d], &Q, &Z1[d]); s != TC2_OK)
        return s;
    }
  }
  LCHK(hipEventRecord(ev.b, x.st));
  LCHK(hipEventSynchronize(ev.b));
  float ms = 0.f;
  LCHK(hipEventElapsedTime(&ms, ev.a, ev.b));
  *out.seconds = ms * 1e-3;
  if (tc2_status s = to_host(x, Z, out.Z); s != TC2_OK) return s;
  if (tc2_status s = to_host(x, Ho, out.H); s != TC2_OK) return s;
  for (int d = 0; d < n_dir; ++d) {
    if (tc2_status s = to_host(x, H1o[d], &out.H1[d]); s != TC2_OK) return s;
    if (S1)
      if (tc2_status s = to_host(x, Z1[d], &out.Z1[d]); s != TC2_OK) return s;
  }
  return status;
}

// Z X Z, or (with Z1 and X1) Z1 X Z + Z X1 Z + Z X Z1 = (Z1 X + Z X1) Z + (Z X) Z1.
tc2_status congruence_impl(const tc2_bsr* Zh, const tc2_bsr* Xh, const tc2_bsr* Z1h,
                           const tc2_bsr* X1h, const tc2_lowdin_options* o, tc2_bsr* out,
                           double* seconds) {
  if (!Zh || !Xh || !out || (!Z1h) != (!X1h)) return TC2_EINVAL;
  if (tc2_status s = check_opts(o, false); s != TC2_OK) return s;
  const int nb = Zh->nb, b = Zh->b;
  if (nb < 1 || b < 1 || b > BP || nb > MAX_NB) return TC2_EINVAL;
  if (tc2_status s = validate_bsr(*Zh, nb, b); s != TC2_OK) return s;
  if (tc2_status s = validate_bsr(*Xh, nb, b); s != TC2_OK) return s;
  if (Z1h) {
    if (tc2_status s = validate_bsr(*Z1h, nb, b); s != TC2_OK) return s;
    if (tc2_status s = validate_bsr(*X1h, nb, b); s != TC2_OK) return s;
  }
  Ctx x;
  if (tc2_status s = start(o, x); s != TC2_OK) return s;
  Events ev;
  LCHK(hipEventCreate(&ev.a));
  LCHK(hipEventCreate(&ev.b));
  GMat Z, X, Z1, X1, Q, Q1, C;
  if (tc2_status s = from_bsr(*Zh, x.st, Z); s != TC2_OK) return s;
  if (tc2_status s = from_bsr(*Xh, x.st, X); s != TC2_OK) return s;
  if (Z1h) {
    if (tc2_status s = from_bsr(*Z1h, x.st, Z1); s != TC2_OK) return s;
    if (tc2_status s = from_bsr(*X1h, x.st, X1); s != TC2_OK) return s;
  }
  LCHK(hipEventRecord(ev.a, x.st));
  if (tc2_status s = product(x, Z, X, false, o->eps, Q); s != TC2_OK) return s;
  if (!Z1h) {
    if (tc2_status s = product(x, Q, Z, true, o->eps, C); s != TC2_OK) return s;
  } else {
    if (tc2_status s = product(x, Z1, X, false, o->eps, Q1, &Z, &X1); s != TC2_OK) return s;
    if (tc2_status s = product(x, Q1, Z, true, o->eps, C, &Q, &Z1); s != TC2_OK) return s;
  }
  LCHK(hipEventRecord(ev.b, x.st));
  LCHK(hipEventSynchronize(ev.b));
  float ms = 0.f;
  LCHK(hipEventElapsedTime(&ms, ev.a, ev.b));
  if (seconds) *seconds = ms * 1e-3;
  return to_host(x, C, out);
}

}  // namespace

extern "C" TC2_API tc2_status tc2_lowdin(const tc2_bsr* S, const tc2_bsr* H, int32_t n_dir,
                                         const tc2_bsr* H1, const tc2_lowdin_options* opts,
                                         tc2_lowdin_result* res) {
  if (!res) return TC2_EINVAL;
  std::memset(res, 0, sizeof(*res));
  tc2_status s;
  try {
    s = lowdin_core(S, H, n_dir, H1, nullptr, opts,
                    LowdinOut{&res->iters, &res->resid, &res->lambda, &res->seconds, &res->Z,
                              &res->H, res->H1, nullptr});
  } catch (...) {
    s = TC2_ENOMEM;
  }
  if (s < 0) {  // no partial outputs on failure
    release(&res->Z);
    release(&res->H);
    for (tc2_bsr& m : res->H1) release(&m);
  }
  res->status = s;
  return s;
}

extern "C" TC2_API tc2_status tc2_lowdin_response(const tc2_bsr* S, const tc2_bsr* H,
                                                  int32_t n_dir, const tc2_bsr* H1,
                                                  const tc2_bsr* S1,
                                                  const tc2_lowdin_options* opts,
                                                  tc2_lowdin_response_result* res) {
  if (!res) return TC2_EINVAL;
  std::memset(res, 0, sizeof(*res));
  tc2_status s;
  if (n_dir > 0 && !S1) {
    s = TC2_EINVAL;
  } else {
    try {
      s = lowdin_core(S, H, n_dir, H1, n_dir > 0 ? S1 : nullptr, opts,
                      LowdinOut{&res->iters, &res->resid, &res->lambda, &res->seconds, &res->Z,
                                &res->H, res->H1, res->Z1});
    } catch (...) {
      s = TC2_ENOMEM;
    }
  }
  if (s < 0) {
    release(&res->Z);
    release(&res->H);
    for (tc2_bsr& m : res->H1) release(&m);
    for (tc2_bsr& m : res->Z1) release(&m);
  }
  res->status = s;
  return s;
}

extern "C" TC2_API tc2_status tc2_congruence(const tc2_bsr* Z, const tc2_bsr* X,
                                             const tc2_lowdin_options* opts, tc2_bsr* out,
                                             double* seconds) {
  if (!out) return TC2_EINVAL;
  std::memset(out, 0, sizeof(*out));
  tc2_status s;
  try {
    s = congruence_impl(Z, X, nullptr, nullptr, opts, out, seconds);
  } catch (...) {
    s = TC2_ENOMEM;
  }
  if (s < 0) release(out);
  return s;
}

extern "C" TC2_API tc2_status tc2_congruence_response(const tc2_bsr* Z, const tc2_bsr* Z1,
                                                      const tc2_bsr* X, const tc2_bsr* X1,
                                                      const tc2_lowdin_options* opts,
                                                      tc2_bsr* out, double* seconds) {
  if (!out) return TC2_EINVAL;
  std::memset(out, 0, sizeof(*out));
  tc2_status s;
  if (!Z1 || !X1) {
    s = TC2_EINVAL;
  } else {
    try {
      s = congruence_impl(Z, X, Z1, X1, opts, out, seconds);
    } catch (...) {
      s = TC2_ENOMEM;
    }
  }
  if (s < 0) release(out);
  return s;
}

extern "C" TC2_API void tc2_bsr_release(tc2_bsr* m) { release(m); }
