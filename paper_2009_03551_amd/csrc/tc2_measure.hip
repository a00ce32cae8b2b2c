// Measurement and export entry points of the TC2 solver context:
//  * the exact count of useful block products of every update (count_useful),
//    as the work of one update of Eq. TC2 / TC2-CPSCF (Sec. 2.2) is defined on
//    the stored blocks of each matrix and the outputs the filter of Sec. 2.3
//    keeps;
//  * complete block rows of the current iterate (tc2_export_rows), for
//    checks of sampled rows of large systems;
//  * the current iterate entry by entry (tc2_export_entries) and its
//    comparison with entries held by the caller (tc2_compare_entries), so that
//    two solves of a system too large to export whole can be compared on the
//    device, in chunks.
#include "tc2_context.h"
#include "tc2_device.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

using namespace tc2;

namespace {

#define HIPCHK(x)                                                        \
  do {                                                                   \
    hipError_t e_ = (x);                                                 \
    if (e_ != hipSuccess) {                                              \
      if (ctx && ctx->verbose)                                           \
        fprintf(stderr, "tc2: %s failed: %s\n", #x, hipGetErrorString(e_)); \
      return e_ == hipErrorOutOfMemory ? TC2_ENOMEM : TC2_EDEVICE;       \
    }                                                                    \
  } while (0)

// ------------------------------------------------------------------ masks
// Bit m of mask[e] is set when block m (0: X0, 1 + d: X1_d) of entry e has a
// nonzero element.  One wave per entry.
template <typename T>
__global__ void k_block_masks(long long nnz, int D, const T* __restrict__ xv,
                              unsigned char* __restrict__ mask, const int* nnz_dev) {
  const int lane = threadIdx.x & 63;
  if (nnz_dev) nnz = min(nnz, (long long)*nnz_dev);
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long e = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; e < nnz; e += nwaves) {
    unsigned bits = 0u;
    for (int m = 0; m <= D; ++m) {
      const T* x = xv + ((size_t)e * (1 + D) + m) * BS;
      bool nz = false;
#pragma unroll
      for (int j = 0; j < 4; ++j) nz |= x[lane + 64 * j] != (T)0;
      if (__ballot(nz) != 0ull) bits |= 1u << m;
    }
    if (lane == 0) mask[e] = (unsigned char)bits;
  }
}

// New entry e <- its staged block, with the mask of its nonzero matrices and
// (bn given) the Frobenius norm of each of its blocks, in one pass, one wave
// per entry.  The stage holds C_IJ row-major: entry (I, J) needs it
// column-major (a transpose), the mirrored entry (J, I) needs C_IJ^T
// column-major, i.e. the stage as it is (bit 0 of new_src).  Lane l handles
// elements l + 64 j of each tile, as k_block_masks and k_block_norms do, and
// sums their squares in the same order with the same wave reduction, so the
// norms equal theirs bit for bit.  An update whose stage overflowed is run
// again: then nothing is written.
template <typename T>
__global__ void k_gather_masks(long long nnz, int D, const int* __restrict__ new_src,
                               const T* __restrict__ stage, T* __restrict__ xv,
                               unsigned char* __restrict__ mask, float* __restrict__ bn,
                               const int* nnz_dev, const int* skip_flag) {
  if (skip_flag && *skip_flag) return;
  const int lane = threadIdx.x & 63;
  if (nnz_dev) nnz = min(nnz, (long long)*nnz_dev);
  const int per = (1 + D) * BS;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long e = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; e < nnz; e += nwaves) {
    const int src = new_src[e];
    unsigned bits = 0u;
    for (int m = 0; m <= D; ++m) {
      const T* sb = stage + (size_t)(src >> 1) * per + m * BS;
      T* xb = xv + (size_t)e * per + m * BS;
      bool nz = false;
      double ss = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = lane + 64 * j;  // c * 16 + r of the column-major tile
        const T v = (src & 1) ? sb[q] : sb[(q & 15) * BP + (q >> 4)];
        xb[q] = v;
        nz |= v != (T)0;
        const double dv = (double)v;
        ss += dv * dv;
      }
      if (__ballot(nz) != 0ull) bits |= 1u << m;
      if (bn) {
        ss = wave_sum(ss);
        if (lane == 0) bn[(size_t)e * (1 + D) + m] = (float)sqrt(ss);
      }
    }
    if (lane == 0) mask[e] = (unsigned char)bits;
  }
}

// ------------------------------------------------------------------ useful products
// One wave per row I of the new pattern.  For every new entry (I, J >= I) of
// a system that took part in the update, the common columns K of the old rows
// I and J give the block triples; a triple counts one product for X0 X0 when
// X0_IK and X0_JK are both nonzero and the new block of X0 is nonzero (kept),
// and one product each for X0_IK X1_JK^T and X1_IK X0_JK^T when the operand
// blocks are nonzero and the new block of X1_d is nonzero.  The counts go to
// acc[system * 4 + kind].
struct UsefulArgs {
  int nb, D, kind;
  const int* orp;
  const int* oci;
  const unsigned char* omask;
  const int* nrp;
  const int* nci;
  const unsigned char* nmask;
  const int* sys_of;
  const int* active;
  unsigned long long* acc;
};

__global__ void k_useful(UsefulArgs a) {
  const int lane = threadIdx.x & 63;
  const int nwaves = (int)(((long long)gridDim.x * blockDim.x) >> 6);
  for (int I = (int)(((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6); I < a.nb;
       I += nwaves) {
    const int sys = a.sys_of[I];
    if (!a.active[sys]) continue;
    const int i0 = a.orp[I], i1 = a.orp[I + 1];
    unsigned long long row_total = 0;
    for (int e = a.nrp[I]; e < a.nrp[I + 1]; ++e) {
      const int J = a.nci[e];
      if (J < I) continue;
      const unsigned nm = a.nmask[e];
      if (!nm) continue;
      const int j0 = a.orp[J], nj = a.orp[J + 1] - j0;
      unsigned n00 = 0, n1[MAXD] = {0, 0, 0};
      for (int p = i0 + lane; p < i1; p += 64) {
        const int q = bsearch_eq(a.oci + j0, nj, a.oci[p]);
        if (q < 0) continue;
        const unsigned ma = a.omask[p], mb = a.omask[j0 + q];
        n00 += (ma & mb & 1u);
        for (int d = 0; d < a.D; ++d)
          n1[d] += (ma & (mb >> (1 + d)) & 1u) + ((ma >> (1 + d)) & mb & 1u);
      }
      unsigned long long c = 0;
      if (nm & 1u) c += (unsigned long long)n00;
      for (int d = 0; d < a.D; ++d)
        if ((nm >> (1 + d)) & 1u) c += (unsigned long long)n1[d];
      row_total += c;
    }
    // wave sum of the per-lane counts
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) row_total += __shfl_xor(row_total, o, 64);
    if (lane == 0 && row_total) atomicAdd(&a.acc[(size_t)sys * 4 + a.kind], row_total);
  }
}

static unsigned grid_waves(long long n, int waves_per_block) {
  const long long want = (n + waves_per_block - 1) / waves_per_block;
  return (unsigned)std::max(1LL, std::min(want, 1LL << 20));
}

// ------------------------------------------------------------------ gathers
// Entries ent[0..n) of matrix m (all 1 + D matrices when m < 0) as compact
// row-major b x b FP64 blocks.
template <typename T>
__global__ void k_gather_entries(long long n, int D, int m, int b, const long long* ent,
                                 long long first, const T* __restrict__ xv, double* out) {
  const int bb = b * b;
  const int nm = m < 0 ? 1 + D : 1;
  const long long total = n * nm * bb;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long i = idx / (nm * bb);
    const int rem = (int)(idx - i * nm * bb);
    const int mm = rem / bb, rc = rem - mm * bb;
    const int r = rc / b, c = rc - r * b;
    const long long e = ent ? ent[i] : first + i;
    const int mat = m < 0 ? mm : m;
    out[idx] = (double)xv[((size_t)e * (1 + D) + mat) * BS + c * BP + r];
  }
}

// ------------------------------------------------------------------ comparison
// Caller entries (row, col, values) against matrix m of the iterate: the
// largest |given - stored| over the given entries (stored = 0 where the
// iterate has no such entry), and found[e] set for the entries met.  One wave
// per given entry.  The maximum of non-negative doubles is taken on their bit
// patterns, which order the same way, so the result does not depend on the
// order of the waves.
// stats: [0] max over entries both sides hold, [1] max over entries only
// the caller gave, [2] max over entries only the iterate holds (bit patterns
// of non-negative doubles), [3] entries only the caller gave, [4] entries only
// the iterate holds, [5] max Frobenius norm of a block held by one side only
template <typename T>
__global__ void k_compare_given(long long n, int D, int m, int b, const int* __restrict__ rows,
                                const int* __restrict__ cols, const double* __restrict__ vals,
                                const int* __restrict__ rp, const int* __restrict__ ci,
                                const T* __restrict__ xv, unsigned char* found,
                                unsigned long long* stats) {
  const int lane = threadIdx.x & 63;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  double mx_both = 0.0, mx_only = 0.0, nrm_only = 0.0;
  unsigned long long n_only = 0;
  for (long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n; i += nwaves) {
    const int I = rows[i], J = cols[i];
    const int r0 = rp[I];
    const int q = bsearch_eq(ci + r0, rp[I + 1] - r0, J);
    const long long e = q >= 0 ? (long long)r0 + q : -1;
    if (e >= 0 && lane == 0) found[e] = 1;
    double mx = 0.0, ss = 0.0;
    for (int rc = lane; rc < b * b; rc += 64) {
      const int r = rc / b, c = rc - r * b;
      const double x = e >= 0 ? (double)xv[((size_t)e * (1 + D) + m) * BS + c * BP + r] : 0.0;
      const double v = vals[(size_t)i * b * b + rc];
      mx = fmax(mx, fabs(v - x));
      ss += v * v;
    }
    if (e >= 0) {
      mx_both = fmax(mx_both, mx);
    } else {
      ss = wave_sum(ss);
      if (ss > 0.0) {
        mx_only = fmax(mx_only, mx);
        nrm_only = fmax(nrm_only, sqrt(ss));
        n_only += 1;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mx_both = fmax(mx_both, __shfl_xor(mx_both, o, 64));
    mx_only = fmax(mx_only, __shfl_xor(mx_only, o, 64));
  }
  if (lane == 0) {
    if (mx_both > 0.0) atomicMax(&stats[0], (unsigned long long)__double_as_longlong(mx_both));
    if (mx_only > 0.0) atomicMax(&stats[1], (unsigned long long)__double_as_longlong(mx_only));
    if (nrm_only > 0.0) atomicMax(&stats[5], (unsigned long long)__double_as_longlong(nrm_only));
    if (n_only) atomicAdd(&stats[3], n_only);
  }
}

// Entries of the iterate that the caller did not give: their largest
// |stored|, count (nonzero blocks only) and largest Frobenius norm.
template <typename T>
__global__ void k_compare_missing(long long nnz, int D, int m, const T* __restrict__ xv,
                                  const unsigned char* __restrict__ found,
                                  unsigned long long* stats) {
  const int lane = threadIdx.x & 63;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  double mx = 0.0, nrm = 0.0;
  unsigned long long cnt = 0;
  for (long long e = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; e < nnz; e += nwaves) {
    if (found[e]) continue;
    const T* x = xv + ((size_t)e * (1 + D) + m) * BS;
    double bm = 0.0, ss = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double v = (double)x[lane + 64 * j];
      bm = fmax(bm, fabs(v));
      ss += v * v;
    }
    ss = wave_sum(ss);
    if (ss > 0.0) {
      mx = fmax(mx, bm);
      nrm = fmax(nrm, sqrt(ss));
      cnt += 1;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if (lane == 0) {
    if (mx > 0.0) atomicMax(&stats[2], (unsigned long long)__double_as_longlong(mx));
    if (nrm > 0.0) atomicMax(&stats[5], (unsigned long long)__double_as_longlong(nrm));
    if (cnt) atomicAdd(&stats[4], cnt);
  }
}

// A device buffer of one call, freed on return.
struct Tmp {
  void* p = nullptr;
  ~Tmp() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t n) { return tc2::dev_malloc(&p, n < 256 ? 256 : n); }
  template <typename T> T* as() const { return (T*)p; }
};

}  // namespace

// ====================================================================== counting
namespace tc2 {

void launch_block_masks(hipStream_t st, int prec, long long nnz, int D, const void* xv,
                        unsigned char* mask, const int* nnz_dev) {
  if (nnz == 0) return;
  const unsigned g = grid_waves(nnz, 4);
  if (prec == P_FP64)
    hipLaunchKernelGGL(k_block_masks<double>, dim3(g), dim3(256), 0, st, nnz, D,
                       (const double*)xv, mask, nnz_dev);
  else
    hipLaunchKernelGGL(k_block_masks<float>, dim3(g), dim3(256), 0, st, nnz, D,
                       (const float*)xv, mask, nnz_dev);
}

void launch_gather_masks(hipStream_t st, int prec, long long nnz, int D, const int* new_src,
                         const void* stage, void* xv, unsigned char* mask, float* bn,
                         const int* nnz_dev, const int* skip_flag) {
  if (nnz == 0) return;
  const unsigned g = grid_waves(nnz, 4);
  if (prec == P_FP64)
    hipLaunchKernelGGL(k_gather_masks<double>, dim3(g), dim3(256), 0, st, nnz, D, new_src,
                       (const double*)stage, (double*)xv, mask, bn, nnz_dev, skip_flag);
  else
    hipLaunchKernelGGL(k_gather_masks<float>, dim3(g), dim3(256), 0, st, nnz, D, new_src,
                       (const float*)stage, (float*)xv, mask, bn, nnz_dev, skip_flag);
}

tc2_status mask_iterate(tc2_ctx* ctx, hipStream_t st) {
  const int c = ctx->cur;
  const long long nnz = ctx->nnz[c];
  HIPCHK(ctx->mask[c].reserve((size_t)std::max(nnz, 1LL)));
  launch_block_masks(st, ctx->cur_prec, nnz, ctx->D, ctx->xv[c].p, ctx->mask[c].as<unsigned char>(),
                     nullptr);
  HIPCHK(hipGetLastError());
  return TC2_OK;
}

// The masks of the new iterate were computed by the update itself.
tc2_status count_update(tc2_ctx* ctx, hipStream_t st) {
  const int n = ctx->cur, o = n ^ 1;
  UsefulArgs a{};
  a.nb = ctx->nb;
  a.D = ctx->D;
  a.kind = ctx->last_kind;
  a.orp = ctx->rp[o].as<int>();
  a.oci = ctx->ci[o].as<int>();
  a.omask = ctx->mask[o].as<unsigned char>();
  a.nrp = ctx->rp[n].as<int>();
  a.nci = ctx->ci[n].as<int>();
  a.nmask = ctx->mask[n].as<unsigned char>();
  a.sys_of = ctx->sys_of.as<int>();
  a.active = ctx->active.as<int>();
  a.acc = ctx->useful_acc.as<unsigned long long>();
  hipLaunchKernelGGL(k_useful, dim3(grid_waves(ctx->nb, 4)), dim3(256), 0, st, a);
  HIPCHK(hipGetLastError());
  return TC2_OK;
}

}  // namespace tc2

// ====================================================================== ABI
namespace {

tc2_status export_rows_impl(tc2_ctx* ctx, int32_t system, const int32_t* rows, int32_t n_rows,
                            tc2_bsr* x0, tc2_bsr* x1) {
  if (!ctx || !x0 || (n_rows > 0 && !rows) || n_rows < 0) return TC2_EINVAL;
  if (system < 0 || system >= ctx->nsys || !ctx->have_iterate) return TC2_EINVAL;
  if (ctx->D > 0 && !x1) return TC2_EINVAL;
  const SysInfo& si = ctx->sys[system];
  for (int i = 0; i < n_rows; ++i)
    if (rows[i] < 0 || rows[i] >= si.nb) return TC2_EINVAL;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->own;
  HIPCHK(hipStreamSynchronize(ctx->run.st ? ctx->run.st : st));
  const int c = ctx->cur, D = ctx->D, b = ctx->b, nb = ctx->nb;
  std::vector<int> rp(nb + 1);
  HIPCHK(hipMemcpy(rp.data(), ctx->rp[c].p, (size_t)(nb + 1) * 4, hipMemcpyDeviceToHost));
  std::vector<char> want(si.nb, 0);
  for (int i = 0; i < n_rows; ++i) want[rows[i]] = 1;
  // entries of the wanted rows, in row order
  std::vector<long long> ent;
  std::vector<int32_t> col;
  std::vector<int64_t> out_rp(si.nb + 1, 0);
  for (int i = 0; i < si.nb; ++i) {
    out_rp[i + 1] = out_rp[i];
    if (!want[i]) continue;
    const int I = si.row0 + i, n = rp[I + 1] - rp[I];
    std::vector<int> cs(n);
    if (n) HIPCHK(hipMemcpy(cs.data(), ctx->ci[c].as<int>() + rp[I], (size_t)n * 4, hipMemcpyDeviceToHost));
    for (int k = 0; k < n; ++k) {
      ent.push_back((long long)rp[I] + k);
      col.push_back(cs[k] - si.row0);
    }
    out_rp[i + 1] += n;
  }
  const long long ne = (long long)ent.size();
  const size_t bb = (size_t)b * b;
  std::vector<double> vals((size_t)ne * (1 + D) * bb);
  if (ne) {
    Tmp dent, dout;
    HIPCHK(dent.alloc((size_t)ne * 8));
    HIPCHK(dout.alloc(vals.size() * 8));
    HIPCHK(hipMemcpy(dent.p, ent.data(), (size_t)ne * 8, hipMemcpyHostToDevice));
    const long long total = (long long)vals.size();
    const unsigned g = (unsigned)std::min<long long>((total + 255) / 256, 1 << 20);
    if (ctx->cur_prec == P_FP64)
      hipLaunchKernelGGL(k_gather_entries<double>, dim3(g), dim3(256), 0, st, ne, D, -1, b,
                         dent.as<long long>(), 0LL, ctx->xv[c].as<double>(), dout.as<double>());
    else
      hipLaunchKernelGGL(k_gather_entries<float>, dim3(g), dim3(256), 0, st, ne, D, -1, b,
                         dent.as<long long>(), 0LL, ctx->xv[c].as<float>(), dout.as<double>());
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(vals.data(), dout.p, vals.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  // library-allocated outputs (released with tc2_bsr_release)
  tc2_bsr* outs[1 + MAXD] = {x0, nullptr, nullptr, nullptr};
  for (int d = 0; d < D; ++d) outs[1 + d] = &x1[d];
  for (int m = 0; m <= D; ++m) *outs[m] = tc2_bsr{0, 0, nullptr, nullptr, nullptr};
  for (int m = 0; m <= D; ++m) {
    int64_t* orp = (int64_t*)malloc(sizeof(int64_t) * ((size_t)si.nb + 1));
    int32_t* oci = (int32_t*)malloc(sizeof(int32_t) * (size_t)std::max(ne, 1LL));
    double* ov = (double*)malloc(sizeof(double) * (size_t)std::max(ne, 1LL) * bb);
    if (!orp || !oci || !ov) {
      free(orp);
      free(oci);
      free(ov);
      for (int k = 0; k < m; ++k) tc2_bsr_release(outs[k]);
      return TC2_ENOMEM;
    }
    memcpy(orp, out_rp.data(), sizeof(int64_t) * ((size_t)si.nb + 1));
    if (ne) memcpy(oci, col.data(), sizeof(int32_t) * (size_t)ne);
    for (long long i = 0; i < ne; ++i)
      memcpy(ov + (size_t)i * bb, vals.data() + ((size_t)i * (1 + D) + m) * bb, bb * sizeof(double));
    *outs[m] = tc2_bsr{si.nb, b, orp, oci, ov};
  }
  return TC2_OK;
}

tc2_status export_entries_impl(tc2_ctx* ctx, int32_t matrix, int64_t first, int64_t count,
                               int32_t* rows, int32_t* cols, double* vals) {
  if (!ctx || !ctx->have_iterate || matrix < 0 || matrix > ctx->D || first < 0 || count < 0)
    return TC2_EINVAL;
  const int c = ctx->cur, nb = ctx->nb, b = ctx->b;
  if (first + count > ctx->nnz[c]) return TC2_EINVAL;
  if (count == 0) return TC2_OK;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->own;
  HIPCHK(hipStreamSynchronize(ctx->run.st ? ctx->run.st : st));
  if (rows || cols) {
    std::vector<int> rp(nb + 1);
    HIPCHK(hipMemcpy(rp.data(), ctx->rp[c].p, (size_t)(nb + 1) * 4, hipMemcpyDeviceToHost));
    if (cols)
      HIPCHK(hipMemcpy(cols, ctx->ci[c].as<int>() + first, (size_t)count * 4, hipMemcpyDeviceToHost));
    if (rows) {
      int I = (int)(std::upper_bound(rp.begin(), rp.end(), (int)first) - rp.begin()) - 1;
      for (int64_t k = 0; k < count; ++k) {
        while (rp[I + 1] <= first + k) ++I;
        rows[k] = I;
      }
    }
  }
  if (vals) {
    Tmp dout;
    const size_t bb = (size_t)b * b;
    HIPCHK(dout.alloc((size_t)count * bb * 8));
    const long long total = count * (long long)bb;
    const unsigned g = (unsigned)std::min<long long>((total + 255) / 256, 1 << 20);
    if (ctx->cur_prec == P_FP64)
      hipLaunchKernelGGL(k_gather_entries<double>, dim3(g), dim3(256), 0, st, (long long)count,
                         ctx->D, matrix, b, (const long long*)nullptr, (long long)first,
                         ctx->xv[c].as<double>(), dout.as<double>());
    else
      hipLaunchKernelGGL(k_gather_entries<float>, dim3(g), dim3(256), 0, st, (long long)count,
                         ctx->D, matrix, b, (const long long*)nullptr, (long long)first,
                         ctx->xv[c].as<float>(), dout.as<double>());
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(vals, dout.p, (size_t)count * bb * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  return TC2_OK;
}

tc2_status compare_entries_impl(tc2_ctx* ctx, int32_t matrix, int64_t n, const int32_t* rows,
                                const int32_t* cols, const double* vals, double* max_abs,
                                double* detail) {
  if (!ctx || !ctx->have_iterate || !max_abs || matrix < 0 || matrix > ctx->D || n < 0 ||
      (n > 0 && (!rows || !cols || !vals)))
    return TC2_EINVAL;
  const int c = ctx->cur, nb = ctx->nb, b = ctx->b, D = ctx->D;
  for (int64_t k = 0; k < n; ++k) {
    if (rows[k] < 0 || rows[k] >= nb || cols[k] < 0 || cols[k] >= nb) return TC2_EINVAL;
    if (k > 0 && (rows[k] < rows[k - 1] || (rows[k] == rows[k - 1] && cols[k] <= cols[k - 1])))
      return TC2_EINVAL;
  }
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = ctx->own;
  HIPCHK(hipStreamSynchronize(ctx->run.st ? ctx->run.st : st));
  const long long nnz = ctx->nnz[c];
  const size_t bb = (size_t)b * b;
  Tmp drows, dcols, dvals, dfound, dmax;
  HIPCHK(drows.alloc((size_t)std::max<int64_t>(n, 1) * 4));
  HIPCHK(dcols.alloc((size_t)std::max<int64_t>(n, 1) * 4));
  HIPCHK(dfound.alloc((size_t)std::max(nnz, 1LL)));
  HIPCHK(dmax.alloc(6 * 8));
  HIPCHK(hipMemsetAsync(dfound.p, 0, (size_t)std::max(nnz, 1LL), st));
  HIPCHK(hipMemsetAsync(dmax.p, 0, 6 * 8, st));
  if (n) {
    HIPCHK(hipMemcpyAsync(drows.p, rows, (size_t)n * 4, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dcols.p, cols, (size_t)n * 4, hipMemcpyHostToDevice, st));
  }
  // values in chunks of at most 1 Mi entries
  const int64_t chunk = std::min<int64_t>(std::max<int64_t>(n, 1), 1 << 20);
  HIPCHK(dvals.alloc((size_t)chunk * bb * 8));
  for (int64_t k0 = 0; k0 < n; k0 += chunk) {
    const int64_t m = std::min<int64_t>(chunk, n - k0);
    HIPCHK(hipMemcpyAsync(dvals.p, vals + (size_t)k0 * bb, (size_t)m * bb * 8, hipMemcpyHostToDevice, st));
    const unsigned g = grid_waves(m, 4);
    if (ctx->cur_prec == P_FP64)
      hipLaunchKernelGGL(k_compare_given<double>, dim3(g), dim3(256), 0, st, (long long)m, D, matrix, b,
                         drows.as<int>() + k0, dcols.as<int>() + k0, dvals.as<double>(),
                         ctx->rp[c].as<int>(), ctx->ci[c].as<int>(), ctx->xv[c].as<double>(),
                         dfound.as<unsigned char>(), dmax.as<unsigned long long>());
    else
      hipLaunchKernelGGL(k_compare_given<float>, dim3(g), dim3(256), 0, st, (long long)m, D, matrix, b,
                         drows.as<int>() + k0, dcols.as<int>() + k0, dvals.as<double>(),
                         ctx->rp[c].as<int>(), ctx->ci[c].as<int>(), ctx->xv[c].as<float>(),
                         dfound.as<unsigned char>(), dmax.as<unsigned long long>());
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));  // the chunk buffer is reused
  }
  if (nnz) {
    const unsigned g = grid_waves(nnz, 4);
    if (ctx->cur_prec == P_FP64)
      hipLaunchKernelGGL(k_compare_missing<double>, dim3(g), dim3(256), 0, st, nnz, D, matrix,
                         ctx->xv[c].as<double>(), dfound.as<unsigned char>(),
                         dmax.as<unsigned long long>());
    else
      hipLaunchKernelGGL(k_compare_missing<float>, dim3(g), dim3(256), 0, st, nnz, D, matrix,
                         ctx->xv[c].as<float>(), dfound.as<unsigned char>(),
                         dmax.as<unsigned long long>());
    HIPCHK(hipGetLastError());
  }
  unsigned long long bits[6] = {0, 0, 0, 0, 0, 0};
  HIPCHK(hipMemcpyAsync(bits, dmax.p, 6 * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double v[6];
  for (int k = 0; k < 6; ++k) {
    if (k == 3 || k == 4) v[k] = (double)bits[k];
    else memcpy(&v[k], &bits[k], 8);
  }
  *max_abs = std::max(v[0], std::max(v[1], v[2]));
  if (detail)
    for (int k = 0; k < 6; ++k) detail[k] = v[k];
  return TC2_OK;
}

}  // namespace

extern "C" {

TC2_API tc2_status tc2_export_rows(tc2_ctx* ctx, int32_t system, const int32_t* rows,
                                   int32_t n_rows, tc2_bsr* x0, tc2_bsr* x1) {
  try {
    return export_rows_impl(ctx, system, rows, n_rows, x0, x1);
  } catch (const std::bad_alloc&) {
    return TC2_ENOMEM;
  } catch (...) {
    return TC2_EDEVICE;
  }
}

TC2_API tc2_status tc2_iterate_size(tc2_ctx* ctx, int64_t* nnz) {
  if (!ctx || !nnz || !ctx->have_iterate) return TC2_EINVAL;
  *nnz = ctx->nnz[ctx->cur];
  return TC2_OK;
}

TC2_API tc2_status tc2_export_entries(tc2_ctx* ctx, int32_t matrix, int64_t first, int64_t count,
                                      int32_t* rows, int32_t* cols, double* vals) {
  try {
    return export_entries_impl(ctx, matrix, first, count, rows, cols, vals);
  } catch (const std::bad_alloc&) {
    return TC2_ENOMEM;
  } catch (...) {
    return TC2_EDEVICE;
  }
}

TC2_API tc2_status tc2_compare_entries(tc2_ctx* ctx, int32_t matrix, int64_t n, const int32_t* rows,
                                       const int32_t* cols, const double* vals, double* max_abs,
                                       double* detail) {
  try {
    return compare_entries_impl(ctx, matrix, n, rows, cols, vals, max_abs, detail);
  } catch (const std::bad_alloc&) {
    return TC2_ENOMEM;
  } catch (...) {
    return TC2_EDEVICE;
  }
}

}  // extern "C"
