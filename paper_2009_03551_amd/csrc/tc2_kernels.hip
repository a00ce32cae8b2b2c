// HIP kernels of the TC2 / TC2-CPSCF solver for gfx950 (MI355X).
//
// One iteration of the recursion (Sec. 2.2, Eq. TC2 and Eq. TC2-CPSCF) is
//   symbolic  : upper-triangle pattern of X*X by row-wise union (Gustavson's
//               row formulation, Algorithm 1, restricted to J >= I), built in
//               an LDS bitmap;
//   numeric   : one 64-lane wave per candidate block (I, J): intersect the
//               sorted column lists of rows I and J, then accumulate
//               X0_IK X0_KJ, X0_IK X1_KJ + X1_IK X0_KJ over the common K with
//               MFMA on padded 16 x 16 tiles; fused epilogue: branch combine,
//               block Frobenius norms, drop (filter of Sec. 2.3), traces and
//               band-energy partial sums;
//   compact   : kept upper blocks -> new sorted symmetric pattern + values.
#include "tc2_device.h"

namespace tc2 {

// ------------------------------------------------------------------ Gershgorin
// Bounds of the spectrum of H (Sec. 2.2): per scalar row i, H_ii -+ sum_{j!=i} |H_ij|.
__global__ void k_gershgorin(int nb, int b, const int* rp, const int* ci, const double* hv,
                             double* rowlo, double* rowhi) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nb * b) return;
  int I = g / b, r = g - I * b;
  double sum = 0.0, centre = 0.0;
  for (int e = rp[I]; e < rp[I + 1]; ++e) {
    const double* blk = hv + (size_t)e * BS;
    bool diag = ci[e] == I;
    for (int c = 0; c < b; ++c) {
      double v = blk[c * BP + r];
      if (diag && c == r) centre = v; else sum += fabs(v);
    }
  }
  rowlo[g] = centre - sum;
  rowhi[g] = centre + sum;
}

__global__ void k_sys_minmax(const int* sys_start, const int* sys_end, int b, const double* rowlo,
                             const double* rowhi, double* emin, double* emax) {
  __shared__ double slo[256], shi[256];
  int s = blockIdx.x;
  long g0 = (long)sys_start[s] * b, g1 = (long)sys_end[s] * b;
  double lo = INFINITY, hi = -INFINITY;
  for (long g = g0 + threadIdx.x; g < g1; g += blockDim.x) {
    lo = fmin(lo, rowlo[g]);
    hi = fmax(hi, rowhi[g]);
  }
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + o]);
      shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    emin[s] = slo[0];
    emax[s] = shi[0];
  }
}

// ------------------------------------------------------------------ init
// X0 = (emax I - H)/(emax - emin), X1_d = -H1_d/(emax - emin)  (Sec. 2.2).
struct InitPtrs {
  const int* src_h1[MAXD];
  const double* h1v[MAXD];
};

template <typename T>
__global__ void k_init(long long n, int D, int b, const int* row_of, const int* ci,
                       const int* src_h, InitPtrs p, const double* hv, const int* sys_of,
                       const double* emin, const double* emax, const int* mode, T* xv) {
  // grid-stride: a dispatch covers at most 2^32 work-items
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (long long)gridDim.x * blockDim.x) {
    int per = (1 + D) * BS;
    long long e = idx / per;
    int rem = (int)(idx - e * per);
    int m = rem / BS, q = rem - m * BS;
    int c = q / BP, r = q - c * BP;
    int I = row_of[e], J = ci[e];
    int s = sys_of[I];
    double v = 0.0;
    if (r < b && c < b) {
      int md = mode[s];
      if (md == 0) {
        double W = emax[s] - emin[s];
        if (m == 0) {
          int eh = src_h[e];
          double h = eh >= 0 ? hv[(size_t)eh * BS + q] : 0.0;
          double d = (I == J && r == c) ? emax[s] : 0.0;
          v = (d - h) / W;
        } else {
          int eh = p.src_h1[m - 1][e];
          double h = eh >= 0 ? p.h1v[m - 1][(size_t)eh * BS + q] : 0.0;
          v = -h / W;
        }
      } else if (md == 2) {
        v = (m == 0 && I == J && r == c) ? 1.0 : 0.0;
      }
    }
    xv[idx] = (T)v;
  }
}

// ------------------------------------------------------------------ symbolic
// Upper-triangle candidate pattern of the product: for row I the union over
// K in row(I) of {J in row(K) : J >= I}.  Pass 0 counts, pass 1 writes the
// sorted columns.
__global__ __launch_bounds__(256) void k_symbolic(int pass, SymArgs a) {
  extern __shared__ unsigned sbits[];
  __shared__ int sscan[256];
  const int I = blockIdx.x;
  const int s = a.sys_of[I];
  const int lo = I, nbits = a.sys_end[s] - I;
  const int nwords = (nbits + 31) >> 5;
  const int t = threadIdx.x;
  const int r0 = a.rp[I], r1 = a.rp[I + 1];
  if (!a.active[s]) {  // stopped systems are carried by the copy-through kernel
    if (pass == 0 && t == 0) a.cand_cnt[I] = 0;
    return;
  }
  for (int w = t; w < nwords; w += blockDim.x) sbits[w] = 0u;
  __syncthreads();
  const int wave = t >> 6, lane = t & 63, nw = blockDim.x >> 6;
  for (int e = r0 + wave; e < r1; e += nw) {
    int K = a.ci[e];
    int f0 = a.rp[K], f1 = a.rp[K + 1];
    for (int f = f0 + lane; f < f1; f += 64) {
      int J = a.ci[f];
      if (J >= I) {
        int o = J - lo;
        atomicOr(&sbits[o >> 5], 1u << (o & 31));
      }
    }
  }
  __syncthreads();
  // contiguous word range per thread, block-wide exclusive scan of popcounts
  int per = (nwords + blockDim.x - 1) / blockDim.x;
  int w0 = t * per, w1 = min(nwords, w0 + per);
  int cnt = 0;
  for (int w = w0; w < w1; ++w) cnt += __popc(sbits[w]);
  sscan[t] = cnt;
  __syncthreads();
  if (pass == 0) {
    for (int o = 128; o > 0; o >>= 1) {
      if (t < o) sscan[t] += sscan[t + o];
      __syncthreads();
    }
    if (t == 0) a.cand_cnt[I] = sscan[0];
    return;
  }
  // Hillis-Steele inclusive scan
  for (int o = 1; o < 256; o <<= 1) {
    int v = (t >= o) ? sscan[t - o] : 0;
    __syncthreads();
    sscan[t] += v;
    __syncthreads();
  }
  int pos = a.cand_rp[I] + sscan[t] - cnt;
  for (int w = w0; w < w1; ++w) {
    unsigned x = sbits[w];
    while (x) {
      int bit = __ffs(x) - 1;
      x &= x - 1;
      a.cand_ci[pos++] = lo + (w << 5) + bit;
    }
  }
}

// ------------------------------------------------------------------ scans
// Exclusive scan of n ints into out[0..n] (out[n] = total), single block.
__global__ __launch_bounds__(1024) void k_scan(int n, const int* in, int* out, int* total) {
  __shared__ int s[1024];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 1024) {
    int i = base + threadIdx.x;
    int v = i < n ? in[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      int u = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
      __syncthreads();
      s[threadIdx.x] += u;
      __syncthreads();
    }
    if (i < n) out[i] = carry + s[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[n] = carry;
    if (total) *total = carry;
  }
}

__global__ void k_items_count(int nb, const int* cand_rp, int* item_cnt) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nb) return;
  int n = cand_rp[I + 1] - cand_rp[I];
  item_cnt[I] = (n + CHUNK - 1) / CHUNK;
}

__global__ void k_items(int nb, const int* cand_rp, const int* item_rp, int* item_row,
                        int* item_c0) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nb) return;
  int k0 = item_rp[I], k1 = item_rp[I + 1];
  for (int k = k0; k < k1; ++k) {
    item_row[k] = I;
    item_c0[k] = cand_rp[I] + (k - k0) * CHUNK;
  }
}

__global__ void k_sys_items(int nsys, int mult, const int* sys_start, const int* sys_end,
                            const int* item_rp, int* lo, int* hi) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys) return;
  lo[s] = mult * item_rp[sys_start[s]];
  hi[s] = mult * item_rp[sys_end[s]];
}

// ------------------------------------------------------------------ numeric
constexpr int MAXM_LDS = 4096;  // row-I column list cached in LDS up to this length

template <typename T, int D>
__global__ __launch_bounds__(256) void k_numeric(NumArgs a) {
  __shared__ int scol[MAXM_LDS];
  __shared__ double spart[4][NQ];
  const int item = blockIdx.x;
  const int I = a.item_row[item];
  const int c0 = a.item_c0[item];
  const int c1 = min(c0 + CHUNK, a.cand_rp[I + 1]);
  const int r0 = a.rp[I], mI = a.rp[I + 1] - r0;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int s = a.sys_of[I];
  const bool square = a.branch[s] != 0;
  const double eps = a.eps[s];
  const int* rowI = a.ci + r0;
  if (mI <= MAXM_LDS) {
    for (int p = t; p < mI; p += blockDim.x) scol[p] = rowI[p];
    rowI = scol;
  }
  __syncthreads();

  const T* X = (const T*)a.xv;
  const size_t stride = (size_t)(1 + D) * BS;
  EpiCtx E{a.xv, stride, a.h_rp, a.h_ci, a.h_v, {a.h1_rp[0], a.h1_rp[1], a.h1_rp[2]},
           {a.h1_ci[0], a.h1_ci[1], a.h1_ci[2]}, {a.h1_v[0], a.h1_v[1], a.h1_v[2]}, a.stage,
           a.kept_ij, a.stage_count, a.stage_cap, a.overflow, a.bad};
  double q[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) q[k] = 0.0;
  unsigned long long issued = 0;

  for (int c = c0 + wave; c < c1; c += 4) {
    const int J = a.cand_ci[c];
    Acc<T> acc[1 + D];
#pragma unroll
    for (int m = 0; m <= D; ++m)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[m].v[j] = 0;
    int npairs = 0;
    const int f0 = a.rp[J], f1 = a.rp[J + 1];
    for (int base = f0; base < f1; base += 64) {
      const int f = base + lane;
      int pos = -1;
      if (f < f1) pos = bsearch_eq(rowI, mI, a.ci[f]);
      const bool found = pos >= 0;
      const unsigned long long mask = __ballot(found);
      const int n = __popcll(mask);
      if (n == 0) continue;
      const int my = __popcll(mask & ((1ull << lane) - 1ull));
      const int dst = found ? my : n + (lane - my);
      const int vI = __builtin_amdgcn_ds_permute(dst << 2, r0 + pos);
      const int vJ = __builtin_amdgcn_ds_permute(dst << 2, f);
      npairs += n;
      for (int i = 0; i < n; ++i) {
        const int pI = __builtin_amdgcn_readlane(vI, i);
        const int pJ = __builtin_amdgcn_readlane(vJ, i);
        const T* xa = X + (size_t)pI * stride + lane;
        const T* xb = X + (size_t)pJ * stride + lane;
        for (int kk = 0; kk < a.ksteps; ++kk) {
          const T a0 = xa[kk * 64], b0 = xb[kk * 64];
          mfma(acc[0], a0, b0);
#pragma unroll
          for (int d = 0; d < D; ++d) {
            const T a1 = xa[(1 + d) * BS + kk * 64], b1 = xb[(1 + d) * BS + kk * 64];
            mfma(acc[1 + d], a0, b1);
            mfma(acc[1 + d], a1, b0);
          }
        }
      }
    }
    issued += (unsigned long long)npairs * (1 + 2 * D);  // block products
    const int pIJ = bsearch_eq(rowI, mI, J);
    epilogue<T, D>(E, acc, I, J, pIJ >= 0 ? r0 + pIJ : -1, square, eps, npairs, s, q);
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NQ; ++k) spart[wave][k] = q[k];
    if (issued) atomicAdd(a.exec_pairs, issued);
  }
  __syncthreads();
  if (t < NQ) {
    double sum = spart[0][t];
    for (int w = 1; w < 4; ++w) sum += spart[w][t];
    a.partial[(size_t)item * NQ + t] = sum;
  }
}

// ------------------------------------------------------------------ measure
// Scalars of the current iterate (Tr X0, ||X0||_F^2, band energies, alpha)
// straight from its stored blocks; used for the initial matrices.  One wave
// per row, entries J >= I weighted by 2 off the diagonal.
template <typename T, int D>
__global__ __launch_bounds__(64) void k_measure(MeasArgs a) {
  const int I = blockIdx.x;
  const int lane = threadIdx.x;
  const T* X = (const T*)a.xv;
  const size_t stride = (size_t)(1 + D) * BS;
  double q[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) q[k] = 0.0;
  for (int e = a.rp[I]; e < a.rp[I + 1]; ++e) {
    const int J = a.ci[e];
    if (J < I) continue;
    const double w = (J == I) ? 1.0 : 2.0;
    int eh = -1;
    for (int f = a.h_rp[I]; f < a.h_rp[I + 1]; ++f)
      if (a.h_ci[f] == J) { eh = f; break; }
    for (int m = 0; m <= D; ++m) {
      double tr = 0.0, ss = 0.0, dh = 0.0, d1 = 0.0;
      int e1 = -1;
      if (m > 0)
        for (int f = a.h1_rp[m - 1][I]; f < a.h1_rp[m - 1][I + 1]; ++f)
          if (a.h1_ci[m - 1][f] == J) { e1 = f; break; }
      for (int j = 0; j < 4; ++j) {
        const int qd = lane + 64 * j;
        const double x = (double)X[(size_t)e * stride + m * BS + qd];
        if (J == I && (qd & 15) == (qd >> 4)) tr += x;
        ss += x * x;
        if (eh >= 0) dh += x * a.h_v[(size_t)eh * BS + qd];
        if (e1 >= 0) d1 += x * a.h1_v[m - 1][(size_t)e1 * BS + qd];
      }
      tr = wave_sum(tr);
      ss = wave_sum(ss);
      dh = wave_sum(dh);
      d1 = wave_sum(d1);
      if (m == 0) {
        q[Q_TR0] += tr;
        q[Q_FRO0] += w * ss;
        q[Q_E0] += w * dh;
      } else {
        q[Q_TR1 + m - 1] += tr;
        q[Q_E1 + m - 1] += w * dh;
        q[Q_AL + m - 1] += w * d1;
      }
    }
  }
  if (lane < NQ) {
    double out = 0.0;
#pragma unroll
    for (int k = 0; k < NQ; ++k) out = (lane == k) ? q[k] : out;
    a.partial[(size_t)I * NQ + lane] = out;
  }
}

// ------------------------------------------------------------------ compaction
__global__ void k_compact_count(CompactArgs a, int n_kept) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (a.n_kept_dev) n_kept = min(n_kept, *a.n_kept_dev);
  if (k >= n_kept) return;
  int2 ij = a.kept_ij[k];
  atomicAdd(&a.rowcnt[ij.x], 1);
  if (ij.y != ij.x) atomicAdd(&a.rowcnt[ij.y], 1);
}

__global__ void k_compact_scatter(CompactArgs a, int n_kept) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (a.n_kept_dev) n_kept = min(n_kept, *a.n_kept_dev);
  if (k >= n_kept) return;
  int2 ij = a.kept_ij[k];
  int p = a.new_rp[ij.x] + atomicAdd(&a.cursor[ij.x], 1);
  a.tmp_ci[p] = ij.y;
  a.tmp_src[p] = 2 * k;
  if (ij.y != ij.x) {
    int p2 = a.new_rp[ij.y] + atomicAdd(&a.cursor[ij.y], 1);
    a.tmp_ci[p2] = ij.x;
    a.tmp_src[p2] = 2 * k + 1;
  }
}

// Sort each new row by column: rank of a column = number of set bits below it
// in an LDS bitmap over the system's column range.
__global__ __launch_bounds__(256) void k_row_sort(CompactArgs a) {
  extern __shared__ unsigned sm[];
  __shared__ int sscan[256];
  const int R = blockIdx.x;
  const int s = a.sys_of[R];
  const int lo = a.sys_start[s], nbits = a.sys_end[s] - lo;
  const int nwords = (nbits + 31) >> 5;
  unsigned* bits = sm;
  unsigned* pre = sm + nwords;
  const int t = threadIdx.x;
  const int p0 = a.new_rp[R], p1 = a.new_rp[R + 1];
  for (int w = t; w < nwords; w += blockDim.x) bits[w] = 0u;
  __syncthreads();
  for (int p = p0 + t; p < p1; p += blockDim.x) {
    int o = a.tmp_ci[p] - lo;
    atomicOr(&bits[o >> 5], 1u << (o & 31));
  }
  __syncthreads();
  int per = (nwords + blockDim.x - 1) / blockDim.x;
  int w0 = t * per, w1 = min(nwords, w0 + per);
  int cnt = 0;
  for (int w = w0; w < w1; ++w) cnt += __popc(bits[w]);
  sscan[t] = cnt;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    int v = (t >= o) ? sscan[t - o] : 0;
    __syncthreads();
    sscan[t] += v;
    __syncthreads();
  }
  int run = sscan[t] - cnt;
  for (int w = w0; w < w1; ++w) {
    pre[w] = run;
    run += __popc(bits[w]);
  }
  __syncthreads();
  for (int p = p0 + t; p < p1; p += blockDim.x) {
    int col = a.tmp_ci[p];
    int o = col - lo;
    int w = o >> 5;
    int rank = pre[w] + __popc(bits[w] & ((1u << (o & 31)) - 1u));
    a.new_ci[p0 + rank] = col;
    a.new_src[p0 + rank] = a.tmp_src[p];
  }
}

// new entry e <- staged block: the stage holds C_IJ row-major; entry (I, J)
// needs it column-major (a transpose), the mirrored entry (J, I) needs
// C_IJ^T column-major, i.e. the stage as it is.
template <typename T>
__global__ void k_gather(long long n, int D, const int* new_src, const T* stage, T* xv,
                         const int* nnz_dev, const int* skip_flag) {
  // an update whose stage overflowed is run again: its values must not be
  // written over the iterate that the repeated products read
  if (skip_flag && *skip_flag) return;
  // four consecutive elements per thread: one column segment (c, r..r+3) of a
  // column-major tile, a 4-vector store; the source is the same segment of
  // the stage (mirrored entry) or four rows of one column (transpose)
  typedef T T4 __attribute__((ext_vector_type(4)));
  const int per = (1 + D) * BS;
  if (nnz_dev) n = min(n, (long long)*nnz_dev * per);
  const long long n4 = n >> 2;
  for (long long i4 = (long long)blockIdx.x * blockDim.x + threadIdx.x; i4 < n4;
       i4 += (long long)gridDim.x * blockDim.x) {
    const long long idx = i4 << 2;
    const long long e = idx / per;
    const int rem = (int)(idx - e * per);
    const int m = rem / BS, qd = rem - m * BS;  // qd = c*16 + r, r % 4 == 0
    const int src = new_src[e];
    const T* sb = stage + (size_t)(src >> 1) * per + m * BS;
    T4 v;
    if (src & 1) {
      v = *(const T4*)(sb + qd);
    } else {
      const int c = qd >> 4, r = qd & 15;
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = sb[(r + i) * BP + c];
    }
    *(T4*)(xv + idx) = v;
  }
}

// ------------------------------------------------------------------ reductions
// Per system, the partial sums of its work items in a fixed order.  Thread t
// adds the items t, t + RT, ... in one pass (the NQ sums of an item are
// contiguous, so a wave reads consecutive memory); the wave sums follow a
// fixed butterfly and the waves are added in wave order.
constexpr int RT = 1024;
__global__ __launch_bounds__(RT) void k_reduce(const int* lo, const int* hi,
                                               const double* partial, double* scal) {
  __shared__ double sh[RT / 64][NQ];
  const int s = blockIdx.x;
  const int t = threadIdx.x, w = t >> 6;
  double v[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) v[k] = 0.0;
  const int end = hi[s];
  for (int i = lo[s] + t; i < end; i += RT) {
    const double* p = partial + (size_t)i * NQ;
#pragma unroll
    for (int k = 0; k < NQ; ++k) v[k] += p[k];
  }
#pragma unroll
  for (int k = 0; k < NQ; ++k) v[k] = wave_sum(v[k]);
  if ((t & 63) == 0) {
#pragma unroll
    for (int k = 0; k < NQ; ++k) sh[w][k] = v[k];
  }
  __syncthreads();
  if (t < NQ) {
    double acc = 0.0;
    for (int j = 0; j < RT / 64; ++j) acc += sh[j][t];
    scal[s * NQ + t] = acc;
  }
}

// ------------------------------------------------------------------ export / convert
template <typename T>
__global__ void k_export(long long n, int D, int m, int b, const T* xv, double* out) {
  const int bb = b * b;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (long long)gridDim.x * blockDim.x) {
    long long e = idx / bb;
    int rem = (int)(idx - e * bb);
    int r = rem / b, c = rem - r * b;
    out[idx] = (double)xv[((size_t)e * (1 + D) + m) * BS + c * BP + r];
  }
}

template <typename A, typename B>
__global__ void k_convert(long long n, const A* in, B* out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    out[i] = (B)in[i];
}

__global__ void k_fill_int(int* p, int v, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

// ================================================================== launchers
static inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }
// Grid of a grid-stride elementwise kernel: enough blocks to fill the chip
// several times over, while blocks x threads stays far below 2^32 (a dispatch
// counts its work-items in 32 bits).
static inline unsigned sblk(long long n, int bs) {
  long long g = (n + bs - 1) / bs;
  return (unsigned)(g < 65536 ? (g > 0 ? g : 1) : 65536);
}

void launch_gershgorin(hipStream_t st, int nb, int b, const int* rp, const int* ci,
                       const double* hv, double* rowlo, double* rowhi) {
  long long n = (long long)nb * b;
  if (n == 0) return;
  hipLaunchKernelGGL(k_gershgorin, dim3(nblk(n, 256)), dim3(256), 0, st, nb, b, rp, ci, hv,
                     rowlo, rowhi);
}

void launch_sys_minmax(hipStream_t st, int nsys, const int* sys_start, const int* sys_end,
                       int b, const double* rowlo, const double* rowhi, double* emin,
                       double* emax) {
  hipLaunchKernelGGL(k_sys_minmax, dim3(nsys), dim3(256), 0, st, sys_start, sys_end, b, rowlo,
                     rowhi, emin, emax);
}

void launch_init(hipStream_t st, int prec, int nnz, int D, int b, const int* row_of,
                 const int* ci, const int* src_h, const int* const* src_h1, const double* hv,
                 const double* const* h1v, const int* sys_of, const double* emin,
                 const double* emax, const int* mode, void* xv) {
  InitPtrs p{};
  for (int d = 0; d < D; ++d) {
    p.src_h1[d] = src_h1[d];
    p.h1v[d] = h1v[d];
  }
  long long n = (long long)nnz * (1 + D) * BS;
  if (n == 0) return;
  if (prec == P_FP64)
    hipLaunchKernelGGL(k_init<double>, dim3(sblk(n, 256)), dim3(256), 0, st, n, D, b, row_of, ci,
                       src_h, p, hv, sys_of, emin, emax, mode, (double*)xv);
  else
    hipLaunchKernelGGL(k_init<float>, dim3(sblk(n, 256)), dim3(256), 0, st, n, D, b, row_of, ci,
                       src_h, p, hv, sys_of, emin, emax, mode, (float*)xv);
}

void launch_symbolic(hipStream_t st, int pass, const SymArgs& a) {
  if (a.nb == 0) return;
  // dynamic LDS: bitmap of the largest system window (host checks the limit)
  size_t lds = (size_t)((a.max_sys_atoms + 31) / 32) * 4;
  hipLaunchKernelGGL(k_symbolic, dim3(a.nb), dim3(256), lds, st, pass, a);
}

void launch_scan(hipStream_t st, int n, const int* in, int* out, int* total) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, n, in, out, total);
}

void launch_items_count(hipStream_t st, int nb, const int* cand_rp, int* item_cnt) {
  if (nb == 0) return;
  hipLaunchKernelGGL(k_items_count, dim3(nblk(nb, 256)), dim3(256), 0, st, nb, cand_rp, item_cnt);
}

void launch_items(hipStream_t st, int nb, const int* cand_rp, const int* item_rp, int* item_row,
                  int* item_c0) {
  if (nb == 0) return;
  hipLaunchKernelGGL(k_items, dim3(nblk(nb, 256)), dim3(256), 0, st, nb, cand_rp, item_rp,
                     item_row, item_c0);
}

void launch_sys_items(hipStream_t st, int nsys, int mult, const int* sys_start,
                      const int* sys_end, const int* item_rp, int* lo, int* hi) {
  hipLaunchKernelGGL(k_sys_items, dim3(nblk(nsys, 64)), dim3(64), 0, st, nsys, mult, sys_start,
                     sys_end, item_rp, lo, hi);
}

template <typename T>
static void numeric_d(hipStream_t st, const NumArgs& a) {
  switch (a.D) {
    case 0: hipLaunchKernelGGL((k_numeric<T, 0>), dim3(a.n_items), dim3(256), 0, st, a); break;
    case 1: hipLaunchKernelGGL((k_numeric<T, 1>), dim3(a.n_items), dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_numeric<T, 2>), dim3(a.n_items), dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((k_numeric<T, 3>), dim3(a.n_items), dim3(256), 0, st, a); break;
  }
}

void launch_numeric(hipStream_t st, int prec, const NumArgs& a) {
  if (a.n_items == 0) return;
  if (prec == P_FP64) numeric_d<double>(st, a);
  else numeric_d<float>(st, a);
}

template <typename T>
static void measure_d(hipStream_t st, const MeasArgs& a) {
  switch (a.D) {
    case 0: hipLaunchKernelGGL((k_measure<T, 0>), dim3(a.nb), dim3(64), 0, st, a); break;
    case 1: hipLaunchKernelGGL((k_measure<T, 1>), dim3(a.nb), dim3(64), 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_measure<T, 2>), dim3(a.nb), dim3(64), 0, st, a); break;
    default: hipLaunchKernelGGL((k_measure<T, 3>), dim3(a.nb), dim3(64), 0, st, a); break;
  }
}

void launch_measure(hipStream_t st, int prec, const MeasArgs& a) {
  if (a.nb == 0) return;
  if (prec == P_FP64) measure_d<double>(st, a);
  else measure_d<float>(st, a);
}

void launch_compact_count(hipStream_t st, const CompactArgs& a, int n_kept) {
  if (n_kept == 0) return;
  hipLaunchKernelGGL(k_compact_count, dim3(nblk(n_kept, 256)), dim3(256), 0, st, a, n_kept);
}

void launch_compact_scatter(hipStream_t st, const CompactArgs& a, int n_kept) {
  if (n_kept == 0) return;
  hipLaunchKernelGGL(k_compact_scatter, dim3(nblk(n_kept, 256)), dim3(256), 0, st, a, n_kept);
}

void launch_row_sort(hipStream_t st, const CompactArgs& a) {
  if (a.nb == 0) return;
  size_t lds = (size_t)((a.max_sys_atoms + 31) / 32) * 8;
  hipLaunchKernelGGL(k_row_sort, dim3(a.nb), dim3(256), lds, st, a);
}

void launch_gather(hipStream_t st, int prec, int nnz, int D, const int* new_src,
                   const void* stage, void* xv, const int* nnz_dev, const int* skip_flag) {
  long long n = (long long)nnz * (1 + D) * BS;
  if (n == 0) return;
  if (prec == P_FP64)
    hipLaunchKernelGGL(k_gather<double>, dim3(sblk(n / 4, 256)), dim3(256), 0, st, n, D, new_src,
                       (const double*)stage, (double*)xv, nnz_dev, skip_flag);
  else
    hipLaunchKernelGGL(k_gather<float>, dim3(sblk(n / 4, 256)), dim3(256), 0, st, n, D, new_src,
                       (const float*)stage, (float*)xv, nnz_dev, skip_flag);
}

void launch_reduce(hipStream_t st, int nsys, const int* lo, const int* hi,
                   const double* partial, double* scal) {
  hipLaunchKernelGGL(k_reduce, dim3(nsys), dim3(RT), 0, st, lo, hi, partial, scal);
}

void launch_export(hipStream_t st, int prec, int nnz, int D, int m, int b, const void* xv,
                   double* out) {
  long long n = (long long)nnz * b * b;
  if (n == 0) return;
  if (prec == P_FP64)
    hipLaunchKernelGGL(k_export<double>, dim3(sblk(n, 256)), dim3(256), 0, st, n, D, m, b,
                       (const double*)xv, out);
  else
    hipLaunchKernelGGL(k_export<float>, dim3(sblk(n, 256)), dim3(256), 0, st, n, D, m, b,
                       (const float*)xv, out);
}

void launch_convert(hipStream_t st, int from_prec, int to_prec, long long n, const void* in,
                    void* out) {
  if (n == 0) return;
  bool f64in = from_prec == P_FP64, f64out = to_prec == P_FP64;
  if (f64in && !f64out)
    hipLaunchKernelGGL((k_convert<double, float>), dim3(sblk(n, 256)), dim3(256), 0, st, n,
                       (const double*)in, (float*)out);
  else if (!f64in && f64out)
    hipLaunchKernelGGL((k_convert<float, double>), dim3(sblk(n, 256)), dim3(256), 0, st, n,
                       (const float*)in, (double*)out);
}

void launch_fill_int(hipStream_t st, int* p, int v, long long n) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_int, dim3(sblk(n, 256)), dim3(256), 0, st, p, v, n);
}

}  // namespace tc2
