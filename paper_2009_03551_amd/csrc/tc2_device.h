// Device-side helpers shared by the kernel translation units.
#pragma once
#include "tc2_internal.h"

namespace tc2 {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// first index p in [0, n) with a[p] == key, or -1 (a sorted ascending)
__device__ __forceinline__ int bsearch_eq(const int* a, int n, int key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    int v = a[mid];
    if (v < key) lo = mid + 1; else hi = mid;
  }
  return (lo < n && a[lo] == key) ? lo : -1;
}

// Accumulator of one 16 x 16 output tile.  The MFMA result layout differs
// between the f64 and f32 instructions (checked on the device):
//   f64 16x16x4: lane l, register j holds row l/16 + 4j, column l%16;
//   f32 16x16x4: lane l, register j holds row 4(l/16) + j, column l%16.
template <typename T> struct Acc;
template <> struct Acc<double> {
  d4 v;
  __device__ static int row(int l, int j) { return (l >> 4) + 4 * j; }
};
template <> struct Acc<float> {
  f4 v;
  __device__ static int row(int l, int j) { return 4 * (l >> 4) + j; }
};
// FP64 sums of f32 MFMA tiles (same element layout as Acc<float>): each
// column block's FP32 product is added here, so that the long sum over the
// common columns K runs in FP64.
struct AccW {
  d4 v;
  __device__ static int row(int l, int j) { return 4 * (l >> 4) + j; }
};

__device__ __forceinline__ void mfma(Acc<double>& c, double a, double b) {
  c.v = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c.v, 0, 0, 0);
}
__device__ __forceinline__ void mfma(Acc<float>& c, float a, float b) {
  c.v = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c.v, 0, 0, 0);
}

// bfloat16 operand of v_mfma_f32_16x16x16_bf16 from a column-major FP32 16 x 16
// tile: lane l holds elements (row l%16, k = 4(l/16) + i), i < 4, rounded to
// nearest even.  The same read gives the B operand of X_IK X_JK^T.
__device__ __forceinline__ s4 bf16_frag(const float* tile, int lane) {
  s4 v;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const __bf16 h = (__bf16)tile[(4 * (lane >> 4) + i) * BP + (lane & 15)];
    v[i] = __builtin_bit_cast(short, h);
  }
  return v;
}

// The same fragment as bf16_frag, each value split into three bfloat16 parts
// v = h + m + l + r: h = bf16(v), m = bf16(v - h), l = bf16(v - h - m) (the
// differences are exact in FP32), so that the parts carry 24 significant bits.
__device__ __forceinline__ void bf16_split3(const float* tile, int lane, s4& h, s4& m, s4& l) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float v = tile[(4 * (lane >> 4) + i) * BP + (lane & 15)];
    const __bf16 bh = (__bf16)v;
    const float r1 = v - (float)bh;
    const __bf16 bm = (__bf16)r1;
    const __bf16 bl = (__bf16)(r1 - (float)bm);
    h[i] = __builtin_bit_cast(short, bh);
    m[i] = __builtin_bit_cast(short, bm);
    l[i] = __builtin_bit_cast(short, bl);
  }
}

__device__ __forceinline__ void mfma_bf16(Acc<float>& c, s4 a, s4 b) {
  c.v = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c.v, 0, 0, 0);
}

// Skip network parameter offsets (see tc2_mlp.hip); in LDS, W2 is stored
// transposed (W2T[k][j] = W2[j][k]) so that lane j reads row k contiguously.
constexpr int MLP_W1 = 0, MLP_B1 = 512, MLP_W2 = 576, MLP_B2 = 4672, MLP_W3 = 4736, MLP_B3 = 4800;

// Logit of the skip network for one feature vector (wave-uniform), one hidden
// unit per lane; th points to the LDS copy with W2 transposed.
__device__ __forceinline__ float mlp_logit_wave(const float* th, const float* f, int lane) {
  float a1 = th[MLP_B1 + lane];
#pragma unroll
  for (int i = 0; i < MLP_NF; ++i) a1 += th[MLP_W1 + lane * MLP_NF + i] * f[i];
  const float h1 = fmaxf(a1, 0.f);
  float a2 = th[MLP_B2 + lane];
#pragma unroll 8
  for (int k = 0; k < MLP_NH; ++k)
    a2 += th[MLP_W2 + k * MLP_NH + lane] * __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, h1), k));
  const float h2 = fmaxf(a2, 0.f);
  return (float)wave_sum((double)(th[MLP_W3 + lane] * h2)) + th[MLP_B3];
}

// Pointers used by the fused epilogue of the numeric kernels.
struct EpiCtx {
  const void* xv;
  size_t stride;             // elements per entry ((1+D)*BS)
  const int* h_rp;
  const int* h_ci;
  const double* h_v;
  const int* h1_rp[MAXD];
  const int* h1_ci[MAXD];
  const double* h1_v[MAXD];
  void* stage;
  int2* kept_ij;
  int* stage_count;
  int stage_cap;
  int* overflow;
  int* bad;
};

// Epilogue of one output block C_IJ (accumulators of X0*X0 and of
// X0*X1_d + X1_d*X0) for the TC2 update (Sec. 2.2): combine with the branch
// (SQUARE: C; DOUBLE: 2X - C), round to the working precision, Frobenius
// norm of each matrix's block, drop below eps (filter of Sec. 2.3, never on
// the diagonal), append the kept block to the stage as the upper block
// (min(I,J), max(I,J)) row-major, and add Tr, ||X0||_F^2, Tr(X H), Tr(X1 H1)
// contributions (weight 2 off the diagonal) to q.  eIJ is the entry of the
// old block (I, J) or -1.  A is the accumulator type (its element layout and
// precision).  Called by a whole wave.
template <typename T, int D, typename A = Acc<T>>
__device__ __forceinline__ bool epilogue(const EpiCtx& E, const A* acc, int I, int J,
                                         int eIJ, bool square, double eps, int npairs, int sys,
                                         double* q) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15;
  const bool diag = (I == J);
  const T* X = (const T*)E.xv;
  double v[1 + D][4];
#pragma unroll
  for (int m = 0; m <= D; ++m)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = A::row(lane, j);
      const double c = (double)acc[m].v[j];
      double x = c;
      if (!square) {
        const double old = eIJ >= 0 ? (double)X[(size_t)eIJ * E.stride + m * BS + col * BP + r] : 0.0;
        x = 2.0 * old - c;
      }
      v[m][j] = (double)(T)x;
    }
  double nrm2[1 + D];
  bool keep[1 + D];
  bool any = false, bad = false;
#pragma unroll
  for (int m = 0; m <= D; ++m) {
    double ss = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      ss += v[m][j] * v[m][j];
      bad |= !isfinite(v[m][j]);
    }
    nrm2[m] = wave_sum(ss);
    keep[m] = diag || !(sqrt(nrm2[m]) < eps);
    any |= keep[m];
  }
  if (__ballot(bad) != 0ull && lane == 0) atomicOr(&E.bad[sys], 1);
  if (any) {
    int slot = 0;
    if (lane == 0) slot = atomicAdd(E.stage_count, 1);
    slot = __builtin_amdgcn_readfirstlane(slot);
    if (slot < E.stage_cap) {
      T* st = (T*)E.stage + (size_t)slot * E.stride;
      const bool tr = I > J;  // the stage holds the upper block (J, I) = C_IJ^T
#pragma unroll
      for (int m = 0; m <= D; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = A::row(lane, j);
          st[m * BS + (tr ? col * BP + r : r * BP + col)] = keep[m] ? (T)v[m][j] : (T)0;
        }
      if (lane == 0) E.kept_ij[slot] = tr ? make_int2(J, I) : make_int2(I, J);
    } else if (lane == 0) {
      atomicOr(E.overflow, 1);
    }
  }
  const double w = diag ? 1.0 : 2.0;
  if (any) q[Q_TRIP] += (double)npairs;
  if (diag) {
#pragma unroll
    for (int m = 0; m <= D; ++m) {
      double tr = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) tr += (A::row(lane, j) == col) ? v[m][j] : 0.0;
      tr = wave_sum(tr);
      if (m == 0) q[Q_TR0] += tr; else q[Q_TR1 + m - 1] += tr;
    }
  }
  if (keep[0]) q[Q_FRO0] += w * nrm2[0];
  int eh = -1;
  for (int e = E.h_rp[I]; e < E.h_rp[I + 1]; ++e)
    if (E.h_ci[e] == J) { eh = e; break; }
  if (eh >= 0) {
    const double* hb = E.h_v + (size_t)eh * BS;
#pragma unroll
    for (int m = 0; m <= D; ++m) {
      if (!keep[m]) continue;
      double dot = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) dot += v[m][j] * hb[col * BP + A::row(lane, j)];
      dot = wave_sum(dot);
      if (m == 0) q[Q_E0] += w * dot; else q[Q_E1 + m - 1] += w * dot;
    }
  }
#pragma unroll
  for (int d = 0; d < D; ++d) {
    if (!keep[1 + d]) continue;
    int e1 = -1;
    for (int e = E.h1_rp[d][I]; e < E.h1_rp[d][I + 1]; ++e)
      if (E.h1_ci[d][e] == J) { e1 = e; break; }
    if (e1 >= 0) {
      const double* hb = E.h1_v[d] + (size_t)e1 * BS;
      double dot = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) dot += v[1 + d][j] * hb[col * BP + A::row(lane, j)];
      dot = wave_sum(dot);
      q[Q_AL + d] += w * dot;
    }
  }
  return any;
}

}  // namespace tc2
