// Clustered-tile numeric kernel of the TC2 / TC2-CPSCF update for gfx950.
//
// Atoms are grouped into clusters of up to CS = 8 nearby atoms.  A work item
// is a tile of output blocks (I in cluster P) x (J in cluster Q) for P <= Q;
// it walks the common columns K of the two clusters' row panels once and, for
// every K, stages the present blocks X_JK of cluster Q in LDS while each wave
// holds the MFMA fragments of its X_IK in registers.  Every staged block then
// feeds up to 8 block products instead of one, which cuts the L2/HBM operand
// traffic of the row-by-row product (Algorithm 1) several-fold.  The
// accumulators and the fused epilogue (branch combine, Frobenius drop,
// traces and band energies) are the same as in the one-wave-per-block kernel.
#include "tc2_device.h"

namespace tc2 {

// ------------------------------------------------------------------ cluster panels
// Panel of cluster P: sorted union of the columns of its atoms' rows, with the
// entry index of (I_s, K) for every member s (-1 when absent).  The union is
// an LDS bitmap over the system's atoms; pass 1 ranks each member entry in it
// (prefix popcounts), so no search is needed.
constexpr int PNT = 1024;  // threads of the panel and tile kernels

__device__ __forceinline__ int block_exclusive_scan(int v, int* ssc) {
  const int t = threadIdx.x;
  ssc[t] = v;
  __syncthreads();
  for (int o = 1; o < PNT; o <<= 1) {
    const int u = (t >= o) ? ssc[t - o] : 0;
    __syncthreads();
    ssc[t] += u;
    __syncthreads();
  }
  return ssc[t] - v;  // ssc[PNT-1] holds the total
}

__global__ __launch_bounds__(PNT) void k_panels(int pass, PanelArgs a) {
  extern __shared__ unsigned sbits[];  // nwords bits, then nwords prefix counts
  __shared__ int sscan[PNT];
  const int P = blockIdx.x;
  const int sys = a.clus_sys[P];
  const int t = threadIdx.x;
  if (!a.active[sys]) {
    if (pass == 0 && t == 0) a.panel_cnt[P] = 0;
    return;
  }
  const int lo = a.sys_start[sys], nbits = a.sys_end[sys] - lo;
  const int nwords = (nbits + 31) >> 5;
  unsigned* pre = sbits + nwords;
  for (int w = t; w < nwords; w += PNT) sbits[w] = 0u;
  __syncthreads();
  for (int s = 0; s < CS; ++s) {
    const int I = a.clus_atom[P * CS + s];
    if (I < 0) continue;
    for (int e = a.rp[I] + t; e < a.rp[I + 1]; e += PNT) {
      const int o = a.ci[e] - lo;
      atomicOr(&sbits[o >> 5], 1u << (o & 31));
    }
  }
  __syncthreads();
  const int per = (nwords + PNT - 1) / PNT;
  const int w0 = t * per, w1 = min(nwords, w0 + per);
  int cnt = 0;
  for (int w = w0; w < w1; ++w) cnt += __popc(sbits[w]);
  const int before = block_exclusive_scan(cnt, sscan);
  if (pass == 0) {
    if (t == PNT - 1) a.panel_cnt[P] = sscan[PNT - 1];
    return;
  }
  const int base = a.panel_rp[P];
  int run = before;
  for (int w = w0; w < w1; ++w) {
    pre[w] = run;
    unsigned x = sbits[w];
    while (x) {
      const int bit = __ffs(x) - 1;
      x &= x - 1;
      const int pos = base + run++;
      a.panel_k[pos] = lo + (w << 5) + bit;
#pragma unroll
      for (int s = 0; s < CS; ++s) a.panel_e[(size_t)pos * CS + s] = -1;
    }
  }
  __syncthreads();  // ranks in LDS and the -1 fill precede the entry writes
  for (int s = 0; s < CS; ++s) {
    const int I = a.clus_atom[P * CS + s];
    if (I < 0) continue;
    for (int e = a.rp[I] + t; e < a.rp[I + 1]; e += PNT) {
      const int o = a.ci[e] - lo, w = o >> 5;
      const int rank = (int)pre[w] + __popc(sbits[w] & ((1u << (o & 31)) - 1u));
      a.panel_e[(size_t)(base + rank) * CS + s] = e;
    }
  }
}

// Tiles of cluster P: the clusters Q >= P holding an atom J with a column K in
// common with some atom of P (cluster-level symbolic product).  Pass 0 builds
// the cluster bitmap, keeps it in tile_bits and bounds the number of output
// blocks of the tiles; pass 1 writes the tiles from the kept bitmap.
__global__ __launch_bounds__(PNT) void k_tiles(int pass, PanelArgs a) {
  extern __shared__ unsigned sbits[];
  __shared__ int sscan[PNT];
  __shared__ long long spairs[PNT];
  const int P = blockIdx.x;
  const int sys = a.clus_sys[P];
  const int t = threadIdx.x;
  if (!a.active[sys]) {
    if (pass == 0 && t == 0) {
      a.tile_cnt[P] = 0;
      a.tile_pairs[P] = 0;
    }
    return;
  }
  const int nbits = a.csys_end[sys] - P;
  const int nwords = (nbits + 31) >> 5;
  unsigned* gbits = a.tile_bits + (size_t)P * a.tile_words;
  if (pass == 0) {
    for (int w = t; w < nwords; w += PNT) sbits[w] = 0u;
    __syncthreads();
    const int wave = t >> 6, lane = t & 63, nw = PNT >> 6;
    for (int idx = a.panel_rp[P] + wave; idx < a.panel_rp[P + 1]; idx += nw) {
      const int K = a.panel_k[idx];
      for (int f = a.rp[K] + lane; f < a.rp[K + 1]; f += 64) {
        const int Q = a.atom_clus[a.ci[f]];
        if (Q >= P) {
          const int o = Q - P;
          atomicOr(&sbits[o >> 5], 1u << (o & 31));
        }
      }
    }
    __syncthreads();
    for (int w = t; w < nwords; w += PNT) gbits[w] = sbits[w];
  } else {
    for (int w = t; w < nwords; w += PNT) sbits[w] = gbits[w];
    __syncthreads();
  }
  const int per = (nwords + PNT - 1) / PNT;
  const int w0 = t * per, w1 = min(nwords, w0 + per);
  int cnt = 0;
  for (int w = w0; w < w1; ++w) cnt += __popc(sbits[w]);
  if (pass == 0) {
    int nP = 0;
    for (int s = 0; s < CS; ++s) nP += a.clus_atom[P * CS + s] >= 0;
    long long pairs = 0;
    for (int w = w0; w < w1; ++w) {
      unsigned x = sbits[w];
      while (x) {
        const int bit = __ffs(x) - 1;
        x &= x - 1;
        const int Q = P + (w << 5) + bit;
        int nQ = 0;
        for (int s = 0; s < CS; ++s) nQ += a.clus_atom[Q * CS + s] >= 0;
        pairs += (Q == P) ? (long long)nP * (nP + 1) / 2 : (long long)nP * nQ;
      }
    }
    sscan[t] = cnt;
    spairs[t] = pairs;
    __syncthreads();
    for (int o = PNT / 2; o > 0; o >>= 1) {
      if (t < o) {
        sscan[t] += sscan[t + o];
        spairs[t] += spairs[t + o];
      }
      __syncthreads();
    }
    if (t == 0) {
      a.tile_cnt[P] = sscan[0];
      a.tile_pairs[P] = spairs[0];
    }
    return;
  }
  int pos = a.tile_rp[P] + block_exclusive_scan(cnt, sscan);
  for (int w = w0; w < w1; ++w) {
    unsigned x = sbits[w];
    while (x) {
      const int bit = __ffs(x) - 1;
      x &= x - 1;
      a.tile_p[pos] = P;
      a.tile_q[pos] = P + (w << 5) + bit;
      ++pos;
    }
  }
}

// ------------------------------------------------------------------ tile numeric
// A block owns a sub-tile of SP rows of cluster P x TQ columns of cluster Q
// (a tile of 8 x 8 output blocks is split into (8/SP)(8/TQ) blocks).  Wave
// w = h TQ + v owns the "diagonal" outputs (I_s, J_t) with t = (s + v) mod TQ
// for the SP / WS rows s of part h, so that for any column K every wave has
// about the same number of present block pairs.  The common columns K of the two panels are walked in
// groups of KG; for each group the present blocks X_{I_s K} and X_{J_t K} are
// copied straight from global memory into LDS with global_load_lds (16 B per
// lane), double-buffered so that the copy of group g+1 overlaps the MFMAs of
// group g.
typedef __attribute__((address_space(3))) void lds_void;

// W (FP32 values only): the FP32 MFMA product of each column block K is added
// to FP64 accumulators, so that only the short sum inside one block runs in
// FP32 and the long sum over K runs in FP64.
// FK: the block size needs all four K-steps of the padded tile (b > 12), so
// the K-step loop has no exit test and the compiler can overlap the LDS reads
// of one step with the MFMAs of the previous one.
// WS waves share each column of the sub-tile (WS > 1: several waves per SIMD,
// so that one wave's bookkeeping overlaps another's matrix operations).
template <typename T, int D, int SP, int TQ, bool BF, bool W, bool FK, int WS>
__global__ __launch_bounds__(TQ * WS * 64) void k_tile_numeric(TileArgs a) {
  constexpr int PER = (1 + D) * BS;                       // elements per entry
  constexpr int EB = PER * (int)sizeof(T);                // bytes per entry
  constexpr int NE = SP + TQ;                             // entries per column K
  constexpr int KG = (65536 / (NE * EB)) > 0 ? (65536 / (NE * EB)) : 1;
  constexpr int NW = TQ * WS;                             // waves
  constexpr int NT = NW * 64;
  constexpr int NO = SP / WS;                             // outputs per wave
  static_assert(SP % WS == 0, "rows of the sub-tile split evenly over the waves of a column");
  constexpr int KLMAX = 2048;
  constexpr int SUBS = (CS / SP) * (CS / TQ);
  __shared__ __attribute__((aligned(16))) T buf[2][KG][NE][PER];
  __shared__ int sflag[2][KG][NE];
  __shared__ int2 kl[KLMAX];
  __shared__ int wcount[NW];
  __shared__ int sIA[SP], sJB[TQ];
  __shared__ unsigned sown[SP];  // row s: bit t set when output (I_s, J_t) is computed
  __shared__ int s_any;
  __shared__ double spart[NW][NQ];
  __shared__ int s_lb;

  // One sub-tile per block, or (a.work set) a persistent grid in which every
  // block takes the next sub-tile from an atomic counter until all are done;
  // the sub-tile count then comes from the device (tile_rp[nc]).
  const int total = (a.n_tiles_dev ? *a.n_tiles_dev : a.n_tiles) * SUBS;
  for (int it = 0;; ++it) {
  int lb;
  if (a.work) {
    if (threadIdx.x == 0) s_lb = atomicAdd(a.work, 1);
    __syncthreads();
    lb = s_lb;
  } else {
    lb = it == 0 ? (int)blockIdx.x : total;
  }
  if (lb >= total) break;
  const int tile = lb / SUBS, sub = lb - tile * SUBS;
  const int ph = sub / (CS / TQ), qh = sub - ph * (CS / TQ);
  const int P = a.tile_p[tile], Q = a.tile_q[tile];
  // threadIdx-derived values are made opaque per sub-tile, so that the
  // compiler does not hoist per-lane addresses out of the sub-tile loop and
  // keep them live across it (register pressure)
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  const int lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);  // wave-uniform (scalar)
  const int sys = a.clus_sys[P];
  const bool square = a.branch[sys] != 0;
  const double eps = a.eps[sys];
  if (t == 0) s_any = 0;
  if (t < SP) sIA[t] = a.clus_atom[P * CS + ph * SP + t];
  if (t < TQ) sJB[t] = a.clus_atom[Q * CS + qh * TQ + t];
  __syncthreads();

  // outputs of this wave: o -> (row so[o], column to[o])
  int Io[NO], Jo[NO], so[NO], to[NO];
  bool owned[NO];
  bool any_owned = false;
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    so[o] = (wave / TQ) * NO + o;
    to[o] = (so[o] + wave % TQ) % TQ;
    Io[o] = sIA[so[o]];
    Jo[o] = sJB[to[o]];
    owned[o] = Io[o] >= 0 && Jo[o] >= 0 && (P != Q || Io[o] <= Jo[o]);
    any_owned |= owned[o];
  }
  if (any_owned && lane == 0) s_any = 1;
  __syncthreads();
  if (!s_any) {  // e.g. the lower sub-tiles of a diagonal tile: no work, zero sums
    if (t < NQ) a.partial[(size_t)lb * NQ + t] = 0.0;
    continue;
  }

  const T* X = (const T*)a.xv;
  Acc<T> acc[W ? 1 : NO][W ? 1 : 1 + D];
  AccW wacc[W ? NO : 1][W ? 1 + D : 1];
#pragma unroll
  for (int o = 0; o < NO; ++o)
#pragma unroll
    for (int m = 0; m <= D; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if constexpr (W) wacc[o][m].v[r] = 0.0;
        else acc[o][m].v[r] = 0;
      }
  int np[NO];
#pragma unroll
  for (int o = 0; o < NO; ++o) np[o] = 0;

  const int pp0 = a.panel_rp[P], pp1 = a.panel_rp[P + 1];
  const int pq0 = a.panel_rp[Q], nq = a.panel_rp[Q + 1] - pq0;

  // Entries of column group g (KG columns x NE blocks), one per lane: lane
  // gi*NE + x holds the entry of block x of column g*KG + gi, or -1.  Loaded
  // one group ahead, so that issuing the copies never waits on this load.
  static_assert(KG * NE <= 64, "entries of a column group exceed one wave");
  auto load_entries = [&](int g, int nm) {
    int e = -1;
    if (lane < KG * NE) {
      const int gi = lane / NE, x = lane - gi * NE;
      const int m = g * KG + gi;
      if (m < nm) {
        const int2 pq = kl[m];
        e = (x < SP) ? a.panel_e[(size_t)pq.x * CS + ph * SP + x]
                     : a.panel_e[(size_t)pq.y * CS + qh * TQ + (x - SP)];
      }
    }
    return e;
  };
  // Masks of the nonzero matrices of the entries eg (lane-distributed as the
  // entries); all bits set when no masks are given
  auto load_masks = [&](int eg) {
    return eg < 0 ? 0 : (a.xmask ? (int)a.xmask[eg] : 0xff);
  };
  // Copy the blocks of a column group (entries eg, as load_entries) into
  // buffer bb.  A block that meets no present partner of a computed output in
  // its column is not copied (marked absent): no product needs it.
  auto issue = [&](int eg, int bb) {
    const unsigned long long pm = __ballot(eg >= 0);
#pragma unroll
    for (int gi = 0; gi < KG; ++gi) {
      const unsigned mA = (unsigned)(pm >> (gi * NE)) & ((1u << SP) - 1u);
      const unsigned mB = (unsigned)(pm >> (gi * NE + SP)) & ((1u << TQ) - 1u);
      unsigned colsA = 0;  // columns t with a present A block in an owned row
#pragma unroll
      for (int r = 0; r < SP; ++r) colsA |= ((mA >> r) & 1u) ? sown[r] : 0u;
      for (int x = wave; x < NE; x += NW) {
        int e = __builtin_amdgcn_readlane(eg, gi * NE + x);
        const bool need = (x < SP) ? (sown[x] & mB) != 0u : ((colsA >> (x - SP)) & 1u) != 0u;
        if (!need) e = -1;
        if (lane == 0) sflag[bb][gi][x] = e;
        if (e >= 0) {
          const char* src = (const char*)(X + (size_t)e * PER) + lane * 16;
          char* dst = (char*)&buf[bb][gi][x][0];
#pragma unroll
          for (int i = 0; i < EB / 1024; ++i)
            __builtin_amdgcn_global_load_lds((const void*)(src + i * 1024),
                                             (lds_void*)(dst + i * 1024), 16, 0, 0);
        }
      }
    }
  };

  // common columns of the chunk [base, end) of P's panel with Q's panel -> kl;
  // with `useful`, only the columns where some computed output (I_s, J_t)
  // has both blocks X_{I_s K} and X_{J_t K} present
  auto build_kl = [&](int base, int end, bool useful) {
    int nm = 0;
    for (int c0 = base; c0 < end; c0 += NT) {
      const int idx = c0 + t;
      int j = -1;
      if (idx < end) j = (P == Q) ? idx - pp0 : bsearch_eq(a.panel_k + pq0, nq, a.panel_k[idx]);
      if (useful && j >= 0) {
        unsigned mB = 0u, use = 0u;
        const int* eb = a.panel_e + (size_t)(pq0 + j) * CS + qh * TQ;
        for (int u = 0; u < TQ; ++u) mB |= (eb[u] >= 0) ? (1u << u) : 0u;
        const int* ea = a.panel_e + (size_t)idx * CS + ph * SP;
        for (int r = 0; r < SP; ++r) use |= (ea[r] >= 0) ? (sown[r] & mB) : 0u;
        if (!use) j = -1;
      }
      const bool found = j >= 0;
      const unsigned long long mask = __ballot(found);
      if (lane == 0) wcount[wave] = __popcll(mask);
      __syncthreads();
      int off = nm, tot = 0;
      for (int w = 0; w < NW; ++w) {
        const int c = wcount[w];
        off += (w < wave) ? c : 0;
        tot += c;
      }
      if (found) kl[off + __popcll(mask & ((1ull << lane) - 1ull))] = make_int2(idx, pq0 + j);
      nm += tot;
      __syncthreads();
    }
    return nm;
  };

  // lane o of each wave: entry of the old block (I_o, J_o), or -1
  int my_e = -1;
  {
    int Il = -1, Jl = -1;
#pragma unroll
    for (int o = 0; o < NO; ++o)
      if (lane == o) { Il = Io[o]; Jl = Jo[o]; }
    if (lane < NO && Il >= 0 && Jl >= 0) {
      const int r0 = a.rp[Il];
      const int f = bsearch_eq(a.ci + r0, a.rp[Il + 1] - r0, Jl);
      my_e = f >= 0 ? r0 + f : -1;
    }
  }

  // ---- exact screen: ||C_IJ|| <= sum_K ||A_IK|| ||B_KJ|| (+ 2 ||X_IJ|| on the
  // DOUBLE branch); an off-diagonal output whose bound is below eps for X0
  // and every X1_d is certainly dropped, so its products are skipped.  The
  // learned screen then evaluates the skip network on features of the
  // remaining outputs and skips those it predicts to be dropped; features and
  // the true outcome can be logged for training.
  // columns of P's panel taken per pass (a smaller chunk can be forced to test
  // the multi-pass path on small inputs)
  const int KLC = (a.kl_chunk > 0 && a.kl_chunk < KLMAX) ? a.kl_chunk : KLMAX;
  int my_slot = -1;  // lane o: log slot of output o
  if (a.skip || a.log_cap > 0) {
    constexpr int THF = 4864;  // floats reserved for the network at the start of buf
    constexpr int NSF = (int)((sizeof(buf) / 4 - THF) / (NE * (1 + D)));  // columns per norm round
    float* th = (float*)&buf[0][0][0][0];
    float* ns = th + THF;
    if (a.skip == 2) {
      for (int p = t; p < MLP_NP; p += NT) {
        float v = a.mlp[p];
        int q = p;
        if (p >= MLP_W2 && p < MLP_B2) {  // transpose W2 (j, k) -> (k, j)
          const int j = (p - MLP_W2) / MLP_NH, k = (p - MLP_W2) - j * MLP_NH;
          q = MLP_W2 + k * MLP_NH + j;
        }
        th[q] = v;
      }
    }
    double bsum[NO][1 + D];
    float bmax[NO];
    int bcnt[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      bmax[o] = 0.f;
      bcnt[o] = 0;
#pragma unroll
      for (int m = 0; m <= D; ++m) bsum[o][m] = 0.0;
    }
    for (int base = pp0; base < pp1; base += KLC) {
      const int nm = build_kl(base, min(pp1, base + KLC), false);
      for (int r0 = 0; r0 < nm; r0 += NSF) {
        const int nr = min(NSF, nm - r0);
        for (int i = t; i < nr * NE; i += NT) {
          const int m = i / NE, x = i - m * NE;
          const int2 pq = kl[r0 + m];
          const int e = (x < SP) ? a.panel_e[(size_t)pq.x * CS + ph * SP + x]
                                 : a.panel_e[(size_t)pq.y * CS + qh * TQ + (x - SP)];
#pragma unroll
          for (int mm = 0; mm <= D; ++mm)
            ns[(m * NE + x) * (1 + D) + mm] = e >= 0 ? a.bn[(size_t)e * (1 + D) + mm] : -1.f;
        }
        __syncthreads();
        for (int m = lane; m < nr; m += 64) {
          const float* nk = ns + (size_t)m * NE * (1 + D);
#pragma unroll
          for (int o = 0; o < NO; ++o) {
            const float* na = nk + so[o] * (1 + D);
            const float* nb = nk + (SP + to[o]) * (1 + D);
            if (na[0] < 0.f || nb[0] < 0.f) continue;  // block absent
            bcnt[o] += 1;
            bmax[o] = fmaxf(bmax[o], na[0] * nb[0]);
            bsum[o][0] += (double)na[0] * nb[0];
#pragma unroll
            for (int d = 0; d < D; ++d)
              bsum[o][1 + d] += (double)na[0] * nb[1 + d] + (double)na[1 + d] * nb[0];
          }
        }
        __syncthreads();
      }
    }
    int nlog = 0;
    unsigned netskip_mask = 0u;  // outputs skipped by the network (bit o)
    bool logit_o[NO];
    float feat[MLP_NF];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      logit_o[o] = false;
      const int eIJ = __builtin_amdgcn_readlane(my_e, o);
      double bnd[1 + D];
      bool drop = owned[o] && Io[o] != Jo[o];
#pragma unroll
      for (int m = 0; m <= D; ++m) {
        bnd[m] = wave_sum(bsum[o][m]);
        if (!square && eIJ >= 0) bnd[m] += 2.0 * (double)a.bn[(size_t)eIJ * (1 + D) + m];
        // a relative margin covers the rounding of the float block norms
        drop = drop && bnd[m] * (1.0 + 1e-6) < eps;
      }
      if (a.skip && drop) {
        owned[o] = false;
        if (lane == 0) atomicAdd(a.screened, 1ull);
        continue;
      }
      if (!owned[o] || Io[o] == Jo[o]) continue;
      // features of the candidate (scaled logs relative to eps)
      const int cnt = (int)wave_sum((double)bcnt[o]);
      float mx = bmax[o];
#pragma unroll
      for (int sh = 32; sh > 0; sh >>= 1) mx = fmaxf(mx, __shfl_xor(mx, sh, 64));
      double b1 = 0.0;
#pragma unroll
      for (int d = 0; d < D; ++d) b1 = fmax(b1, bnd[1 + d]);
      const double le = log10(eps > 0.0 ? eps : 1e-300);
      feat[0] = (float)(0.1 * (log10(fmax(bnd[0], 1e-300)) - le));
      feat[1] = (float)(0.1 * (log10(fmax(b1, 1e-300)) - le));
      feat[2] = (float)(0.1 * (log10(fmax((double)mx, 1e-300)) - le));
      feat[3] = (float)(0.5 * log10(1.0 + cnt));
      double r = 0.0;
      if (a.xyz) {
        double d2 = 0.0;
        for (int k = 0; k < 3; ++k) {
          const double dd = a.xyz[3 * Io[o] + k] - a.xyz[3 * Jo[o] + k];
          d2 += dd * dd;
        }
        r = sqrt(d2);
      }
      feat[4] = (float)(0.1 * r);
      feat[5] = eIJ >= 0 ? (float)(0.1 * (log10(fmax((double)a.bn[(size_t)eIJ * (1 + D)], 1e-300)) - le))
                         : -3.f;
      feat[6] = 0.05f * (float)a.iter;
      feat[7] = square ? 1.f : 0.f;
      bool net_skip = false;
      float z = 0.f;
      if (a.skip == 2) {
        z = mlp_logit_wave(th, feat, lane);
        // the network may skip only an output whose exact bound is below
        // mlp_cap * eps for every matrix, and never, on the DOUBLE branch, a
        // stored block whose 2 ||X_IJ|| alone reaches eps
        bool allowed = true;
        double bmx = 0.0;
#pragma unroll
        for (int m = 0; m <= D; ++m) {
          allowed = allowed && bnd[m] < (double)a.mlp_cap * eps;
          if (!square && eIJ >= 0) allowed = allowed && 2.0 * (double)a.bn[(size_t)eIJ * (1 + D) + m] < eps;
          bmx = fmax(bmx, bnd[m]);
        }
        net_skip = allowed && z > a.mlp_z;
        if (net_skip && lane == 0) {
          atomicAdd(a.mlp_skipped, 1ull);
          atomicAdd(&a.mlp_bsum[sys], bmx);
        }
      }
      if (a.log_cap > 0) {
        logit_o[o] = true;
        // features (and the logit) to a slot claimed below; the wave keeps them
        // in its private scratch until then
        if (lane <= MLP_NF) {
          float v = z;
#pragma unroll
          for (int i = 0; i < MLP_NF; ++i) v = (lane == i) ? feat[i] : v;
          ns[wave * NO * (MLP_NF + 1) + o * (MLP_NF + 1) + lane] = v;
        }
        ++nlog;
      }
      if (net_skip) {
        owned[o] = false;
        netskip_mask |= 1u << o;
      }
    }
    if (a.log_cap > 0 && nlog > 0) {
      int base_slot = 0;
      if (lane == 0) base_slot = (int)atomicAdd(a.log_count, (unsigned long long)nlog);
      base_slot = __builtin_amdgcn_readfirstlane(base_slot);
      int rank = 0;
#pragma unroll
      for (int o = 0; o < NO; ++o) {
        if (!logit_o[o]) continue;
        const long long slot = (long long)base_slot + rank++;
        if (slot < a.log_cap) {
          const float* v = ns + wave * NO * (MLP_NF + 1) + o * (MLP_NF + 1);
          if (lane < MLP_NF) a.log_x[slot * MLP_NF + lane] = v[lane];
          if (lane == 0 && a.log_z) a.log_z[slot] = v[MLP_NF];
          // the outcome of an output the network skipped is not known
          if (lane == 0 && ((netskip_mask >> o) & 1u)) a.log_y[slot] = -1.f;
          if (lane == o) my_slot = (int)slot;
        }
      }
    }
    __syncthreads();  // the network and the scratch in buf are dead from here
    any_owned = false;
#pragma unroll
    for (int o = 0; o < NO; ++o) any_owned |= owned[o];
  }

  // outputs computed by this wave (bit o) and by this block (row masks)
  unsigned own_mask = 0u;
#pragma unroll
  for (int o = 0; o < NO; ++o) own_mask |= owned[o] ? (1u << o) : 0u;
  own_mask = __builtin_amdgcn_readfirstlane(own_mask);
  if (t < SP) sown[t] = 0u;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int o = 0; o < NO; ++o)
      if (owned[o]) atomicOr(&sown[so[o]], 1u << to[o]);
  }
  __syncthreads();

  // Products of one column block K (buffer bb, slot gi) for the present
  // outputs pm (K-steps of 4 up to the block size).  mk holds, lane gi*NE + x,
  // the mask of the nonzero matrices of block x of the column: a product with
  // a zero operand block is not issued (it would add exact zeros).
  unsigned long long nprod = 0;  // block products issued by this wave
  auto column = [&](unsigned pm, int bb, int gi, int mk) {
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      if (!((pm >> o) & 1u)) continue;
      const unsigned ma = (unsigned)__builtin_amdgcn_readlane(mk, gi * NE + so[o]);
      const unsigned mb = (unsigned)__builtin_amdgcn_readlane(mk, gi * NE + SP + to[o]);
      // enabled products: bit 0 X0 X0; bit 1 + d X0 X1_d; bit 1 + MAXD + d X1_d X0
      unsigned en = ma & mb & 1u;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        en |= ((ma & (mb >> (1 + d))) & 1u) << (1 + d);
        en |= (((ma >> (1 + d)) & mb) & 1u) << (1 + MAXD + d);
      }
      en = __builtin_amdgcn_readfirstlane(en);
      if (!en) continue;
      nprod += __popc(en);
      const T* xa = &buf[bb][gi][so[o]][0];
      const T* xb = &buf[bb][gi][SP + to[o]][0];
      if constexpr (BF && W) {
        // bfloat16 three-way split: each operand value v = h + m + l; the six
        // cross products above 2^-24 of the leading term (l h, h l, m m, m h,
        // h m, h h, smallest first) run as 16x16x16 bfloat16 MFMAs into an
        // FP32 temporary per column block, which is added to the FP64 sums
        s4 ah[1 + D], am[1 + D], al[1 + D], bh[1 + D], bm[1 + D], bl[1 + D];
#pragma unroll
        for (int m = 0; m <= D; ++m) {
          bf16_split3((const float*)xa + m * BS, lane, ah[m], am[m], al[m]);
          bf16_split3((const float*)xb + m * BS, lane, bh[m], bm[m], bl[m]);
        }
        Acc<float> tmp[1 + D];
#pragma unroll
        for (int m = 0; m <= D; ++m)
#pragma unroll
          for (int r = 0; r < 4; ++r) tmp[m].v[r] = 0.f;
        auto prod3 = [&](Acc<float>& c, int ma, int mb) {
          mfma_bf16(c, al[ma], bh[mb]);
          mfma_bf16(c, ah[ma], bl[mb]);
          mfma_bf16(c, am[ma], bm[mb]);
          mfma_bf16(c, am[ma], bh[mb]);
          mfma_bf16(c, ah[ma], bm[mb]);
          mfma_bf16(c, ah[ma], bh[mb]);
        };
        if (en & 1u) prod3(tmp[0], 0, 0);
#pragma unroll
        for (int d = 0; d < D; ++d) {
          if ((en >> (1 + d)) & 1u) prod3(tmp[1 + d], 0, 1 + d);
          if ((en >> (1 + MAXD + d)) & 1u) prod3(tmp[1 + d], 1 + d, 0);
        }
        if (en & 1u) {
#pragma unroll
          for (int r = 0; r < 4; ++r) wacc[o][0].v[r] += (double)tmp[0].v[r];
        }
#pragma unroll
        for (int d = 0; d < D; ++d)
          if ((en >> (1 + d)) & ((1u << MAXD) | 1u)) {
#pragma unroll
            for (int r = 0; r < 4; ++r) wacc[o][1 + d].v[r] += (double)tmp[1 + d].v[r];
          }
      } else if constexpr (BF) {
        // bfloat16 operands: one 16x16x16 MFMA per block product
        const s4 a0 = bf16_frag((const float*)xa, lane), b0 = bf16_frag((const float*)xb, lane);
        if (en & 1u) mfma_bf16(acc[o][0], a0, b0);
#pragma unroll
        for (int d = 0; d < D; ++d) {
          if ((en >> (1 + d)) & 1u) {
            const s4 b1 = bf16_frag((const float*)xb + (1 + d) * BS, lane);
            mfma_bf16(acc[o][1 + d], a0, b1);
          }
          if ((en >> (1 + MAXD + d)) & 1u) {
            const s4 a1 = bf16_frag((const float*)xa + (1 + d) * BS, lane);
            mfma_bf16(acc[o][1 + d], a1, b0);
          }
        }
      } else {
        // Every operand fragment of the output's column blocks is read from
        // LDS at once (one wait); X0's fragments serve all of its products.
        // Each enabled product then runs its K-steps as one straight block.
        T fa[1 + D][4], fb[1 + D][4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          if (!FK && kk >= a.ksteps) break;
#pragma unroll
          for (int m = 0; m <= D; ++m) {
            fa[m][kk] = xa[m * BS + lane + kk * 64];
            fb[m][kk] = xb[m * BS + lane + kk * 64];
          }
        }
        // W: this column's FP32 products go to temporaries, then to the FP64 sums
        Acc<T> tmp[W ? 1 + D : 1];
        if constexpr (W) {
#pragma unroll
          for (int m = 0; m <= D; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) tmp[m].v[r] = 0.f;
        }
        Acc<T>* dst = W ? tmp : &acc[W ? 0 : o][0];
        auto prod = [&](Acc<T>& cc, const T* ra, const T* rb) {
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            if (!FK && kk >= a.ksteps) break;
            mfma(cc, ra[kk], rb[kk]);
          }
        };
        if (en & 1u) prod(dst[0], fa[0], fb[0]);
#pragma unroll
        for (int d = 0; d < D; ++d) {
          if ((en >> (1 + d)) & 1u) prod(dst[1 + d], fa[0], fb[1 + d]);
          if ((en >> (1 + MAXD + d)) & 1u) prod(dst[1 + d], fa[1 + d], fb[0]);
        }
        if constexpr (W) {
          if (en & 1u) {
#pragma unroll
            for (int r = 0; r < 4; ++r) wacc[o][0].v[r] += (double)tmp[0].v[r];
          }
#pragma unroll
          for (int d = 0; d < D; ++d)
            if ((en >> (1 + d)) & ((1u << MAXD) | 1u)) {
#pragma unroll
              for (int r = 0; r < 4; ++r) wacc[o][1 + d].v[r] += (double)tmp[1 + d].v[r];
            }
        }
      }
    }
  };

  for (int base = pp0; base < pp1; base += KLC) {
    // ---- common columns of this chunk of P's panel with Q's panel
    const int end = min(pp1, base + KLC);
    const int nm = build_kl(base, end, true);
    // ---- pipelined products over the common columns
    const int ngroups = (nm + KG - 1) / KG;
    int e_next = 0, m_cur = 0, m_next = 0;
    if (ngroups > 0) {
      const int e0 = load_entries(0, nm);
      issue(e0, 0);
      m_cur = load_masks(e0);
      e_next = load_entries(1, nm);
    }
    for (int g = 0; g < ngroups; ++g) {
      const int bb = g & 1;
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
      if (g + 1 < ngroups) {
        issue(e_next, bb ^ 1);
        m_next = load_masks(e_next);
        e_next = load_entries(g + 2, nm);
      }
      if (any_owned) {
#pragma unroll
        for (int gi = 0; gi < KG; ++gi) {
          if (g * KG + gi >= nm) break;
          // outputs with both blocks present in this column, as a wave-uniform
          // mask: the branches below are scalar, and each present output runs
          // its products for the column as one straight block
          const unsigned pe = (unsigned)__ballot(lane < NE && sflag[bb][gi][lane < NE ? lane : 0] >= 0);
          unsigned pm = 0u;
#pragma unroll
          for (int o = 0; o < NO; ++o) pm |= ((pe >> so[o]) & (pe >> (SP + to[o])) & 1u) << o;
          pm = __builtin_amdgcn_readfirstlane(pm & own_mask);
#pragma unroll
          for (int o = 0; o < NO; ++o) np[o] += (int)((pm >> o) & 1u);
          column(pm, bb, gi, m_cur);
        }
      }
      m_cur = m_next;
    }
    __syncthreads();
  }

  // ---- epilogue: lane o looks up the old block (I_o, J_o) for output o
  EpiCtx E{a.xv, (size_t)PER, a.h_rp, a.h_ci, a.h_v, {a.h1_rp[0], a.h1_rp[1], a.h1_rp[2]},
           {a.h1_ci[0], a.h1_ci[1], a.h1_ci[2]}, {a.h1_v[0], a.h1_v[1], a.h1_v[2]}, a.stage,
           a.kept_ij, a.stage_count, a.stage_cap, a.overflow, a.bad};
  double q[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) q[k] = 0.0;
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    const int eIJ = __builtin_amdgcn_readlane(my_e, o);
    const int slot = __builtin_amdgcn_readlane(my_slot, o);
    if (!owned[o]) continue;
    bool kept = false;
    if (np[o] > 0) {
      if constexpr (W)
        kept = epilogue<T, D, AccW>(E, wacc[o], Io[o], Jo[o], eIJ, square, eps, np[o], sys, q);
      else
        kept = epilogue<T, D>(E, acc[o], Io[o], Jo[o], eIJ, square, eps, np[o], sys, q);
    }
    if (slot >= 0 && lane == 0) a.log_y[slot] = kept ? 0.f : 1.f;  // label: dropped
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NQ; ++k) spart[wave][k] = q[k];
    if (nprod) atomicAdd(a.exec_pairs, nprod);
  }
  __syncthreads();
  if (t < NQ) {
    double sum = 0.0;
    for (int w = 0; w < NW; ++w) sum += spart[w][t];
    a.partial[(size_t)lb * NQ + t] = sum;
  }
  }  // sub-tiles
}

// ------------------------------------------------------------------ copy-through
// One wave per entry (I, J >= I) of a stopped system: its blocks go to the
// stage unchanged (row-major upper block).
template <typename T>
__global__ void k_copy_through(CopyArgs a) {
  const int lane = threadIdx.x & 63;
  const int nnz = a.rp[a.nb];
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long w = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < nnz;
       w += nwaves) {
    const int e = (int)w;
    int lo = 0, hi = a.nb;  // row of entry e
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (a.rp[mid] <= e) lo = mid; else hi = mid;
    }
    const int I = lo, J = a.ci[e];
    if (J < I || a.active[a.sys_of[I]]) continue;
    int slot = 0;
    if (lane == 0) slot = atomicAdd(a.stage_count, 1);
    slot = __builtin_amdgcn_readfirstlane(slot);
    if (slot >= a.stage_cap) {
      if (lane == 0) atomicOr(a.overflow, 1);
      continue;
    }
    const int per = (1 + a.D) * BS;
    const T* X = (const T*)a.xv + (size_t)e * per;
    T* st = (T*)a.stage + (size_t)slot * per;
    for (int q = lane; q < per; q += 64) {
      const int m = q / BS, qq = q - m * BS;  // stage index qq = r*16 + c
      const int r = qq >> 4, c = qq & 15;
      st[q] = X[m * BS + c * BP + r];
    }
    if (lane == 0) a.kept_ij[slot] = make_int2(I, J);
  }
}

// ------------------------------------------------------------------ block norms
// Frobenius norm of every stored block of every matrix (float), one wave per
// entry; used by the screens.
template <typename T>
__global__ void k_block_norms(long long nnz, int D, const T* xv, float* bn, const int* nnz_dev) {
  const int lane = threadIdx.x & 63;
  if (nnz_dev) nnz = min(nnz, (long long)*nnz_dev);
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long e = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; e < nnz;
       e += nwaves) {
    for (int m = 0; m <= D; ++m) {
      const T* x = xv + ((size_t)e * (1 + D) + m) * BS;
      double ss = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double v = (double)x[lane + 64 * j];
        ss += v * v;
      }
      ss = wave_sum(ss);
      if (lane == 0) bn[(size_t)e * (1 + D) + m] = (float)sqrt(ss);
    }
  }
}

void launch_block_norms(hipStream_t st, int prec, long long nnz, int D, const void* xv, float* bn,
                        const int* nnz_dev) {
  if (nnz == 0) return;
  // one wave per entry, waves loop over entries beyond 2^24 blocks of 4 waves
  const long long want = (nnz + 3) / 4;
  const unsigned blocks = (unsigned)(want < (1 << 20) ? want : (1 << 20));
  if (prec == P_FP64)
    hipLaunchKernelGGL(k_block_norms<double>, dim3(blocks), dim3(256), 0, st, nnz, D,
                       (const double*)xv, bn, nnz_dev);
  else
    hipLaunchKernelGGL(k_block_norms<float>, dim3(blocks), dim3(256), 0, st, nnz, D,
                       (const float*)xv, bn, nnz_dev);
}

// ================================================================== launchers
void launch_panels(hipStream_t st, int pass, const PanelArgs& a) {
  if (a.nc == 0) return;
  const size_t lds = (size_t)((a.max_sys_atoms + 31) / 32) * 8;  // bitmap + prefix counts
  hipLaunchKernelGGL(k_panels, dim3(a.nc), dim3(PNT), lds, st, pass, a);
}

void launch_tiles(hipStream_t st, int pass, const PanelArgs& a) {
  if (a.nc == 0) return;
  const size_t lds = (size_t)a.tile_words * 4;
  hipLaunchKernelGGL(k_tiles, dim3(a.nc), dim3(PNT), lds, st, pass, a);
}

// Sub-tile shapes (rows of cluster P x columns of cluster Q per workgroup).
// Which ones exist depends on the kernel kind and D: the accumulators of a
// wave ((1 + D) tiles per owned output) must stay within its register budget.
constexpr int SHAPE_SP[TS_N] = {8, 4, 8, 4};
constexpr int SHAPE_TQ[TS_N] = {8, 8, 4, 4};

constexpr bool shape_ok(int kind, int D, int s) {
  return ((kind == K_FP64 || kind == K_WIDE) && D >= 2)
             ? s == TS_4x4
             : (s == TS_8x8 || ((D == 1 || D == 3) && s == TS_4x8) ||
                (D == 1 && kind != K_BF16 && s == TS_8x4));
}

bool tile_shape_available(int kind, int D, int shape) {
  return kind >= 0 && kind < 4 && D >= 0 && D <= MAXD && shape >= 0 && shape < TS_N &&
         shape_ok(kind, D, shape);
}

int tile_shape_default(int kind, int D) {
  return ((kind == K_FP64 || kind == K_WIDE) && D >= 2) ? TS_4x4 : TS_8x8;
}

int tile_subs(int shape) { return (CS / SHAPE_SP[shape]) * (CS / SHAPE_TQ[shape]); }

const char* tile_shape_name(int shape) {
  static const char* names[TS_N] = {"8x8", "4x8", "8x4", "4x4"};
  return (shape >= 0 && shape < TS_N) ? names[shape] : "?";
}

// Blocks of a persistent launch: enough to fill every CU at the kernel's
// occupancy (computed once per instance).
template <typename T, int D, int SP, int TQ, bool BF, bool W, bool FK, int WS>
static unsigned resident_blocks() {
  static int per_cu = -1, cus = 0;
  if (per_cu < 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_tile_numeric<T, D, SP, TQ, BF, W, FK, WS>,
                                                     TQ * WS * 64, 0) != hipSuccess || n < 1) {
      cus = 256;
      n = 1;
    }
    per_cu = n;
  }
  return (unsigned)(per_cu * cus);
}

template <typename T, int D, int SP, int TQ, bool BF, bool W, bool FK, int WS>
static void tile_go_w(hipStream_t st, const TileArgs& a) {
  unsigned G = (unsigned)a.n_tiles * (unsigned)((CS / SP) * (CS / TQ));
  if (a.work) {  // persistent: never more blocks than sub-tiles or than fit at once
    const unsigned R = resident_blocks<T, D, SP, TQ, BF, W, FK, WS>();
    G = G < R ? G : R;
  }
  hipLaunchKernelGGL((k_tile_numeric<T, D, SP, TQ, BF, W, FK, WS>), dim3(G), dim3(TQ * WS * 64), 0,
                     st, a);
}

// Waves per sub-tile column.  The 4 x 4 sub-tile with two or three
// directions (FP64, and the kinds with FP64 sums: FP32 products and the
// bfloat16 split) runs sixteen waves (four per column, one output each, four
// per SIMD); the 8 x 8 sub-tile with at most one direction (FP64, FP32 with
// FP64 sums) sixteen (two per column, four outputs each); the other kinds and
// shapes one wave per column.
template <typename T, int D, int SP, int TQ, bool BF, bool W, bool FK>
static void tile_go_k(hipStream_t st, const TileArgs& a) {
  if constexpr (D >= 2 && SP == 4 && TQ == 4 && (sizeof(T) == 8 || W)) {
    if (a.waves_per_column != 1) return tile_go_w<T, D, SP, TQ, BF, W, FK, 4>(st, a);
  }
  if constexpr (D <= 1 && SP == 8 && TQ == 8 && (sizeof(T) == 8 || (W && !BF))) {
    if (a.waves_per_column != 1) return tile_go_w<T, D, SP, TQ, BF, W, FK, 2>(st, a);
  }
  tile_go_w<T, D, SP, TQ, BF, W, FK, 1>(st, a);
}

template <typename T, int D, bool BF, bool W, int S>
static void tile_go(hipStream_t st, const TileArgs& a) {
  constexpr int SP = SHAPE_SP[S], TQ = SHAPE_TQ[S];
  // bfloat16 products take the whole padded K in one MFMA: no K-step loop
  if constexpr (!BF) {
    if (a.ksteps == 4) return tile_go_k<T, D, SP, TQ, BF, W, true>(st, a);
  }
  tile_go_k<T, D, SP, TQ, BF, W, false>(st, a);
}

// false when the shape does not exist for this kind
template <typename T, int D, bool BF, bool W>
static bool tile_shape_go(hipStream_t st, const TileArgs& a) {
  // the bfloat16 split with FP64 sums has the accumulators of the FP32 kind with FP64 sums
  constexpr int KIND = sizeof(T) == 8 ? K_FP64 : (W ? K_WIDE : (BF ? K_BF16 : K_FP32));
  switch (a.shape) {
    case TS_8x8:
      if constexpr (shape_ok(KIND, D, TS_8x8)) { tile_go<T, D, BF, W, TS_8x8>(st, a); return true; }
      break;
    case TS_4x8:
      if constexpr (shape_ok(KIND, D, TS_4x8)) { tile_go<T, D, BF, W, TS_4x8>(st, a); return true; }
      break;
    case TS_8x4:
      if constexpr (shape_ok(KIND, D, TS_8x4)) { tile_go<T, D, BF, W, TS_8x4>(st, a); return true; }
      break;
    case TS_4x4:
      if constexpr (shape_ok(KIND, D, TS_4x4)) { tile_go<T, D, BF, W, TS_4x4>(st, a); return true; }
      break;
    default: break;
  }
  return false;
}

template <typename T, int D>
static bool tile_launch(hipStream_t st, const TileArgs& a) {
  if constexpr (sizeof(T) == 4) {
    if (a.bf16) return a.wide ? tile_shape_go<T, D, true, true>(st, a) : tile_shape_go<T, D, true, false>(st, a);
    if (a.wide) return tile_shape_go<T, D, false, true>(st, a);
  }
  return tile_shape_go<T, D, false, false>(st, a);
}

template <typename T>
static bool tile_d(hipStream_t st, const TileArgs& a) {
  switch (a.D) {
    case 0: return tile_launch<T, 0>(st, a);
    case 1: return tile_launch<T, 1>(st, a);
    case 2: return tile_launch<T, 2>(st, a);
    default: return tile_launch<T, 3>(st, a);
  }
}

bool launch_tile_numeric(hipStream_t st, int prec, const TileArgs& a) {
  if (a.n_tiles == 0) return true;
  if (prec == P_FP64) return tile_d<double>(st, a);
  return tile_d<float>(st, a);
}

void launch_copy_through(hipStream_t st, int prec, const CopyArgs& a, int nnz) {
  if (nnz == 0) return;
  const long long want = ((long long)nnz + 3) / 4;
  const unsigned blocks = (unsigned)(want < (1 << 20) ? want : (1 << 20));
  if (prec == P_FP64) hipLaunchKernelGGL(k_copy_through<double>, dim3(blocks), dim3(256), 0, st, a);
  else hipLaunchKernelGGL(k_copy_through<float>, dim3(blocks), dim3(256), 0, st, a);
}

}  // namespace tc2
