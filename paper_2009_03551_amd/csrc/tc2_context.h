// The solver context behind the opaque tc2_ctx of include/tc2.h: device
// buffers, the merged problem, the state of a solve in progress and the
// counters it reports.  Shared by the runtime (setup, the update loop) and the
// measurement entry points (row export, iterate export and comparison, exact
// useful-flop counting).
#pragma once

#include "tc2_internal.h"
#include "../../include/tc2.h"

#include <string>
#include <utility>
#include <vector>

namespace tc2 {

// ------------------------------------------------------------------ device buffers
// Buffers of at least VM_MIN bytes live in a reserved virtual range with
// physical chunks mapped as they grow, taken from and given back to a pool
// per device (tc2_memory.hip); smaller ones are plain allocations.
struct DBuf;
constexpr size_t VM_MIN = (size_t)64 << 20;
hipError_t vm_grow(DBuf& b, size_t n);     // map up to >= n bytes, contents kept
void vm_release(DBuf& b);                  // chunks back to the pool, range freed
hipError_t dev_malloc(void** p, size_t n); // hipMalloc, retried after pool_trim
void pool_trim();                          // pooled chunks of the device to the GPU driver

struct DBuf {
  void* p = nullptr;
  size_t cap = 0;
  bool vm = false;                         // p is a virtual range (see above)
  size_t va = 0;                           // its reserved bytes
  int dev = 0;
  std::vector<hipMemGenericAllocationHandle_t> chunks;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void release() {
    if (vm) {
      vm_release(*this);
      return;
    }
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  // grow to at least n bytes (contents are not preserved)
  hipError_t reserve(size_t n) {
    if (n <= cap && p) return hipSuccess;
    if (vm || n >= VM_MIN) {
      if (!vm) release();
      const hipError_t e = vm_grow(*this, n);
      if (e != hipErrorNotSupported) return e;
      (void)hipGetLastError();
    }
    release();
    size_t want = n < 256 ? 256 : n;
    hipError_t e = dev_malloc(&p, want);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    cap = want;
    return hipSuccess;
  }
  // grow to at least n bytes; a plain allocation grows by at least a quarter
  // of its capacity, so that a buffer that grows over many updates is
  // reallocated a few times instead of at every update (contents are not
  // preserved)
  hipError_t reserve_grow(size_t n) {
    if (n <= cap && p) return hipSuccess;
    if (vm || n >= VM_MIN) return reserve(n);
    const size_t g = cap + cap / 4;
    return reserve(n > g ? n : g);
  }
  // grow to at least n bytes keeping the first `keep` bytes (a virtual range
  // keeps them by mapping more chunks; a plain allocation is copied on
  // stream st into its replacement, then freed)
  hipError_t grow_keep(size_t n, size_t keep, hipStream_t st) {
    if (n <= cap && p) return hipSuccess;
    if (vm) return vm_grow(*this, n);
    if (n >= VM_MIN) {
      DBuf t;
      hipError_t e = vm_grow(t, n);
      if (e == hipSuccess) {
        if (p && keep) {
          e = hipMemcpyAsync(t.p, p, keep < cap ? keep : cap, hipMemcpyDeviceToDevice, st);
          if (e == hipSuccess) e = hipStreamSynchronize(st);
          if (e != hipSuccess) return e;
        }
        release();
        swap(t);
        return hipSuccess;
      }
      if (e != hipErrorNotSupported) return e;
      (void)hipGetLastError();
    }
    const size_t g = cap + cap / 4;
    const size_t want = n > g ? n : g;
    void* q = nullptr;
    hipError_t e = dev_malloc(&q, want);
    if (e != hipSuccess) return e;
    if (p && keep) {
      e = hipMemcpyAsync(q, p, keep < cap ? keep : cap, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        (void)hipFree(q);
        return e;
      }
    }
    release();
    p = q;
    cap = want;
    return hipSuccess;
  }
  void swap(DBuf& o) {
    std::swap(p, o.p);
    std::swap(cap, o.cap);
    std::swap(vm, o.vm);
    std::swap(va, o.va);
    std::swap(dev, o.dev);
    chunks.swap(o.chunks);
  }
  template <typename T> T* as() const { return (T*)p; }
};

// Page-locked host memory for the small per-update transfers: copies to and
// from it are plain DMAs, where pageable memory goes through staging copies.
struct HostPin {
  void* p = nullptr;
  size_t cap = 0;
  HostPin() = default;
  HostPin(const HostPin&) = delete;
  HostPin& operator=(const HostPin&) = delete;
  ~HostPin() {
    if (p) (void)hipHostFree(p);
  }
  hipError_t reserve(size_t n) {
    if (n <= cap && p) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    hipError_t e = hipHostMalloc(&p, n, hipHostMallocDefault);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    cap = n;
    return hipSuccess;
  }
};

struct HostBsr {
  std::vector<int64_t> row_ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

struct SysInfo {
  int row0 = 0, nb = 0;
  int64_t n_occ = 0;
  double eps = 0, tol = 0;
  int max_iter = 0;
  std::string replay;
  int mode = 0;  // 0 iterate, 1 trivial zero (Nocc = 0), 2 trivial identity (Nocc = N)
};

struct SysState {
  bool active = false;
  int k = 0;
  double prev[1 + 2 * MAXD] = {0};
  std::vector<double> iota;
  std::string branches;
  int closing_left = 0;
  int closing_first = 1;
  tc2_status status = TC2_OK;
  double trip = 0;                     // union-pattern block triples on kept outputs
  double nominal = 0;                  // full-product block triples (sum of m_K^2)
};

// State of the solve in progress: tc2_run runs a whole solve; tc2_advance may
// stop between two updates and continue from here.
struct RunState {
  bool open = false;                   // a solve has begun and not finished
  hipStream_t st = nullptr;
  std::vector<SysState> ss;
  std::vector<double> emin, emax, scal;
  std::vector<int> mode, active, branch, bad;
  std::vector<unsigned long long> nominal;
  size_t pin_nominal = 0;
  int phase = 0;                       // 0: working precision, 1: closing FP64 pair
  int updates = 0;
  bool later_stage = false, reduced = false;
  unsigned long long exec_pairs = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

}  // namespace tc2

struct tc2_ctx {
  int device = 0;
  hipStream_t own = nullptr;
  int nsys = 0, D = 0, b = 0, nb = 0, prec = tc2::P_FP64, closing = 0, verbose = 0, export_m = 0;
  int profile = 0;
  hipEvent_t pev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  double ms_sym = 0, ms_num = 0, ms_cmp = 0;
  double ms_num_kind[4] = {0, 0, 0, 0};
  int launches_kind[4] = {0, 0, 0, 0};
  int last_kind = 0;                // kernel kind of the last update
  int num_launches = 0;
  int max_sys_atoms = 0;
  std::vector<tc2::SysInfo> sys;
  // host copies kept for export
  std::vector<int> h_sys_of;
  // device: systems
  tc2::DBuf sys_of, sys_start, sys_end, active, branch, mode, eps, emin, emax, bad;
  // device: H and H1
  tc2::DBuf h_rp, h_ci, h_v;
  tc2::DBuf h1_rp[tc2::MAXD], h1_ci[tc2::MAXD], h1_v[tc2::MAXD];
  // initial pattern (union of H and H1 patterns) and its sources
  int nnz0 = 0;
  tc2::DBuf x0_rp, x0_ci, x0_row, src_h, src_h1[tc2::MAXD];
  // iterate: the pattern (rp, ci) is double buffered; the values are held in
  // one buffer, xv[cur] (an update writes the new values over the old ones
  // once its products have read them; the other slot is empty except during
  // a precision switch)
  tc2::DBuf rp[2], ci[2], xv[2];
  int nnz[2] = {0, 0};
  int cur = 0;
  int cur_prec = tc2::P_FP64;
  bool have_iterate = false;      // a solve has produced (or begun) an iterate
  // work buffers
  tc2::DBuf cand_cnt, cand_rp, cand_ci, item_cnt, item_rp, item_row, item_c0, partial;
  tc2::DBuf stage, kept_ij, counters, exec_pairs, rowcnt, cursor, tmp_ci, tmp_src, new_src;
  tc2::HostPin pin_graph;         // per-update readback of the graph path
  tc2::HostPin pin_loop;          // active / branch flags in, bad / nominal out
  tc2::DBuf sys_lo, sys_hi, scal, rowlo, rowhi, xfer;
  long long stage_cap = 0;
  int kernel = 0;                 // 0 tiled, 1 one wave per block
  int fp64_first = 0;             // leading FP64 updates of a reduced-precision solve
  int op_bf16 = 0;                // current stage rounds MFMA operands to bfloat16
  int wide = 0;                   // FP32 stages: FP64 sums over the column blocks
  int shape[4] = {0, 0, 0, 0};    // sub-tile shape per kernel kind
  bool tuned[4] = {false, false, false, false};
  int tune = 0;                   // 1: measure the shapes once per kind
  std::string tune_cache;         // file of tuned shapes ("" = none)
  std::string arch;               // device architecture name (cache key)
  long long prev_out_bound = -1;  // candidate outputs of the previous update
  double ms_tune = 0.0;
  bool kind_used[4] = {false, false, false, false};
  int skip = 0;                   // 1: exact norm-bound screen, 2: + skip network
  int skip_now = 0;               // the screen of the current update (2 falls back
                                  // to 1 once the network's budget is spent)
  float mlp_cap = 4.f;            // network skips only outputs with bound < mlp_cap * eps
  double mlp_budget = 0.0;        // per system and solve: sum of the bounds of the
                                  // outputs the network may skip (0: no limit)
  tc2::DBuf mlp_bsum;             // per system: that sum so far in this solve
  int mlp_updates = 0;            // updates run with the network in this solve
  tc2::DBuf bn, screened;         // block norms, skip counters [exact, network]
  bool bn_valid = false;          // bn holds the norms of the current iterate
                                  // (written by the last captured update's gather)
  tc2::DBuf nominal;              // per system: sum over rows K of m_K^2, this update
  unsigned long long screened_total = 0, mlp_total = 0;
  tc2::DBuf mlp;                  // skip network parameters
  float mlp_z = 0.f;              // logit of the skip threshold
  tc2::DBuf xyz;                  // merged positions (all problems gave them)
  bool have_xyz = false;
  long long log_cap = 0, log_n = 0;
  tc2::DBuf log_x, log_y, log_z, log_count;
  int update_index = 0;
  // per-entry masks of the nonzero matrices of each pattern buffer (see
  // mask_iterate), and the exact useful-flop count (count_useful): per system
  // x kernel kind, the useful block products on kept outputs
  int count_useful = 0;
  std::string metrics_log;        // JSONL file of per-update scalars ("" = none)
  int solve_index = 0;            // solves begun by this context
  tc2::DBuf mask[2];
  tc2::DBuf useful_acc;           // nsys x 4 kinds, unsigned long long
  // test knobs (environment, read at setup): shorter panel passes in the
  // tiled kernel, and a tiny stage that overflows every update
  int test_kl_chunk = 0;
  long long test_stage_cap = 0;
  int test_no_zero_skip = 0;      // issue every product (masks not passed to the kernel)
  int test_waves_per_column = 0;  // 1: one wave per sub-tile column in every numeric kernel
  std::vector<int> h_active;      // host copy of the active flags
  // clusters
  int nc = 0, max_sys_clusters = 0;
  long long tile_bound = 0;       // most tiles an update can have (P <= Q per system)
  tc2::DBuf clus_atom, clus_sys, atom_clus, csys_start, csys_end;
  // graph-captured updates (tiled kernel): one executable graph per iterate
  // buffer, valid while the key (buffers, sizes, kind, shape) is unchanged
  int graph = 0;                  // option: capture updates in hipGraphs
  bool graph_ok = true;           // false after a capture the runtime refused
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipGraphExec_t gexec_post[2] = {nullptr, nullptr};  // profiling: the part after the products
  std::vector<unsigned long long> gkey[2];
  long long kept_prev = 0, kept_prev2 = 0, kept_prev3 = 0;  // kept upper blocks, last updates
  int graph_updates = 0, graph_captures = 0;
  // branch and stopping decisions on the device (device_loop): per-system
  // records, parameters and the flag word the host polls
  int device_loop = 0;            // option: updates replayed between two polls
  int dl_updates = 0;             // updates of this solve decided on the device
  int dl_last = 0;                // updates of the last device-loop solve (batch sizing)
  long long dl_cap = 0;           // dense bound of the kept upper blocks
  tc2::DBuf dl_state, dl_param, dl_word;
  tc2::HostPin pin_dl;            // the word and the records, read back
  tc2::DBuf panel_cnt, panel_rp, panel_k, panel_e, tile_cnt, tile_rp, tile_pairs, tile_p, tile_q;
  tc2::DBuf tile_bits;            // cluster bitmaps kept between the two tile passes
  // the solve in progress
  tc2::RunState run;
  // results
  std::vector<tc2::HostBsr> out_x0;
  std::vector<tc2::HostBsr> out_x1[tc2::MAXD];
};

namespace tc2 {

inline size_t prec_bytes(int prec) { return prec == P_FP64 ? 8 : 4; }

// Exact useful-flop count of one update (tc2_measure.hip): masks of the new
// iterate, then the block triples of the update on kept outputs into
// ctx->useful_acc under the kernel kind of the update.
tc2_status count_update(tc2_ctx* ctx, hipStream_t st);
// Masks of the nonzero matrices of every entry of the current iterate (bit m
// of mask[e] set when block m of entry e has a nonzero element).  The numeric
// kernel issues no product with a zero operand block; the useful count uses
// the masks of the old and the new iterate.
tc2_status mask_iterate(tc2_ctx* ctx, hipStream_t st);
// The same for nnz entries of xv (at most *nnz_dev when given), as stream work.
void launch_block_masks(hipStream_t st, int prec, long long nnz, int D, const void* xv,
                        unsigned char* mask, const int* nnz_dev);
// The gather of the new values from the stage (at most nnz entries, *nnz_dev
// when given) together with their masks and, bn given, their block norms (as
// k_block_norms computes them), in one pass; nothing is written when
// *skip_flag is set (an overflowed stage: the update runs again).
void launch_gather_masks(hipStream_t st, int prec, long long nnz, int D, const int* new_src,
                         const void* stage, void* xv, unsigned char* mask, float* bn,
                         const int* nnz_dev, const int* skip_flag);

}  // namespace tc2
