// Internal declarations shared by the TC2 runtime and its kernels.
//
// Device data layout (one merged block-diagonal matrix for a batch of
// systems; every system has nb_s atom rows, all with the same block size b):
//
//  * pattern: int32 row pointer rp[nb+1] and sorted column indices ci[nnz]
//    holding BOTH triangles of the symmetric pattern;
//  * values: for entry e and matrix m (m = 0 for X0, 1..D for X1_d) one
//    padded 16 x 16 tile at ((e*(1+D) + m) * 256), stored COLUMN-major
//    (element (r, c) at c*16 + r) and zero outside the b x b corner.  With
//    this layout the MFMA A and B fragments of a block product are single
//    contiguous 64-lane loads (see the numeric kernel);
//  * H and H1_d are stored the same way (one matrix per value array).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tc2 {

constexpr int BP = 16;        // padded block dimension
constexpr int BS = BP * BP;   // elements per padded block
constexpr int MAXD = 3;       // field directions
constexpr int NQ = 4 + 3 * MAXD;  // per-work-item partial sums (see Q_*)
constexpr int CHUNK = 32;     // candidates per numeric work item
constexpr int MAX_SYS_BITS = 1 << 19;  // atoms per system (symbolic bitmap)
constexpr int CS = 8;         // atoms per cluster (tiled numeric kernel)
constexpr int MLP_NF = 8;     // skip network: input features
constexpr int MLP_NH = 64;    // hidden units per layer
constexpr int MLP_NP = MLP_NH * MLP_NF + MLP_NH + MLP_NH * MLP_NH + MLP_NH + MLP_NH + 1;

// partial-sum slots
enum {
  Q_TR0 = 0,   // Tr X0
  Q_FRO0 = 1,  // ||X0||_F^2
  Q_E0 = 2,    // Tr(X0 H)
  Q_TRIP = 3,  // block triples landing on kept output blocks
  Q_TR1 = 4,   // Tr X1_d           (4 .. 4+D-1)
  Q_E1 = 4 + MAXD,       // Tr(X1_d H)
  Q_AL = 4 + 2 * MAXD,   // Tr(X1_d H1_d)
};

enum Prec { P_FP64 = 0, P_FP32 = 1, P_BF16 = 2 };

// Kinds of the tiled numeric kernel: FP64 values; FP32 values with FP32 sums;
// FP32 values with bfloat16 MFMA operands; FP32 values with FP64 sums over the
// column blocks.
enum Kind { K_FP64 = 0, K_FP32 = 1, K_BF16 = 2, K_WIDE = 3 };
// Sub-tile shapes of the tiled kernel: rows of cluster P x columns of cluster Q
enum TileShape { TS_8x8 = 0, TS_4x8 = 1, TS_8x4 = 2, TS_4x4 = 3 };
constexpr int TS_N = 4;

struct SymArgs {
  int nb;
  const int* rp;        // current pattern
  const int* ci;
  const int* sys_of;    // row -> system
  const int* sys_end;   // system -> one past its last row
  const int* active;    // system -> 1 while iterating
  const int* cand_rp;   // fill pass only
  int* cand_cnt;        // count pass output (nb)
  int* cand_ci;         // fill pass output
  int max_sys_atoms;    // largest system (LDS bitmap size)
};

struct MeasArgs {
  int nb;
  int D;
  const int* rp;
  const int* ci;
  const void* xv;
  const int* h_rp;
  const int* h_ci;
  const double* h_v;
  const int* h1_rp[MAXD];
  const int* h1_ci[MAXD];
  const double* h1_v[MAXD];
  double* partial;      // nb x NQ
};

struct NumArgs {
  int nb;
  int D;
  int b;
  int ksteps;               // ceil(b/4): K-steps of 4 in the padded tile
  const int* rp;            // current pattern
  const int* ci;
  const void* xv;           // current values (T)
  const int* cand_rp;       // upper-triangle candidates
  const int* cand_ci;
  const int* item_row;      // work item -> row
  const int* item_c0;       // work item -> first candidate
  int n_items;
  const int* sys_of;
  const int* active;
  const int* branch;        // system -> 1 SQUARE, 0 DOUBLE
  const double* eps;        // system -> drop threshold
  // H and H1 (for the band energies and alpha), FP64 padded column-major
  const int* h_rp;
  const int* h_ci;
  const double* h_v;
  const int* h1_rp[MAXD];
  const int* h1_ci[MAXD];
  const double* h1_v[MAXD];
  // outputs
  void* stage;              // kept upper blocks, row-major tiles (T)
  int2* kept_ij;            // slot -> (I, J)
  int* stage_count;         // atomic slot counter
  int stage_cap;
  int* overflow;            // set when stage_count would exceed stage_cap
  int* bad;                 // set when a NaN/Inf is produced
  double* partial;          // n_items x NQ
  unsigned long long* exec_pairs;  // block triples issued (all candidates)
};

// Cluster row panels: for cluster P the sorted union of the columns K of its
// atoms' rows, with the entry index of (I_s, K) for each member s (-1 absent).
struct PanelArgs {
  int nc;
  const int* rp;
  const int* ci;
  const int* clus_atom;   // nc x CS, -1 padded
  const int* clus_sys;    // cluster -> system
  const int* sys_start;
  const int* sys_end;
  const int* csys_start;  // system -> first cluster
  const int* csys_end;
  const int* atom_clus;   // atom -> cluster
  const int* active;
  int max_sys_atoms;
  int max_sys_clusters;
  // panels
  int* panel_cnt;         // nc
  const int* panel_rp;    // nc+1
  int* panel_k;
  int* panel_e;           // 8 per panel entry
  // tiles
  int* tile_cnt;          // nc
  long long* tile_pairs;  // nc: upper bound of output pairs of the tiles of P
  const int* tile_rp;     // nc+1
  int* tile_p;
  int* tile_q;
  unsigned* tile_bits;    // nc x tile_words: cluster bitmap of pass 0 for pass 1
  int tile_words;         // (max_sys_clusters + 31) / 32
};

struct TileArgs {
  int D;
  int bf16;               // FP32 values, MFMA operands rounded to bfloat16
  int wide;               // FP32 values, per-block products summed in FP64
  int shape;              // TileShape (must exist for the kind and D)
  int* work;              // nullptr: one block per sub-tile; else a zeroed
                          // counter and a persistent grid (see the kernel)
  const int* n_tiles_dev; // nullptr, or the tile count on the device
  int skip;               // 0 none, 1 exact norm-bound screen, 2 bound + network
  const float* bn;        // block norms (nnz x (1+D)) when skip != 0 or logging
  const unsigned char* xmask;  // per entry: bit m set when block m is nonzero (products of a
                               // zero block are not issued); nullptr: every product issued
  unsigned long long* screened;  // outputs skipped by the exact screen
  const float* mlp;       // skip network parameters (MLP_NP), skip == 2
  float mlp_z;            // skip when the logit exceeds this (logit of the threshold)
  float mlp_cap;          // the network may skip only outputs whose bound is < mlp_cap * eps
  unsigned long long* mlp_skipped;
  double* mlp_bsum;       // per system: sum of the bounds of the outputs the network skipped
  const double* xyz;      // merged atom positions or nullptr
  int iter;               // update index (feature)
  float* log_x;           // logged features (log_cap x MLP_NF)
  float* log_y;           // logged labels (1 = dropped, 0 = kept, -1 = skipped by the network)
  float* log_z;           // logged logits of the in-kernel network (skip == 2), or nullptr
  unsigned long long* log_count;
  long long log_cap;      // 0: no logging
  int kl_chunk;           // 0: default panel pass length
  int ksteps;
  int waves_per_column;   // 1: one wave per column of the 4 x 4 sub-tile (tests compare)
  int n_tiles;
  const int* rp;
  const int* ci;
  const void* xv;
  const int* tile_p;
  const int* tile_q;
  const int* clus_atom;
  const int* clus_sys;
  const int* panel_rp;
  const int* panel_k;
  const int* panel_e;
  const int* branch;
  const double* eps;
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
  double* partial;        // n_tiles x NQ
  unsigned long long* exec_pairs;  // block products issued
};

// Rows of systems that stopped iterating: their upper blocks go to the stage
// unchanged.
struct CopyArgs {
  int nb;
  int D;
  const int* rp;
  const int* ci;
  const void* xv;
  const int* sys_of;
  const int* active;
  void* stage;
  int2* kept_ij;
  int* stage_count;
  int stage_cap;
  int* overflow;
};

struct CompactArgs {
  int nb;
  int D;
  const int* stage_count;
  const int2* kept_ij;
  int* rowcnt;        // nb (zeroed)
  int* cursor;        // nb (zeroed)
  const int* new_rp;  // nb+1
  int* tmp_ci;
  int* tmp_src;
  int* new_ci;
  int* new_src;
  const int* sys_of;
  const int* sys_start;
  const int* sys_end;
  int max_sys_atoms;
  const int* n_kept_dev;  // nullptr, or the kept count on the device (then
                          // clamped to the host count, the stage capacity)
};

// hipMalloc that, when the device is out of memory, first returns the chunks
// the solver keeps pooled for reuse to the driver and tries again
hipError_t dev_malloc(void** p, size_t n);

// kernels (launch wrappers), all asynchronous on `st`
void launch_gershgorin(hipStream_t st, int nb, int b, const int* rp, const int* ci,
                       const double* hv, double* rowlo, double* rowhi);
void launch_sys_minmax(hipStream_t st, int nsys, const int* sys_start, const int* sys_end,
                       int b, const double* rowlo, const double* rowhi, double* emin, double* emax);
void launch_init(hipStream_t st, int prec, int nnz, int D, int b, const int* row_of,
                 const int* ci, const int* src_h, const int* const* src_h1,
                 const double* hv, const double* const* h1v, const int* sys_of,
                 const double* emin, const double* emax, const int* mode, void* xv);
void launch_symbolic(hipStream_t st, int pass, const SymArgs& a);
void launch_scan(hipStream_t st, int n, const int* in, int* out, int* total);
void launch_items(hipStream_t st, int nb, const int* cand_rp, const int* item_rp,
                  int* item_row, int* item_c0);
void launch_items_count(hipStream_t st, int nb, const int* cand_rp, int* item_cnt);
void launch_numeric(hipStream_t st, int prec, const NumArgs& a);
void launch_measure(hipStream_t st, int prec, const MeasArgs& a);
void launch_panels(hipStream_t st, int pass, const PanelArgs& a);
void launch_tiles(hipStream_t st, int pass, const PanelArgs& a);
bool launch_tile_numeric(hipStream_t st, int prec, const TileArgs& a);  // false: no such shape
bool tile_shape_available(int kind, int D, int shape);
int tile_shape_default(int kind, int D);
int tile_subs(int shape);  // workgroups per tile of 8 x 8 output blocks
const char* tile_shape_name(int shape);
void launch_copy_through(hipStream_t st, int prec, const CopyArgs& a, int nnz);
// nnz_dev (optional): the entry count on the device, at most nnz (the grid)
void launch_block_norms(hipStream_t st, int prec, long long nnz, int D, const void* xv, float* bn,
                        const int* nnz_dev = nullptr);
void launch_compact_count(hipStream_t st, const CompactArgs& a, int n_kept);
void launch_compact_scatter(hipStream_t st, const CompactArgs& a, int n_kept);
void launch_row_sort(hipStream_t st, const CompactArgs& a);
// nnz_dev (optional): the new entry count on the device, at most nnz;
// skip_flag (optional): nothing is written when *skip_flag is nonzero
void launch_gather(hipStream_t st, int prec, int nnz, int D, const int* new_src,
                   const void* stage, void* xv, const int* nnz_dev = nullptr,
                   const int* skip_flag = nullptr);
void launch_reduce(hipStream_t st, int nsys, const int* sys_item_lo, const int* sys_item_hi,
                   const double* partial, double* scal);
void launch_sys_items(hipStream_t st, int nsys, int mult, const int* sys_start, const int* sys_end,
                      const int* item_rp, int* lo, int* hi);
void launch_export(hipStream_t st, int prec, int nnz, int D, int m, int b, const void* xv,
                   double* out);
void launch_convert(hipStream_t st, int from_prec, int to_prec, long long n, const void* in,
                    void* out);
void launch_fill_int(hipStream_t st, int* p, int v, long long n);

}  // namespace tc2
