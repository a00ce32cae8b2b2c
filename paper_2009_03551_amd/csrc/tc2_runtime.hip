// Host runtime of the TC2 / TC2-CPSCF solver: the C ABI of include/tc2.h.
//
// tc2_setup validates and uploads the problems (a batch is merged into one
// block-diagonal matrix with a system id per atom row); tc2_run drives the
// recursion of Sec. 2.2 (Eq. TC2 coupled with Eq. TC2-CPSCF) on the device,
// one merged kernel sequence per update, and applies the stopping rule of
// Sec. 2.3 (band-energy change below the tolerance) per system.
#include "tc2_internal.h"
#include "tc2_context.h"
#include "tc2_decide.h"
#include "tc2_host.h"
#include "../../include/tc2.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace tc2;

namespace {

// Block triples (I, K, J) of the full product X X on the current pattern, per
// active system: the sum over rows K of m_K^2, m_K the stored blocks of row K
// (the pattern is symmetric).  This is the nominal count of a full sparse
// product, as the paper accounts the work of an update, against which the
// kept-output count of the kernels is the useful one.
__global__ void k_nominal(int nb, const int* rp, const int* sys_of, const int* active,
                          unsigned long long* acc) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x) {
    const int s = sys_of[i];
    if (!active[s]) continue;
    const unsigned long long m = (unsigned long long)(rp[i + 1] - rp[i]);
    atomicAdd(&acc[s], m * m);
  }
}

}  // namespace


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


// padded, column-major device image of a batch of BSR matrices (FP64)
void pack_blocks(const tc2_bsr& m, int b, std::vector<double>& out) {
  int64_t nnz = m.row_ptr[m.nb];
  size_t off = out.size();
  out.resize(off + (size_t)nnz * BS, 0.0);
  for (int64_t e = 0; e < nnz; ++e)
    for (int r = 0; r < b; ++r)
      for (int c = 0; c < b; ++c)
        out[off + (size_t)e * BS + c * BP + r] = m.val[(e * b + r) * b + c];
}

template <typename T>
tc2_status upload(tc2_ctx* ctx, DBuf& d, const std::vector<T>& h) {
  HIPCHK(d.reserve(h.size() * sizeof(T)));
  if (!h.empty()) HIPCHK(hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return TC2_OK;
}

// merged row pointer / columns (int32) of a matrix family over the batch
void merge_pattern(const std::vector<const tc2_bsr*>& ms, const std::vector<SysInfo>& sys,
                   std::vector<int>& rp, std::vector<int>& ci) {
  rp.assign(1, 0);
  ci.clear();
  for (size_t s = 0; s < ms.size(); ++s) {
    const tc2_bsr* m = ms[s];
    for (int i = 0; i < m->nb; ++i) {
      for (int64_t p = m->row_ptr[i]; p < m->row_ptr[i + 1]; ++p) ci.push_back(sys[s].row0 + m->col[p]);
      rp.push_back((int)ci.size());
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ host checks
namespace tc2 {

tc2_status validate_bsr(const tc2_bsr& m, int nb, int b) {
  if (m.nb != nb || m.b != b) return TC2_EINVAL;
  if (!m.row_ptr || (!m.col && m.row_ptr[nb] > 0) || (!m.val && m.row_ptr[nb] > 0)) return TC2_EINVAL;
  if (m.row_ptr[0] != 0) return TC2_EINVAL;
  for (int i = 0; i < nb; ++i) {
    if (m.row_ptr[i + 1] < m.row_ptr[i]) return TC2_EINVAL;
    for (int64_t p = m.row_ptr[i]; p < m.row_ptr[i + 1]; ++p) {
      if (m.col[p] < 0 || m.col[p] >= nb) return TC2_EINVAL;
      if (p > m.row_ptr[i] && m.col[p] <= m.col[p - 1]) return TC2_EINVAL;
    }
  }
  if (m.row_ptr[nb] > (int64_t)0x7fffffff / 2) return TC2_EOVERFLOW;
  // symmetric pattern
  for (int i = 0; i < nb; ++i)
    for (int64_t p = m.row_ptr[i]; p < m.row_ptr[i + 1]; ++p) {
      int j = m.col[p];
      const int32_t* b0 = m.col + m.row_ptr[j];
      const int32_t* b1 = m.col + m.row_ptr[j + 1];
      if (!std::binary_search(b0, b1, i)) return TC2_ENONSYM;
    }
  int64_t nv = m.row_ptr[nb] * (int64_t)b * b;
  for (int64_t k = 0; k < nv; ++k)
    if (!std::isfinite(m.val[k])) return TC2_ENAN;
  return TC2_OK;
}

bool has_diag(const tc2_bsr& m, int nb) {
  for (int i = 0; i < nb; ++i)
    if (!std::binary_search(m.col + m.row_ptr[i], m.col + m.row_ptr[i + 1], i)) return false;
  return true;
}

tc2_status select_gfx950(int device, std::string* arch) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return TC2_EDEVICE;
  if (device < 0 || device >= ndev) return TC2_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return TC2_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return TC2_EDEVICE;
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TC2_EDEVICE;
  if (arch) arch->assign(prop.gcnArchName, strcspn(prop.gcnArchName, ":"));
  return TC2_OK;
}

}  // namespace tc2

// ====================================================================== ABI
extern "C" {

const char* tc2_version(void) { return "tc2-mi355x 0.1 (gfx950)"; }

const char* tc2_strerror(tc2_status s) {
  switch (s) {
    case TC2_OK: return "ok";
    case TC2_NOT_CONVERGED: return "not converged within max_iter";
    case TC2_FLOOR_REACHED: return "stopped at the precision floor (stall guard)";
    case TC2_EINVAL: return "invalid argument";
    case TC2_ENOMEM: return "out of memory";
    case TC2_EDEVICE: return "device error or no gfx950 device";
    case TC2_ENONSYM: return "pattern not symmetric or diagonal block missing";
    case TC2_EDEGENERATE: return "degenerate spectrum bounds (emax == emin)";
    case TC2_ENAN: return "NaN or Inf encountered";
    case TC2_EOVERFLOW: return "size exceeds the index range";
  }
  return "unknown status";
}

void tc2_free(tc2_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  const int dev = ctx->device;
  if (ctx->own) (void)hipStreamDestroy(ctx->own);
  for (hipEvent_t& e : ctx->pev)
    if (e) (void)hipEventDestroy(e);
  for (hipGraphExec_t& g : ctx->gexec)
    if (g) (void)hipGraphExecDestroy(g);
  for (hipGraphExec_t& g : ctx->gexec_post)
    if (g) (void)hipGraphExecDestroy(g);
  if (ctx->run.ev0) (void)hipEventDestroy(ctx->run.ev0);
  if (ctx->run.ev1) (void)hipEventDestroy(ctx->run.ev1);
  delete ctx;
  (void)dev;
}

tc2_status tc2_trim_memory(int32_t device) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return TC2_EINVAL;
  }
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return TC2_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return TC2_EDEVICE;
  tc2::pool_trim();
  (void)hipSetDevice(cur);
  return TC2_OK;
}

// ---- tuned sub-tile shapes.  The cache file holds one JSON object per line,
//   {"key": "<arch>/<kind>/D<d>/k<ksteps>/s<skip>", "shape": "<SPxTQ>", "ms": {...}}
// keyed by what changes the best shape: kernel kind, directions, K-steps per
// block (block size) and screening.  Later lines win.
static const char* kind_name(int k) {
  static const char* n[4] = {"fp64", "fp32", "bf16", "fp32w"};
  return n[k];
}

static std::string tune_key(const tc2_ctx* ctx, int kind) {
  char buf[160];
  snprintf(buf, sizeof(buf), "%s/%s/D%d/k%d/s%d", ctx->arch.c_str(), kind_name(kind), ctx->D,
           (ctx->b + 3) / 4, ctx->skip);
  return buf;
}

static void tune_load(tc2_ctx* ctx) {
  if (ctx->tune_cache.empty()) return;
  FILE* f = fopen(ctx->tune_cache.c_str(), "r");
  if (!f) return;
  std::string keys[4];
  for (int k = 0; k < 4; ++k) keys[k] = "\"key\": \"" + tune_key(ctx, k) + "\"";
  char line[1024];
  while (fgets(line, sizeof(line), f)) {
    for (int k = 0; k < 4; ++k) {
      if (!strstr(line, keys[k].c_str())) continue;
      const char* p = strstr(line, "\"shape\": \"");
      if (!p) continue;
      p += 10;
      for (int sh = 0; sh < TS_N; ++sh) {
        const char* nm = tile_shape_name(sh);
        if (strncmp(p, nm, strlen(nm)) == 0 && p[strlen(nm)] == '"' &&
            tile_shape_available(k, ctx->D, sh)) {
          ctx->shape[k] = sh;
          ctx->tuned[k] = true;
        }
      }
    }
  }
  fclose(f);
}

static void tune_store(const tc2_ctx* ctx, int kind, const float* ms) {
  if (ctx->tune_cache.empty()) return;
  FILE* f = fopen(ctx->tune_cache.c_str(), "a");
  if (!f) return;
  fprintf(f, "{\"key\": \"%s\", \"shape\": \"%s\", \"ms\": {", tune_key(ctx, kind).c_str(),
          tile_shape_name(ctx->shape[kind]));
  bool first = true;
  for (int sh = 0; sh < TS_N; ++sh) {
    if (ms[sh] < 0.f) continue;
    fprintf(f, "%s\"%s\": %.4f", first ? "" : ", ", tile_shape_name(sh), ms[sh]);
    first = false;
  }
  fprintf(f, "}}\n");
  fclose(f);
}

static tc2_status setup_impl(const tc2_problem* probs, int32_t np, const tc2_options* o,
                             tc2_ctx** out) {
  tc2_ctx* ctx = nullptr;
  if (!out) return TC2_EINVAL;
  *out = nullptr;
  if (!probs || np < 1 || !o) return TC2_EINVAL;
  if (o->precision < 0 || o->precision > 2) return TC2_EINVAL;
  if (o->closing_fp64 != 0 && o->closing_fp64 != 2) return TC2_EINVAL;
  if (o->skip < 0 || o->skip > 2) return TC2_EINVAL;
  if ((o->skip != 0 || o->log_capacity > 0) && o->numeric_kernel != 0) return TC2_EINVAL;
  if (o->skip == 2) {
    if (!o->mlp_weights || !(o->mlp_threshold > 0.f && o->mlp_threshold < 1.f)) return TC2_EINVAL;
    if (!(o->mlp_bound_cap >= 0.f) || !(o->mlp_budget >= 0.0) || !std::isfinite(o->mlp_budget))
      return TC2_EINVAL;
    for (int p = 0; p < MLP_NP; ++p)
      if (!std::isfinite(o->mlp_weights[p])) return TC2_ENAN;
  }
  if (o->log_capacity < 0 || o->log_capacity > ((int64_t)1 << 31)) return TC2_EINVAL;
  if (o->wide_accumulate < 0 || o->wide_accumulate > 1) return TC2_EINVAL;
  if (o->wide_accumulate && o->numeric_kernel != 0) return TC2_EINVAL;
  if (o->tune < 0 || o->tune > 1 || (o->tune && o->numeric_kernel != 0)) return TC2_EINVAL;
  if (o->graph < 0 || o->graph > 1 || (o->graph && o->numeric_kernel != 0)) return TC2_EINVAL;
  if (o->numeric_kernel < 0 || o->numeric_kernel > 1) return TC2_EINVAL;
  if (o->precision == P_BF16 && o->numeric_kernel != 0) return TC2_EINVAL;
  if (o->fp64_first < 0 || o->fp64_first > TC2_MAX_ITER) return TC2_EINVAL;
  if (o->count_useful < 0 || o->count_useful > 1) return TC2_EINVAL;
  if (o->device_loop < 0 || o->device_loop > TC2_MAX_ITER) return TC2_EINVAL;
  const int b = probs[0].H.b, D = probs[0].n_dir;
  if (b < 1 || b > BP || D < 0 || D > MAXD) return TC2_EINVAL;
  int64_t nb_tot = 0;
  int max_atoms = 0;
  for (int s = 0; s < np; ++s) {
    const tc2_problem& p = probs[s];
    if (p.H.b != b || p.n_dir != D) return TC2_EINVAL;
    if (p.H.nb < 1) return TC2_EINVAL;
    if (!(p.eps_drop >= 0.0) || !(p.tol > 0.0) || !std::isfinite(p.eps_drop)) return TC2_EINVAL;
    if (p.max_iter < 1 || p.max_iter > TC2_MAX_ITER) return TC2_EINVAL;
    int64_t N = (int64_t)p.H.nb * b;
    if (p.n_occ < 0 || p.n_occ > N) return TC2_EINVAL;
    if (p.replay) {
      size_t L = strlen(p.replay);
      if (L < 1 || L > TC2_MAX_ITER) return TC2_EINVAL;
      for (size_t k = 0; k < L; ++k)
        if (p.replay[k] != 'S' && p.replay[k] != 'D') return TC2_EINVAL;
    }
    tc2_status st = validate_bsr(p.H, p.H.nb, b);
    if (st != TC2_OK) return st;
    if (!has_diag(p.H, p.H.nb)) return TC2_ENONSYM;
    for (int d = 0; d < D; ++d) {
      st = validate_bsr(p.H1[d], p.H.nb, b);
      if (st != TC2_OK) return st;
    }
    nb_tot += p.H.nb;
    max_atoms = std::max(max_atoms, p.H.nb);
  }
  if (nb_tot > (1 << 26) || max_atoms > MAX_SYS_BITS) return TC2_EOVERFLOW;

  std::string arch;
  if (o->device < 0 || o->device >= 64) return TC2_EDEVICE;
  if (tc2_status st = select_gfx950(o->device, &arch); st != TC2_OK) return st;

  ctx = new (std::nothrow) tc2_ctx();
  if (!ctx) return TC2_ENOMEM;
  ctx->device = o->device;
  ctx->nsys = np;
  ctx->D = D;
  ctx->b = b;
  ctx->nb = (int)nb_tot;
  ctx->prec = o->precision;
  ctx->closing = o->closing_fp64;
  ctx->verbose = o->verbose;
  ctx->export_m = o->export_matrices;
  ctx->max_sys_atoms = max_atoms;
  ctx->profile = o->profile;
  ctx->kernel = o->numeric_kernel;
  ctx->fp64_first = o->fp64_first;
  ctx->skip = o->skip;
  ctx->skip_now = o->skip;
  if (o->skip == 2) {
    ctx->mlp_cap = o->mlp_bound_cap > 0.f ? o->mlp_bound_cap : 4.f;
    ctx->mlp_budget = o->mlp_budget;
  }
  ctx->log_cap = o->log_capacity;
  ctx->wide = o->wide_accumulate;
  ctx->tune = o->tune;
  if (o->tune_cache) ctx->tune_cache = o->tune_cache;
  ctx->graph = o->graph;
  ctx->device_loop = o->device_loop;
  ctx->count_useful = o->count_useful;
  if (o->metrics_log) ctx->metrics_log = o->metrics_log;
  ctx->arch = arch;
  for (int k = 0; k < 4; ++k) ctx->shape[k] = tile_shape_default(k, D);
  if (ctx->tune) tune_load(ctx);
  if (const char* v = getenv("TC2_TEST_KL_CHUNK")) ctx->test_kl_chunk = std::max(0, atoi(v));
  if (const char* v = getenv("TC2_TEST_STAGE_CAP")) ctx->test_stage_cap = std::max(0LL, atoll(v));
  if (const char* v = getenv("TC2_TEST_NO_ZERO_SKIP")) ctx->test_no_zero_skip = atoi(v) != 0;
  if (const char* v = getenv("TC2_TEST_WAVES_PER_COLUMN")) ctx->test_waves_per_column = atoi(v);
  tc2_status st = TC2_OK;
  auto fail = [&](tc2_status s) {
    tc2_free(ctx);
    return s;
  };
  if (hipStreamCreateWithFlags(&ctx->own, hipStreamNonBlocking) != hipSuccess) return fail(TC2_EDEVICE);
  if (ctx->profile)
    for (hipEvent_t& e : ctx->pev)
      if (hipEventCreate(&e) != hipSuccess) return fail(TC2_EDEVICE);

  // systems
  std::vector<int> sys_of(nb_tot), sys_start(np), sys_end(np), mode(np);
  std::vector<double> eps(np);
  int row = 0;
  ctx->sys.resize(np);
  for (int s = 0; s < np; ++s) {
    const tc2_problem& p = probs[s];
    SysInfo& si = ctx->sys[s];
    si.row0 = row;
    si.nb = p.H.nb;
    si.n_occ = p.n_occ;
    si.eps = p.eps_drop;
    si.tol = p.tol;
    si.max_iter = p.max_iter;
    if (p.replay) si.replay = p.replay;
    int64_t N = (int64_t)p.H.nb * b;
    si.mode = p.n_occ == 0 ? 1 : (p.n_occ == N ? 2 : 0);
    for (int i = 0; i < p.H.nb; ++i) sys_of[row + i] = s;
    sys_start[s] = row;
    sys_end[s] = row + p.H.nb;
    mode[s] = si.mode;
    eps[s] = p.eps_drop;
    row += p.H.nb;
  }
  ctx->h_sys_of = sys_of;
  if ((st = upload(ctx, ctx->sys_of, sys_of)) != TC2_OK) return fail(st);
  if ((st = upload(ctx, ctx->sys_start, sys_start)) != TC2_OK) return fail(st);
  if ((st = upload(ctx, ctx->sys_end, sys_end)) != TC2_OK) return fail(st);
  if ((st = upload(ctx, ctx->mode, mode)) != TC2_OK) return fail(st);
  if ((st = upload(ctx, ctx->eps, eps)) != TC2_OK) return fail(st);
  std::vector<int> zeros(np, 0);
  if ((st = upload(ctx, ctx->active, zeros)) != TC2_OK) return fail(st);
  if (ctx->nominal.reserve((size_t)np * 8) != hipSuccess) return fail(TC2_ENOMEM);
  if ((st = upload(ctx, ctx->branch, zeros)) != TC2_OK) return fail(st);
  if ((st = upload(ctx, ctx->bad, zeros)) != TC2_OK) return fail(st);
  if (ctx->emin.reserve(np * 8) || ctx->emax.reserve(np * 8)) return fail(TC2_ENOMEM);

  // H, H1 merged
  std::vector<const tc2_bsr*> hs(np);
  for (int s = 0; s < np; ++s) hs[s] = &probs[s].H;
  std::vector<int> rp, ci;
  std::vector<double> vals;
  merge_pattern(hs, ctx->sys, rp, ci);
  for (int s = 0; s < np; ++s) pack_blocks(probs[s].H, b, vals);
  if ((st = upload(ctx, ctx->h_rp, rp)) != TC2_OK) return fail(st);
  if ((st = upload(ctx, ctx->h_ci, ci)) != TC2_OK) return fail(st);
  if ((st = upload(ctx, ctx->h_v, vals)) != TC2_OK) return fail(st);
  std::vector<int> hrp = rp, hci = ci;
  std::vector<std::vector<int>> h1rp(D), h1ci(D);
  for (int d = 0; d < D; ++d) {
    std::vector<const tc2_bsr*> m1(np);
    for (int s = 0; s < np; ++s) m1[s] = &probs[s].H1[d];
    vals.clear();
    merge_pattern(m1, ctx->sys, h1rp[d], h1ci[d]);
    for (int s = 0; s < np; ++s) pack_blocks(probs[s].H1[d], b, vals);
    if ((st = upload(ctx, ctx->h1_rp[d], h1rp[d])) != TC2_OK) return fail(st);
    if ((st = upload(ctx, ctx->h1_ci[d], h1ci[d])) != TC2_OK) return fail(st);
    if ((st = upload(ctx, ctx->h1_v[d], vals)) != TC2_OK) return fail(st);
  }
  // initial pattern: union of H and the H1_d patterns, with source entries
  std::vector<int> xrp(1, 0), xci, xrow, sh;
  std::vector<std::vector<int>> sh1(D);
  for (int I = 0; I < ctx->nb; ++I) {
    std::vector<int> cols(hci.begin() + hrp[I], hci.begin() + hrp[I + 1]);
    for (int d = 0; d < D; ++d) cols.insert(cols.end(), h1ci[d].begin() + h1rp[d][I], h1ci[d].begin() + h1rp[d][I + 1]);
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    for (int J : cols) {
      xci.push_back(J);
      xrow.push_back(I);
      auto f = std::lower_bound(hci.begin() + hrp[I], hci.begin() + hrp[I + 1], J);
      sh.push_back((f != hci.begin() + hrp[I + 1] && *f == J) ? (int)(f - hci.begin()) : -1);
      for (int d = 0; d < D; ++d) {
        auto g = std::lower_bound(h1ci[d].begin() + h1rp[d][I], h1ci[d].begin() + h1rp[d][I + 1], J);
        sh1[d].push_back((g != h1ci[d].begin() + h1rp[d][I + 1] && *g == J) ? (int)(g - h1ci[d].begin()) : -1);
      }
    }
    xrp.push_back((int)xci.size());
  }
  ctx->nnz0 = (int)xci.size();
  if ((st = upload(ctx, ctx->x0_rp, xrp)) != TC2_OK) return fail(st);
  if ((st = upload(ctx, ctx->x0_ci, xci)) != TC2_OK) return fail(st);
  if ((st = upload(ctx, ctx->x0_row, xrow)) != TC2_OK) return fail(st);
  if ((st = upload(ctx, ctx->src_h, sh)) != TC2_OK) return fail(st);
  for (int d = 0; d < D; ++d)
    if ((st = upload(ctx, ctx->src_h1[d], sh1[d])) != TC2_OK) return fail(st);
  // clusters of up to CS nearby atoms for the tiled kernel: atoms in Morton
  // order of their positions (grid step = shortest distance between two atoms
  // coupled in H), or in index order without positions, cut into runs of CS
  {
    std::vector<int> clus_atom, clus_sys, atom_clus(nb_tot), csys_start(np), csys_end(np);
    int maxc = 0;
    for (int s = 0; s < np; ++s) {
      const tc2_problem& p = probs[s];
      const int n = p.H.nb, row0 = ctx->sys[s].row0;
      std::vector<int> order(n);
      for (int i = 0; i < n; ++i) order[i] = i;
      if (p.xyz) {
        for (int i = 0; i < 3 * n; ++i)
          if (!std::isfinite(p.xyz[i])) return fail(TC2_ENAN);
        double h = 0.0;
        for (int i = 0; i < n; ++i)
          for (int64_t e = p.H.row_ptr[i]; e < p.H.row_ptr[i + 1]; ++e) {
            const int j = p.H.col[e];
            if (j == i) continue;
            double d2 = 0.0;
            for (int k = 0; k < 3; ++k) d2 += (p.xyz[3 * i + k] - p.xyz[3 * j + k]) * (p.xyz[3 * i + k] - p.xyz[3 * j + k]);
            const double d = std::sqrt(d2);
            if (d > 0.0 && (h == 0.0 || d < h)) h = d;
          }
        if (!(h > 0.0)) h = 1.0;
        double lo3[3] = {INFINITY, INFINITY, INFINITY};
        for (int i = 0; i < n; ++i)
          for (int k = 0; k < 3; ++k) lo3[k] = std::min(lo3[k], p.xyz[3 * i + k]);
        std::vector<uint64_t> key(n);
        for (int i = 0; i < n; ++i) {
          uint64_t code = 0;
          uint64_t q[3];
          for (int k = 0; k < 3; ++k) {
            double v = std::floor((p.xyz[3 * i + k] - lo3[k]) / h + 0.5);
            q[k] = (uint64_t)std::min(std::max(v, 0.0), 2097151.0);
          }
          for (int bit = 20; bit >= 0; --bit)
            for (int k = 0; k < 3; ++k) code = (code << 1) | ((q[k] >> bit) & 1u);
          key[i] = code;
        }
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return key[x] < key[y]; });
      }
      csys_start[s] = (int)clus_sys.size();
      for (int k = 0; k < n; k += CS) {
        std::vector<int> mem(order.begin() + k, order.begin() + std::min(n, k + CS));
        std::sort(mem.begin(), mem.end());
        const int cidx = (int)clus_sys.size();
        clus_sys.push_back(s);
        for (int j = 0; j < CS; ++j) clus_atom.push_back(j < (int)mem.size() ? row0 + mem[j] : -1);
        for (int m : mem) atom_clus[row0 + m] = cidx;
      }
      csys_end[s] = (int)clus_sys.size();
      maxc = std::max(maxc, csys_end[s] - csys_start[s]);
    }
    ctx->nc = (int)clus_sys.size();
    ctx->max_sys_clusters = maxc;
    for (int s = 0; s < np; ++s) {
      const long long m = csys_end[s] - csys_start[s];
      ctx->tile_bound += m * (m + 1) / 2;
    }
    // with fewer cluster pairs than compute units, one workgroup per pair
    // leaves most units idle and each runs the whole column loop of its
    // pair: the FP64 kind, 8x8 by default, then takes the 4x8 sub-tile (two
    // workgroups per pair; on a 64-atom chain the products took 0.155 ms per
    // update instead of 0.216), unless a tuned shape was loaded
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess) {
      (void)hipGetLastError();
      n_cu = 0;
    }
    if (!ctx->tuned[K_FP64] && ctx->shape[K_FP64] == TS_8x8 && ctx->tile_bound < n_cu &&
        tile_shape_available(K_FP64, D, TS_4x8))
      ctx->shape[K_FP64] = TS_4x8;
    if ((st = upload(ctx, ctx->clus_atom, clus_atom)) != TC2_OK) return fail(st);
    if ((st = upload(ctx, ctx->clus_sys, clus_sys)) != TC2_OK) return fail(st);
    if ((st = upload(ctx, ctx->atom_clus, atom_clus)) != TC2_OK) return fail(st);
    if ((st = upload(ctx, ctx->csys_start, csys_start)) != TC2_OK) return fail(st);
    if ((st = upload(ctx, ctx->csys_end, csys_end)) != TC2_OK) return fail(st);
  }
  // positions (a feature of the skip network) and the network itself
  {
    bool all = true;
    for (int s = 0; s < np; ++s) all = all && probs[s].xyz != nullptr;
    if (all) {
      std::vector<double> xyz;
      for (int s = 0; s < np; ++s) xyz.insert(xyz.end(), probs[s].xyz, probs[s].xyz + 3 * (size_t)probs[s].H.nb);
      if ((st = upload(ctx, ctx->xyz, xyz)) != TC2_OK) return fail(st);
      ctx->have_xyz = true;
    }
    if (o->skip == 2) {
      if (ctx->mlp_bsum.reserve((size_t)np * 8) != hipSuccess) return fail(TC2_ENOMEM);
      std::vector<float> th(o->mlp_weights, o->mlp_weights + MLP_NP);
      if ((st = upload(ctx, ctx->mlp, th)) != TC2_OK) return fail(st);
      ctx->mlp_z = std::log(o->mlp_threshold / (1.f - o->mlp_threshold));
    }
    if (ctx->log_cap > 0) {
      if (ctx->log_x.reserve((size_t)ctx->log_cap * MLP_NF * 4) ||
          ctx->log_y.reserve((size_t)ctx->log_cap * 4) ||
          ctx->log_z.reserve((size_t)ctx->log_cap * 4) || ctx->log_count.reserve(8))
        return fail(TC2_ENOMEM);
    }
  }
  if (ctx->rowlo.reserve((size_t)ctx->nb * b * 8) || ctx->rowhi.reserve((size_t)ctx->nb * b * 8))
    return fail(TC2_ENOMEM);
  if (hipDeviceSynchronize() != hipSuccess) return fail(TC2_EDEVICE);
  *out = ctx;
  return TC2_OK;
}

tc2_status tc2_setup(const tc2_problem* problems, int32_t n_problems, const tc2_options* opts,
                     tc2_ctx** out) {
  try {
    return setup_impl(problems, n_problems, opts, out);
  } catch (const std::bad_alloc&) {
    return TC2_ENOMEM;
  } catch (...) {
    return TC2_EINVAL;
  }
}

}  // extern "C"

// ====================================================================== solve
namespace {

// Copy the current iterate into fresh buffers of another precision.
tc2_status convert_iterate(tc2_ctx* ctx, hipStream_t st, int to_prec) {
  ctx->bn_valid = false;  // the norms of the converted values are taken anew
  int c = ctx->cur;
  long long n = (long long)ctx->nnz[c] * (1 + ctx->D) * BS;
  DBuf& dst = ctx->xv[c ^ 1];
  // the stage is sized in the old precision and reserved again by the next
  // update: release it first, so that both copies of the values fit
  HIPCHK(hipStreamSynchronize(st));
  ctx->stage.release();
  HIPCHK(dst.reserve((size_t)n * prec_bytes(to_prec)));
  launch_convert(st, ctx->cur_prec, to_prec, n, ctx->xv[c].p, dst.p);
  // move the pattern along
  HIPCHK(ctx->rp[c ^ 1].reserve((size_t)(ctx->nb + 1) * 4));
  HIPCHK(ctx->ci[c ^ 1].reserve((size_t)std::max(1, ctx->nnz[c]) * 4));
  HIPCHK(hipMemcpyAsync(ctx->rp[c ^ 1].p, ctx->rp[c].p, (size_t)(ctx->nb + 1) * 4, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(ctx->ci[c ^ 1].p, ctx->ci[c].p, (size_t)ctx->nnz[c] * 4, hipMemcpyDeviceToDevice, st));
  ctx->nnz[c ^ 1] = ctx->nnz[c];
  ctx->cur = c ^ 1;
  ctx->cur_prec = to_prec;
  // the values in the old precision are no longer needed
  HIPCHK(hipStreamSynchronize(st));
  ctx->xv[c].release();
  return mask_iterate(ctx, st);
}

// Scalars of the current iterate into host memory (nsys x NQ).
tc2_status measure(tc2_ctx* ctx, hipStream_t st, std::vector<double>& scal) {
  const int c = ctx->cur;
  MeasArgs m{};
  m.nb = ctx->nb;
  m.D = ctx->D;
  m.rp = ctx->rp[c].as<int>();
  m.ci = ctx->ci[c].as<int>();
  m.xv = ctx->xv[c].p;
  m.h_rp = ctx->h_rp.as<int>();
  m.h_ci = ctx->h_ci.as<int>();
  m.h_v = ctx->h_v.as<double>();
  for (int d = 0; d < ctx->D; ++d) {
    m.h1_rp[d] = ctx->h1_rp[d].as<int>();
    m.h1_ci[d] = ctx->h1_ci[d].as<int>();
    m.h1_v[d] = ctx->h1_v[d].as<double>();
  }
  HIPCHK(ctx->partial.reserve((size_t)std::max(ctx->nb, 1) * NQ * 8));
  m.partial = ctx->partial.as<double>();
  launch_measure(st, ctx->cur_prec, m);
  HIPCHK(ctx->scal.reserve((size_t)ctx->nsys * NQ * 8));
  launch_reduce(st, ctx->nsys, ctx->sys_start.as<int>(), ctx->sys_end.as<int>(), ctx->partial.as<double>(),
                ctx->scal.as<double>());
  scal.resize((size_t)ctx->nsys * NQ);
  HIPCHK(hipMemcpyAsync(scal.data(), ctx->scal.p, scal.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return TC2_OK;
}

// Zero the per-system nominal counters and count this update's full-product
// triples on the pattern rp (stream work; also recorded into update graphs).
tc2_status count_nominal(tc2_ctx* ctx, hipStream_t st, const int* rp) {
  launch_fill_int(st, ctx->nominal.as<int>(), 0, 2LL * ctx->nsys);
  const unsigned g = (unsigned)std::min(65535, (ctx->nb + 255) / 256);
  hipLaunchKernelGGL(k_nominal, dim3(g), dim3(256), 0, st, ctx->nb, rp, ctx->sys_of.as<int>(),
                     ctx->active.as<int>(), ctx->nominal.as<unsigned long long>());
  HIPCHK(hipGetLastError());
  return TC2_OK;
}

// One update of every active system: candidates (atom-level symbolic product
// or cluster panels + tiles), numeric products with the fused epilogue,
// copy-through of stopped systems, compaction into the next pattern.  Leaves
// the per-system scalars of the new iterate in `scal`.
tc2_status step(tc2_ctx* ctx, hipStream_t st, std::vector<double>& scal,
                unsigned long long& exec_pairs_total) {
  const int c = ctx->cur, n = c ^ 1;
  const int nb = ctx->nb, D = ctx->D;
  const size_t tile = (size_t)(1 + D) * BS * prec_bytes(ctx->cur_prec);
  HIPCHK(ctx->counters.reserve(64));
  int* cnt = ctx->counters.as<int>();  // [0] scan total, [1] stage count, [2] overflow, [4] work counter
  int hcnt[4];
  const bool tiled = ctx->kernel == 0;
  bool any_stopped = false;
  for (int s = 0; s < ctx->nsys; ++s) any_stopped |= !ctx->h_active[s];

  if (ctx->profile) HIPCHK(hipEventRecord(ctx->pev[0], st));
  if (tc2_status r = count_nominal(ctx, st, ctx->rp[c].as<int>()); r != TC2_OK) return r;
  int n_work = 0;          // work items (atom path) or tile blocks (tiled path)
  long long out_bound = 0; // upper bound of computed output blocks
  const int kind = ctx->cur_prec == P_FP64 ? K_FP64
                   : ((ctx->op_bf16 && !ctx->wide) ? K_BF16 : (ctx->wide ? K_WIDE : K_FP32));
  const int wide_now = kind == K_WIDE ? 1 : 0;
  int mult = tiled ? tile_subs(ctx->shape[kind]) : 1;
  if (tiled) ctx->kind_used[kind] = true;
  ctx->last_kind = kind;
  if (!tiled) {
    // ---- atom-level symbolic product and work items
    HIPCHK(ctx->cand_cnt.reserve((size_t)nb * 4));
    HIPCHK(ctx->cand_rp.reserve((size_t)(nb + 1) * 4));
    SymArgs sa{};
    sa.nb = nb;
    sa.rp = ctx->rp[c].as<int>();
    sa.ci = ctx->ci[c].as<int>();
    sa.sys_of = ctx->sys_of.as<int>();
    sa.sys_end = ctx->sys_end.as<int>();
    sa.active = ctx->active.as<int>();
    sa.cand_cnt = ctx->cand_cnt.as<int>();
    sa.cand_rp = ctx->cand_rp.as<int>();
    sa.max_sys_atoms = ctx->max_sys_atoms;
    launch_symbolic(st, 0, sa);
    launch_scan(st, nb, ctx->cand_cnt.as<int>(), ctx->cand_rp.as<int>(), cnt);
    HIPCHK(hipMemcpyAsync(hcnt, cnt, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int ncand = hcnt[0];
    out_bound = ncand;
    HIPCHK(ctx->cand_ci.reserve((size_t)std::max(ncand, 1) * 4));
    sa.cand_ci = ctx->cand_ci.as<int>();
    launch_symbolic(st, 1, sa);
    HIPCHK(ctx->item_cnt.reserve((size_t)nb * 4));
    HIPCHK(ctx->item_rp.reserve((size_t)(nb + 1) * 4));
    launch_items_count(st, nb, ctx->cand_rp.as<int>(), ctx->item_cnt.as<int>());
    launch_scan(st, nb, ctx->item_cnt.as<int>(), ctx->item_rp.as<int>(), cnt);
    HIPCHK(hipMemcpyAsync(hcnt, cnt, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    n_work = hcnt[0];
    HIPCHK(ctx->item_row.reserve((size_t)std::max(n_work, 1) * 4));
    HIPCHK(ctx->item_c0.reserve((size_t)std::max(n_work, 1) * 4));
    launch_items(st, nb, ctx->cand_rp.as<int>(), ctx->item_rp.as<int>(), ctx->item_row.as<int>(),
                 ctx->item_c0.as<int>());
    HIPCHK(ctx->sys_lo.reserve((size_t)ctx->nsys * 4));
    HIPCHK(ctx->sys_hi.reserve((size_t)ctx->nsys * 4));
    launch_sys_items(st, ctx->nsys, 1, ctx->sys_start.as<int>(), ctx->sys_end.as<int>(),
                     ctx->item_rp.as<int>(), ctx->sys_lo.as<int>(), ctx->sys_hi.as<int>());
  } else {
    // ---- cluster panels and tiles
    const int nc = ctx->nc;
    HIPCHK(ctx->panel_cnt.reserve((size_t)nc * 4));
    HIPCHK(ctx->panel_rp.reserve((size_t)(nc + 1) * 4));
    HIPCHK(ctx->tile_cnt.reserve((size_t)nc * 4));
    HIPCHK(ctx->tile_rp.reserve((size_t)(nc + 1) * 4));
    HIPCHK(ctx->tile_pairs.reserve((size_t)nc * 8));
    PanelArgs pa{};
    pa.nc = nc;
    pa.rp = ctx->rp[c].as<int>();
    pa.ci = ctx->ci[c].as<int>();
    pa.clus_atom = ctx->clus_atom.as<int>();
    pa.clus_sys = ctx->clus_sys.as<int>();
    pa.sys_start = ctx->sys_start.as<int>();
    pa.sys_end = ctx->sys_end.as<int>();
    pa.csys_start = ctx->csys_start.as<int>();
    pa.csys_end = ctx->csys_end.as<int>();
    pa.atom_clus = ctx->atom_clus.as<int>();
    pa.active = ctx->active.as<int>();
    pa.max_sys_atoms = ctx->max_sys_atoms;
    pa.max_sys_clusters = ctx->max_sys_clusters;
    pa.panel_cnt = ctx->panel_cnt.as<int>();
    pa.panel_rp = ctx->panel_rp.as<int>();
    pa.tile_cnt = ctx->tile_cnt.as<int>();
    pa.tile_pairs = ctx->tile_pairs.as<long long>();
    pa.tile_rp = ctx->tile_rp.as<int>();
    pa.tile_words = (ctx->max_sys_clusters + 31) / 32;
    HIPCHK(ctx->tile_bits.reserve((size_t)std::max(nc, 1) * pa.tile_words * 4));
    pa.tile_bits = ctx->tile_bits.as<unsigned>();
    launch_panels(st, 0, pa);
    launch_scan(st, nc, ctx->panel_cnt.as<int>(), ctx->panel_rp.as<int>(), cnt);
    HIPCHK(hipMemcpyAsync(hcnt, cnt, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int npanel = hcnt[0];
    HIPCHK(ctx->panel_k.reserve((size_t)std::max(npanel, 1) * 4));
    HIPCHK(ctx->panel_e.reserve((size_t)std::max(npanel, 1) * CS * 4));
    pa.panel_k = ctx->panel_k.as<int>();
    pa.panel_e = ctx->panel_e.as<int>();
    launch_panels(st, 1, pa);
    launch_tiles(st, 0, pa);
    launch_scan(st, nc, ctx->tile_cnt.as<int>(), ctx->tile_rp.as<int>(), cnt);
    std::vector<long long> pairs(nc);
    HIPCHK(hipMemcpyAsync(hcnt, cnt, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(pairs.data(), ctx->tile_pairs.p, (size_t)nc * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int ntiles = hcnt[0];
    for (long long v : pairs) out_bound += v;
    HIPCHK(ctx->tile_p.reserve((size_t)std::max(ntiles, 1) * 4));
    HIPCHK(ctx->tile_q.reserve((size_t)std::max(ntiles, 1) * 4));
    pa.tile_p = ctx->tile_p.as<int>();
    pa.tile_q = ctx->tile_q.as<int>();
    launch_tiles(st, 1, pa);
    n_work = ntiles;
    HIPCHK(ctx->sys_lo.reserve((size_t)ctx->nsys * 4));
    HIPCHK(ctx->sys_hi.reserve((size_t)ctx->nsys * 4));
  }
  // room for the partial sums of any sub-tile shape (at most 4 per tile)
  HIPCHK(ctx->partial.reserve((size_t)std::max((long long)n_work * (tiled ? 4 : 1), (long long)nb) * NQ * 8));
  if (ctx->profile) HIPCHK(hipEventRecord(ctx->pev[1], st));

  // ---- numeric (retried with a larger stage if it overflows).  The stage
  // holds every possible output block when that fits a modest budget.
  if (any_stopped) out_bound += ctx->nnz[c];
  if (ctx->test_stage_cap > 0) {
    ctx->stage_cap = ctx->test_stage_cap;  // forces the overflow / retry path
  } else {
    const size_t budget = (size_t)16 << 30;
    if ((size_t)out_bound * tile <= budget) ctx->stage_cap = std::max<long long>(ctx->stage_cap, out_bound);
    else if (ctx->stage_cap == 0) ctx->stage_cap = std::max(ctx->nnz[c], nb) + 1024;
  }
  if (ctx->profile) {
    HIPCHK(hipEventSynchronize(ctx->pev[1]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->pev[0], ctx->pev[1]));
    ctx->ms_sym += ms;
  }
  HIPCHK(ctx->exec_pairs.reserve(8));
  const bool screen = tiled && (ctx->skip_now != 0 || ctx->log_cap > 0);
  if (screen) {
    HIPCHK(ctx->bn.reserve((size_t)std::max(ctx->nnz[c], 1) * (1 + D) * 4));
    HIPCHK(ctx->screened.reserve(16));
    launch_block_norms(st, ctx->cur_prec, ctx->nnz[c], D, ctx->xv[c].p, ctx->bn.as<float>());
  }
  int n_kept = 0;
  unsigned long long log_before = 0;  // restored if the numeric step is retried
  if (tiled && ctx->log_cap > 0) {
    HIPCHK(hipMemcpyAsync(&log_before, ctx->log_count.p, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  auto tile_args = [&](int cap, int shape) {
    TileArgs ta{};
    ta.D = D;
    ta.ksteps = (ctx->b + 3) / 4;
    ta.n_tiles = n_work;
    ta.rp = ctx->rp[c].as<int>();
    ta.ci = ctx->ci[c].as<int>();
    ta.xv = ctx->xv[c].p;
    ta.tile_p = ctx->tile_p.as<int>();
    ta.tile_q = ctx->tile_q.as<int>();
    ta.clus_atom = ctx->clus_atom.as<int>();
    ta.clus_sys = ctx->clus_sys.as<int>();
    ta.panel_rp = ctx->panel_rp.as<int>();
    ta.panel_k = ctx->panel_k.as<int>();
    ta.panel_e = ctx->panel_e.as<int>();
    ta.branch = ctx->branch.as<int>();
    ta.eps = ctx->eps.as<double>();
    ta.h_rp = ctx->h_rp.as<int>();
    ta.h_ci = ctx->h_ci.as<int>();
    ta.h_v = ctx->h_v.as<double>();
    for (int d = 0; d < D; ++d) {
      ta.h1_rp[d] = ctx->h1_rp[d].as<int>();
      ta.h1_ci[d] = ctx->h1_ci[d].as<int>();
      ta.h1_v[d] = ctx->h1_v[d].as<double>();
    }
    ta.stage = ctx->stage.p;
    ta.kept_ij = ctx->kept_ij.as<int2>();
    ta.stage_count = cnt + 1;
    ta.stage_cap = cap;
    ta.shape = shape;
    ta.work = cnt + 4;  // persistent launch: sub-tiles from a counter zeroed with cnt
    ta.overflow = cnt + 2;
    ta.bad = ctx->bad.as<int>();
    ta.partial = ctx->partial.as<double>();
    ta.exec_pairs = ctx->exec_pairs.as<unsigned long long>();
    ta.bf16 = (ctx->op_bf16 && ctx->cur_prec == P_FP32) ? 1 : 0;
    ta.wide = wide_now;
    ta.skip = ctx->skip_now;
    ta.xmask = ctx->test_no_zero_skip ? nullptr : ctx->mask[c].as<unsigned char>();
    ta.waves_per_column = ctx->test_waves_per_column;
    ta.bn = screen ? ctx->bn.as<float>() : nullptr;
    ta.screened = screen ? ctx->screened.as<unsigned long long>() : nullptr;
    ta.mlp_skipped = screen ? ctx->screened.as<unsigned long long>() + 1 : nullptr;
    ta.mlp = ctx->skip_now == 2 ? ctx->mlp.as<float>() : nullptr;
    ta.mlp_z = ctx->mlp_z;
    ta.mlp_cap = ctx->mlp_cap;
    ta.mlp_bsum = ctx->skip_now == 2 ? ctx->mlp_bsum.as<double>() : nullptr;
    ta.xyz = ctx->have_xyz ? ctx->xyz.as<double>() : nullptr;
    ta.iter = ctx->update_index;
    ta.log_cap = ctx->log_cap;
    ta.log_x = ctx->log_cap > 0 ? ctx->log_x.as<float>() : nullptr;
    ta.log_y = ctx->log_cap > 0 ? ctx->log_y.as<float>() : nullptr;
    ta.log_z = ctx->log_cap > 0 ? ctx->log_z.as<float>() : nullptr;
    ta.log_count = ctx->log_cap > 0 ? ctx->log_count.as<unsigned long long>() : nullptr;
    ta.kl_chunk = ctx->test_kl_chunk;
    return ta;
  };

  // ---- autotuning of the sub-tile shape: once per kernel kind, at the first
  // update past the peak of the candidate outputs (representative of the
  // densest updates, which dominate the solve), every available shape runs
  // this update's products twice (warm-up, then timed); the fastest is kept
  // and appended to the cache file.  The products are recomputed below.
  if (tiled && ctx->tune && !ctx->tuned[kind] && ctx->log_cap == 0 && n_work > 0 &&
      ctx->prev_out_bound >= 0 && out_bound <= ctx->prev_out_bound) {
    float ms_s[TS_N];
    int best = ctx->shape[kind];
    float best_ms = 3.0e38f;
    const int cap = (int)std::min<long long>(std::max<long long>(ctx->stage_cap, 1), out_bound);
    HIPCHK(ctx->stage.reserve((size_t)cap * tile));
    HIPCHK(ctx->kept_ij.reserve((size_t)cap * 8));
    hipEvent_t t0, t1;
    HIPCHK(hipEventCreate(&t0));
    HIPCHK(hipEventCreate(&t1));
    for (int sh = 0; sh < TS_N; ++sh) {
      ms_s[sh] = -1.f;
      if (!tile_shape_available(kind, D, sh)) continue;
      const TileArgs ta = tile_args(cap, sh);
      for (int rep = 0; rep < 2; ++rep) {
        launch_fill_int(st, cnt, 0, 8);
        launch_fill_int(st, ctx->exec_pairs.as<int>(), 0, 2);
        if (screen) launch_fill_int(st, ctx->screened.as<int>(), 0, 4);
        HIPCHK(hipEventRecord(t0, st));
        if (!launch_tile_numeric(st, ctx->cur_prec, ta)) return TC2_EINVAL;
        HIPCHK(hipGetLastError());
        HIPCHK(hipEventRecord(t1, st));
        HIPCHK(hipEventSynchronize(t1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, t0, t1));
        ctx->ms_tune += ms;
        ms_s[sh] = ms;
      }
      if (ms_s[sh] < best_ms) {
        best_ms = ms_s[sh];
        best = sh;
      }
      if (ctx->verbose)
        fprintf(stderr, "tc2 tune %s: shape %s %.3f ms\n", tune_key(ctx, kind).c_str(),
                tile_shape_name(sh), ms_s[sh]);
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    ctx->shape[kind] = best;
    ctx->tuned[kind] = true;
    tune_store(ctx, kind, ms_s);
    mult = tile_subs(best);
  }
  ctx->prev_out_bound = out_bound;
  if (tiled)
    launch_sys_items(st, ctx->nsys, mult, ctx->csys_start.as<int>(), ctx->csys_end.as<int>(),
                     ctx->tile_rp.as<int>(), ctx->sys_lo.as<int>(), ctx->sys_hi.as<int>());

  unsigned long long pairs = 0;
  for (int attempt = 0;; ++attempt) {
    int cap = (int)std::min<long long>(std::max<long long>(ctx->stage_cap, 1), out_bound > 0 ? out_bound : 1);
    HIPCHK(ctx->stage.reserve((size_t)cap * tile));
    HIPCHK(ctx->kept_ij.reserve((size_t)cap * 8));
    launch_fill_int(st, cnt, 0, 8);
    launch_fill_int(st, ctx->exec_pairs.as<int>(), 0, 2);
    if (ctx->profile) HIPCHK(hipEventRecord(ctx->pev[2], st));
    if (!tiled) {
      NumArgs na{};
      na.nb = nb;
      na.D = D;
      na.b = ctx->b;
      na.ksteps = (ctx->b + 3) / 4;
      na.rp = ctx->rp[c].as<int>();
      na.ci = ctx->ci[c].as<int>();
      na.xv = ctx->xv[c].p;
      na.cand_rp = ctx->cand_rp.as<int>();
      na.cand_ci = ctx->cand_ci.as<int>();
      na.item_row = ctx->item_row.as<int>();
      na.item_c0 = ctx->item_c0.as<int>();
      na.n_items = n_work;
      na.sys_of = ctx->sys_of.as<int>();
      na.active = ctx->active.as<int>();
      na.branch = ctx->branch.as<int>();
      na.eps = ctx->eps.as<double>();
      na.h_rp = ctx->h_rp.as<int>();
      na.h_ci = ctx->h_ci.as<int>();
      na.h_v = ctx->h_v.as<double>();
      for (int d = 0; d < D; ++d) {
        na.h1_rp[d] = ctx->h1_rp[d].as<int>();
        na.h1_ci[d] = ctx->h1_ci[d].as<int>();
        na.h1_v[d] = ctx->h1_v[d].as<double>();
      }
      na.stage = ctx->stage.p;
      na.kept_ij = ctx->kept_ij.as<int2>();
      na.stage_count = cnt + 1;
      na.stage_cap = cap;
      na.overflow = cnt + 2;
      na.bad = ctx->bad.as<int>();
      na.partial = ctx->partial.as<double>();
      na.exec_pairs = ctx->exec_pairs.as<unsigned long long>();
      launch_numeric(st, ctx->cur_prec, na);
    } else {
      TileArgs ta = tile_args(cap, ctx->shape[kind]);
      if (screen) launch_fill_int(st, ctx->screened.as<int>(), 0, 4);
      if (!launch_tile_numeric(st, ctx->cur_prec, ta)) return TC2_EINVAL;
    }
    HIPCHK(hipGetLastError());
    if (ctx->profile) HIPCHK(hipEventRecord(ctx->pev[3], st));
    if (any_stopped) {
      CopyArgs ca{};
      ca.nb = nb;
      ca.D = D;
      ca.rp = ctx->rp[c].as<int>();
      ca.ci = ctx->ci[c].as<int>();
      ca.xv = ctx->xv[c].p;
      ca.sys_of = ctx->sys_of.as<int>();
      ca.active = ctx->active.as<int>();
      ca.stage = ctx->stage.p;
      ca.kept_ij = ctx->kept_ij.as<int2>();
      ca.stage_count = cnt + 1;
      ca.stage_cap = cap;
      ca.overflow = cnt + 2;
      launch_copy_through(st, ctx->cur_prec, ca, ctx->nnz[c]);
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemcpyAsync(hcnt, cnt, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&pairs, ctx->exec_pairs.p, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (ctx->profile) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ctx->pev[2], ctx->pev[3]));
      ctx->ms_num += ms;
      ctx->num_launches++;
      ctx->ms_num_kind[kind] += ms;
      ctx->launches_kind[kind]++;
    }
    if (!hcnt[2]) {
      n_kept = hcnt[1];
      break;
    }
    if (tiled && ctx->log_cap > 0)
      HIPCHK(hipMemcpyAsync(ctx->log_count.p, &log_before, 8, hipMemcpyHostToDevice, st));
    // overflow: the counter still counts every kept block
    ctx->stage_cap = (int)std::min<long long>((long long)hcnt[1] * 5 / 4 + 1024, out_bound);
    if (attempt > 3) return TC2_ENOMEM;
  }
  exec_pairs_total += pairs;
  if (screen) {
    unsigned long long sc[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(sc, ctx->screened.p, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    ctx->screened_total += sc[0];
    ctx->mlp_total += sc[1];
  }
  if (tiled && ctx->skip_now == 2) {
    // the network's budget: once the bounds of the outputs it skipped add up
    // to more than mlp_budget for some system, the rest of the solve runs
    // with the exact screen alone
    ctx->mlp_updates++;
    if (ctx->mlp_budget > 0.0) {
      std::vector<double> bs(ctx->nsys);
      HIPCHK(hipMemcpyAsync(bs.data(), ctx->mlp_bsum.p, (size_t)ctx->nsys * 8, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      for (double v : bs)
        if (v > ctx->mlp_budget) ctx->skip_now = 1;
      if (ctx->skip_now == 1 && ctx->verbose)
        fprintf(stderr, "tc2: skip network budget spent after %d updates\n", ctx->mlp_updates);
    }
  }
  if (ctx->verbose) {
    float ms = 0.f;
    if (ctx->profile) (void)hipEventElapsedTime(&ms, ctx->pev[2], ctx->pev[3]);
    fprintf(stderr, "tc2 step: %s work=%d (x%d) out_bound=%lld kept=%d pairs=%llu numeric %.3f ms\n",
            tiled ? "tiles" : "items", n_work, mult, out_bound, n_kept, pairs, ms);
  }
  ctx->stage_cap = std::max(ctx->stage_cap, (long long)n_kept * 5 / 4 + 1024);

  // ---- compaction into the new pattern
  if (ctx->profile) HIPCHK(hipEventRecord(ctx->pev[0], st));
  HIPCHK(ctx->rowcnt.reserve((size_t)nb * 4));
  HIPCHK(ctx->cursor.reserve((size_t)nb * 4));
  HIPCHK(ctx->rp[n].reserve((size_t)(nb + 1) * 4));
  launch_fill_int(st, ctx->rowcnt.as<int>(), 0, nb);
  launch_fill_int(st, ctx->cursor.as<int>(), 0, nb);
  CompactArgs ca{};
  ca.nb = nb;
  ca.D = D;
  ca.kept_ij = ctx->kept_ij.as<int2>();
  ca.rowcnt = ctx->rowcnt.as<int>();
  ca.cursor = ctx->cursor.as<int>();
  ca.new_rp = ctx->rp[n].as<int>();
  ca.sys_of = ctx->sys_of.as<int>();
  ca.sys_start = ctx->sys_start.as<int>();
  ca.sys_end = ctx->sys_end.as<int>();
  ca.max_sys_atoms = ctx->max_sys_atoms;
  launch_compact_count(st, ca, n_kept);
  launch_scan(st, nb, ctx->rowcnt.as<int>(), ctx->rp[n].as<int>(), cnt);
  HIPCHK(hipMemcpyAsync(hcnt, cnt, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const int nnz_new = hcnt[0];
  HIPCHK(ctx->tmp_ci.reserve((size_t)std::max(nnz_new, 1) * 4));
  HIPCHK(ctx->tmp_src.reserve((size_t)std::max(nnz_new, 1) * 4));
  HIPCHK(ctx->new_src.reserve((size_t)std::max(nnz_new, 1) * 4));
  HIPCHK(ctx->ci[n].reserve((size_t)std::max(nnz_new, 1) * 4));
  // the products and the copy-through have read the old values (the stream
  // was synchronised above): the new values go into the same buffer
  ctx->xv[n].release();
  HIPCHK(ctx->xv[c].reserve_grow((size_t)std::max(nnz_new, 1) * tile));
  ca.tmp_ci = ctx->tmp_ci.as<int>();
  ca.tmp_src = ctx->tmp_src.as<int>();
  ca.new_ci = ctx->ci[n].as<int>();
  ca.new_src = ctx->new_src.as<int>();
  launch_compact_scatter(st, ca, n_kept);
  launch_row_sort(st, ca);
  // the new values and the masks of their nonzero matrices, in one pass
  HIPCHK(ctx->mask[n].reserve((size_t)std::max(nnz_new, 1)));
  launch_gather_masks(st, ctx->cur_prec, nnz_new, D, ctx->new_src.as<int>(), ctx->stage.p,
                      ctx->xv[c].p, ctx->mask[n].as<unsigned char>(), nullptr, nullptr, nullptr);
  HIPCHK(hipGetLastError());
  ctx->xv[c].swap(ctx->xv[n]);
  ctx->nnz[n] = nnz_new;
  ctx->cur = n;
  ctx->bn_valid = false;
  if (ctx->profile) HIPCHK(hipEventRecord(ctx->pev[1], st));

  // ---- per-system scalars of the new iterate
  HIPCHK(ctx->scal.reserve((size_t)ctx->nsys * NQ * 8));
  launch_reduce(st, ctx->nsys, ctx->sys_lo.as<int>(), ctx->sys_hi.as<int>(), ctx->partial.as<double>(),
                ctx->scal.as<double>());
  scal.resize((size_t)ctx->nsys * NQ);
  HIPCHK(hipMemcpyAsync(scal.data(), ctx->scal.p, scal.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  if (ctx->profile) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->pev[0], ctx->pev[1]));
    ctx->ms_cmp += ms;
  }
  return TC2_OK;
}

// One update of the tiled path as a single captured hipGraph: panels, tiles,
// block norms, the persistent numeric kernel (sub-tiles taken from an atomic
// counter, their count read on the device), copy-through, compaction and the
// per-system reductions.  No size is read back in between: buffers are sized
// from bounds known before the update (panel entries <= stored blocks, tiles
// <= tile_bound, new entries <= 2 x stage capacity) and from an estimate of
// the kept blocks; when the stage overflows, the update is run again with a
// larger stage (the iterate it reads is untouched).  The graph is replayed as
// long as the buffers, sizes and kernel choice it captured are unchanged.
// Returns TC2_OK, an error, or 1 when the runtime refused the capture (the
// caller then runs the update without a graph).
// A graph-mode buffer that cannot be allocated (its bounds are looser than
// the exact sizes of the update without a graph) switches the context back
// to updates without graphs; only buffers of the next iterate and work
// buffers are reserved here, never the current iterate.
#define GRESERVE(x)                                                      \
  do {                                                                   \
    hipError_t e_ = (x);                                                 \
    if (e_ == hipErrorOutOfMemory) {                                     \
      (void)hipGetLastError();                                           \
      for (DBuf* b_ : {&ctx->stage, &ctx->kept_ij, &ctx->tmp_ci, &ctx->tmp_src, \
                       &ctx->new_src, &ctx->ci[n]})                        \
        b_->release();                                                   \
      return 1;                                                          \
    }                                                                    \
    if (e_ != hipSuccess) return TC2_EDEVICE;                            \
  } while (0)

int step_graph(tc2_ctx* ctx, hipStream_t st, std::vector<double>& scal,
               unsigned long long& exec_pairs_total, bool dl = false) {
  const int c = ctx->cur, n = c ^ 1;
  const int nb = ctx->nb, D = ctx->D, nc = ctx->nc;
  const int kind = ctx->cur_prec == P_FP64 ? K_FP64
                   : ((ctx->op_bf16 && !ctx->wide) ? K_BF16 : (ctx->wide ? K_WIDE : K_FP32));
  const int shape = ctx->shape[kind];
  const int mult = tile_subs(shape);
  const size_t tile = (size_t)(1 + D) * BS * prec_bytes(ctx->cur_prec);
  const bool screen = ctx->skip_now != 0;
  // with the decisions on the device the host does not know which systems
  // have stopped: the copy-through is always part of the update
  bool any_stopped = dl;
  if (!dl)
    for (int s = 0; s < ctx->nsys; ++s) any_stopped |= !ctx->h_active[s];
  ctx->kind_used[kind] = true;
  ctx->last_kind = kind;
  const long long nnz_c = ctx->nnz[c];

  // kept-block estimate: the last count grown by the larger of the last two
  // growth factors; with the decisions on the device, the dense bound (no update can
  // overflow it, so none needs a size from the host)
  long long est;
  if (dl) {
    est = ctx->dl_cap;
  } else if (ctx->kept_prev == 0) {
    est = 2 * nnz_c + 1024;
  } else {
    // the larger of the last two growth factors: the growth of the kept
    // count varies from one update to the next (cube30: 2.45, 1.98, 1.07,
    // 1.53, 1.10, 1.43, ...), and an update that overflows its stage runs
    // its products again; 2.5 after the first update
    double g = 2.5;
    if (ctx->kept_prev2 > 0) {
      g = (double)ctx->kept_prev / (double)ctx->kept_prev2;
      if (ctx->kept_prev3 > 0) g = std::max(g, (double)ctx->kept_prev2 / (double)ctx->kept_prev3);
    }
    g = std::min(2.5, std::max(1.0, g));
    est = (long long)(ctx->kept_prev * g * 1.1) + 1024;
  }
  // geometric buckets (steps of 2^(1/4)): the capacity is part of the graph
  // key, so updates whose estimates share a bucket replay the same graph
  if (!dl) {
    double v = 1024.0;
    while (v < (double)est) v *= 1.189207115002721;
    est = (long long)v;
    if (ctx->test_stage_cap > 0) est = ctx->test_stage_cap;
  }
  est = std::min<long long>(est, INT32_MAX / 2);
  // entries of the current pattern the panel buffers must hold: the
  // host's count, or the bound of any pattern under the dense stage bound
  const long long ent_c = dl ? 2 * est : nnz_c;

  int hcnt[8];
  unsigned long long pairs = 0, sc[2] = {0, 0};
  int nnz_new = 0;
  for (int attempt = 0;; ++attempt) {
    const int cap = (int)est;
    GRESERVE(ctx->counters.reserve(64));
    GRESERVE(ctx->exec_pairs.reserve(8));
    GRESERVE(ctx->panel_cnt.reserve((size_t)nc * 4));
    GRESERVE(ctx->panel_rp.reserve((size_t)(nc + 1) * 4));
    GRESERVE(ctx->tile_cnt.reserve((size_t)nc * 4));
    GRESERVE(ctx->tile_rp.reserve((size_t)(nc + 1) * 4));
    GRESERVE(ctx->tile_pairs.reserve((size_t)nc * 8));
    const int tile_words = (ctx->max_sys_clusters + 31) / 32;
    GRESERVE(ctx->tile_bits.reserve((size_t)std::max(nc, 1) * tile_words * 4));
    GRESERVE(ctx->panel_k.reserve((size_t)std::max<long long>(ent_c, 1) * 4));
    GRESERVE(ctx->panel_e.reserve((size_t)std::max<long long>(ent_c, 1) * CS * 4));
    GRESERVE(ctx->tile_p.reserve((size_t)std::max<long long>(ctx->tile_bound, 1) * 4));
    GRESERVE(ctx->tile_q.reserve((size_t)std::max<long long>(ctx->tile_bound, 1) * 4));
    GRESERVE(ctx->partial.reserve((size_t)std::max(ctx->tile_bound * 4, (long long)nb) * NQ * 8));
    GRESERVE(ctx->sys_lo.reserve((size_t)ctx->nsys * 4));
    GRESERVE(ctx->sys_hi.reserve((size_t)ctx->nsys * 4));
    GRESERVE(ctx->stage.reserve((size_t)cap * tile));
    GRESERVE(ctx->kept_ij.reserve((size_t)cap * 8));
    GRESERVE(ctx->rowcnt.reserve((size_t)nb * 4));
    GRESERVE(ctx->cursor.reserve((size_t)nb * 4));
    GRESERVE(ctx->rp[n].reserve((size_t)(nb + 1) * 4));
    const size_t cap2 = (size_t)2 * cap;
    GRESERVE(ctx->tmp_ci.reserve(cap2 * 4));
    GRESERVE(ctx->tmp_src.reserve(cap2 * 4));
    GRESERVE(ctx->new_src.reserve(cap2 * 4));
    GRESERVE(ctx->ci[n].reserve(cap2 * 4));
    GRESERVE(ctx->mask[n].reserve(cap2));
    // one value buffer holds the current values and receives the new ones:
    // it grows, keeping the current values, to the larger of the two
    ctx->xv[n].release();
    GRESERVE(ctx->xv[c].grow_keep(std::max<size_t>(cap2, (size_t)nnz_c) * tile, (size_t)nnz_c * tile, st));
    // entries the value buffer can hold: a bound of the current entries for
    // the kernels that read their count from the device
    const long long cap_c = std::max<long long>((long long)(ctx->xv[c].cap / tile), 1);
    // the gather of the last captured update wrote the block norms of the
    // current iterate into bn, unless bn must grow now (growing drops them)
    const size_t bn_need = (size_t)cap_c * (1 + D) * 4;
    const bool norms_ready = screen && ctx->bn_valid && ctx->bn.p && ctx->bn.cap >= bn_need;
    if (screen) {
      GRESERVE(ctx->bn.reserve(bn_need));
      GRESERVE(ctx->screened.reserve(16));
    }
    GRESERVE(ctx->scal.reserve((size_t)ctx->nsys * NQ * 8));
    GRESERVE(ctx->pin_graph.reserve(64 + (size_t)ctx->nsys * NQ * 8));
    int* cnt = ctx->counters.as<int>();  // [1] stage count [2] overflow [4] work counter

    // what the graph captures: everything that would change a launch
    const std::vector<unsigned long long> key = {
        (unsigned long long)kind, (unsigned long long)shape, (unsigned long long)screen,
        (unsigned long long)any_stopped, (unsigned long long)cap, (unsigned long long)cap_c,
        (unsigned long long)ctx->profile, (unsigned long long)(uintptr_t)st, (unsigned long long)dl,
        (unsigned long long)norms_ready,
        (uintptr_t)ctx->xv[c].p, (uintptr_t)ctx->rp[c].p, (uintptr_t)ctx->ci[c].p,
        (uintptr_t)ctx->rp[n].p, (uintptr_t)ctx->ci[n].p,
        (uintptr_t)ctx->panel_k.p, (uintptr_t)ctx->panel_e.p, (uintptr_t)ctx->tile_p.p,
        (uintptr_t)ctx->tile_q.p, (uintptr_t)ctx->partial.p, (uintptr_t)ctx->bn.p,
        (uintptr_t)ctx->stage.p, (uintptr_t)ctx->kept_ij.p, (uintptr_t)ctx->tmp_ci.p,
        (uintptr_t)ctx->tmp_src.p, (uintptr_t)ctx->new_src.p, (uintptr_t)ctx->scal.p,
        (uintptr_t)ctx->counters.p, (uintptr_t)ctx->screened.p, (uintptr_t)ctx->exec_pairs.p,
        (uintptr_t)ctx->rowcnt.p, (uintptr_t)ctx->cursor.p, (uintptr_t)ctx->sys_lo.p,
        (uintptr_t)ctx->sys_hi.p, (uintptr_t)ctx->panel_cnt.p, (uintptr_t)ctx->panel_rp.p,
        (uintptr_t)ctx->tile_cnt.p, (uintptr_t)ctx->tile_rp.p, (uintptr_t)ctx->tile_pairs.p,
        (uintptr_t)ctx->tile_bits.p, (uintptr_t)ctx->nominal.p, (uintptr_t)ctx->mask[c].p,
        (uintptr_t)ctx->mask[n].p};
    // the three parts of the update, as stream work (captured or not)
    auto rec_pre = [&]() {
      (void)count_nominal(ctx, st, ctx->rp[c].as<int>());
      PanelArgs pa{};
      pa.nc = nc;
      pa.rp = ctx->rp[c].as<int>();
      pa.ci = ctx->ci[c].as<int>();
      pa.clus_atom = ctx->clus_atom.as<int>();
      pa.clus_sys = ctx->clus_sys.as<int>();
      pa.sys_start = ctx->sys_start.as<int>();
      pa.sys_end = ctx->sys_end.as<int>();
      pa.csys_start = ctx->csys_start.as<int>();
      pa.csys_end = ctx->csys_end.as<int>();
      pa.atom_clus = ctx->atom_clus.as<int>();
      pa.active = ctx->active.as<int>();
      pa.max_sys_atoms = ctx->max_sys_atoms;
      pa.max_sys_clusters = ctx->max_sys_clusters;
      pa.panel_cnt = ctx->panel_cnt.as<int>();
      pa.panel_rp = ctx->panel_rp.as<int>();
      pa.tile_cnt = ctx->tile_cnt.as<int>();
      pa.tile_pairs = ctx->tile_pairs.as<long long>();
      pa.tile_rp = ctx->tile_rp.as<int>();
      pa.panel_k = ctx->panel_k.as<int>();
      pa.panel_e = ctx->panel_e.as<int>();
      pa.tile_p = ctx->tile_p.as<int>();
      pa.tile_q = ctx->tile_q.as<int>();
      pa.tile_bits = ctx->tile_bits.as<unsigned>();
      pa.tile_words = tile_words;
      launch_panels(st, 0, pa);
      launch_scan(st, nc, ctx->panel_cnt.as<int>(), ctx->panel_rp.as<int>(), cnt);
      launch_panels(st, 1, pa);
      launch_tiles(st, 0, pa);
      launch_scan(st, nc, ctx->tile_cnt.as<int>(), ctx->tile_rp.as<int>(), cnt);
      launch_tiles(st, 1, pa);
      launch_sys_items(st, ctx->nsys, mult, ctx->csys_start.as<int>(), ctx->csys_end.as<int>(),
                       ctx->tile_rp.as<int>(), ctx->sys_lo.as<int>(), ctx->sys_hi.as<int>());
      if (screen) {
        launch_fill_int(st, ctx->screened.as<int>(), 0, 4);
        if (!norms_ready)
          launch_block_norms(st, ctx->cur_prec, cap_c, D, ctx->xv[c].p, ctx->bn.as<float>(),
                             ctx->rp[c].as<int>() + nb);
      }
      launch_fill_int(st, cnt, 0, 8);
      launch_fill_int(st, ctx->exec_pairs.as<int>(), 0, 2);
    };
    auto rec_num = [&]() -> bool {
      TileArgs ta{};
      ta.D = D;
      ta.ksteps = (ctx->b + 3) / 4;
      ta.n_tiles = (int)std::min<long long>(ctx->tile_bound, INT32_MAX / 4);
      ta.n_tiles_dev = ctx->tile_rp.as<int>() + nc;
      ta.work = cnt + 4;
      ta.rp = ctx->rp[c].as<int>();
      ta.ci = ctx->ci[c].as<int>();
      ta.xv = ctx->xv[c].p;
      ta.tile_p = ctx->tile_p.as<int>();
      ta.tile_q = ctx->tile_q.as<int>();
      ta.clus_atom = ctx->clus_atom.as<int>();
      ta.clus_sys = ctx->clus_sys.as<int>();
      ta.panel_rp = ctx->panel_rp.as<int>();
      ta.panel_k = ctx->panel_k.as<int>();
      ta.panel_e = ctx->panel_e.as<int>();
      ta.branch = ctx->branch.as<int>();
      ta.eps = ctx->eps.as<double>();
      ta.h_rp = ctx->h_rp.as<int>();
      ta.h_ci = ctx->h_ci.as<int>();
      ta.h_v = ctx->h_v.as<double>();
      for (int d = 0; d < D; ++d) {
        ta.h1_rp[d] = ctx->h1_rp[d].as<int>();
        ta.h1_ci[d] = ctx->h1_ci[d].as<int>();
        ta.h1_v[d] = ctx->h1_v[d].as<double>();
      }
      ta.stage = ctx->stage.p;
      ta.kept_ij = ctx->kept_ij.as<int2>();
      ta.stage_count = cnt + 1;
      ta.stage_cap = cap;
      ta.overflow = cnt + 2;
      ta.bad = ctx->bad.as<int>();
      ta.partial = ctx->partial.as<double>();
      ta.exec_pairs = ctx->exec_pairs.as<unsigned long long>();
      ta.bf16 = (ctx->op_bf16 && ctx->cur_prec == P_FP32) ? 1 : 0;
      ta.wide = kind == K_WIDE ? 1 : 0;
      ta.shape = shape;
      ta.skip = ctx->skip_now;
      ta.xmask = ctx->test_no_zero_skip ? nullptr : ctx->mask[c].as<unsigned char>();
      ta.waves_per_column = ctx->test_waves_per_column;
      ta.bn = screen ? ctx->bn.as<float>() : nullptr;
      ta.screened = screen ? ctx->screened.as<unsigned long long>() : nullptr;
      ta.mlp_skipped = screen ? ctx->screened.as<unsigned long long>() + 1 : nullptr;
      ta.kl_chunk = ctx->test_kl_chunk;
      return launch_tile_numeric(st, ctx->cur_prec, ta);
    };
    auto rec_post = [&]() {
      if (any_stopped) {
        CopyArgs ca{};
        ca.nb = nb;
        ca.D = D;
        ca.rp = ctx->rp[c].as<int>();
        ca.ci = ctx->ci[c].as<int>();
        ca.xv = ctx->xv[c].p;
        ca.sys_of = ctx->sys_of.as<int>();
        ca.active = ctx->active.as<int>();
        ca.stage = ctx->stage.p;
        ca.kept_ij = ctx->kept_ij.as<int2>();
        ca.stage_count = cnt + 1;
        ca.stage_cap = cap;
        ca.overflow = cnt + 2;
        launch_copy_through(st, ctx->cur_prec, ca, (int)cap_c);
      }
      launch_fill_int(st, ctx->rowcnt.as<int>(), 0, nb);
      launch_fill_int(st, ctx->cursor.as<int>(), 0, nb);
      CompactArgs cm{};
      cm.nb = nb;
      cm.D = D;
      cm.kept_ij = ctx->kept_ij.as<int2>();
      cm.rowcnt = ctx->rowcnt.as<int>();
      cm.cursor = ctx->cursor.as<int>();
      cm.new_rp = ctx->rp[n].as<int>();
      cm.sys_of = ctx->sys_of.as<int>();
      cm.sys_start = ctx->sys_start.as<int>();
      cm.sys_end = ctx->sys_end.as<int>();
      cm.max_sys_atoms = ctx->max_sys_atoms;
      cm.n_kept_dev = cnt + 1;
      cm.tmp_ci = ctx->tmp_ci.as<int>();
      cm.tmp_src = ctx->tmp_src.as<int>();
      cm.new_ci = ctx->ci[n].as<int>();
      cm.new_src = ctx->new_src.as<int>();
      launch_compact_count(st, cm, cap);
      launch_scan(st, nb, ctx->rowcnt.as<int>(), ctx->rp[n].as<int>(), cnt);
      launch_compact_scatter(st, cm, cap);
      launch_row_sort(st, cm);
      // the gather (with the masks of the new values) writes over the current
      // values: skipped when the stage overflowed (the update is then run
      // again from those values)
      launch_gather_masks(st, ctx->cur_prec, (long long)cap2, D, ctx->new_src.as<int>(),
                          ctx->stage.p, ctx->xv[c].p, ctx->mask[n].as<unsigned char>(),
                          screen ? ctx->bn.as<float>() : nullptr, ctx->rp[n].as<int>() + nb,
                          cnt + 2);
      launch_reduce(st, ctx->nsys, ctx->sys_lo.as<int>(), ctx->sys_hi.as<int>(),
                    ctx->partial.as<double>(), ctx->scal.as<double>());
      if (dl) {
        // branch and stopping decisions for the next update, on the device
        DecideArgs da{};
        da.nsys = ctx->nsys;
        da.D = D;
        da.init = 0;
        da.scal = ctx->scal.as<double>();
        da.bad = ctx->bad.as<int>();
        da.nominal = ctx->nominal.as<unsigned long long>();
        da.exec_pairs = ctx->exec_pairs.as<unsigned long long>();
        da.screened = screen ? ctx->screened.as<unsigned long long>() : nullptr;
        da.overflow = cnt + 2;
        da.param = ctx->dl_param.as<DecideParam>();
        da.state = ctx->dl_state.as<DecideSys>();
        da.active = ctx->active.as<int>();
        da.branch = ctx->branch.as<int>();
        da.word = ctx->dl_word.as<DecideWord>();
        launch_decide(st, da);
      }
    };
    // capture of a part sequence into an executable graph; false if refused
    auto capture = [&](hipGraphExec_t* out, bool with_pre, bool with_num, bool with_post) {
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return false;
      }
      bool ok = true;
      if (with_pre) rec_pre();
      if (with_num) ok = rec_num();
      if (with_post) rec_post();
      if (hipGetLastError() != hipSuccess) ok = false;
      hipGraph_t graph = nullptr;
      const hipError_t ee = hipStreamEndCapture(st, &graph);
      if (ee != hipSuccess || !ok || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return false;
      }
      const hipError_t ie = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) {
        *out = nullptr;
        (void)hipGetLastError();
        return false;
      }
      return true;
    };
    // one graph for the whole update; when profiling, the products run as a
    // direct launch between a graph before and a graph after them, so that
    // stream events can time them
    if (!ctx->gexec[c] || ctx->gkey[c] != key) {
      for (hipGraphExec_t* g : {&ctx->gexec[c], &ctx->gexec_post[c]})
        if (*g) {
          (void)hipGraphExecDestroy(*g);
          *g = nullptr;
        }
      const bool ok = ctx->profile
                          ? capture(&ctx->gexec[c], true, false, false) &&
                                capture(&ctx->gexec_post[c], false, false, true)
                          : capture(&ctx->gexec[c], true, true, true);
      if (!ok) return 1;
      ctx->gkey[c] = key;
      ctx->graph_captures++;
    }
    if (ctx->profile) {
      HIPCHK(hipEventRecord(ctx->pev[0], st));
      HIPCHK(hipGraphLaunch(ctx->gexec[c], st));
      HIPCHK(hipEventRecord(ctx->pev[1], st));
      HIPCHK(hipEventRecord(ctx->pev[2], st));
      if (!rec_num()) return TC2_EINVAL;
      HIPCHK(hipGetLastError());
      HIPCHK(hipEventRecord(ctx->pev[3], st));
      HIPCHK(hipEventRecord(ctx->pev[4], st));
      HIPCHK(hipGraphLaunch(ctx->gexec_post[c], st));
      HIPCHK(hipEventRecord(ctx->pev[5], st));
    } else {
      HIPCHK(hipGraphLaunch(ctx->gexec[c], st));
    }
    if (dl) {
      // nothing is read back: the device has taken the decisions, and the
      // host polls their flag word every device_loop updates
      ctx->xv[c].swap(ctx->xv[n]);
      ctx->cur = n;
      ctx->bn_valid = screen;
      return TC2_OK;
    }
    // counters, pairs, new entries, screen counts and scalars, read back
    // through page-locked memory: [hcnt 32 B | pairs 8 | nnz_new 8 | sc 16 | scal]
    scal.resize((size_t)ctx->nsys * NQ);
    char* pin = (char*)ctx->pin_graph.p;
    HIPCHK(hipMemcpyAsync(pin, cnt, sizeof(hcnt), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(pin + 32, ctx->exec_pairs.p, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(pin + 40, ctx->rp[n].as<int>() + nb, 4, hipMemcpyDeviceToHost, st));
    if (screen) HIPCHK(hipMemcpyAsync(pin + 48, ctx->screened.p, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(pin + 64, ctx->scal.p, scal.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    memcpy(hcnt, pin, sizeof(hcnt));
    memcpy(&pairs, pin + 32, 8);
    memcpy(&nnz_new, pin + 40, 4);
    if (screen) memcpy(sc, pin + 48, 16);
    memcpy(scal.data(), pin + 64, scal.size() * 8);
    if (ctx->profile) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ctx->pev[0], ctx->pev[1]));
      ctx->ms_sym += ms;
      HIPCHK(hipEventElapsedTime(&ms, ctx->pev[2], ctx->pev[3]));
      ctx->ms_num += ms;
      ctx->ms_num_kind[kind] += ms;
      ctx->num_launches++;
      ctx->launches_kind[kind]++;
      HIPCHK(hipEventElapsedTime(&ms, ctx->pev[4], ctx->pev[5]));
      ctx->ms_cmp += ms;
    }
    if (!hcnt[2]) break;
    // stage overflow: the counter still counts every kept block
    est = std::min<long long>((long long)hcnt[1] * 5 / 4 + 1024, INT32_MAX / 2);
    if (attempt > 3) return TC2_ENOMEM;
  }
  exec_pairs_total += pairs;
  if (screen) {
    ctx->screened_total += sc[0];
    ctx->mlp_total += sc[1];
  }
  ctx->kept_prev3 = ctx->kept_prev2;
  ctx->kept_prev2 = ctx->kept_prev;
  ctx->kept_prev = hcnt[1];
  ctx->stage_cap = std::max<long long>(ctx->stage_cap, (long long)hcnt[1] * 5 / 4 + 1024);
  ctx->xv[c].swap(ctx->xv[n]);
  ctx->nnz[n] = nnz_new;
  ctx->cur = n;
  ctx->bn_valid = screen;  // the gather wrote the new iterate's block norms
  ctx->graph_updates++;
  if (ctx->verbose)
    fprintf(stderr, "tc2 step (graph): kept=%d pairs=%llu new entries=%d captures=%d\n", hcnt[1],
            pairs, nnz_new, ctx->graph_captures);
  return TC2_OK;
}

// energies vector used by the stopping test: E0, E1_d, alpha_d
void energies(const double* q, int D, double* e) {
  e[0] = q[Q_E0];
  for (int d = 0; d < D; ++d) {
    e[1 + d] = q[Q_E1 + d];
    e[1 + D + d] = q[Q_AL + d];
  }
}

tc2_status export_results(tc2_ctx* ctx, hipStream_t st) {
  const int c = ctx->cur, D = ctx->D, b = ctx->b, nb = ctx->nb;
  const int nnz = ctx->nnz[c];
  std::vector<int> rp(nb + 1), ci(std::max(nnz, 1));
  HIPCHK(hipMemcpyAsync(rp.data(), ctx->rp[c].p, (size_t)(nb + 1) * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(ci.data(), ctx->ci[c].p, (size_t)nnz * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(ctx->xfer.reserve((size_t)std::max(nnz, 1) * b * b * 8));
  std::vector<double> v((size_t)nnz * b * b);
  ctx->out_x0.assign(ctx->nsys, HostBsr());
  for (int d = 0; d < MAXD; ++d) ctx->out_x1[d].assign(d < D ? ctx->nsys : 0, HostBsr());
  for (int m = 0; m <= D; ++m) {
    launch_export(st, ctx->cur_prec, nnz, D, m, b, ctx->xv[c].p, ctx->xfer.as<double>());
    HIPCHK(hipMemcpyAsync(v.data(), ctx->xfer.p, v.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int s = 0; s < ctx->nsys; ++s) {
      const SysInfo& si = ctx->sys[s];
      HostBsr& hb = (m == 0) ? ctx->out_x0[s] : ctx->out_x1[m - 1][s];
      hb.row_ptr.assign(1, 0);
      hb.col.clear();
      hb.val.clear();
      for (int i = 0; i < si.nb; ++i) {
        int I = si.row0 + i;
        for (int p = rp[I]; p < rp[I + 1]; ++p) {
          hb.col.push_back(ci[p] - si.row0);
          hb.val.insert(hb.val.end(), v.begin() + (size_t)p * b * b, v.begin() + (size_t)(p + 1) * b * b);
        }
        hb.row_ptr.push_back((int64_t)hb.col.size());
      }
    }
  }
  return TC2_OK;
}

// Whether the solve in progress has finished: no system is active and no
// stage switch is pending (the next stage would reactivate systems).
bool solve_finished(const tc2_ctx* ctx) {
  const RunState& R = ctx->run;
  for (int s = 0; s < ctx->nsys; ++s)
    if (R.ss[s].active) return false;
  if (R.phase == 0 && ctx->op_bf16 && !ctx->wide) return false;
  if (R.phase == 0 && R.reduced && ctx->closing == 2) return false;
  return true;
}

// Start of a solve: counters reset, Gershgorin bounds, the initial matrices
// and their scalars (every system restarts from H).
tc2_status begin_solve(tc2_ctx* ctx, hipStream_t st) {
  RunState& R = ctx->run;
  const int nsys = ctx->nsys, D = ctx->D, b = ctx->b, nb = ctx->nb;
  R.open = false;
  R.st = st;
  R.ss.assign(nsys, SysState());
  ctx->ms_sym = ctx->ms_num = ctx->ms_cmp = 0.0;
  for (int k = 0; k < 4; ++k) {
    ctx->ms_num_kind[k] = 0.0;
    ctx->launches_kind[k] = 0;
  }
  ctx->ms_tune = 0.0;
  ctx->prev_out_bound = -1;
  ctx->kept_prev = ctx->kept_prev2 = ctx->kept_prev3 = 0;
  ctx->dl_updates = 0;
  ctx->bn_valid = false;
  ctx->graph_updates = 0;
  ctx->graph_captures = 0;
  for (bool& u : ctx->kind_used) u = false;
  ctx->screened_total = 0;
  ctx->mlp_total = 0;
  ctx->log_n = 0;
  if (ctx->log_cap > 0) launch_fill_int(st, ctx->log_count.as<int>(), 0, 2);
  ctx->num_launches = 0;
  ctx->skip_now = ctx->skip;
  ctx->mlp_updates = 0;
  if (ctx->skip == 2) launch_fill_int(st, ctx->mlp_bsum.as<int>(), 0, 2LL * nsys);
  if (ctx->count_useful) {
    HIPCHK(ctx->useful_acc.reserve((size_t)nsys * 4 * 8));
    launch_fill_int(st, ctx->useful_acc.as<int>(), 0, 8LL * nsys);
  }
  if (!R.ev0) HIPCHK(hipEventCreate(&R.ev0));
  if (!R.ev1) HIPCHK(hipEventCreate(&R.ev1));
  HIPCHK(hipEventRecord(R.ev0, st));

  // ---- Gershgorin bounds and the initial matrices
  R.emin.assign(nsys, 0.0);
  R.emax.assign(nsys, 0.0);
  launch_gershgorin(st, nb, b, ctx->h_rp.as<int>(), ctx->h_ci.as<int>(), ctx->h_v.as<double>(),
                    ctx->rowlo.as<double>(), ctx->rowhi.as<double>());
  launch_sys_minmax(st, nsys, ctx->sys_start.as<int>(), ctx->sys_end.as<int>(), b, ctx->rowlo.as<double>(),
                    ctx->rowhi.as<double>(), ctx->emin.as<double>(), ctx->emax.as<double>());
  HIPCHK(hipMemcpyAsync(R.emin.data(), ctx->emin.p, nsys * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(R.emax.data(), ctx->emax.p, nsys * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  R.mode.assign(nsys, 0);
  R.active.assign(nsys, 0);
  R.branch.assign(nsys, 0);
  R.bad.assign(nsys, 0);
  R.nominal.assign(nsys, 0);
  R.pin_nominal = ((size_t)nsys * 12 + 7) / 8 * 8;  // after three int arrays
  HIPCHK(ctx->pin_loop.reserve(R.pin_nominal + (size_t)nsys * 8));
  for (int s = 0; s < nsys; ++s) {
    R.mode[s] = ctx->sys[s].mode;
    R.ss[s].status = TC2_OK;
    if (R.mode[s] == 0 && !(R.emax[s] > R.emin[s])) {
      R.ss[s].status = TC2_EDEGENERATE;
      R.mode[s] = 1;  // placeholder result; status reports the error
    }
    if (R.mode[s] == 0) R.ss[s].active = true;
  }
  HIPCHK(hipMemcpyAsync(ctx->mode.p, R.mode.data(), nsys * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ctx->bad.p, R.bad.data(), nsys * 4, hipMemcpyHostToDevice, st));
  // reduced precision keeps FP32 values; BF16 rounds the MFMA operands only.
  // fp64_first leading updates run in FP64 before the switch.
  const int start_prec = (ctx->prec == P_FP64 || ctx->fp64_first > 0) ? P_FP64 : P_FP32;
  ctx->cur = 0;
  ctx->cur_prec = start_prec;
  ctx->nnz[0] = ctx->nnz0;
  ctx->stage_cap = 0;
  const size_t tile = (size_t)(1 + D) * BS * prec_bytes(start_prec);
  // the value buffer of the last solve (in either slot) is kept for this one
  if (ctx->xv[1].cap > ctx->xv[0].cap) ctx->xv[0].swap(ctx->xv[1]);
  ctx->xv[1].release();
  HIPCHK(ctx->rp[0].reserve((size_t)(nb + 1) * 4));
  HIPCHK(ctx->ci[0].reserve((size_t)std::max(ctx->nnz0, 1) * 4));
  HIPCHK(ctx->xv[0].reserve((size_t)std::max(ctx->nnz0, 1) * tile));
  HIPCHK(hipMemcpyAsync(ctx->rp[0].p, ctx->x0_rp.p, (size_t)(nb + 1) * 4, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(ctx->ci[0].p, ctx->x0_ci.p, (size_t)ctx->nnz0 * 4, hipMemcpyDeviceToDevice, st));
  {
    const int* src1[MAXD] = {nullptr, nullptr, nullptr};
    const double* h1v[MAXD] = {nullptr, nullptr, nullptr};
    for (int d = 0; d < D; ++d) {
      src1[d] = ctx->src_h1[d].as<int>();
      h1v[d] = ctx->h1_v[d].as<double>();
    }
    launch_init(st, start_prec, ctx->nnz0, D, b, ctx->x0_row.as<int>(), ctx->x0_ci.as<int>(),
                ctx->src_h.as<int>(), src1, ctx->h_v.as<double>(), h1v, ctx->sys_of.as<int>(),
                ctx->emin.as<double>(), ctx->emax.as<double>(), ctx->mode.as<int>(), ctx->xv[0].p);
  }
  ctx->have_iterate = true;
  tc2_status st0 = measure(ctx, st, R.scal);
  if (st0 != TC2_OK) return st0;
  for (int s = 0; s < nsys; ++s) {
    energies(&R.scal[(size_t)s * NQ], D, R.ss[s].prev);
    R.branch[s] = R.scal[(size_t)s * NQ + Q_TR0] >= (double)ctx->sys[s].n_occ ? 1 : 0;
  }
  st0 = mask_iterate(ctx, st);
  if (st0 != TC2_OK) return st0;
  // stages of a reduced-precision solve: [FP64 x fp64_first] -> [BF16] -> FP32
  // -> closing FP64 pair; each reduced stage runs to its own stopping test.
  R.reduced = ctx->prec != P_FP64;
  ctx->op_bf16 = ctx->prec == P_BF16 ? 1 : 0;
  R.phase = 0;
  R.updates = 0;
  R.later_stage = false;
  R.exec_pairs = 0;
  R.open = true;
  ctx->solve_index++;
  return TC2_OK;
}

// One JSON line per system that took part in the update just run: the
// scalars of the new iterate, the stopping quantities and the stored blocks.
void log_update(tc2_ctx* ctx, const std::vector<int>& was_active, const std::vector<double>& dmax,
                const std::vector<int>& cnt) {
  FILE* f = fopen(ctx->metrics_log.c_str(), "a");
  if (!f) return;
  static const char* kinds[4] = {"fp64", "fp32", "bf16", "fp32w"};
  const RunState& R = ctx->run;
  for (int s = 0; s < ctx->nsys; ++s) {
    if (!was_active[s]) continue;
    const SysState& S = R.ss[s];
    const double* q = &R.scal[(size_t)s * NQ];
    fprintf(f, "{\"solve\": %d, \"system\": %d, \"update\": %d, \"branch\": \"%c\", "
               "\"kind\": \"%s\", \"phase\": %d, \"tr_x0\": %.17g, \"e0\": %.17g, \"iota\": %.17g, "
               "\"dmax\": %.17g, \"nnzb\": %d",
            ctx->solve_index, s, S.k, S.branches.back(), kinds[ctx->last_kind], R.phase, q[Q_TR0],
            q[Q_E0], q[Q_TR0] - q[Q_FRO0], dmax[s], cnt[s + 1] - cnt[s]);
    const char* names[3] = {"tr_x1", "e1", "alpha"};
    const int base[3] = {Q_TR1, Q_E1, Q_AL};
    for (int k = 0; k < 3; ++k) {
      fprintf(f, ", \"%s\": [", names[k]);
      for (int d = 0; d < ctx->D; ++d) fprintf(f, "%s%.17g", d ? ", " : "", q[base[k] + d]);
      fprintf(f, "]");
    }
    fprintf(f, ", \"active\": %s, \"status\": %d}\n", S.active ? "true" : "false", (int)S.status);
  }
  fclose(f);
}

// One update of every active system, preceded by the stage switch that is
// due (BF16 -> FP32, reduced stage -> closing FP64 pair).  *done is set, and
// no update runs, when the solve has finished.
tc2_status advance_one(tc2_ctx* ctx, bool* done) {
  RunState& R = ctx->run;
  hipStream_t st = R.st;
  const int nsys = ctx->nsys, D = ctx->D;
  std::vector<SysState>& ss = R.ss;
  *done = false;
  for (;;) {
    bool any = false;
    for (int s = 0; s < nsys; ++s) {
      R.active[s] = ss[s].active ? 1 : 0;
      any |= ss[s].active;
      if (ss[s].active) {
        const std::string& rep = ctx->sys[s].replay;
        if (R.phase == 0 && !rep.empty()) R.branch[s] = rep[ss[s].k] == 'S' ? 1 : 0;
        ss[s].branches.push_back(R.branch[s] ? 'S' : 'D');
      }
    }
    if (any) break;
    if (R.phase == 0 && ctx->op_bf16 && !ctx->wide) {
      // BF16 stage done: continue with FP32 operands from where it stopped
      ctx->op_bf16 = 0;
      R.later_stage = true;
      for (int s = 0; s < nsys; ++s)
        if (R.mode[s] == 0 && ss[s].status >= 0 && ctx->sys[s].replay.empty()) {
          ss[s].active = true;
          ss[s].iota.clear();
        }
      continue;
    }
    if (R.phase == 0 && R.reduced && ctx->closing == 2) {
      // closing pair in FP64: trace rule, then the opposite branch
      tc2_status cs = convert_iterate(ctx, st, P_FP64);
      if (cs != TC2_OK) return cs;
      R.phase = 1;
      for (int s = 0; s < nsys; ++s)
        if (R.mode[s] == 0 && ss[s].status >= 0) {
          ss[s].active = true;
          ss[s].closing_left = 2;
          ss[s].closing_first = R.branch[s];
        }
      continue;
    }
    *done = true;
    return TC2_OK;
  }
  // flags in and status out through page-locked memory (the previous
  // update's stream synchronisation guarantees its copies have completed):
  // [active | branch | bad] ints, then nominal counts
  char* pin = (char*)ctx->pin_loop.p;
  memcpy(pin, R.active.data(), nsys * 4);
  memcpy(pin + (size_t)nsys * 4, R.branch.data(), nsys * 4);
  HIPCHK(hipMemcpyAsync(ctx->active.p, pin, nsys * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ctx->branch.p, pin + (size_t)nsys * 4, nsys * 4, hipMemcpyHostToDevice, st));
  ctx->h_active = R.active;
  ctx->update_index = R.updates;
  tc2_status r = TC2_OK;
  {
    const int kind_now = ctx->cur_prec == P_FP64 ? K_FP64
                         : ((ctx->op_bf16 && !ctx->wide) ? K_BF16 : (ctx->wide ? K_WIDE : K_FP32));
    // the closing pair runs as direct launches: two updates gain nothing
    // from a captured graph, and sizing their FP64 buffers exactly (not by
    // the graph's bounds) lets them fit in the buffers the reduced stage
    // already holds
    const bool use_graph = ctx->graph && ctx->graph_ok && ctx->kernel == 0 &&
                           ctx->log_cap == 0 && ctx->skip_now != 2 && R.phase == 0 &&
                           (!ctx->tune || ctx->tuned[kind_now]);
    int g = 1;
    if (use_graph) {
      g = step_graph(ctx, st, R.scal, R.exec_pairs);
      if (g == 1) ctx->graph_ok = false;  // the runtime refused the capture
    }
    r = g == 1 ? step(ctx, st, R.scal, R.exec_pairs) : (tc2_status)g;
  }
  if (r != TC2_OK) return r;
  ++R.updates;
  // exact useful count of this update, while the old iterate is still held
  if (ctx->count_useful && (r = count_update(ctx, st)) != TC2_OK) return r;
  if (R.reduced && R.phase == 0 && ctx->cur_prec == P_FP64 && R.updates >= ctx->fp64_first) {
    r = convert_iterate(ctx, st, P_FP32);
    if (r != TC2_OK) return r;
  }
  HIPCHK(hipMemcpyAsync(pin + (size_t)nsys * 8, ctx->bad.p, nsys * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(pin + R.pin_nominal, ctx->nominal.p, nsys * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  memcpy(R.bad.data(), pin + (size_t)nsys * 8, nsys * 4);
  memcpy(R.nominal.data(), pin + R.pin_nominal, nsys * 8);
  std::vector<int> was_active(R.active);
  std::vector<double> dmaxs(nsys, 0.0);
  for (int s = 0; s < nsys; ++s) {
    if (!ss[s].active) continue;
    SysState& S = ss[s];
    const SysInfo& si = ctx->sys[s];
    const double* q = &R.scal[(size_t)s * NQ];
    S.k++;
    S.trip += q[Q_TRIP];
    S.nominal += (double)R.nominal[s];
    double cur[1 + 2 * MAXD];
    energies(q, D, cur);
    const double iota = q[Q_TR0] - q[Q_FRO0];
    S.iota.push_back(iota);
    double dmax = 0.0;
    for (int k = 0; k < 1 + 2 * D; ++k) dmax = std::max(dmax, std::fabs(cur[k] - S.prev[k]));
    dmaxs[s] = dmax;
    std::copy(cur, cur + 1 + 2 * D, S.prev);
    if (ctx->verbose)
      fprintf(stderr, "tc2 sys %d it %d %c tr-nocc %.3e iota %.3e E0 %.12f dmax %.3e\n", s, S.k,
              S.branches.back(), q[Q_TR0] - (double)si.n_occ, iota, cur[0], dmax);
    if (R.bad[s]) {
      S.status = TC2_ENAN;
      S.active = false;
      continue;
    }
    if (R.phase == 1) {
      // closing pair: the second step takes the branch opposite to the first
      if (--S.closing_left == 0) S.active = false;
      else R.branch[s] = S.closing_first ? 0 : 1;
      continue;
    }
    const double tol = ctx->cur_prec == P_FP64 ? si.tol
                                               : std::max(si.tol, (ctx->op_bf16 && !ctx->wide) ? 1e-3 : 1e-6);
    bool stop = false;
    if (!si.replay.empty()) {
      if (S.k == (int)si.replay.size()) {
        stop = true;
        S.status = TC2_OK;
      }
    } else if (S.k >= 2 && dmax < tol) {
      stop = true;
      S.status = TC2_OK;
    } else if (ctx->op_bf16 && !ctx->wide && S.k >= 3 && std::fabs(iota) < 1e-2 * (double)si.n_occ) {
      // bfloat16 stage: hand over to FP32 while the spectrum of X0 is still
      // well inside (0, 1), before bfloat16 rounding can push it out
      stop = true;
      S.status = TC2_OK;
    } else if (S.iota.size() >= 3 && (std::fabs(iota) < 1.0 || R.later_stage) &&
               std::fabs(iota) >= std::fabs(S.iota[S.iota.size() - 3])) {
      // precision floor; in a stage that starts from a reduced-precision
      // iterate, also a growing |iota| (eigenvalues pushed out of [0, 1])
      stop = true;
      S.status = TC2_FLOOR_REACHED;
    } else if (S.k >= si.max_iter) {
      stop = true;
      S.status = TC2_NOT_CONVERGED;
    }
    if (stop) S.active = false;
    R.branch[s] = q[Q_TR0] >= (double)si.n_occ ? 1 : 0;
  }
  if (!ctx->metrics_log.empty()) {
    // stored blocks per system, from the new row pointer at the system
    // boundaries: cnt[s + 1] - cnt[s]
    std::vector<int> rp(ctx->nb + 1), cnt(nsys + 1, 0);
    HIPCHK(hipMemcpyAsync(rp.data(), ctx->rp[ctx->cur].p, (size_t)(ctx->nb + 1) * 4,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int s = 0; s < nsys; ++s)
      cnt[s + 1] = cnt[s] + (rp[ctx->sys[s].row0 + ctx->sys[s].nb] - rp[ctx->sys[s].row0]);
    log_update(ctx, was_active, dmaxs, cnt);
  }
  return TC2_OK;
}

// Useful block products counted so far in this solve, per system and kernel
// kind (count_useful), read from the device.
tc2_status read_useful(tc2_ctx* ctx, hipStream_t st, std::vector<unsigned long long>& acc) {
  acc.assign((size_t)ctx->nsys * 4, 0ull);
  if (!ctx->count_useful) return TC2_OK;
  HIPCHK(hipMemcpyAsync(acc.data(), ctx->useful_acc.p, acc.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return TC2_OK;
}

// End of a solve: timing, final scalars from the stored iterate, the export
// and the per-system results.
tc2_status finish_solve(tc2_ctx* ctx, tc2_result* res) {
  RunState& R = ctx->run;
  hipStream_t st = R.st;
  const int nsys = ctx->nsys, D = ctx->D, b = ctx->b, nb = ctx->nb;
  R.open = false;
  HIPCHK(hipEventRecord(R.ev1, st));
  if (ctx->log_cap > 0) {
    unsigned long long n = 0;
    HIPCHK(hipMemcpyAsync(&n, ctx->log_count.p, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    ctx->log_n = std::min<long long>((long long)n, ctx->log_cap);
  }
  HIPCHK(hipEventSynchronize(R.ev1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, R.ev0, R.ev1));
  std::vector<unsigned long long> acc;
  if (tc2_status s0 = read_useful(ctx, st, acc); s0 != TC2_OK) return s0;

  // final scalars straight from the stored iterate
  std::vector<double> scal;
  tc2_status st0 = measure(ctx, st, scal);
  if (st0 != TC2_OK) return st0;
  if (ctx->export_m) {
    st0 = export_results(ctx, st);
    if (st0 != TC2_OK) return st0;
  }
  std::vector<int> final_rp(nb + 1);
  HIPCHK(hipMemcpyAsync(final_rp.data(), ctx->rp[ctx->cur].p, (size_t)(nb + 1) * 4,
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  tc2_status worst = TC2_OK;
  const double b3 = 2.0 * b * b * b;
  const double kst = (double)((b + 3) / 4) * 4;
  for (int s = 0; s < nsys; ++s) {
    tc2_result& Rs = res[s];
    const SysState& S = R.ss[s];
    memset(&Rs, 0, sizeof(Rs));
    const double* q = &scal[(size_t)s * NQ];
    Rs.status = S.status;
    Rs.iters = S.k;
    Rs.tr_x0 = q[Q_TR0];
    Rs.idem_err = q[Q_TR0] - q[Q_FRO0];
    Rs.e0 = q[Q_E0];
    for (int d = 0; d < D; ++d) {
      Rs.trace_x1h1[d] = q[Q_AL + d];
      Rs.tr_x1[d] = q[Q_TR1 + d];
      Rs.e1[d] = q[Q_E1 + d];
    }
    Rs.emin = R.emin[s];
    Rs.emax = R.emax[s];
    Rs.seconds = ms * 1e-3;
    Rs.union_flops = S.trip * b3 * (1 + 2 * D);
    Rs.nominal_flops = S.nominal * b3 * (1 + 2 * D);
    Rs.executed_flops = (s == 0) ? (double)R.exec_pairs * 2.0 * BP * BP * kst : 0.0;
    strncpy(Rs.branches, S.branches.c_str(), TC2_MAX_ITER + 3);
    Rs.ms_symbolic = ctx->ms_sym;
    Rs.ms_numeric = ctx->ms_num;
    for (int k = 0; k < 4; ++k) {
      Rs.useful_flops_kind[k] = (double)acc[(size_t)s * 4 + k] * b3;
      Rs.useful_flops += Rs.useful_flops_kind[k];
      Rs.ms_numeric_kind[k] = ctx->ms_num_kind[k];
      Rs.numeric_launches_kind[k] = ctx->launches_kind[k];
    }
    Rs.graph_updates = ctx->graph_updates;
    Rs.graph_captures = ctx->graph_captures;
    Rs.device_loop_updates = ctx->dl_updates;
    Rs.ms_compact = ctx->ms_cmp;
    Rs.numeric_launches = ctx->num_launches;
    for (int k = 0; k < 4; ++k) Rs.tile_shape[k] = ctx->kind_used[k] ? ctx->shape[k] : -1;
    Rs.ms_tune = ctx->ms_tune;
    Rs.screened_blocks = (s == 0) ? (int64_t)ctx->screened_total : 0;
    Rs.mlp_skipped_blocks = (s == 0) ? (int64_t)ctx->mlp_total : 0;
    Rs.mlp_updates = ctx->mlp_updates;
    Rs.kept_blocks = final_rp[ctx->sys[s].row0 + ctx->sys[s].nb] - final_rp[ctx->sys[s].row0];
    if (ctx->export_m) {
      HostBsr& x0 = ctx->out_x0[s];
      Rs.X0 = tc2_bsr{ctx->sys[s].nb, b, x0.row_ptr.data(), x0.col.data(), x0.val.data()};
      for (int d = 0; d < D; ++d) {
        HostBsr& x1 = ctx->out_x1[d][s];
        Rs.X1[d] = tc2_bsr{ctx->sys[s].nb, b, x1.row_ptr.data(), x1.col.data(), x1.val.data()};
      }
    }
    if (Rs.status < 0 && (worst >= 0 || Rs.status < worst)) worst = Rs.status;
    else if (worst >= 0 && Rs.status > worst) worst = Rs.status;
  }
  return worst;
}

// Whether the solve just begun can take its branch and stopping decisions
// on the device (device_loop): FP64 updates in captured graphs with nothing
// that needs the host between two updates, and a dense stage bound within
// TC2_DEVICE_LOOP_MAX_BYTES.  Sets ctx->dl_cap.
bool device_loop_eligible(tc2_ctx* ctx) {
  const RunState& R = ctx->run;
  if (ctx->device_loop <= 0 || !ctx->graph || !ctx->graph_ok || ctx->kernel != 0) return false;
  if (ctx->prec != P_FP64 || R.reduced || ctx->cur_prec != P_FP64 || ctx->skip_now == 2) return false;
  // a shape still to be tuned times its first update outside a graph
  if (!ctx->metrics_log.empty() || ctx->log_cap > 0 || (ctx->tune && !ctx->tuned[K_FP64]) ||
      ctx->count_useful || ctx->profile)
    return false;
  long long cap = 0;
  for (const SysInfo& si : ctx->sys) {
    if (!si.replay.empty()) return false;
    cap += (long long)si.nb * (si.nb + 1) / 2;
  }
  const double tile = (double)(1 + ctx->D) * BS * 8;
  if ((double)cap * tile > (double)TC2_DEVICE_LOOP_MAX_BYTES) return false;
  ctx->dl_cap = cap;
  return true;
}

// The updates of a solve with the decisions on the device: the update graphs
// (each ending with k_decide) are replayed device_loop times between two
// polls of the flag word, until no system is active.  The device records are
// then copied into the host state, which finish_solve reports.  *used is
// false when the solve is not eligible (the host loop runs it); a capture the
// runtime refuses hands the rest of the solve to the host loop.
tc2_status run_device_loop(tc2_ctx* ctx, bool* used) {
  RunState& R = ctx->run;
  hipStream_t st = R.st;
  const int nsys = ctx->nsys, D = ctx->D, nb = ctx->nb;
  *used = false;
  if (!device_loop_eligible(ctx)) return TC2_OK;
  const int c0 = ctx->cur;
  const size_t nnz = (size_t)ctx->nnz[c0], cap2 = (size_t)2 * ctx->dl_cap;
  const size_t tile = (size_t)(1 + D) * BS * 8;
  // the current pattern's buffers at the bound, contents kept: no update
  // replayed between two polls grows (and so frees) a buffer in use
  {
    hipError_t e = ctx->ci[c0].grow_keep(cap2 * 4, nnz * 4, st);
    if (e == hipSuccess) e = ctx->mask[c0].grow_keep(cap2, nnz, st);
    if (e == hipSuccess) e = ctx->xv[c0].grow_keep(cap2 * tile, nnz * tile, st);
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      return TC2_OK;
    }
    HIPCHK(e);
  }
  const size_t rec = (size_t)nsys * sizeof(DecideSys);
  const size_t off_rec = 64, off_act = off_rec + rec, off_br = off_act + (size_t)nsys * 4,
               off_nnz = (off_br + (size_t)nsys * 4 + 7) / 8 * 8, off_prm = off_nnz + 8;
  HIPCHK(ctx->dl_param.reserve((size_t)nsys * sizeof(DecideParam)));
  HIPCHK(ctx->dl_state.reserve(rec));
  HIPCHK(ctx->dl_word.reserve(sizeof(DecideWord)));
  HIPCHK(ctx->pin_dl.reserve(off_prm + (size_t)nsys * sizeof(DecideParam)));
  char* pin = (char*)ctx->pin_dl.p;
  DecideParam* prm = (DecideParam*)(pin + off_prm);
  int* act = (int*)(pin + off_act);
  int max_it = 0;
  for (int s = 0; s < nsys; ++s) {
    prm[s].n_occ = (double)ctx->sys[s].n_occ;
    prm[s].tol = ctx->sys[s].tol;
    prm[s].max_iter = ctx->sys[s].max_iter;
    prm[s].pad = 0;
    R.active[s] = R.ss[s].active ? 1 : 0;
    act[s] = R.active[s];
    max_it = std::max(max_it, ctx->sys[s].max_iter);
  }
  HIPCHK(hipMemcpyAsync(ctx->dl_param.p, prm, (size_t)nsys * sizeof(DecideParam),
                        hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ctx->active.p, act, (size_t)nsys * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(ctx->dl_state.p, 0, rec, st));
  HIPCHK(hipMemsetAsync(ctx->dl_word.p, 0, sizeof(DecideWord), st));
  {
    // the first update's branch, from the initial scalars
    DecideArgs da{};
    da.nsys = nsys;
    da.D = D;
    da.init = 1;
    da.scal = ctx->scal.as<double>();
    da.param = ctx->dl_param.as<DecideParam>();
    da.state = ctx->dl_state.as<DecideSys>();
    da.active = ctx->active.as<int>();
    da.branch = ctx->branch.as<int>();
    da.word = ctx->dl_word.as<DecideWord>();
    launch_decide(st, da);
    HIPCHK(hipGetLastError());
  }
  *used = true;
  ctx->h_active = R.active;
  DecideWord w{};
  auto poll = [&]() -> tc2_status {
    HIPCHK(hipMemcpyAsync(pin, ctx->dl_word.p, sizeof(DecideWord), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    memcpy(&w, pin, sizeof(DecideWord));
    return TC2_OK;
  };
  // batches of device_loop updates; within the update count of the last
  // device-loop solve of this context, a batch ends there, and past it the
  // flag word is polled after every update, so that a solve like the last
  // one launches no update after its last stop.  Without such a solve,
  // batches of at most 4 bound the updates launched after the last stop.
  const int expect = ctx->dl_last;
  bool handed_over = false;
  int launched = 0;
  for (;;) {
    int batch = ctx->device_loop;
    if (expect > 0) batch = launched < expect ? std::min(batch, expect - launched) : 1;
    else batch = std::min(batch, 4);
    for (int k = 0; k < batch && launched < max_it; ++k, ++launched) {
      const int g = step_graph(ctx, st, R.scal, R.exec_pairs, true);
      if (g == 1) {
        ctx->graph_ok = false;
        handed_over = true;
        break;
      }
      if (g != TC2_OK) return (tc2_status)g;
    }
    if (tc2_status r = poll(); r != TC2_OK) return r;
    if (w.overflow) return TC2_ENOMEM;
    if (handed_over || !w.any_active || launched >= max_it) break;
  }
  // the device records into the host state
  HIPCHK(hipMemcpyAsync(pin + off_rec, ctx->dl_state.p, rec, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(pin + off_act, ctx->active.p, (size_t)nsys * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(pin + off_br, ctx->branch.p, (size_t)nsys * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(pin + off_nnz, ctx->rp[ctx->cur].as<int>() + nb, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const DecideSys* recs = (const DecideSys*)(pin + off_rec);
  const int* br = (const int*)(pin + off_br);
  for (int s = 0; s < nsys; ++s) {
    SysState& S = R.ss[s];
    if (!S.active) continue;  // trivial or degenerate: never iterated
    const DecideSys& d = recs[s];
    S.k = d.k;
    S.status = (tc2_status)d.status;
    S.active = act[s] != 0;
    S.branches.assign(d.branches, (size_t)d.k);
    S.trip = d.trip;
    S.nominal = (double)d.nominal;
    std::copy(d.prev, d.prev + 1 + 2 * D, S.prev);
    // the last two iotas, in order: enough for the stall guard's k - 2
    S.iota.clear();
    if (d.k >= 2) S.iota.push_back(d.iota2);
    if (d.k >= 1) S.iota.push_back(d.iota1);
    R.active[s] = act[s];
    R.branch[s] = br[s];
  }
  ctx->h_active = R.active;
  int nnz_now = 0;
  memcpy(&nnz_now, pin + off_nnz, 4);
  ctx->nnz[ctx->cur] = nnz_now;
  ctx->kept_prev = ctx->kept_prev2 = ctx->kept_prev3 = 0;
  R.updates += w.updates;
  R.exec_pairs += w.exec_pairs;
  ctx->screened_total += w.screened[0];
  ctx->mlp_total += w.screened[1];
  ctx->graph_updates += w.updates;
  ctx->dl_updates += w.updates;
  if (!handed_over) ctx->dl_last = w.updates;
  return TC2_OK;
}

tc2_status run_impl(tc2_ctx* ctx, void* stream, tc2_result* res) {
  if (!ctx || !res) return TC2_EINVAL;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = stream ? (hipStream_t)stream : ctx->own;
  tc2_status r = begin_solve(ctx, st);
  if (r != TC2_OK) return r;
  if (ctx->device_loop > 0) {
    bool used = false;
    if ((r = run_device_loop(ctx, &used)) != TC2_OK) {
      ctx->run.open = false;
      return r;
    }
  }
  for (;;) {
    bool done = false;
    if ((r = advance_one(ctx, &done)) != TC2_OK) {
      ctx->run.open = false;
      return r;
    }
    if (done) break;
  }
  return finish_solve(ctx, res);
}

tc2_status advance_impl(tc2_ctx* ctx, void* stream, int32_t max_updates, tc2_progress* prog,
                        tc2_result* res) {
  if (!ctx || !prog || !res || max_updates < 0) return TC2_EINVAL;
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = stream ? (hipStream_t)stream : ctx->own;
  memset(prog, 0, sizeof(*prog));
  RunState& R = ctx->run;
  tc2_status worst = TC2_OK;
  const double b3 = 2.0 * ctx->b * ctx->b * ctx->b;
  const double kst = (double)((ctx->b + 3) / 4) * 4;
  auto useful_total = [&](double* out) -> tc2_status {
    std::vector<unsigned long long> acc;
    if (tc2_status s0 = read_useful(ctx, st, acc); s0 != TC2_OK) return s0;
    double t = 0.0;
    for (unsigned long long v : acc) t += (double)v;
    *out = t * b3;
    return TC2_OK;
  };
  double u0 = 0.0;
  unsigned long long p0 = 0;
  if (R.open) {
    R.st = st;
    if (tc2_status s0 = useful_total(&u0); s0 != TC2_OK) return s0;
    p0 = R.exec_pairs;
  }
  auto bank = [&]() -> tc2_status {  // add the open solve's work since u0/p0 to prog
    double u = 0.0;
    if (tc2_status s0 = useful_total(&u); s0 != TC2_OK) return s0;
    prog->useful_flops += u - u0;
    prog->executed_flops += (double)(R.exec_pairs - p0) * 2.0 * BP * BP * kst;
    return TC2_OK;
  };
  tc2_status r;
  while (prog->updates < max_updates) {
    if (!R.open) {
      if ((r = begin_solve(ctx, st)) != TC2_OK) return r;
      u0 = 0.0;
      p0 = 0;
    }
    bool done = false;
    if ((r = advance_one(ctx, &done)) != TC2_OK) {
      R.open = false;
      return r;
    }
    if (done) {
      if ((r = bank()) != TC2_OK) return r;
      worst = finish_solve(ctx, res);
      if (worst < 0) return worst;
      prog->solves_completed++;
      continue;
    }
    prog->updates++;
  }
  if (R.open && solve_finished(ctx)) {
    if ((r = bank()) != TC2_OK) return r;
    worst = finish_solve(ctx, res);
    if (worst < 0) return worst;
    prog->solves_completed++;
  } else if (R.open) {
    if ((r = bank()) != TC2_OK) return r;
  }
  prog->solve_open = R.open ? 1 : 0;
  return worst;
}

}  // namespace

extern "C" tc2_status tc2_run(tc2_ctx* ctx, void* hip_stream, tc2_result* res) {
  try {
    return run_impl(ctx, hip_stream, res);
  } catch (const std::bad_alloc&) {
    return TC2_ENOMEM;
  } catch (...) {
    return TC2_EDEVICE;
  }
}

extern "C" tc2_status tc2_advance(tc2_ctx* ctx, void* hip_stream, int32_t max_updates,
                                  tc2_progress* prog, tc2_result* res) {
  try {
    return advance_impl(ctx, hip_stream, max_updates, prog, res);
  } catch (const std::bad_alloc&) {
    return TC2_ENOMEM;
  } catch (...) {
    return TC2_EDEVICE;
  }
}

extern "C" int64_t tc2_log_copy(tc2_ctx* ctx, float* x, float* y, float* z, int64_t cap) {
  if (!ctx || cap < 0 || (cap > 0 && (!x || !y))) return TC2_EINVAL;
  if (ctx->log_cap <= 0) return 0;
  if (hipSetDevice(ctx->device) != hipSuccess) return TC2_EDEVICE;
  const long long n = std::min<long long>(ctx->log_n, cap);
  if (n == 0) return 0;
  if (hipMemcpy(x, ctx->log_x.p, (size_t)n * MLP_NF * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(y, ctx->log_y.p, (size_t)n * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      (z && hipMemcpy(z, ctx->log_z.p, (size_t)n * 4, hipMemcpyDeviceToHost) != hipSuccess))
    return TC2_EDEVICE;
  return n;
}
