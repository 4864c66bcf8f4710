// C ABI of libpriest.so: validation, problem construction and launch
// sequencing.  All arithmetic of the planner runs in the kernels of
// project.hip (projection), cem.hip (selection / refit / Cholesky) and
// kkt.hip (one-time FP64 KKT factorisation); this file builds the Bernstein
// basis and Q on the host in FP64 and orders the launches.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "priest_internal.h"

using namespace priest;

// Workspace of priest_plan_static: one array per GPU, held until the
// process ends.  Its size covers the largest single-problem plan
// (n_samples 8192, D = 48 needs 1.57 MiB).  In host code `scratch` is only a
// stand-in for the device symbol: kernels and copies take the per-device
// address that hipGetSymbolAddress returns (static_scratch_ptr).
constexpr size_t kStaticWorkspaceBytes = size_t(2) << 20;
static_assert(kStaticWorkspaceBytes == PRIEST_STATIC_WORKSPACE_BYTES, "header and library disagree");
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(PRIEST_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Bernstein polynomial B_{i,n}(tau); zero outside 0 <= i <= n.
double bern(int i, int n, double tau) {
  if (i < 0 || i > n || n < 0) return 0.0;
  return binom(n, i) * std::pow(tau, i) * std::pow(1.0 - tau, n - i);
}

struct GraphEntry {
  std::vector<uint64_t> key;
  hipGraphExec_t exec = nullptr;
};

size_t align256(size_t n) { return (n + 255) & ~static_cast<size_t>(255); }

struct TuneEntry {
  int N, P, mode, bf16;
  TileCfg cfg;
  std::vector<float> ms;
};

// PRIEST_AUTOTUNE=0 in the environment turns the autotuner off.
bool autotune_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("PRIEST_AUTOTUNE");
    return !(e && e[0] == '0');
  }();
  return on;
}

bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return true;
  return st != hipStreamCaptureStatusNone;
}

constexpr int kMaxDevices = 64;
struct StaticScratch {
  std::mutex mu;
  void* ptr[kMaxDevices] = {};
  hipError_t err[kMaxDevices] = {};
  bool looked_up[kMaxDevices] = {};
};
StaticScratch& static_scratch() {
  static StaticScratch* s = new StaticScratch();  // lives until exit
  return *s;
}

// Looks up this device's copy of `scratch` once; `dev` must be current.
void static_scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  StaticScratch& ss = static_scratch();
  std::lock_guard<std::mutex> lk(ss.mu);
  if (ss.looked_up[dev]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  ss.looked_up[dev] = true;
  ss.err[dev] = e;
  ss.ptr[dev] = (e == hipSuccess) ? ptr : nullptr;
}

// This device's address of `scratch` (null if the lookup failed or never ran).
void* static_scratch_ptr(int dev, hipError_t* err) {
  *err = hipErrorInvalidDevice;
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  StaticScratch& ss = static_scratch();
  std::lock_guard<std::mutex> lk(ss.mu);
  if (!ss.looked_up[dev]) return nullptr;
  *err = ss.err[dev];
  return ss.ptr[dev];
}

}  // namespace

struct priest_problem {
  priest_problem_desc desc{};
  int D = 0, E = 0;
  int rowsel[6] = {0, 0, 0, 0, 0, 0};
  float* dW = nullptr;     // [K][3][nv]
  float* dM11 = nullptr;   // [nv][nv]
  float* dPi = nullptr;    // [nv][nv]
  float* dM12 = nullptr;   // [nv][6]
  double* d64 = nullptr;   // scratch for the FP64 factorisation
  std::vector<float> hW, hM11, hPi, hM12;
  float bscale[3] = {0.0f, 0.0f, 0.0f};  // ProjArgs::bscale
  std::mutex graph_mu;
  std::vector<GraphEntry> graphs;
  int device = 0;
  size_t lds_limit = 0;
  // projection tile shape: autotuner results per (N, n_problems, mode, bf16)
  std::mutex tune_mu;
  std::vector<TuneEntry> tuned;
  bool forced = false;
  TileCfg force_cfg{4, 1, 0};
  TileCfg last_cfg{4, 1, 0};
  int last_tuned = 0;
};

namespace {

int32_t validate_desc(const priest_problem_desc* d) {
  if (!d) return fail(PRIEST_ERR_INVALID, "desc is NULL");
  if (d->dims != 2 && d->dims != 3) return fail(PRIEST_ERR_INVALID, "dims must be 2 or 3");
  if (d->n_coeff < 2 || d->n_coeff > PRIEST_MAX_COEFF)
    return fail(PRIEST_ERR_INVALID, "n_coeff must be in [2, %d]", PRIEST_MAX_COEFF);
  if (d->n_steps < 2 || d->n_steps > PRIEST_MAX_STEPS)
    return fail(PRIEST_ERR_INVALID, "n_steps must be in [2, %d]", PRIEST_MAX_STEPS);
  if (d->n_obs < 0 || d->n_obs > PRIEST_MAX_OBS)
    return fail(PRIEST_ERR_INVALID, "n_obs must be in [0, %d]", PRIEST_MAX_OBS);
  if (!(std::isfinite(d->horizon) && d->horizon > 0))
    return fail(PRIEST_ERR_INVALID, "horizon must be finite and > 0");
  if (!(std::isfinite(d->rho) && d->rho >= 0)) return fail(PRIEST_ERR_INVALID, "rho must be finite and >= 0");
  if (!(d->v_max > 0) || std::isnan(d->v_max)) return fail(PRIEST_ERR_INVALID, "v_max must be > 0");
  if (!(d->a_max > 0) || std::isnan(d->a_max)) return fail(PRIEST_ERR_INVALID, "a_max must be > 0");
  if (d->bc_mask & ~63u) return fail(PRIEST_ERR_INVALID, "bc_mask has unknown bits");
  if (d->precision != PRIEST_FP32 && d->precision != PRIEST_BF16_MIXED)
    return fail(PRIEST_ERR_INVALID, "unknown precision");
  if (d->n_refine_fp32 < 0) return fail(PRIEST_ERR_INVALID, "n_refine_fp32 must be >= 0");
  if (d->use_bounds != 0 && d->use_bounds != 1) return fail(PRIEST_ERR_INVALID, "use_bounds must be 0 or 1");
  if (d->obs_model != PRIEST_OBS_VELOCITY && d->obs_model != PRIEST_OBS_PATH)
    return fail(PRIEST_ERR_INVALID, "unknown obstacle model");
  if (d->reserved2 != 0) return fail(PRIEST_ERR_INVALID, "reserved2 must be 0");
  if (d->use_bounds)
    for (int x = 0; x < d->dims; ++x)
      if (std::isnan(d->s_min[x]) || std::isnan(d->s_max[x]) || !(d->s_min[x] <= d->s_max[x]))
        return fail(PRIEST_ERR_INVALID, "workspace bounds of axis %d need s_min <= s_max", x);
  int E = 0;
  for (int i = 0; i < 6; ++i) E += (d->bc_mask >> i) & 1;
  if (E > d->n_coeff)
    return fail(PRIEST_ERR_SINGULAR, "%d boundary rows exceed %d coefficients per axis", E, d->n_coeff);
  return PRIEST_OK;
}

int32_t validate_cem(const priest_cem_params* c, int dims) {
  if (!c) return fail(PRIEST_ERR_INVALID, "cem params are NULL");
  const priest_cost& k = c->cost;
  if (k.reserved != 0) return fail(PRIEST_ERR_INVALID, "cost.reserved must be 0");
  if (k.kind != PRIEST_COST_SMOOTH && k.kind != PRIEST_COST_WEIGHTED)
    return fail(PRIEST_ERR_INVALID, "unknown cost kind");
  if (k.kind == PRIEST_COST_WEIGHTED) {
    const float w[4] = {k.w_acc, k.w_curv, k.w_path, k.w_steer};
    for (float x : w)
      if (!(std::isfinite(x) && x >= 0.0f)) return fail(PRIEST_ERR_INVALID, "cost weights must be finite and >= 0");
    if (!(std::isfinite(k.eps) && k.eps > 0.0f)) return fail(PRIEST_ERR_INVALID, "cost.eps must be > 0");
    if (k.w_steer > 0.0f && dims != 2) return fail(PRIEST_ERR_INVALID, "the steering cost is 2D only");
    if (k.w_steer > 0.0f && !(std::isfinite(k.wheelbase) && k.wheelbase > 0.0f))
      return fail(PRIEST_ERR_INVALID, "cost.wheelbase must be > 0");
  }
  if (c->n_samples < 1 || c->n_samples > 8192)
    return fail(PRIEST_ERR_INVALID, "n_samples must be in [1, 8192] for planning");
  if (c->n_cem < 1) return fail(PRIEST_ERR_INVALID, "n_cem must be >= 1");
  if (c->n_proj_iters < 0) return fail(PRIEST_ERR_INVALID, "n_proj_iters must be >= 0");
  if (c->n_proj < 1 || c->n_proj > c->n_samples)
    return fail(PRIEST_ERR_INVALID, "n_proj must be in [1, n_samples]");
  if (c->n_elite < 1 || c->n_elite > c->n_proj)
    return fail(PRIEST_ERR_INVALID, "n_elite must be in [1, n_proj]");
  if (!(std::isfinite(c->sigma) && c->sigma >= 0 && c->sigma <= 1))
    return fail(PRIEST_ERR_INVALID, "sigma must be in [0, 1]");
  if (!(std::isfinite(c->gamma) && c->gamma > 0)) return fail(PRIEST_ERR_INVALID, "gamma must be > 0");
  if (!(std::isfinite(c->cov_jitter) && c->cov_jitter >= 0))
    return fail(PRIEST_ERR_INVALID, "cov_jitter must be finite and >= 0");
  if (c->update != PRIEST_UPDATE_MPPI && c->update != PRIEST_UPDATE_CMA)
    return fail(PRIEST_ERR_INVALID, "unknown update rule");
  if (c->reserved_f != 0.0f) return fail(PRIEST_ERR_INVALID, "reserved_f must be 0");
  return PRIEST_OK;
}

ProjArgs base_args(const priest_problem* p) {
  ProjArgs a{};
  const auto& d = p->desc;
  a.dims = d.dims;
  a.nv = d.n_coeff;
  a.K = d.n_steps;
  a.M = d.n_obs;
  a.rho = static_cast<float>(d.rho);
  a.dt = static_cast<float>(d.horizon / (d.n_steps - 1));
  a.vmax = static_cast<float>(d.v_max);
  a.amax = static_cast<float>(d.a_max);
  a.traj = d.obs_model == PRIEST_OBS_PATH ? 1 : 0;
  a.box.on = d.use_bounds;
  for (int x = 0; x < 3; ++x) {
    a.box.lo[x] = d.use_bounds ? static_cast<float>(d.s_min[x]) : -INFINITY;
    a.box.hi[x] = d.use_bounds ? static_cast<float>(d.s_max[x]) : INFINITY;
  }
  a.bf16_iters = 0;
  a.W = p->dW;
  a.M11 = p->dM11;
  a.Pi = p->dPi;
  a.M12 = p->dM12;
  for (int x = 0; x < 3; ++x) a.bscale[x] = p->bscale[x];
  return a;
}

// Mixed precision: BF16 MFMA operands for all but the last n_refine_fp32
// projection iterations.
int bf16_iters(const priest_problem* p, int n_iter) {
  if (p->desc.precision != PRIEST_BF16_MIXED) return 0;
  const int n = n_iter - p->desc.n_refine_fp32;
  return n > 0 ? n : 0;
}

int32_t check_lds(const priest_problem* p, const ProjArgs& a) {
  const size_t need = project_lds_bytes(a);
  if (need > p->lds_limit)
    return fail(PRIEST_ERR_INVALID, "problem shape needs %zu B of LDS per block (limit %zu)", need,
                p->lds_limit);
  return PRIEST_OK;
}

// Per problem: projected samples, residuals, costs, Cholesky factor, CMA
// evolution path, status, the obstacle records of a projection launch whose
// waves draw (problem, group) pairs (3 float4 per obstacle) and that
// launch's counter (used in problem 0's block only).
struct PlanLayout {
  size_t xb, resid, c1, L, pc, status, grec, gq, per_problem;
};

PlanLayout plan_layout(int D, int N, int M) {
  PlanLayout l{};
  size_t o = 0;
  l.xb = o;     o += align256(sizeof(float) * static_cast<size_t>(N) * D);
  l.resid = o;  o += align256(sizeof(float) * N);
  l.c1 = o;     o += align256(sizeof(float) * N);
  l.L = o;      o += align256(sizeof(float) * D * D);
  l.pc = o;     o += align256(sizeof(float) * D);
  l.status = o; o += align256(sizeof(int32_t));
  l.grec = o;   o += align256(sizeof(float) * 12 * static_cast<size_t>(M));
  l.gq = o;     o += align256(sizeof(int32_t));
  l.per_problem = o;
  return l;
}

// Profiling hook: event pairs around projection launches (see priest.h).
struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending, pool;
  bool count_pairs = false;
  unsigned long long* pairs_dev = nullptr;  // device counter, kept until exit
  int pairs_device = -1;
};
Profiler& profiler() {
  static Profiler* p = new Profiler();  // lives until exit
  return *p;
}

// launch_project, timed by events when profiling is on and the stream is not
// being captured: the launch itself stamps the kernel's start and end into
// them, so profiling adds no commands to the stream between kernels.
hipError_t launch_project_timed(const ProjArgs& a, int P, hipStream_t s) {
  Profiler& pr = profiler();
  std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
  ProjArgs b = a;
  {
    std::lock_guard<std::mutex> lk(pr.mu);
    if (pr.count_pairs && !stream_capturing(s)) b.pair_count = pr.pairs_dev;
    if (pr.on && !stream_capturing(s)) {
      if (!pr.pool.empty()) {
        ev = pr.pool.back();
        pr.pool.pop_back();
      } else {
        hipError_t e = hipEventCreate(&ev.first);
        if (e == hipSuccess) e = hipEventCreate(&ev.second);
        if (e != hipSuccess) return e;
      }
    }
  }
  const hipError_t e = launch_project(b, P, s, ev.first, ev.second);
  if (ev.first) {
    std::lock_guard<std::mutex> lk(pr.mu);
    pr.pending.push_back(ev);
  }
  return e;
}

struct PlanArgs {
  ProjArgs a;
  CemArgs ca;
};

// Launch arguments of the plan loop for n_problems problems of shape p, with
// the default tile shape.
PlanArgs plan_args(priest_problem* p, int32_t P, const float* bc, const float* obs,
                   const priest_cem_params* c, float* mu, float* cov, uint64_t seed,
                   uint32_t stream_base, const float* noise, const priest_plan_out* out, char* ws) {
  (void)P;
  const int D = p->D, N = c->n_samples;
  const PlanLayout pl = plan_layout(D, N, p->desc.n_obs);
  // per-problem workspace blocks are laid out [problem][...]: strides in floats
  const int64_t wstride = static_cast<int64_t>(pl.per_problem / sizeof(float));
  float* wxb = reinterpret_cast<float*>(ws + pl.xb);
  float* wr = reinterpret_cast<float*>(ws + pl.resid);
  float* wc = reinterpret_cast<float*>(ws + pl.c1);
  float* wL = reinterpret_cast<float*>(ws + pl.L);
  PlanArgs pa{};
  CemArgs& ca = pa.ca;
  ca.D = D;
  ca.N = N;
  ca.n_proj = c->n_proj;
  ca.n_elite = c->n_elite;
  ca.sigma = c->sigma;
  ca.gamma = c->gamma;
  ca.cov_jitter = c->cov_jitter;
  ca.xb = wxb;
  ca.xb_stride = wstride;
  ca.resid = wr;
  ca.c1 = wc;
  ca.n_stride = wstride;
  ca.mu = mu;
  ca.mu_stride = D;
  ca.cov = cov;
  ca.cov_stride = static_cast<int64_t>(D) * D;
  ca.L = wL;
  ca.L_stride = wstride;
  ca.best_xi = out->best_xi;
  ca.best_stride = D;
  ca.best_cost = out->best_cost;
  ca.elite_idx = out->elite_idx;
  ca.proj_idx = out->proj_idx;
  ca.status = out->status;
  ca.chol_only = 0;
  ca.rule = c->update;
  ca.first = 1;
  ca.pc = reinterpret_cast<float*>(ws + pl.pc);
  ca.pc_stride = wstride;

  ProjArgs& a = pa.a;
  a = base_args(p);
  a.N = N;
  a.n_iter = c->n_proj_iters;
  a.bf16_iters = bf16_iters(p, a.n_iter);
  a.mode = noise ? kFromNoise : kFromPhilox;
  a.seed = seed;
  a.stream_base = stream_base;
  a.bc = bc;
  a.bc_stride = static_cast<int64_t>(a.dims) * 6;
  a.obs = obs;
  a.obs_stride = static_cast<int64_t>(a.M) * (a.traj ? a.K * a.dims + 2 : 8);
  a.mu = mu;
  a.mu_stride = D;
  a.L = wL;
  a.L_stride = wstride;
  a.noise = noise;
  a.noise_stride = static_cast<int64_t>(c->n_cem) * N * D;
  a.xi_out = wxb;
  a.xi_out_stride = wstride;
  a.resid = wr;
  a.c1 = wc;
  a.n_stride = wstride;
  a.xi_src_stride = static_cast<int64_t>(N) * D;
  a.grec = reinterpret_cast<float*>(ws + pl.grec);
  a.grec_stride = wstride;
  a.gq = reinterpret_cast<int32_t*>(ws + pl.gq);
  a.cost = CostArgs{c->cost.kind, c->cost.w_acc, c->cost.w_curv, c->cost.w_path,
                    c->cost.w_steer, c->cost.wheelbase, c->cost.eps};
  apply_tiling(a, tile_candidates(a.dims, a.K)[0]);
  return pa;
}

// Enqueues n_cem CEM iterations for n_problems problems.  instrument: the
// projection launches may carry the profiler's events and pair counter
// (false: plain launches that create nothing).
int32_t enqueue_plan(int32_t P, PlanArgs pa, const priest_cem_params* c, const float* noise,
                     const priest_plan_out* out, hipStream_t s, bool instrument = true) {
  ProjArgs a = pa.a;
  CemArgs ca = pa.ca;
  const int D = ca.D, N = ca.N;
  ca.chol_only = 1;  // (also sets every status word to PRIEST_OK)
  HIP_TRY(launch_cem(ca, P, s));
  ca.chol_only = 0;
  for (int l = 0; l < c->n_cem; ++l) {
    a.iter = l;
    a.noise = noise ? noise + static_cast<int64_t>(l) * N * D : nullptr;
    const bool last = (l == c->n_cem - 1);
    a.xi_src = last ? out->xi : nullptr;
    a.resid2 = last ? out->resid : nullptr;
    a.c12 = last ? out->c1 : nullptr;
    a.xi_out2 = last ? out->xi_bar : nullptr;
    if (instrument) HIP_TRY(launch_project_timed(a, P, s));
    else HIP_TRY(launch_project(a, P, s));
    ca.first = (l == 0) ? 1 : 0;
    // the selection outputs describe the last iteration; without the ordered
    // constraint-elite set the refit selects without sorting
    ca.elite_idx = last ? pa.ca.elite_idx : nullptr;
    ca.proj_idx = last ? pa.ca.proj_idx : nullptr;
    HIP_TRY(launch_cem(ca, P, s));
  }
  return PRIEST_OK;
}

bool tiling_cached(priest_problem* p, const ProjArgs& a, int P) {
  std::lock_guard<std::mutex> lk(p->tune_mu);
  if (p->forced) return true;
  const int bf = a.bf16_iters > 0;
  for (const TuneEntry& e : p->tuned)
    if (e.N == a.N && e.P == P && e.mode == a.mode && e.bf16 == bf) return true;
  return false;
}

// Tile shape for a projection of `a` over P problems: the forced shape, a
// cached autotuner result, or, when `trial` is given and tuning is possible,
// the fastest candidate measured on `trial` (which writes only scratch).
// Otherwise the default shape.
int32_t resolve_tiling(priest_problem* p, const ProjArgs& a, int P, hipStream_t s,
                       const ProjArgs* trial, TileCfg* out) {
  std::lock_guard<std::mutex> lk(p->tune_mu);
  const std::vector<TileCfg> cands = tile_candidates(a.dims, a.K);
  p->last_tuned = 0;
  if (p->forced) {
    *out = p->force_cfg;
    p->last_cfg = *out;
    return PRIEST_OK;
  }
  const int bf = a.bf16_iters > 0;
  for (const TuneEntry& e : p->tuned)
    if (e.N == a.N && e.P == P && e.mode == a.mode && e.bf16 == bf) {
      *out = e.cfg;
      p->last_cfg = *out;
      p->last_tuned = 1;
      return PRIEST_OK;
    }
  *out = cands[0];
  p->last_cfg = *out;
  if (!trial || !autotune_enabled() || stream_capturing(s)) return PRIEST_OK;
  std::vector<float> ms;
  HIP_TRY(time_tilings(*trial, P, p->lds_limit, s, cands, &ms));
  const int best = pick_tiling(ms);
  p->tuned.push_back(TuneEntry{a.N, P, a.mode, bf, cands[best], ms});
  *out = cands[best];
  p->last_cfg = *out;
  p->last_tuned = 1;
  return PRIEST_OK;
}

ProjArgs trial_args(const ProjArgs& a);

// Picks (and applies) the projection tile shape of a plan loop: before any
// capture, since timing synchronises the stream; the trial needs the first
// draw's Cholesky factor, which the loop itself recomputes.
int32_t plan_tiling(priest_problem* p, PlanArgs& pa, int32_t P, hipStream_t s, TileCfg* cfg) {
  int32_t st = check_lds(p, pa.a);
  if (st != PRIEST_OK) return st;
  if (pa.a.n_iter > 0 && autotune_enabled() && !tiling_cached(p, pa.a, P) && !stream_capturing(s)) {
    CemArgs chol = pa.ca;
    chol.chol_only = 1;
    chol.status = nullptr;
    HIP_TRY(launch_cem(chol, P, s));
    const ProjArgs t = trial_args(pa.a);
    st = resolve_tiling(p, pa.a, P, s, &t, cfg);
  } else {
    st = resolve_tiling(p, pa.a, P, s, nullptr, cfg);
  }
  if (st != PRIEST_OK) return st;
  apply_tiling(pa.a, *cfg);
  return check_lds(p, pa.a);
}

// A shortened copy of `a` for timing: at most 8 iterations (keeping BF16
// iterations if `a` has any, so that the same kernel instance runs).
ProjArgs trial_args(const ProjArgs& a) {
  ProjArgs t = a;
  t.n_iter = std::min(a.n_iter, 8);
  t.bf16_iters = a.bf16_iters > 0 ? std::max(1, std::min(a.bf16_iters, t.n_iter)) : 0;
  t.xi_src = nullptr;
  t.resid2 = nullptr;
  t.c12 = nullptr;
  t.xi_out2 = nullptr;
  return t;
}

}  // namespace

// Helpers shared with the serving runtime (serve.hip).
namespace priest {
int32_t set_error(int32_t code, const char* msg) { return fail(code, "%s", msg); }
ProjArgs problem_args(const priest_problem* p) { return base_args(p); }
int problem_bf16_iters(const priest_problem* p, int n_iter) { return bf16_iters(p, n_iter); }
int32_t problem_check_lds(const priest_problem* p, const ProjArgs& a) { return check_lds(p, a); }
}  // namespace priest

extern "C" {

const char* priest_last_error(void) { return g_err.c_str(); }

int32_t priest_version(void) { return 1; }

int32_t priest_init_problem(const priest_problem_desc* desc, void* stream, priest_problem** out) {
  if (!out) return fail(PRIEST_ERR_INVALID, "out is NULL");
  *out = nullptr;
  const int32_t st = validate_desc(desc);
  if (st != PRIEST_OK) return st;
  const auto& d = *desc;
  const int nv = d.n_coeff, K = d.n_steps, n = nv - 1;
  const double T = d.horizon;
  std::unique_ptr<priest_problem> p(new priest_problem());
  p->desc = d;
  p->D = d.dims * nv;
  int E = 0;
  for (int i = 0; i < 6; ++i)
    if ((d.bc_mask >> i) & 1) p->rowsel[E++] = i;
  p->E = E;
  HIP_TRY(hipGetDevice(&p->device));
  static_scratch_setup(p->device);  // priest_plan_static's workspace on this device
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, p->device));
  p->lds_limit = prop.sharedMemPerBlock;
  if (d.obs_model == PRIEST_OBS_PATH) {  // obstacle paths run the default shape only
    p->forced = true;
    p->force_cfg = TileCfg{4, 1, 0};
  }

  // Bernstein rows (FP64): P, Pdot, Pddot at t_k = k T/(K-1)
  std::vector<double> P(K * nv), Pd(K * nv), Pdd(K * nv);
  for (int k = 0; k < K; ++k) {
    const double tau = static_cast<double>(k) / (K - 1);
    for (int i = 0; i < nv; ++i) {
      P[k * nv + i] = bern(i, n, tau);
      Pd[k * nv + i] = n * (bern(i - 1, n - 1, tau) - bern(i, n - 1, tau)) / T;
      Pdd[k * nv + i] = (n >= 2) ? n * (n - 1) *
                                       (bern(i - 2, n - 2, tau) - 2.0 * bern(i - 1, n - 2, tau) +
                                        bern(i, n - 2, tau)) / (T * T)
                                 : 0.0;
    }
  }
  // Q = I + rho (n_pos P^T P + Pdot^T Pdot + Pddot^T Pddot): n_pos counts the
  // position blocks of F, one per obstacle plus -P and P of the bounds
  const double n_pos = d.n_obs + (d.use_bounds ? 2.0 : 0.0);
  std::vector<double> Q(nv * nv, 0.0);
  for (int i = 0; i < nv; ++i)
    for (int j = 0; j < nv; ++j) {
      double s = 0.0;
      for (int k = 0; k < K; ++k)
        s += n_pos * P[k * nv + i] * P[k * nv + j] + Pd[k * nv + i] * Pd[k * nv + j] +
             Pdd[k * nv + i] * Pdd[k * nv + j];
      Q[i * nv + j] = (i == j ? 1.0 : 0.0) + d.rho * s;
    }
  // boundary block A_ax: rows P_0, Pdot_0, Pddot_0, P_-1, Pdot_-1, Pddot_-1
  std::vector<double> A(std::max(E, 1) * nv, 0.0);
  for (int r = 0; r < E; ++r) {
    const int which = p->rowsel[r];
    const std::vector<double>& src = (which % 3 == 0) ? P : (which % 3 == 1) ? Pd : Pdd;
    const int k = (which < 3) ? 0 : K - 1;
    for (int i = 0; i < nv; ++i) A[r * nv + i] = src[k * nv + i];
  }
  p->hW.resize(static_cast<size_t>(K) * 3 * nv);
  for (int k = 0; k < K; ++k)
    for (int i = 0; i < nv; ++i) {
      p->hW[(k * 3 + 0) * nv + i] = static_cast<float>(P[k * nv + i]);
      p->hW[(k * 3 + 1) * nv + i] = static_cast<float>(Pd[k * nv + i]);
      p->hW[(k * 3 + 2) * nv + i] = static_cast<float>(Pdd[k * nv + i]);
    }
  // Displacement budgets of the whole-horizon shape: a change Delta of the
  // coefficients moves row type d of step t by |W_t,d Delta| <= S_d max|Delta|
  // per axis (S_d = max_t sum_j |W_t,d,j| over the FP32 rows, rounded up), so
  // a slack of sigma (per axis for p, Euclidean for v and a) lasts while the
  // summed max|Delta| stays below sigma / S_d (p) or sigma / (sqrt(dims) S_d).
  for (int x = 0; x < 3; ++x) {
    double sm = 0.0;
    for (int k = 0; k < K; ++k) {
      double r = 0.0;
      for (int i = 0; i < nv; ++i) r += std::fabs(static_cast<double>(p->hW[(k * 3 + x) * nv + i]));
      sm = std::max(sm, r);
    }
    sm *= 1.0 + 1e-6;
    if (x > 0) sm *= std::sqrt(static_cast<double>(d.dims));
    p->bscale[x] = sm > 0.0 ? static_cast<float>((1.0 - 1e-6) / sm) : INFINITY;
  }

  hipStream_t s = static_cast<hipStream_t>(stream);
  double *dQ = nullptr, *dA = nullptr;
  int* dsel = nullptr;
  int* dflag = nullptr;
  auto cleanup = [&]() {
    if (dQ) (void)hipFree(dQ);
    if (dA) (void)hipFree(dA);
    if (dsel) (void)hipFree(dsel);
    if (dflag) (void)hipFree(dflag);
  };
  auto alloc = [&](void** ptr, size_t bytes) -> bool { return hipMalloc(ptr, bytes) == hipSuccess; };
  if (!alloc(reinterpret_cast<void**>(&p->dW), sizeof(float) * p->hW.size()) ||
      !alloc(reinterpret_cast<void**>(&p->dM11), sizeof(float) * nv * nv) ||
      !alloc(reinterpret_cast<void**>(&p->dPi), sizeof(float) * nv * nv) ||
      !alloc(reinterpret_cast<void**>(&p->dM12), sizeof(float) * nv * 6) ||
      !alloc(reinterpret_cast<void**>(&p->d64), sizeof(double) * (2 * nv * nv + nv * 6)) ||
      !alloc(reinterpret_cast<void**>(&dQ), sizeof(double) * nv * nv) ||
      !alloc(reinterpret_cast<void**>(&dA), sizeof(double) * A.size()) ||
      !alloc(reinterpret_cast<void**>(&dsel), sizeof(int) * 6) ||
      !alloc(reinterpret_cast<void**>(&dflag), sizeof(int))) {
    cleanup();
    priest_free_problem(p.release());
    return fail(PRIEST_ERR_NOMEM, "device allocation failed");
  }
  int flag = -99;
  hipError_t e = hipMemcpyAsync(p->dW, p->hW.data(), sizeof(float) * p->hW.size(),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dQ, Q.data(), sizeof(double) * nv * nv, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dA, A.data(), sizeof(double) * A.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(dsel, p->rowsel, sizeof(int) * 6, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_kkt(dQ, dA, nv, E, dsel, p->d64, p->dM11, p->dPi, p->dM12, dflag, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&flag, dflag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  p->hM11.resize(nv * nv);
  p->hPi.resize(nv * nv);
  p->hM12.resize(nv * 6);
  if (e == hipSuccess) e = hipMemcpy(p->hM11.data(), p->dM11, sizeof(float) * nv * nv, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(p->hPi.data(), p->dPi, sizeof(float) * nv * nv, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(p->hM12.data(), p->dM12, sizeof(float) * nv * 6, hipMemcpyDeviceToHost);
  cleanup();
  if (e != hipSuccess) {
    priest_free_problem(p.release());
    return fail(PRIEST_ERR_DEVICE, "problem setup failed: %s", hipGetErrorString(e));
  }
  if (flag != PRIEST_OK) {
    priest_free_problem(p.release());
    return fail(PRIEST_ERR_SINGULAR, "KKT matrix is singular (boundary rows %u linearly dependent)",
                d.bc_mask);
  }
  *out = p.release();
  return PRIEST_OK;
}

int32_t priest_free_problem(priest_problem* p) {
  if (!p) return PRIEST_OK;
  for (auto& g : p->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (p->dW) (void)hipFree(p->dW);
  if (p->dM11) (void)hipFree(p->dM11);
  if (p->dPi) (void)hipFree(p->dPi);
  if (p->dM12) (void)hipFree(p->dM12);
  if (p->d64) (void)hipFree(p->d64);
  delete p;
  return PRIEST_OK;
}

int32_t priest_problem_dim(const priest_problem* p) { return p ? p->D : 0; }

int32_t priest_project(priest_problem* p, const float* bc, const float* obs, const float* xi_in,
                       int32_t N, int32_t n_iter, float* xi_out, float* resid, float* c1,
                       void* stream) {
  if (!p) return fail(PRIEST_ERR_INVALID, "problem is NULL");
  if (N < 0 || N > PRIEST_MAX_SAMPLES) return fail(PRIEST_ERR_INVALID, "N must be in [0, %d]", PRIEST_MAX_SAMPLES);
  if (n_iter < 0) return fail(PRIEST_ERR_INVALID, "n_iter must be >= 0");
  if (!bc || !xi_in || !xi_out) return fail(PRIEST_ERR_INVALID, "bc, xi_in and xi_out are required");
  if (p->desc.n_obs > 0 && !obs) return fail(PRIEST_ERR_INVALID, "obs is required when n_obs > 0");
  if (N == 0) return PRIEST_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ProjArgs a = base_args(p);
  a.N = N;
  a.n_iter = n_iter;
  a.bf16_iters = bf16_iters(p, n_iter);
  a.mode = kFromInput;
  a.bc = bc;
  a.obs = obs;
  a.xi_in = xi_in;
  a.xi_out = xi_out;
  a.resid = resid;
  a.c1 = c1;
  apply_tiling(a, tile_candidates(a.dims, a.K)[0]);
  int32_t st = check_lds(p, a);
  if (st != PRIEST_OK) return st;
  TileCfg cfg{};
  if (n_iter > 0 && autotune_enabled() && !tiling_cached(p, a, 1) && !stream_capturing(s)) {
    // time the candidates with outputs in scratch (xi_in may alias xi_out)
    float* scratch = nullptr;
    const size_t n = static_cast<size_t>(N) * (p->D + 2);
    HIP_TRY(hipMalloc(reinterpret_cast<void**>(&scratch), sizeof(float) * n));
    ProjArgs t = trial_args(a);
    t.xi_out = scratch;
    t.resid = scratch + static_cast<size_t>(N) * p->D;
    t.c1 = t.resid + N;
    st = resolve_tiling(p, a, 1, s, &t, &cfg);
    (void)hipFree(scratch);
  } else {
    st = resolve_tiling(p, a, 1, s, nullptr, &cfg);
  }
  if (st != PRIEST_OK) return st;
  apply_tiling(a, cfg);
  HIP_TRY(launch_project_timed(a, 1, s));
  return PRIEST_OK;
}

int32_t priest_project_batch(priest_problem* p, int32_t n_problems, const float* bc,
                             const float* obs, const float* xi_in, int32_t N, int32_t n_iter,
                             float* xi_out, float* resid, float* c1, void* stream) {
  if (!p) return fail(PRIEST_ERR_INVALID, "problem is NULL");
  if (n_problems < 1) return fail(PRIEST_ERR_INVALID, "n_problems must be >= 1");
  if (N < 0 || N > PRIEST_MAX_SAMPLES) return fail(PRIEST_ERR_INVALID, "N must be in [0, %d]", PRIEST_MAX_SAMPLES);
  if (n_iter < 0) return fail(PRIEST_ERR_INVALID, "n_iter must be >= 0");
  if (!bc || !xi_in || !xi_out) return fail(PRIEST_ERR_INVALID, "bc, xi_in and xi_out are required");
  if (p->desc.n_obs > 0 && !obs) return fail(PRIEST_ERR_INVALID, "obs is required when n_obs > 0");
  if (N == 0) return PRIEST_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ProjArgs a = base_args(p);
  a.N = N;
  a.n_iter = n_iter;
  a.bf16_iters = bf16_iters(p, n_iter);
  a.mode = kFromInput;
  a.bc = bc;
  a.bc_stride = static_cast<int64_t>(a.dims) * 6;
  a.obs = obs;
  a.obs_stride = static_cast<int64_t>(a.M) * (a.traj ? a.K * a.dims + 2 : 8);
  const int64_t nd = static_cast<int64_t>(N) * p->D;
  a.xi_in = xi_in;
  a.xi_in_stride = nd;
  a.xi_out = xi_out;
  a.xi_out_stride = nd;
  a.resid = resid;
  a.c1 = c1;
  a.n_stride = N;
  apply_tiling(a, tile_candidates(a.dims, a.K)[0]);
  int32_t st = check_lds(p, a);
  if (st != PRIEST_OK) return st;
  TileCfg cfg{};
  if (n_iter > 0 && autotune_enabled() && !tiling_cached(p, a, n_problems) && !stream_capturing(s)) {
    // time the candidates with outputs in scratch (xi_in may alias xi_out)
    float* scratch = nullptr;
    const size_t n = static_cast<size_t>(n_problems) * N * (p->D + 2);
    HIP_TRY(hipMalloc(reinterpret_cast<void**>(&scratch), sizeof(float) * n));
    ProjArgs t = trial_args(a);
    t.xi_out = scratch;
    t.resid = scratch + static_cast<size_t>(n_problems) * nd;
    t.c1 = t.resid + static_cast<size_t>(n_problems) * N;
    st = resolve_tiling(p, a, n_problems, s, &t, &cfg);
    (void)hipFree(scratch);
  } else {
    st = resolve_tiling(p, a, n_problems, s, nullptr, &cfg);
  }
  if (st != PRIEST_OK) return st;
  apply_tiling(a, cfg);
  HIP_TRY(launch_project_timed(a, n_problems, s));
  return PRIEST_OK;
}

int32_t priest_project_hist(priest_problem* p, const float* bc, const float* obs,
                            const float* xi_in, int32_t N, int32_t n_iter, float* xi_out,
                            float* resid, float* c1, float* resid_hist, void* stream) {
  if (!p) return fail(PRIEST_ERR_INVALID, "problem is NULL");
  if (N < 0 || N > PRIEST_MAX_SAMPLES) return fail(PRIEST_ERR_INVALID, "N must be in [0, %d]", PRIEST_MAX_SAMPLES);
  if (n_iter < 0) return fail(PRIEST_ERR_INVALID, "n_iter must be >= 0");
  if (!bc || !xi_in || !xi_out || !resid_hist)
    return fail(PRIEST_ERR_INVALID, "bc, xi_in, xi_out and resid_hist are required");
  if (p->desc.n_obs > 0 && !obs) return fail(PRIEST_ERR_INVALID, "obs is required when n_obs > 0");
  if (N == 0) return PRIEST_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  ProjArgs a = base_args(p);
  a.N = N;
  a.n_iter = n_iter;
  a.bf16_iters = bf16_iters(p, n_iter);
  a.mode = kFromInput;
  a.bc = bc;
  a.obs = obs;
  a.xi_in = xi_in;
  a.xi_out = xi_out;
  a.resid = resid;
  a.c1 = c1;
  a.resid_hist = resid_hist;
  apply_tiling(a, tile_candidates(a.dims, a.K)[0]);  // the default shape
  const int32_t st = check_lds(p, a);
  if (st != PRIEST_OK) return st;
  HIP_TRY(launch_project_timed(a, 1, s));
  return PRIEST_OK;
}

int32_t priest_project_unfused_workspace_size(const priest_problem* p, int32_t N, size_t* bytes) {
  if (!p || !bytes) return fail(PRIEST_ERR_INVALID, "problem and bytes are required");
  if (N < 0 || N > PRIEST_MAX_SAMPLES) return fail(PRIEST_ERR_INVALID, "N must be in [0, %d]", PRIEST_MAX_SAMPLES);
  *bytes = unfused_layout(N, p->desc.n_steps, p->desc.dims, p->desc.n_coeff, p->desc.n_obs).total;
  return PRIEST_OK;
}

int32_t priest_project_unfused(priest_problem* p, const float* bc, const float* obs,
                               const float* xi_in, int32_t N, int32_t n_iter, float* xi_out,
                               float* resid, float* c1, void* workspace, size_t workspace_bytes,
                               void* stream) {
  if (!p) return fail(PRIEST_ERR_INVALID, "problem is NULL");
  if (N < 0 || N > PRIEST_MAX_SAMPLES) return fail(PRIEST_ERR_INVALID, "N must be in [0, %d]", PRIEST_MAX_SAMPLES);
  if (n_iter < 0) return fail(PRIEST_ERR_INVALID, "n_iter must be >= 0");
  if (!bc || !xi_in || !xi_out) return fail(PRIEST_ERR_INVALID, "bc, xi_in and xi_out are required");
  if (p->desc.n_obs > 0 && !obs) return fail(PRIEST_ERR_INVALID, "obs is required when n_obs > 0");
  if (p->desc.precision != PRIEST_FP32)
    return fail(PRIEST_ERR_INVALID, "the unfused form is FP32 only");
  if (p->desc.obs_model != PRIEST_OBS_VELOCITY)
    return fail(PRIEST_ERR_INVALID, "the unfused form takes constant-velocity obstacles only");
  if (N == 0) return PRIEST_OK;
  size_t need = 0;
  priest_project_unfused_workspace_size(p, N, &need);
  if (!workspace || workspace_bytes < need)
    return fail(PRIEST_ERR_NOMEM, "workspace has %zu bytes, %zu needed", workspace_bytes, need);
  ProjArgs a = base_args(p);
  a.N = N;
  a.n_iter = n_iter;
  a.bc = bc;
  a.obs = obs;
  HIP_TRY(launch_unfused(a, xi_in, xi_out, resid, c1, static_cast<char*>(workspace),
                         static_cast<hipStream_t>(stream)));
  return PRIEST_OK;
}

int32_t priest_plan_workspace_size(const priest_problem* p, const priest_cem_params* c,
                                   int32_t n_problems, size_t* bytes) {
  if (!p || !bytes) return fail(PRIEST_ERR_INVALID, "problem and bytes are required");
  const int32_t st = validate_cem(c, p->desc.dims);
  if (st != PRIEST_OK) return st;
  if (n_problems < 1) return fail(PRIEST_ERR_INVALID, "n_problems must be >= 1");
  *bytes = plan_layout(p->D, c->n_samples, p->desc.n_obs).per_problem * static_cast<size_t>(n_problems);
  return PRIEST_OK;
}

static int32_t plan_common(priest_problem* p, int32_t P, const float* bc, const float* obs,
                           const priest_cem_params* c, float* mu, float* cov, uint64_t seed,
                           uint32_t stream_base, const float* noise, const priest_plan_out* out,
                           void* workspace, size_t workspace_bytes, int32_t use_graph,
                           void* stream) {
  if (!p) return fail(PRIEST_ERR_INVALID, "problem is NULL");
  int32_t st = validate_cem(c, p->desc.dims);
  if (st != PRIEST_OK) return st;
  if (P < 1) return fail(PRIEST_ERR_INVALID, "n_problems must be >= 1");
  if (!bc || !mu || !cov || !out || !out->best_xi || !out->best_cost || !workspace)
    return fail(PRIEST_ERR_INVALID, "bc, mu, cov, out->best_xi, out->best_cost and workspace are required");
  if (p->desc.n_obs > 0 && !obs) return fail(PRIEST_ERR_INVALID, "obs is required when n_obs > 0");
  size_t need = 0;
  priest_plan_workspace_size(p, c, P, &need);
  if (workspace_bytes < need)
    return fail(PRIEST_ERR_NOMEM, "workspace has %zu bytes, %zu needed", workspace_bytes, need);
  if (cem_lds_bytes(c->n_samples, p->D, c->n_elite) > p->lds_limit)
    return fail(PRIEST_ERR_INVALID, "n_samples too large for the selection kernel");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (use_graph && !s) return fail(PRIEST_ERR_INVALID, "graph capture needs a non-default stream");
  PlanArgs pa = plan_args(p, P, bc, obs, c, mu, cov, seed, stream_base, noise, out,
                          static_cast<char*>(workspace));
  TileCfg cfg{};
  st = plan_tiling(p, pa, P, s, &cfg);
  if (st != PRIEST_OK) return st;
  if (!use_graph) return enqueue_plan(P, pa, c, noise, out, s);
  std::vector<uint64_t> key = {
      static_cast<uint64_t>(P), reinterpret_cast<uint64_t>(bc), reinterpret_cast<uint64_t>(obs),
      reinterpret_cast<uint64_t>(mu), reinterpret_cast<uint64_t>(cov), seed, stream_base,
      reinterpret_cast<uint64_t>(noise), reinterpret_cast<uint64_t>(workspace),
      reinterpret_cast<uint64_t>(s), reinterpret_cast<uint64_t>(out->best_xi),
      reinterpret_cast<uint64_t>(out->best_cost), reinterpret_cast<uint64_t>(out->elite_idx),
      reinterpret_cast<uint64_t>(out->proj_idx), reinterpret_cast<uint64_t>(out->xi),
      reinterpret_cast<uint64_t>(out->xi_bar), reinterpret_cast<uint64_t>(out->resid),
      reinterpret_cast<uint64_t>(out->c1), reinterpret_cast<uint64_t>(out->status)};
  const uint32_t* cw = reinterpret_cast<const uint32_t*>(c);
  for (size_t i = 0; i < sizeof(priest_cem_params) / 4; ++i) key.push_back(cw[i]);
  key.push_back(static_cast<uint64_t>(cfg.axis_slots) | (static_cast<uint64_t>(cfg.row_tiles) << 8) |
                (static_cast<uint64_t>(cfg.persistent) << 16));
  std::lock_guard<std::mutex> lk(p->graph_mu);
  for (auto& g : p->graphs)
    if (g.key == key) {
      HIP_TRY(hipGraphLaunch(g.exec, s));
      return PRIEST_OK;
    }
  HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  st = enqueue_plan(P, pa, c, noise, out, s);
  hipGraph_t graph = nullptr;
  const hipError_t ce = hipStreamEndCapture(s, &graph);
  if (st != PRIEST_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (ce != hipSuccess) return fail(PRIEST_ERR_DEVICE, "stream capture failed: %s", hipGetErrorString(ce));
  GraphEntry g;
  g.key = key;
  const hipError_t ie = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return fail(PRIEST_ERR_DEVICE, "graph instantiate failed: %s", hipGetErrorString(ie));
  if (p->graphs.size() >= 16) {
    (void)hipGraphExecDestroy(p->graphs.front().exec);
    p->graphs.erase(p->graphs.begin());
  }
  p->graphs.push_back(g);
  HIP_TRY(hipGraphLaunch(g.exec, s));
  return PRIEST_OK;
}

int32_t priest_plan(priest_problem* p, const float* bc, const float* obs,
                    const priest_cem_params* c, float* mu, float* cov, uint64_t seed,
                    uint32_t stream_id, const float* noise, const priest_plan_out* out,
                    void* workspace, size_t workspace_bytes, void* stream) {
  return plan_common(p, 1, bc, obs, c, mu, cov, seed, stream_id, noise, out, workspace,
                     workspace_bytes, 0, stream);
}

int32_t priest_plan_static(priest_problem* p, const float* bc, const float* obs,
                           const priest_cem_params* c, float* mu, float* cov, uint64_t seed,
                           uint32_t stream_id, const float* noise, const priest_plan_out* out,
                           void* stream) {
  if (!p) return fail(PRIEST_ERR_INVALID, "problem is NULL");
  int32_t st = validate_cem(c, p->desc.dims);
  if (st != PRIEST_OK) return st;
  if (!bc || !mu || !cov || !out || !out->best_xi || !out->best_cost)
    return fail(PRIEST_ERR_INVALID, "bc, mu, cov, out->best_xi and out->best_cost are required");
  if (p->desc.n_obs > 0 && !obs) return fail(PRIEST_ERR_INVALID, "obs is required when n_obs > 0");
  size_t need = 0;
  priest_plan_workspace_size(p, c, 1, &need);
  if (need > kStaticWorkspaceBytes)
    return fail(PRIEST_ERR_NOMEM, "plan needs %zu bytes of workspace, the static one has %zu", need,
                kStaticWorkspaceBytes);
  if (cem_lds_bytes(c->n_samples, p->D, c->n_elite) > p->lds_limit)
    return fail(PRIEST_ERR_INVALID, "n_samples too large for the selection kernel");
  hipError_t e = hipSuccess;
  void* ws = static_scratch_ptr(p->device, &e);
  if (!ws)
    return fail(PRIEST_ERR_DEVICE, "static workspace of device %d unavailable: %s", p->device,
                hipGetErrorString(e));
  hipStream_t s = static_cast<hipStream_t>(stream);
  PlanArgs pa = plan_args(p, 1, bc, obs, c, mu, cov, seed, stream_id, noise, out,
                          static_cast<char*>(ws));
  // no autotuning (it synchronises and creates timing events): a forced or
  // already tuned shape, else the default one
  TileCfg cfg{};
  st = check_lds(p, pa.a);
  if (st != PRIEST_OK) return st;
  st = resolve_tiling(p, pa.a, 1, s, nullptr, &cfg);
  if (st != PRIEST_OK) return st;
  apply_tiling(pa.a, cfg);
  st = check_lds(p, pa.a);
  if (st != PRIEST_OK) return st;
  return enqueue_plan(1, pa, c, noise, out, s, false);
}

int32_t priest_plan_batch(priest_problem* p, int32_t n_problems, const float* bc,
                          const float* obs, const priest_cem_params* c, float* mu, float* cov,
                          uint64_t seed, uint32_t stream_base, const float* noise,
                          const priest_plan_out* out, void* workspace, size_t workspace_bytes,
                          int32_t use_graph, void* stream) {
  return plan_common(p, n_problems, bc, obs, c, mu, cov, seed, stream_base, noise, out, workspace,
                     workspace_bytes, use_graph, stream);
}

int32_t priest_profile_enable(int32_t on) {
  Profiler& pr = profiler();
  std::lock_guard<std::mutex> lk(pr.mu);
  pr.on = on != 0;
  return PRIEST_OK;
}

int32_t priest_profile_count_pairs(int32_t on) {
  Profiler& pr = profiler();
  std::lock_guard<std::mutex> lk(pr.mu);
  if (on) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (pr.pairs_dev && pr.pairs_device != dev)
      return fail(PRIEST_ERR_INVALID, "pair counting was first enabled on device %d", pr.pairs_device);
    if (!pr.pairs_dev) {
      HIP_TRY(hipMalloc(reinterpret_cast<void**>(&pr.pairs_dev), sizeof(unsigned long long)));
      pr.pairs_device = dev;
    }
    HIP_TRY(hipMemset(pr.pairs_dev, 0, sizeof(unsigned long long)));
  }
  pr.count_pairs = on != 0;
  return PRIEST_OK;
}

int32_t priest_profile_read_pairs(uint64_t* pairs) {
  if (!pairs) return fail(PRIEST_ERR_INVALID, "pairs is required");
  Profiler& pr = profiler();
  std::lock_guard<std::mutex> lk(pr.mu);
  *pairs = 0;
  if (!pr.pairs_dev) return PRIEST_OK;
  HIP_TRY(hipDeviceSynchronize());
  unsigned long long v = 0;
  HIP_TRY(hipMemcpy(&v, pr.pairs_dev, sizeof(v), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(pr.pairs_dev, 0, sizeof(unsigned long long)));
  *pairs = v;
  return PRIEST_OK;
}

int32_t priest_profile_read(int32_t* n_launches, double* total_ms) {
  if (!n_launches || !total_ms) return fail(PRIEST_ERR_INVALID, "n_launches and total_ms are required");
  Profiler& pr = profiler();
  std::vector<std::pair<hipEvent_t, hipEvent_t>> evs;
  {
    std::lock_guard<std::mutex> lk(pr.mu);
    evs.swap(pr.pending);
  }
  double sum = 0.0;
  hipError_t err = hipSuccess;
  for (auto& ev : evs) {
    float ms = 0.0f;
    if (err == hipSuccess) err = hipEventSynchronize(ev.second);
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, ev.first, ev.second);
    sum += ms;
  }
  {
    std::lock_guard<std::mutex> lk(pr.mu);
    for (auto& ev : evs) pr.pool.push_back(ev);
  }
  if (err != hipSuccess) return fail(PRIEST_ERR_DEVICE, "profile read failed: %s", hipGetErrorString(err));
  *n_launches = static_cast<int32_t>(evs.size());
  *total_ms = sum;
  return PRIEST_OK;
}

int32_t priest_tiling_candidates(const priest_problem* p, priest_tiling* out, int32_t max_out,
                                 int32_t* n) {
  if (!p || !n || max_out < 0 || (max_out > 0 && !out))
    return fail(PRIEST_ERR_INVALID, "problem and n are required");
  const std::vector<TileCfg> c = tile_candidates(p->desc.dims, p->desc.n_steps);
  *n = static_cast<int32_t>(c.size());
  for (int32_t i = 0; i < max_out && i < *n; ++i)
    out[i] = priest_tiling{c[i].axis_slots, c[i].row_tiles, c[i].persistent, 0};
  return PRIEST_OK;
}

int32_t priest_set_tiling(priest_problem* p, const priest_tiling* t) {
  if (!p) return fail(PRIEST_ERR_INVALID, "problem is NULL");
  std::lock_guard<std::mutex> lk(p->tune_mu);
  if (p->desc.obs_model == PRIEST_OBS_PATH) {
    if (t && (t->axis_slots != 4 || t->row_tiles != 1 || t->persistent != 0 || t->reserved != 0))
      return fail(PRIEST_ERR_INVALID, "problems with obstacle paths use the default tile shape");
    return PRIEST_OK;
  }
  if (!t) {
    p->forced = false;
    return PRIEST_OK;
  }
  if (!tiling_valid(p->desc.dims, t->axis_slots, t->row_tiles, p->desc.n_steps) ||
      (t->persistent != 0 && t->persistent != 1) || t->reserved != 0)
    return fail(PRIEST_ERR_INVALID, "tiling (%d, %d, %d) is not a candidate for dims %d",
                t->axis_slots, t->row_tiles, t->persistent, p->desc.dims);
  p->forced = true;
  p->force_cfg = TileCfg{t->axis_slots, t->row_tiles, t->persistent};
  return PRIEST_OK;
}

int32_t priest_last_tiling(const priest_problem* p, priest_tiling* out, int32_t* tuned) {
  if (!p || !out) return fail(PRIEST_ERR_INVALID, "problem and out are required");
  std::lock_guard<std::mutex> lk(const_cast<priest_problem*>(p)->tune_mu);
  *out = priest_tiling{p->last_cfg.axis_slots, p->last_cfg.row_tiles, p->last_cfg.persistent, 0};
  if (tuned) *tuned = p->last_tuned;
  return PRIEST_OK;
}

int32_t priest_plan_dpriest(priest_problem* p, int32_t n_groups, const float* bc,
                            const float* obs, const priest_cem_params* c, float* mu, float* cov,
                            uint64_t seed, uint32_t stream_base, const float* noise,
                            const priest_plan_out* out, float* best_xi, float* best_cost,
                            int32_t* best_group, void* workspace, size_t workspace_bytes,
                            void* stream) {
  if (!p) return fail(PRIEST_ERR_INVALID, "problem is NULL");
  int32_t st = validate_cem(c, p->desc.dims);
  if (st != PRIEST_OK) return st;
  if (n_groups < 1) return fail(PRIEST_ERR_INVALID, "n_groups must be >= 1");
  if (!bc || !mu || !cov || !out || !out->best_xi || !out->best_cost || !workspace || !best_xi ||
      !best_cost || !best_group)
    return fail(PRIEST_ERR_INVALID,
                "bc, mu, cov, out->best_xi, out->best_cost, best_xi, best_cost, best_group and "
                "workspace are required");
  if (p->desc.n_obs > 0 && !obs) return fail(PRIEST_ERR_INVALID, "obs is required when n_obs > 0");
  size_t need = 0;
  priest_plan_workspace_size(p, c, n_groups, &need);
  if (workspace_bytes < need)
    return fail(PRIEST_ERR_NOMEM, "workspace has %zu bytes, %zu needed", workspace_bytes, need);
  if (cem_lds_bytes(c->n_samples, p->D, c->n_elite) > p->lds_limit)
    return fail(PRIEST_ERR_INVALID, "n_samples too large for the selection kernel");
  hipStream_t s = static_cast<hipStream_t>(stream);
  PlanArgs pa = plan_args(p, n_groups, bc, obs, c, mu, cov, seed, stream_base, noise, out,
                          static_cast<char*>(workspace));
  // one scene for every distribution
  pa.a.bc_stride = 0;
  pa.a.obs_stride = 0;
  TileCfg cfg{};
  st = plan_tiling(p, pa, n_groups, s, &cfg);
  if (st != PRIEST_OK) return st;
  st = enqueue_plan(n_groups, pa, c, noise, out, s);
  if (st != PRIEST_OK) return st;
  HIP_TRY(launch_pick_best(n_groups, p->D, out->best_xi, out->best_cost, best_xi, best_cost,
                           best_group, s));
  return PRIEST_OK;
}

int32_t priest_debug_offsets(priest_problem* p, const float* bc, const float* obs,
                             const float* xi, int32_t N, float* offsets, void* stream) {
  if (!p || !xi || !offsets) return fail(PRIEST_ERR_INVALID, "problem, xi and offsets are required");
  if (p->desc.n_obs > 0 && !obs) return fail(PRIEST_ERR_INVALID, "obs is required when n_obs > 0");
  if (N < 0 || N > 4096) return fail(PRIEST_ERR_INVALID, "N must be in [0, 4096]");
  (void)bc;
  if (N == 0) return PRIEST_OK;
  ProjArgs a = base_args(p);
  a.N = N;
  a.obs = obs;
  HIP_TRY(launch_debug_offsets(a, xi, offsets, static_cast<hipStream_t>(stream)));
  return PRIEST_OK;
}

int32_t priest_debug_normals(uint64_t seed, uint32_t stream_id, int32_t iter, int32_t N, int32_t D,
                             float* z, void* stream) {
  if (!z || N < 0 || D < 1 || iter < 0) return fail(PRIEST_ERR_INVALID, "bad arguments");
  if (N == 0) return PRIEST_OK;
  HIP_TRY(launch_debug_normals(seed, stream_id, iter, N, D, z, static_cast<hipStream_t>(stream)));
  return PRIEST_OK;
}

int32_t priest_debug_select(int32_t N, int32_t n_proj, int32_t n_elite, const float* r,
                            const float* c1, int32_t* elite_idx, int32_t* proj_idx, void* stream) {
  if (!r || !c1 || !elite_idx || n_elite < 1 || n_proj < n_elite || N < n_proj ||
      N > kCemThreads * 16)
    return fail(PRIEST_ERR_INVALID, "need r, c1, elite_idx and 1 <= n_elite <= n_proj <= N <= %d",
                kCemThreads * 16);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // a one-coefficient problem around the selection: zero rows, mu = 0, Sigma = 1
  float* buf = nullptr;
  const size_t nf = static_cast<size_t>(N) + 8;
  HIP_TRY(hipMalloc(&buf, nf * sizeof(float)));
  std::vector<float> h(nf, 0.0f);
  h[N + 1] = 1.0f;  // cov
  hipError_t e = hipMemcpyAsync(buf, h.data(), nf * sizeof(float), hipMemcpyHostToDevice, s);
  CemArgs ca{};
  ca.D = 1;
  ca.N = N;
  ca.n_proj = n_proj;
  ca.n_elite = n_elite;
  ca.sigma = 0.5f;
  ca.gamma = 1.0f;
  ca.cov_jitter = 0.0f;
  ca.xb = buf;
  ca.resid = r;
  ca.c1 = c1;
  ca.mu = buf + N;
  ca.cov = buf + N + 1;
  ca.L = buf + N + 2;
  ca.best_xi = buf + N + 3;
  ca.best_cost = buf + N + 4;
  ca.elite_idx = elite_idx;
  ca.proj_idx = proj_idx;
  if (e == hipSuccess) e = launch_cem(ca, 1, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  const hipError_t ef = hipFree(buf);
  HIP_TRY(e);
  HIP_TRY(ef);
  return PRIEST_OK;
}

int32_t priest_debug_constants(const priest_problem* p, int32_t which, float* host_out,
                               int32_t count) {
  if (!p || !host_out) return fail(PRIEST_ERR_INVALID, "problem and host_out are required");
  const std::vector<float>* src = nullptr;
  switch (which) {
    case 0: src = &p->hM11; break;
    case 1: src = &p->hPi; break;
    case 2: src = &p->hM12; break;
    case 3: src = &p->hW; break;
    default: return fail(PRIEST_ERR_INVALID, "unknown constant %d", which);
  }
  if (count != static_cast<int32_t>(src->size()))
    return fail(PRIEST_ERR_INVALID, "constant %d has %zu entries, count is %d", which, src->size(), count);
  std::memcpy(host_out, src->data(), sizeof(float) * src->size());
  return PRIEST_OK;
}

}  // extern "C"
