// Continuous-batching planning server: the host runtime of the serving path.
//
// Each step advances every active request by one iteration of Alg. 1:
//   1. one host->device copy of the step's staging block (descriptor tables,
//      new scenes, reset warm starts) and a segment-copy kernel that places
//      the uploads;
//   2. Cholesky of the sampling covariance for requests admitted this step;
//   3. one descriptor-table projection launch per distinct n_steps (draw +
//      eqs. (4)-(7) for every sample, each request on blocks of its own);
//   4. one selection/refit launch over all requests (eqs. (9a)-(9c));
//   5. a gather of finished requests' results and one device->host copy.
// Requests are admitted FIFO at step boundaries when a slot is free, their
// robot has no request in flight and their device state fits the arena
// (first-fit, coalescing).  Work on one stream is ordered, so a finishing
// request's arena block and its robot are released as soon as its last step
// is enqueued; the host reads its result once the step's event completes.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <tuple>
#include <vector>

#include "priest_internal.h"

using namespace priest;

namespace {

double clock_now() {
  static const auto t0 = std::chrono::steady_clock::now();
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

size_t al256(size_t n) { return (n + 255) & ~static_cast<size_t>(255); }

constexpr int kRing = 3;            // staging slots; > max_inflight_steps
constexpr int kMaxActive = 8192;
constexpr int kMaxRobots = 65536;
constexpr int kMaxD = 3 * PRIEST_MAX_COEFF;

// One contiguous 32-bit copy done by one block of seg_copy_kernel.
struct Seg {
  const uint32_t* src;
  uint32_t* dst;
  int32_t n;
  int32_t pad;
};

__global__ void seg_copy_kernel(const Seg* segs) {
  const Seg g = segs[blockIdx.x];
  for (int i = threadIdx.x; i < g.n; i += blockDim.x) g.dst[i] = g.src[i];
}

// First-fit allocator over [0, cap) with coalescing of free neighbours.
class Arena {
 public:
  explicit Arena(size_t cap = 0) : cap_(cap) {
    if (cap) free_[0] = cap;
  }
  bool alloc(size_t n, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, noff = it->first + n;
        free_.erase(it);
        if (rest) free_[noff] = rest;
        used_ += n;
        high_ = std::max(high_, used_);
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t high() const { return high_; }
  size_t cap() const { return cap_; }

 private:
  size_t cap_ = 0, used_ = 0, high_ = 0;
  std::map<size_t, size_t> free_;
};

struct Robot {
  bool busy = false;
  bool init = false;
};

struct Req {
  int64_t id = 0;
  priest_request r{};
  std::vector<float> bc, obs;
  size_t off = 0, bytes = 0;
  int iter = 0;
  bool fresh = true;  // admitted in the step being built
  priest_problem* prob = nullptr;
  double t_admit = 0, t_done = 0;
  // device state inside the arena
  float *dbc = nullptr, *dobs = nullptr, *dxb = nullptr, *dres = nullptr, *dc1 = nullptr,
        *dL = nullptr, *dbest = nullptr, *dcost = nullptr;
  int32_t* dstat = nullptr;
  // result, filled when the final step completes
  float cost = 0;
  int32_t status = 0;
  std::vector<float> best;
};

struct Step {
  hipEvent_t ev = nullptr;
  int slot = 0;
  std::vector<Req*> finishing;  // result row k of the slot's result block
};

struct Slot {
  char* host = nullptr;  // pinned
  char* dev = nullptr;
  size_t cap = 0;
  uint32_t* hres = nullptr;  // pinned [max_active][D + 2]
  uint32_t* dres = nullptr;
};

using ShapeKey = std::tuple<int, int, double>;

}  // namespace

struct priest_server {
  priest_server_config cfg{};
  hipStream_t stream = nullptr;
  int D = 0;
  bool dry = false;
  std::map<ShapeKey, priest_problem*> problems;
  char* arena_base = nullptr;
  Arena arena;
  float* robot_mu = nullptr;   // [max_robots][D]
  float* robot_cov = nullptr;  // [max_robots][D][D]
  std::vector<Robot> robots;
  std::deque<Req*> pending;
  std::vector<Req*> active;
  std::deque<Req*> done;
  std::deque<Step> inflight;
  std::vector<hipEvent_t> event_pool;
  Slot slots[kRing];
  int ring = 0;
  int64_t next_id = 1;
  priest_server_stats st{};
};

namespace {

int32_t sfail(int32_t code, const char* msg) { return set_error(code, msg); }

#define SERVE_TRY(expr)                                                             \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) return sfail(PRIEST_ERR_DEVICE, hipGetErrorString(e_));   \
  } while (0)

size_t footprint(int dims, int D, const priest_request& r) {
  const size_t N = r.n_samples;
  return al256(4 * 6 * static_cast<size_t>(dims)) +
         al256(4 * 8 * static_cast<size_t>(std::max(r.n_obs, 1))) + al256(4 * N * D) +
         2 * al256(4 * N) + al256(4 * static_cast<size_t>(D) * D) +
         al256(4 * static_cast<size_t>(D)) + 2 * al256(4);
}

int32_t get_problem(priest_server* s, int K, int M, double T, priest_problem** out) {
  const ShapeKey key{K, M, T};
  auto it = s->problems.find(key);
  if (it != s->problems.end()) {
    *out = it->second;
    return PRIEST_OK;
  }
  priest_problem_desc d{};
  d.dims = s->cfg.dims;
  d.n_coeff = s->cfg.n_coeff;
  d.n_steps = K;
  d.n_obs = M;
  d.horizon = T;
  d.rho = s->cfg.rho;
  d.v_max = s->cfg.v_max;
  d.a_max = s->cfg.a_max;
  d.bc_mask = s->cfg.bc_mask;
  d.precision = s->cfg.precision;
  d.n_refine_fp32 = s->cfg.n_refine_fp32;
  priest_problem* p = nullptr;
  int32_t st = priest_init_problem(&d, s->stream, &p);
  if (st != PRIEST_OK) return st;
  ProjArgs a = problem_args(p);
  a.N = 4;
  a.mode = kFromPhilox;
  set_default_tiling(a);
  a.blocks_per_problem = 1;
  st = problem_check_lds(p, a);
  if (st != PRIEST_OK) {
    priest_free_problem(p);
    return st;
  }
  s->problems[key] = p;
  *out = p;
  return PRIEST_OK;
}

// Moves the requests of completed steps to `done`.  With `wait`, blocks on
// the oldest in-flight step first.
int32_t harvest(priest_server* s, bool wait) {
  while (!s->inflight.empty()) {
    Step& f = s->inflight.front();
    if (!s->dry) {
      const hipError_t e = wait ? hipEventSynchronize(f.ev) : hipEventQuery(f.ev);
      if (e == hipErrorNotReady) return PRIEST_OK;
      if (e != hipSuccess) return sfail(PRIEST_ERR_DEVICE, hipGetErrorString(e));
      s->event_pool.push_back(f.ev);
    }
    const double now = clock_now();
    const int W = s->D + 2;
    for (size_t k = 0; k < f.finishing.size(); ++k) {
      Req* q = f.finishing[k];
      if (!s->dry) {
        const uint32_t* h = s->slots[f.slot].hres + k * W;
        q->best.resize(s->D);
        std::memcpy(q->best.data(), h, 4 * s->D);
        std::memcpy(&q->cost, h + s->D, 4);
        std::memcpy(&q->status, h + s->D + 1, 4);
      }
      q->t_done = now;
      s->done.push_back(q);
      s->st.completed += 1;
      s->st.sample_iters += static_cast<int64_t>(q->r.n_samples) * q->r.n_proj_iters * q->r.n_cem;
    }
    s->inflight.pop_front();
    wait = false;
  }
  return PRIEST_OK;
}

// Admits pending requests in FIFO order; a request whose robot is busy is
// passed over, a request that does not fit the arena stops admission (no
// overtaking by smaller requests, so large requests cannot starve).
int32_t admit(priest_server* s) {
  for (auto it = s->pending.begin(); it != s->pending.end();) {
    if (static_cast<int>(s->active.size()) >= s->cfg.max_active) break;
    Req* q = *it;
    Robot& rb = s->robots[q->r.robot];
    if (rb.busy) {
      ++it;
      continue;
    }
    if (!s->dry) {
      const int32_t st = get_problem(s, q->r.n_steps, q->r.n_obs, q->r.horizon, &q->prob);
      if (st != PRIEST_OK) return st;
    }
    if (!s->arena.alloc(q->bytes, &q->off)) break;
    if (!s->dry) {
      char* base = s->arena_base + q->off;
      size_t o = 0;
      auto take = [&](size_t n) {
        char* p = base + o;
        o += al256(n);
        return p;
      };
      const size_t D = s->D, N = q->r.n_samples;
      q->dbc = reinterpret_cast<float*>(take(4 * 6 * static_cast<size_t>(s->cfg.dims)));
      q->dobs = reinterpret_cast<float*>(take(4 * 8 * static_cast<size_t>(std::max(q->r.n_obs, 1))));
      q->dxb = reinterpret_cast<float*>(take(4 * N * D));
      q->dres = reinterpret_cast<float*>(take(4 * N));
      q->dc1 = reinterpret_cast<float*>(take(4 * N));
      q->dL = reinterpret_cast<float*>(take(4 * D * D));
      q->dbest = reinterpret_cast<float*>(take(4 * D));
      q->dcost = reinterpret_cast<float*>(take(4));
      q->dstat = reinterpret_cast<int32_t*>(take(4));
    }
    rb.busy = true;
    q->iter = 0;
    q->fresh = true;
    q->t_admit = clock_now();
    s->active.push_back(q);
    s->st.admitted += 1;
    it = s->pending.erase(it);
  }
  s->st.max_active_seen =
      std::max<int64_t>(s->st.max_active_seen, static_cast<int64_t>(s->active.size()));
  return PRIEST_OK;
}

// Straight-line control polygon from the start to the goal position, and
// init_std^2 I.
void reset_state(const priest_server* s, const Req* q, float* mu, float* cov) {
  const int nv = s->cfg.n_coeff, D = s->D;
  for (int ax = 0; ax < s->cfg.dims; ++ax) {
    const float p0 = q->bc[ax * 6 + 0], pf = q->bc[ax * 6 + 3];
    for (int c = 0; c < nv; ++c)
      mu[ax * nv + c] = p0 + (pf - p0) * static_cast<float>(c) / static_cast<float>(nv - 1);
  }
  const float v = s->cfg.init_std * s->cfg.init_std;
  for (int i = 0; i < D * D; ++i) cov[i] = 0.0f;
  for (int d = 0; d < D; ++d) cov[d * D + d] = v;
}

int32_t ensure_slot(priest_server* s, Slot& sl, size_t bytes) {
  if (bytes <= sl.cap) return PRIEST_OK;
  // buffers of this slot may still be read by enqueued work
  SERVE_TRY(hipStreamSynchronize(s->stream));
  if (sl.host) SERVE_TRY(hipHostFree(sl.host));
  if (sl.dev) SERVE_TRY(hipFree(sl.dev));
  sl.host = nullptr;
  sl.dev = nullptr;
  sl.cap = 0;
  const size_t cap = std::max(2 * bytes, static_cast<size_t>(1) << 20);
  if (hipHostMalloc(reinterpret_cast<void**>(&sl.host), cap) != hipSuccess)
    return sfail(PRIEST_ERR_NOMEM, "pinned staging allocation failed");
  if (hipMalloc(reinterpret_cast<void**>(&sl.dev), cap) != hipSuccess)
    return sfail(PRIEST_ERR_NOMEM, "device staging allocation failed");
  sl.cap = cap;
  return PRIEST_OK;
}

CemArgs cem_task(const priest_server* s, const Req* q, bool chol_only) {
  CemArgs c{};
  c.D = s->D;
  c.N = q->r.n_samples;
  c.n_proj = q->r.n_proj;
  c.n_elite = q->r.n_elite;
  c.chol_only = chol_only ? 1 : 0;
  c.sigma = s->cfg.sigma;
  c.gamma = s->cfg.gamma;
  c.cov_jitter = s->cfg.cov_jitter;
  c.xb = q->dxb;
  c.resid = q->dres;
  c.c1 = q->dc1;
  c.mu = s->robot_mu + static_cast<size_t>(q->r.robot) * s->D;
  c.cov = s->robot_cov + static_cast<size_t>(q->r.robot) * s->D * s->D;
  c.L = q->dL;
  c.best_xi = q->dbest;
  c.best_cost = q->dcost;
  c.status = q->dstat;
  return c;
}

// Builds the step's staging block and enqueues its launches.
int32_t launch_step(priest_server* s, int slot_index, const std::vector<Req*>& finishing) {
  Slot& sl = s->slots[slot_index];
  const int n = static_cast<int>(s->active.size());
  const int D = s->D, dims = s->cfg.dims;
  std::vector<Req*> fresh;
  for (Req* q : s->active)
    if (q->fresh) fresh.push_back(q);
  const int nchol = static_cast<int>(fresh.size());
  // projection order: grouped by n_steps, stable within a group
  std::vector<Req*> order(s->active);
  std::stable_sort(order.begin(), order.end(),
                   [](const Req* x, const Req* y) { return x->r.n_steps < y->r.n_steps; });
  int nbuckets = 0;
  for (int i = 0; i < n; ++i)
    if (i == 0 || order[i]->r.n_steps != order[i - 1]->r.n_steps) ++nbuckets;
  // what the new requests upload: scene, and (mu, Sigma) when reset
  enum : uint8_t { kKeep = 0, kResetBoth = 1, kResetCov = 2 };
  std::vector<uint8_t> reset(fresh.size());
  size_t nup = 0;
  int nuseg = 0;
  for (size_t i = 0; i < fresh.size(); ++i) {
    const Req* q = fresh[i];
    const bool init = s->robots[q->r.robot].init;
    if (!init || q->r.warm_start == PRIEST_WARM_RESET) reset[i] = kResetBoth;
    else if (q->r.warm_start == PRIEST_WARM_KEEP_MEAN) reset[i] = kResetCov;
    else reset[i] = kKeep;
    nup += 6 * static_cast<size_t>(dims) + 8 * static_cast<size_t>(q->r.n_obs) + 1;
    nuseg += 2 + (q->r.n_obs > 0 ? 1 : 0);
    if (reset[i] == kResetBoth) {
      nup += D;
      nuseg += 1;
    }
    if (reset[i] != kKeep) {
      nup += static_cast<size_t>(D) * D;
      nuseg += 1;
    }
  }
  const int ngseg = 3 * static_cast<int>(finishing.size());
  // layout of the staging block
  size_t o = 0;
  const size_t o_proj = o;  o += al256(sizeof(ProjArgs) * n);
  const size_t o_cem = o;   o += al256(sizeof(CemArgs) * (nchol + n));
  const size_t o_pre = o;   o += al256(sizeof(int) * (n + nbuckets));
  const size_t o_useg = o;  o += al256(sizeof(Seg) * nuseg);
  const size_t o_gseg = o;  o += al256(sizeof(Seg) * ngseg);
  const size_t o_data = o;  o += al256(4 * nup);
  const int32_t est = ensure_slot(s, sl, o);
  if (est != PRIEST_OK) return est;
  char* h = sl.host;
  char* d = sl.dev;
  ProjArgs* hp = reinterpret_cast<ProjArgs*>(h + o_proj);
  CemArgs* hc = reinterpret_cast<CemArgs*>(h + o_cem);
  int* hpre = reinterpret_cast<int*>(h + o_pre);
  Seg* hus = reinterpret_cast<Seg*>(h + o_useg);
  Seg* hgs = reinterpret_cast<Seg*>(h + o_gseg);
  float* hdata = reinterpret_cast<float*>(h + o_data);
  const uint32_t* ddata = reinterpret_cast<const uint32_t*>(d + o_data);

  // 1. uploads of new requests
  {
    size_t w = 0;
    int k = 0;
    auto up = [&](const float* src, size_t cnt, float* dst) {
      std::memcpy(hdata + w, src, 4 * cnt);
      hus[k++] = Seg{ddata + w, reinterpret_cast<uint32_t*>(dst), static_cast<int32_t>(cnt), 0};
      w += cnt;
    };
    std::vector<float> mu(D), cov(static_cast<size_t>(D) * D);
    for (size_t i = 0; i < fresh.size(); ++i) {
      const Req* q = fresh[i];
      float* rmu = s->robot_mu + static_cast<size_t>(q->r.robot) * D;
      float* rcov = s->robot_cov + static_cast<size_t>(q->r.robot) * D * D;
      up(q->bc.data(), 6 * static_cast<size_t>(dims), q->dbc);
      const float zero = 0.0f;  // status word starts at PRIEST_OK (bit pattern 0)
      up(&zero, 1, reinterpret_cast<float*>(q->dstat));
      if (q->r.n_obs > 0) up(q->obs.data(), 8 * static_cast<size_t>(q->r.n_obs), q->dobs);
      if (reset[i] != kKeep) reset_state(s, q, mu.data(), cov.data());
      if (reset[i] == kResetBoth) up(mu.data(), D, rmu);
      if (reset[i] != kKeep) up(cov.data(), static_cast<size_t>(D) * D, rcov);
      s->robots[q->r.robot].init = true;
    }
  }
  // 2. Cholesky tasks of new requests, then refit tasks of all requests
  int max_N = 1, max_elite = 1;
  for (int i = 0; i < nchol; ++i) hc[i] = cem_task(s, fresh[i], true);
  for (int i = 0; i < n; ++i) {
    const Req* q = s->active[i];
    hc[nchol + i] = cem_task(s, q, false);
    max_N = std::max(max_N, q->r.n_samples);
    max_elite = std::max(max_elite, q->r.n_elite);
  }
  // 3. projection tasks; bucket b's prefix array (count + 1 entries) starts
  //    at hpre[b.pre]
  struct Bucket {
    int K, first, count, blocks, pre;
    size_t lds;
    bool bf;
  };
  std::vector<Bucket> buckets;
  {
    int pw = 0;
    for (int i = 0; i < n; ++i) {
      const Req* q = order[i];
      ProjArgs a = problem_args(q->prob);
      a.N = q->r.n_samples;
      set_default_tiling(a);  // the descriptor-table kernel's shape
      a.blocks_per_problem = (a.N + a.S - 1) / a.S;
      a.n_iter = q->r.n_proj_iters;
      a.bf16_iters = problem_bf16_iters(q->prob, a.n_iter);
      a.mode = kFromPhilox;
      a.iter = q->iter;
      a.stream_base = q->r.stream_id;
      a.seed = s->cfg.seed;
      a.bc = q->dbc;
      a.obs = q->dobs;
      a.mu = s->robot_mu + static_cast<size_t>(q->r.robot) * D;
      a.L = q->dL;
      a.xi_out = q->dxb;
      a.resid = q->dres;
      a.c1 = q->dc1;
      if (buckets.empty() || buckets.back().K != a.K) {
        if (!buckets.empty()) hpre[pw++] = buckets.back().blocks;
        buckets.push_back(Bucket{a.K, i, 0, 0, pw, 0, false});
      }
      Bucket& b = buckets.back();
      hpre[pw++] = b.blocks;
      b.blocks += a.blocks_per_problem;
      b.count += 1;
      b.lds = std::max(b.lds, project_lds_bytes(a));
      b.bf = b.bf || a.bf16_iters > 0;
      hp[i] = a;
    }
    if (!buckets.empty()) hpre[pw++] = buckets.back().blocks;
  }
  // 5. result gathers: row k = (best_xi [D], best_cost, status)
  for (size_t k = 0; k < finishing.size(); ++k) {
    const Req* q = finishing[k];
    uint32_t* row = sl.dres + k * (D + 2);
    hgs[3 * k + 0] = Seg{reinterpret_cast<const uint32_t*>(q->dbest), row, D, 0};
    hgs[3 * k + 1] = Seg{reinterpret_cast<const uint32_t*>(q->dcost), row + D, 1, 0};
    hgs[3 * k + 2] = Seg{reinterpret_cast<const uint32_t*>(q->dstat), row + D + 1, 1, 0};
  }

  SERVE_TRY(hipMemcpyAsync(d, h, o, hipMemcpyHostToDevice, s->stream));
  if (nuseg) {
    hipLaunchKernelGGL(seg_copy_kernel, dim3(nuseg), dim3(256), 0, s->stream,
                       reinterpret_cast<const Seg*>(d + o_useg));
    SERVE_TRY(hipGetLastError());
  }
  if (nchol) {
    const CemTaskLaunch t{reinterpret_cast<const CemArgs*>(d + o_cem), nchol, D, max_N, max_elite};
    SERVE_TRY(launch_cem_tasks(t, s->stream));
  }
  for (const Bucket& b : buckets) {
    const ProjTaskLaunch t{reinterpret_cast<const ProjArgs*>(d + o_proj) + b.first,
                           reinterpret_cast<const int*>(d + o_pre) + b.pre,
                           b.count, b.blocks, dims, b.K, b.bf, b.lds};
    SERVE_TRY(launch_project_tasks(t, s->stream));
  }
  {
    const CemTaskLaunch t{reinterpret_cast<const CemArgs*>(d + o_cem) + nchol, n, D, max_N,
                          max_elite};
    SERVE_TRY(launch_cem_tasks(t, s->stream));
  }
  if (ngseg) {
    hipLaunchKernelGGL(seg_copy_kernel, dim3(ngseg), dim3(64), 0, s->stream,
                       reinterpret_cast<const Seg*>(d + o_gseg));
    SERVE_TRY(hipGetLastError());
    SERVE_TRY(hipMemcpyAsync(sl.hres, sl.dres, 4 * finishing.size() * (D + 2),
                             hipMemcpyDeviceToHost, s->stream));
  }
  return PRIEST_OK;
}

}  // namespace

extern "C" {

double priest_server_now(void) { return clock_now(); }

int32_t priest_server_create(const priest_server_config* cfg, void* stream, priest_server** out) {
  if (!out) return sfail(PRIEST_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!cfg) return sfail(PRIEST_ERR_INVALID, "config is NULL");
  if (cfg->dims != 2 && cfg->dims != 3) return sfail(PRIEST_ERR_INVALID, "dims must be 2 or 3");
  if (cfg->n_coeff < 2 || cfg->n_coeff > PRIEST_MAX_COEFF)
    return sfail(PRIEST_ERR_INVALID, "n_coeff must be in [2, 16]");
  if (cfg->max_active < 1 || cfg->max_active > kMaxActive)
    return sfail(PRIEST_ERR_INVALID, "max_active must be in [1, 8192]");
  if (cfg->max_robots < 1 || cfg->max_robots > kMaxRobots)
    return sfail(PRIEST_ERR_INVALID, "max_robots must be in [1, 65536]");
  if (cfg->max_inflight_steps < 1 || cfg->max_inflight_steps > kRing - 1)
    return sfail(PRIEST_ERR_INVALID, "max_inflight_steps must be 1 or 2");
  if (cfg->memory_budget < 4096) return sfail(PRIEST_ERR_INVALID, "memory_budget must be >= 4096");
  if (cfg->reserved != 0 || (cfg->dry_run != 0 && cfg->dry_run != 1))
    return sfail(PRIEST_ERR_INVALID, "reserved must be 0 and dry_run 0 or 1");
  if (!(cfg->sigma >= 0.0f && cfg->sigma <= 1.0f) || !(cfg->gamma > 0.0f) ||
      !std::isfinite(cfg->gamma) || !(cfg->cov_jitter >= 0.0f) || !std::isfinite(cfg->cov_jitter) ||
      !(cfg->init_std > 0.0f) || !std::isfinite(cfg->init_std))
    return sfail(PRIEST_ERR_INVALID, "bad sampling parameters");
  if (!(std::isfinite(cfg->rho) && cfg->rho >= 0) || !(cfg->v_max > 0) || !(cfg->a_max > 0) ||
      (cfg->bc_mask & ~63u) ||
      (cfg->precision != PRIEST_FP32 && cfg->precision != PRIEST_BF16_MIXED) ||
      cfg->n_refine_fp32 < 0)
    return sfail(PRIEST_ERR_INVALID, "bad problem settings");
  std::unique_ptr<priest_server> s(new priest_server());
  s->cfg = *cfg;
  s->stream = static_cast<hipStream_t>(stream);
  s->D = cfg->dims * cfg->n_coeff;
  s->dry = cfg->dry_run != 0;
  s->arena = Arena(cfg->memory_budget);
  s->robots.resize(cfg->max_robots);
  if (!s->dry) {
    const size_t D = s->D;
    bool ok = hipMalloc(reinterpret_cast<void**>(&s->arena_base), cfg->memory_budget) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&s->robot_mu), 4 * D * cfg->max_robots) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&s->robot_cov), 4 * D * D * cfg->max_robots) == hipSuccess;
    for (Slot& sl : s->slots) {
      const size_t rb = 4 * (D + 2) * static_cast<size_t>(cfg->max_active);
      ok = ok && hipHostMalloc(reinterpret_cast<void**>(&sl.hres), rb) == hipSuccess &&
           hipMalloc(reinterpret_cast<void**>(&sl.dres), rb) == hipSuccess;
    }
    if (!ok) {
      priest_server_destroy(s.release());
      return sfail(PRIEST_ERR_NOMEM, "device or pinned allocation failed");
    }
  }
  *out = s.release();
  return PRIEST_OK;
}

int32_t priest_server_prepare(priest_server* s, int32_t n_steps, int32_t n_obs, double horizon) {
  if (!s) return sfail(PRIEST_ERR_INVALID, "server is NULL");
  if (n_steps < 2 || n_steps > PRIEST_MAX_STEPS || n_obs < 0 || n_obs > PRIEST_MAX_OBS ||
      !(horizon > 0) || !std::isfinite(horizon))
    return sfail(PRIEST_ERR_INVALID, "invalid shape");
  if (s->dry) return PRIEST_OK;
  priest_problem* p = nullptr;
  return get_problem(s, n_steps, n_obs, horizon, &p);
}

int32_t priest_server_submit(priest_server* s, const priest_request* r, int64_t* id) {
  if (!s || !r || !id) return sfail(PRIEST_ERR_INVALID, "server, request and id are required");
  if (r->robot < 0 || r->robot >= s->cfg.max_robots) return sfail(PRIEST_ERR_INVALID, "unknown robot");
  if (r->n_steps < 2 || r->n_steps > PRIEST_MAX_STEPS || r->n_obs < 0 || r->n_obs > PRIEST_MAX_OBS ||
      r->n_samples < 1 || r->n_samples > 8192 || r->n_cem < 1 || r->n_proj_iters < 0 ||
      r->n_proj < 1 || r->n_proj > r->n_samples || r->n_elite < 1 || r->n_elite > r->n_proj ||
      r->warm_start < 0 || r->warm_start > 2 || !(r->horizon > 0) || !std::isfinite(r->horizon) ||
      !r->bc || (r->n_obs > 0 && !r->obs))
    return sfail(PRIEST_ERR_INVALID, "invalid request");
  const int nb = 6 * s->cfg.dims, no = 8 * r->n_obs;
  for (int i = 0; i < nb; ++i)
    if (!std::isfinite(r->bc[i])) return sfail(PRIEST_ERR_INVALID, "non-finite boundary value");
  for (int i = 0; i < no; ++i)
    if (!std::isfinite(r->obs[i])) return sfail(PRIEST_ERR_INVALID, "non-finite obstacle value");
  const size_t bytes = footprint(s->cfg.dims, s->D, *r);
  if (bytes > s->arena.cap()) return sfail(PRIEST_ERR_NOMEM, "request state exceeds the memory budget");
  std::unique_ptr<Req> q(new Req());
  q->r = *r;
  q->r.bc = nullptr;
  q->r.obs = nullptr;
  q->bc.assign(r->bc, r->bc + nb);
  q->obs.assign(r->obs, r->obs + no);
  q->bytes = bytes;
  q->id = s->next_id++;
  *id = q->id;
  s->pending.push_back(q.release());
  s->st.submitted += 1;
  return PRIEST_OK;
}

int32_t priest_server_step(priest_server* s, int32_t* n_active) {
  if (!s) return sfail(PRIEST_ERR_INVALID, "server is NULL");
  if (n_active) *n_active = 0;
  int32_t st = harvest(s, false);
  if (st != PRIEST_OK) return st;
  if (static_cast<int>(s->inflight.size()) >= s->cfg.max_inflight_steps) {
    st = harvest(s, true);
    if (st != PRIEST_OK) return st;
  }
  st = admit(s);
  if (st != PRIEST_OK) return st;
  const int n = static_cast<int>(s->active.size());
  if (n == 0) return PRIEST_OK;
  Step f;
  f.slot = s->ring;
  for (Req* q : s->active)
    if (q->iter + 1 >= q->r.n_cem) f.finishing.push_back(q);
  if (!s->dry) {
    st = launch_step(s, f.slot, f.finishing);
    if (st != PRIEST_OK) return st;
    if (s->event_pool.empty()) {
      hipEvent_t ev;
      SERVE_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      s->event_pool.push_back(ev);
    }
    f.ev = s->event_pool.back();
    s->event_pool.pop_back();
    SERVE_TRY(hipEventRecord(f.ev, s->stream));
  } else {
    for (Req* q : s->active) s->robots[q->r.robot].init = true;
  }
  // work on one stream is ordered: a finished request's arena block and its
  // robot can serve the next step's admissions
  std::vector<Req*> still;
  for (Req* q : s->active) {
    q->fresh = false;
    if (q->iter + 1 >= q->r.n_cem) {
      s->arena.release(q->off, q->bytes);
      s->robots[q->r.robot].busy = false;
    } else {
      q->iter += 1;
      still.push_back(q);
    }
  }
  s->active.swap(still);
  s->inflight.push_back(std::move(f));
  s->ring = (s->ring + 1) % kRing;
  s->st.steps += 1;
  if (n_active) *n_active = n;
  return PRIEST_OK;
}

int32_t priest_server_poll(priest_server* s, priest_result* out, int32_t max_results, int32_t* n) {
  if (!s || !n || max_results < 0 || (max_results > 0 && !out))
    return sfail(PRIEST_ERR_INVALID, "bad arguments");
  *n = 0;
  const int32_t st = harvest(s, false);
  if (st != PRIEST_OK) return st;
  int32_t k = 0;
  while (k < max_results && !s->done.empty()) {
    std::unique_ptr<Req> q(s->done.front());
    s->done.pop_front();
    priest_result& r = out[k++];
    std::memset(&r, 0, sizeof(r));
    r.request_id = q->id;
    r.robot = q->r.robot;
    r.status = q->status;
    r.arrival = q->r.arrival;
    r.t_admit = q->t_admit;
    r.t_done = q->t_done;
    r.best_cost = q->cost;
    for (size_t i = 0; i < q->best.size() && i < static_cast<size_t>(kMaxD); ++i)
      r.best_xi[i] = q->best[i];
  }
  *n = k;
  return PRIEST_OK;
}

int32_t priest_server_flush(priest_server* s) {
  if (!s) return sfail(PRIEST_ERR_INVALID, "server is NULL");
  while (!s->inflight.empty()) {
    const int32_t st = harvest(s, true);
    if (st != PRIEST_OK) return st;
  }
  return PRIEST_OK;
}

int32_t priest_server_counts(const priest_server* s, int32_t* pending, int32_t* active,
                             int32_t* inflight_steps) {
  if (!s) return sfail(PRIEST_ERR_INVALID, "server is NULL");
  if (pending) *pending = static_cast<int32_t>(s->pending.size());
  if (active) *active = static_cast<int32_t>(s->active.size());
  if (inflight_steps) *inflight_steps = static_cast<int32_t>(s->inflight.size());
  return PRIEST_OK;
}

int32_t priest_server_stats_get(const priest_server* s, priest_server_stats* out) {
  if (!s || !out) return sfail(PRIEST_ERR_INVALID, "bad arguments");
  *out = s->st;
  out->arena_used = static_cast<int64_t>(s->arena.used());
  out->arena_budget = static_cast<int64_t>(s->arena.cap());
  out->arena_high_water = static_cast<int64_t>(s->arena.high());
  return PRIEST_OK;
}

int32_t priest_server_robot_state(priest_server* s, int32_t robot, float* host_mu, float* host_cov) {
  if (!s || !host_mu || !host_cov) return sfail(PRIEST_ERR_INVALID, "bad arguments");
  if (robot < 0 || robot >= s->cfg.max_robots || !s->robots[robot].init)
    return sfail(PRIEST_ERR_INVALID, "robot has no state");
  if (s->dry) return PRIEST_OK;
  const size_t D = s->D;
  SERVE_TRY(hipStreamSynchronize(s->stream));
  SERVE_TRY(hipMemcpy(host_mu, s->robot_mu + robot * D, 4 * D, hipMemcpyDeviceToHost));
  SERVE_TRY(hipMemcpy(host_cov, s->robot_cov + robot * D * D, 4 * D * D, hipMemcpyDeviceToHost));
  return PRIEST_OK;
}

int32_t priest_server_destroy(priest_server* s) {
  if (!s) return PRIEST_OK;
  if (!s->dry) (void)hipStreamSynchronize(s->stream);
  for (auto& kv : s->problems) priest_free_problem(kv.second);
  for (Req* q : s->pending) delete q;
  for (Req* q : s->active) delete q;
  for (Req* q : s->done) delete q;
  for (Step& f : s->inflight) {
    // requests of an unfinished step are either still active (deleted
    // above) or finishing in it
    for (Req* q : f.finishing) delete q;
    if (f.ev) (void)hipEventDestroy(f.ev);
  }
  for (hipEvent_t ev : s->event_pool) (void)hipEventDestroy(ev);
  for (Slot& sl : s->slots) {
    if (sl.host) (void)hipHostFree(sl.host);
    if (sl.dev) (void)hipFree(sl.dev);
    if (sl.hres) (void)hipHostFree(sl.hres);
    if (sl.dres) (void)hipFree(sl.dres);
  }
  if (s->robot_mu) (void)hipFree(s->robot_mu);
  if (s->robot_cov) (void)hipFree(s->robot_cov);
  if (s->arena_base) (void)hipFree(s->arena_base);
  delete s;
  return PRIEST_OK;
}

}  // extern "C"
