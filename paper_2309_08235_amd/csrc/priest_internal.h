// Internal declarations shared by the HIP translation units of libpriest.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/priest.h"

namespace priest {

constexpr int kMaxNV = PRIEST_MAX_COEFF;
constexpr int kCemThreads = 512;

// Sample sources of the projection kernel.
enum SampleMode : int32_t {
  kFromInput = 0,   // xi read from xi_in
  kFromPhilox = 1,  // xi = mu + L z, z from Philox4x32-10 + Box-Muller
  kFromNoise = 2,   // xi = mu + L z, z read from `noise`
};

// Arguments of the fused projection kernel.  One launch covers
// n_problems * blocks_per_problem tiles; tile b works on problem
// b / blocks_per_problem, samples [tile*S, tile*S + S) of it.
// Workspace bounds s_min <= p <= s_max per axis (Appendix, G xi <= tau).
struct Box {
  int32_t on;
  float lo[3], hi[3];
};

// Trajectory cost of the final pass (priest_cost; kind 0 = sum ||a||^2).
struct CostArgs {
  int32_t kind;
  float w_acc, w_curv, w_path, w_steer, wheelbase, eps;
};

struct ProjArgs {
  int32_t dims, nv, K, M, N;
  int32_t S;                   // samples per block: 16 / axis_slots (x 16 waves for row_tiles 0)
  int32_t n_iter;              // projection iterations
  int32_t blocks_per_problem;  // ceil(N / S)
  int32_t axis_slots;          // MFMA columns per sample: 4, or 2 (2D only)
  int32_t row_tiles;           // 16-step time blocks per wave: 1 or 2; 0: the whole horizon
  int32_t persistent;          // 1: grid of resident blocks looping over tiles
  int32_t mode;                // SampleMode
  int32_t bf16_iters;          // leading iterations with BF16 MFMA operands (mixed precision)
  int32_t iter;                // CEM iteration (Philox counter word 2)
  uint32_t stream_base;        // Philox counter word 3 = stream_base + problem
  uint64_t seed;               // Philox key
  float rho, dt, vmax, amax;   // vmax/amax may be +inf
  // whole-horizon shape: coefficient displacement allowed per unit of slack
  // of the position (per axis), velocity and acceleration rows (Euclidean):
  // 1 / S_d, S_d = max_t sum_j |W_t,d,j|, times 1 / sqrt(dims) for d > 0
  float bscale[3];
  Box box;                     // workspace bounds (box.on = 0: none)
  int32_t traj;                // 1: obstacle rows are paths [K * dims] + (a, b)
  CostArgs cost;               // c1 of the final pass
  // problem constants (shared by all problems of the launch)
  const float* W;    // [K][3][nv] rows of P, Pdot, Pddot
  const float* M11;  // [nv][nv]
  const float* Pi;   // [nv][nv]  M11 Q
  const float* M12;  // [nv][6]
  // per-problem inputs (stride in floats between consecutive problems)
  const float* bc;  int64_t bc_stride;
  const float* obs; int64_t obs_stride;
  const float* xi_in; int64_t xi_in_stride;
  const float* mu; int64_t mu_stride;
  const float* L; int64_t L_stride;
  const float* noise; int64_t noise_stride;
  // outputs
  float* xi_out; int64_t xi_out_stride;    // [N][D] per problem, required
  float* resid; float* c1; int64_t n_stride;  // [N] per problem, nullable
  float* xi_src; int64_t xi_src_stride;    // drawn samples, nullable
  // optional second copies (caller outputs, dense [problem][N] / [problem][N][D])
  float* resid2; float* c12; float* xi_out2;
  // profiling: (item, obstacle) pairs evaluated after culling, summed over
  // the launch (nullable)
  unsigned long long* pair_count;
  // per-iteration residual history [n_iter][N] (nullable; default shape, one
  // problem)
  float* resid_hist;
  // whole-horizon shape drawing sample groups (persistent = 1): with these
  // set, the launch first writes every problem's obstacle records to `grec`
  // (3 M float4 per problem, stride in floats) and clears the group counter
  // `gq`, and the waves of a grid of resident blocks draw (problem, group)
  // pairs from it; nullable (then each block draws from a counter in LDS)
  float* grec; int64_t grec_stride;
  int32_t* gq;
};

// Arguments of the selection / refit / Cholesky kernel (one block per problem).
struct CemArgs {
  int32_t D, N, n_proj, n_elite;
  int32_t chol_only;     // 1: only L = chol(cov + eps I)
  float sigma, gamma, cov_jitter;
  const float* xb;  int64_t xb_stride;     // projected samples [N][D]
  const float* resid; const float* c1; int64_t n_stride;
  float* mu; int64_t mu_stride;            // in/out
  float* cov; int64_t cov_stride;          // in/out
  float* L; int64_t L_stride;              // out: chol(cov' + eps I)
  float* best_xi; int64_t best_stride;     // [D]
  float* best_cost;                        // [1] per problem
  int32_t* elite_idx; int32_t* proj_idx;   // nullable
  int32_t* status;                         // nullable, [1] per problem
  int32_t rule;                            // 0: eqs. (9a)-(9c); 1: CMA-ES-style covariance
  int32_t first;                           // 1: the evolution path starts at zero
  float* pc; int64_t pc_stride;            // evolution path [D] per problem (rule 1)
};

// Launch descriptions of the descriptor-table kernels (serving path): all
// tasks of one projection launch share dims and n_steps; `tasks`/`prefix`
// are device arrays (prefix[t] = first block of task t, prefix[n] = n_blocks).
struct ProjTaskLaunch {
  const ProjArgs* tasks;
  const int* prefix;
  int n_tasks, n_blocks, dims, K;
  bool bf16;
  size_t lds_bytes;
};
struct CemTaskLaunch {
  const CemArgs* tasks;
  int n_tasks, D, max_N, max_elite;
};

// host-side launchers (defined in the .hip files)
hipError_t launch_project_tasks(const ProjTaskLaunch& t, hipStream_t s);
hipError_t launch_cem_tasks(const CemTaskLaunch& t, hipStream_t s);
size_t project_lds_bytes(const ProjArgs& a);
// row_tiles 0: one wave owns a sample group over the whole horizon (K <= 128)
bool tiling_valid(int dims, int axis_slots, int row_tiles, int K);
int samples_per_block(const ProjArgs& a);  // from a's tile shape and problem size
int project_threads(int K, int row_tiles);
void set_default_tiling(ProjArgs& a);  // 4 axis slots, 1 time block per wave, not persistent
// start / stop: optional events that receive the kernel's own start and end
// times (hipExtLaunchKernel), for profiling without marker commands.
hipError_t launch_project(const ProjArgs& a, int n_problems, hipStream_t s,
                          hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
size_t cem_lds_bytes(int N, int D, int n_elite);
hipError_t launch_cem(const CemArgs& a, int n_problems, hipStream_t s);
hipError_t launch_pick_best(int G, int D, const float* xi, const float* cost, float* best_xi,
                            float* best_cost, int32_t* best_group, hipStream_t s);
hipError_t launch_kkt(const double* Q, const double* A, int nv, int E, const int* rowsel,
                      double* out64, float* M11, float* Pi, float* M12, int* flag,
                      hipStream_t s);
hipError_t launch_debug_offsets(const ProjArgs& a, const float* xi, float* out, hipStream_t s);
hipError_t launch_debug_normals(uint64_t seed, uint32_t stream_id, int iter, int N, int D,
                                float* z, hipStream_t s);

// Tile shape of the projection kernel (tune.hip)
struct TileCfg {
  int axis_slots, row_tiles, persistent;
};
std::vector<TileCfg> tile_candidates(int dims, int K);  // [0] is the default shape
void apply_tiling(ProjArgs& a, const TileCfg& t);
// Times every candidate on `trial` (whose outputs must be safe to overwrite);
// ms[i] < 0 marks a candidate that does not fit.  Synchronises s.
hipError_t time_tilings(const ProjArgs& trial, int n_problems, size_t lds_limit, hipStream_t s,
                        const std::vector<TileCfg>& cands, std::vector<float>* ms);
int pick_tiling(const std::vector<float>& ms);

// Unfused projection (unfused.hip): workspace layout in bytes and launcher.
struct UnfusedLayout {
  size_t pva, delta, r2, xb, lam, w16, cen, g, total;
};
UnfusedLayout unfused_layout(int N, int K, int dims, int nv, int M);
hipError_t launch_unfused(const ProjArgs& a, const float* xi_in, float* xi_out, float* resid,
                          float* c1, char* ws, hipStream_t s);

// api.hip services used by the serving runtime
#define PRIEST_HIDDEN __attribute__((visibility("hidden")))
PRIEST_HIDDEN int32_t set_error(int32_t code, const char* msg);
PRIEST_HIDDEN ProjArgs problem_args(const priest_problem* p);
PRIEST_HIDDEN int problem_bf16_iters(const priest_problem* p, int n_iter);
PRIEST_HIDDEN int32_t problem_check_lds(const priest_problem* p, const ProjArgs& a);

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the Philox S-P network
// with multipliers 0xD2511F53 / 0xCD9E8D57 and Weyl key increments
// 0x9E3779B9 / 0xBB67AE85.
// ---------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t lo0 = 0xD2511F53u * c.x;
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

// (x >> 9 + 1/2) * 2^-23: an open-interval uniform that FP32 holds exactly.
__device__ __forceinline__ float open_uniform(uint32_t x) {
  return (static_cast<float>(x >> 9) + 0.5f) * 1.1920928955078125e-07f;
}

// Four standard normals of counter (i, q, iter, stream) by Box-Muller on
// word pairs (0,1) and (2,3).
__device__ __forceinline__ void philox_normals4(uint64_t seed, uint32_t i, uint32_t q,
                                                uint32_t iter, uint32_t stream, float z[4]) {
  const U4 w = philox10(U4{i, q, iter, stream}, static_cast<uint32_t>(seed),
                        static_cast<uint32_t>(seed >> 32));
  const uint32_t words[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const float u1 = open_uniform(words[2 * p]);
    const float u2 = open_uniform(words[2 * p + 1]);
    const float rad = sqrtf(-2.0f * logf(u1));
    float sn, cs;
    sincospif(2.0f * u2, &sn, &cs);
    z[2 * p] = rad * cs;
    z[2 * p + 1] = rad * sn;
  }
}

}  // namespace priest
