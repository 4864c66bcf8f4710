// Selection, refit and covariance factorisation of the sampling loop (Alg. 1,
// eqs. (9a)-(9c)) on gfx950: one 512-thread block per problem.
//
//   1. ConstraintEliteSet: the n_proj samples with the lowest residual r,
//      ordered by (r, index) - a stable block radix sort of the order-
//      preserving bit patterns of r (ties keep index order);
//   2. EliteSet: the n_elite lowest c_aug = c1 + r among them, ties kept in
//      the order of step 1 (second stable radix sort, on positions);
//   3. weights c_m = exp(-(c_aug_m - delta)/gamma), delta = min c_aug;
//   4. mu' = (1-sigma) mu + sigma sum w xi_bar / sum w,
//      Sigma' = (1-sigma) Sigma + sigma sum w (xi_bar - mu')(xi_bar - mu')^T / sum w;
//   5. L = chol(Sigma' + eps I), eps = cov_jitter tr(Sigma')/D, for the next
//      draw: one wave, lane i holds row i in registers.
// Every sum runs in a fixed order, so results are bitwise reproducible.
#include "priest_internal.h"

#include <hipcub/block/block_radix_sort.hpp>

// Phase markers (no-ops unless a profiling build defines them).
#ifndef PRIEST_CEM_MARK
#define PRIEST_CEM_MARK(i)
#endif

namespace priest {
namespace {

constexpr int kStageFloats = 4096;  // elite rows staged in LDS per chunk

__host__ __device__ inline size_t align16(size_t n) { return (n + 15) & ~static_cast<size_t>(15); }

struct CemLayout {
  size_t proj, elite, w, red, mu, pc, A, stage, total;
};

__host__ __device__ inline CemLayout cem_layout(int D, int n_proj, int n_elite) {
  CemLayout l{};
  size_t o = 0;
  l.proj = o;  o += align16(sizeof(int) * (n_proj > 0 ? n_proj : 1));
  l.elite = o; o += align16(sizeof(int) * (n_elite > 0 ? n_elite : 1));
  l.w = o;     o += align16(sizeof(float) * (n_elite > 0 ? n_elite : 1));
  l.red = o;   o += align16(sizeof(float) * 64);
  l.mu = o;    o += align16(sizeof(float) * D);
  l.pc = o;    o += align16(sizeof(float) * D);
  l.A = o;     o += align16(sizeof(float) * D * D);
  l.stage = o; o += align16(sizeof(float) * kStageFloats);
  l.total = o;
  return l;
}

// Order-preserving map float -> uint32 (NaN ranks as +inf, -0 as +0).
__device__ __forceinline__ uint32_t ordered_bits(float v) {
  if (v != v) v = __int_as_float(0x7f800000);
  if (v == 0.0f) v = 0.0f;
  const uint32_t u = __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ float bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Lower Cholesky of the D x D matrix A (LDS) by one wave, rows padded to DM
// with the identity; lane i keeps row i in registers.  Column j of L is
// broadcast lane by lane with readlane (lane c holds L[c][j], which the
// update of entry c of every row needs), so the factorisation touches LDS
// only to load A and store L.  Writes L back into A (lower triangle).
// Returns false if a pivot is not positive and finite (it is replaced by 1).
template <int DM>
__device__ bool cholesky_wave(float* A, int D, int lane, float* /*col*/) {
  float row[DM];
#pragma unroll
  for (int c = 0; c < DM; ++c)
    row[c] = (lane < D && c < D) ? A[lane * D + c] : (lane == c ? 1.0f : 0.0f);
  bool bad = false;
#pragma unroll
  for (int j = 0; j < DM; ++j) {
    const float piv = bcast(row[j], j);
    const bool b = !(piv > 0.0f) || !(piv < 3.0e38f);
    bad = bad || b;
    // one reciprocal square root per column: l_jj = piv * rsq(piv),
    // l_ij = a_ij * rsq(piv)
    const float inv = b ? 1.0f : __builtin_amdgcn_rsqf(piv);
    const float ljj = b ? 1.0f : piv * inv;
    const float lij = (lane > j) ? row[j] * inv : ((lane == j) ? ljj : row[j]);
    row[j] = lij;
#pragma unroll
    for (int c = j + 1; c < DM; ++c) row[c] = fmaf(-lij, bcast(lij, c), row[c]);
  }
  if (lane < D) {
#pragma unroll
    for (int c = 0; c < DM; ++c)
      if (c <= lane && c < D) A[lane * D + c] = row[c];
  }
  return !bad;
}

using f4 = __attribute__((ext_vector_type(4))) float;

__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Stable selection of the k smallest keys among n (n <= T * IPT): writes the
// values of ranks 0..k-1 to out[] in ascending (key, input position) order.
template <int IPT>
__device__ void select_sorted(const uint32_t* keys_in, const int* vals_in, int n, int k,
                              int* out, void* temp) {
  using Sort = hipcub::BlockRadixSort<uint32_t, kCemThreads, IPT, int>;
  uint32_t key[IPT];
  int val[IPT];
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const int e = threadIdx.x * IPT + i;
    key[i] = (e < n) ? keys_in[e] : 0xffffffffu;
    val[i] = (e < n) ? vals_in[e] : -1;
  }
  Sort(*reinterpret_cast<typename Sort::TempStorage*>(temp)).Sort(key, val);
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const int rnk = threadIdx.x * IPT + i;
    if (rnk < k) out[rnk] = val[i];
  }
}

// One block's work: selection, refit and factorisation for problem `prob`
// of `a`.  Shared by the uniform-batch kernel and the descriptor-table kernel.
template <int IPT, int DM>
__device__ __forceinline__ void cem_block(const CemArgs& a, int prob) {
  using Sort = hipcub::BlockRadixSort<uint32_t, kCemThreads, IPT, int>;
  __shared__ typename Sort::TempStorage sort_tmp;
  __shared__ uint32_t skey[kCemThreads * IPT];
  __shared__ int sval[kCemThreads * IPT];
  extern __shared__ float4 sm4[];
  char* sm = reinterpret_cast<char*>(sm4);
  const int D = a.D, N = a.N, tid = threadIdx.x, T = blockDim.x;
  const CemLayout l = cem_layout(D, a.n_proj, a.n_elite);
  int* proj = reinterpret_cast<int*>(sm + l.proj);
  int* elite = reinterpret_cast<int*>(sm + l.elite);
  float* w = reinterpret_cast<float*>(sm + l.w);
  float* red = reinterpret_cast<float*>(sm + l.red);
  float* muN = reinterpret_cast<float*>(sm + l.mu);
  float* pcN = reinterpret_cast<float*>(sm + l.pc);
  float* A = reinterpret_cast<float*>(sm + l.A);
  float* mu = a.mu + prob * a.mu_stride;
  float* cov = a.cov + prob * a.cov_stride;
  float* L = a.L + prob * a.L_stride;
  PRIEST_CEM_MARK(0);

  if (!a.chol_only) {
    const float* r = a.resid + prob * a.n_stride;
    const float* c1 = a.c1 + prob * a.n_stride;
    const float* xb = a.xb + prob * a.xb_stride;
    // 1. lowest residuals
    for (int i = tid; i < N; i += T) {
      skey[i] = ordered_bits(r[i]);
      sval[i] = i;
    }
    __syncthreads();
    select_sorted<IPT>(skey, sval, N, a.n_proj, proj, &sort_tmp);
    __syncthreads();
    PRIEST_CEM_MARK(1);
    for (int i = tid; i < a.n_proj; i += T)
      if (a.proj_idx) a.proj_idx[prob * a.n_proj + i] = proj[i];
    // 2. lowest c_aug within them; ties keep the order of step 1
    for (int i = tid; i < a.n_proj; i += T) {
      const int s = proj[i];
      skey[i] = ordered_bits(c1[s] + r[s]);
      sval[i] = i;
    }
    __syncthreads();
    select_sorted<IPT>(skey, sval, a.n_proj, a.n_elite, elite, &sort_tmp);
    __syncthreads();
    for (int m = tid; m < a.n_elite; m += T) {
      elite[m] = proj[elite[m]];
      if (a.elite_idx) a.elite_idx[prob * a.n_elite + m] = elite[m];
    }
    __syncthreads();
    PRIEST_CEM_MARK(2);
    // 3. weights; fixed-order sum by the first wave
    const int e0 = elite[0];
    const float delta = c1[e0] + r[e0];
    for (int m = tid; m < a.n_elite; m += T) {
      const int s = elite[m];
      w[m] = expf(-((c1[s] + r[s]) - delta) / a.gamma);
    }
    __syncthreads();
    if (tid < 64) {
      float part = 0.0f, part2 = 0.0f;
      for (int m = tid; m < a.n_elite; m += 64) {
        part += w[m];
        part2 = fmaf(w[m], w[m], part2);
      }
      part = wave_sum(part);
      part2 = wave_sum(part2);
      if (tid == 0) {
        red[0] = part;
        red[1] = part2;
      }
    }
    __syncthreads();
    const float inv_sw = 1.0f / red[0];
    // CMA-ES-style rates (rule 1): variance-effective selection mass and the
    // default learning rates for dimension n = D
    float cc = 0.0f, c1r = 0.0f, cmu = 0.0f, mu_eff = 1.0f;
    if (a.rule == 1) {
      const float n = static_cast<float>(D);
      mu_eff = red[0] * red[0] / red[1];
      cc = (4.0f + mu_eff / n) / (n + 4.0f + 2.0f * mu_eff / n);
      c1r = 2.0f / ((n + 1.3f) * (n + 1.3f) + mu_eff);
      cmu = fminf(1.0f - c1r, 2.0f * (mu_eff - 2.0f + 1.0f / mu_eff) / ((n + 2.0f) * (n + 2.0f) + mu_eff));
    }
    PRIEST_CEM_MARK(3);
    // 4. mean and covariance from elite rows staged in LDS, CH rows at a time
    float* stage = reinterpret_cast<float*>(sm + l.stage);
    const int CH = kStageFloats / D;
    const bool one_chunk = a.n_elite <= CH;
    auto stage_rows = [&](int m0, int nm) {
      for (int i = tid; i < nm * D; i += T) {
        const int m = i / D;
        stage[i] = xb[static_cast<int64_t>(elite[m0 + m]) * D + (i - m * D)];
      }
    };
    // mean: coefficient d gets 4 partial sums (elites m = part mod 4), added
    // in a fixed order; the partials live in A until the covariance is written
    float macc = 0.0f;
    const int part = tid / D, md = tid - part * D;
    for (int m0 = 0; m0 < a.n_elite; m0 += CH) {
      const int nm = min(CH, a.n_elite - m0);
      stage_rows(m0, nm);
      __syncthreads();
      if (part < 4) {
        for (int m = part; m < nm; m += 4) macc = fmaf(w[m0 + m], stage[m * D + md], macc);
      }
      if (!one_chunk) __syncthreads();
    }
    if (part < 4) A[tid] = macc;
    __syncthreads();
    if (tid < D) {
      const float sm4 = (A[tid] + A[D + tid]) + (A[2 * D + tid] + A[3 * D + tid]);
      const float mw = sm4 * inv_sw;
      muN[tid] = (1.0f - a.sigma) * mu[tid] + a.sigma * mw;
      if (a.rule == 1) {
        const float p0 = a.first ? 0.0f : a.pc[prob * a.pc_stride + tid];
        pcN[tid] = fmaf(sqrtf(cc * (2.0f - cc) * mu_eff), mw - mu[tid], (1.0f - cc) * p0);
      }
    }
    __syncthreads();
    PRIEST_CEM_MARK(4);
    // covariance about the new mean, sum_m w_m (x_m - mu')(x_m - mu')^T (rule
    // 1: about the current mean), on MFMA 16x16x4: wave v computes
    // lower-triangle tile v of the ceil(D/16)^2 tiles, elites four at a time
    // (two accumulation chains, added at the end)
    const float* cen = (a.rule == 1) ? mu : muN;
    const int wv = tid >> 6, lane = tid & 63;
    const int nt = (D + 15) / 16;
    int ti = 0, tj = 0;
    {
      int v = wv;
      while (ti < nt && v > ti) {
        v -= ti + 1;
        ++ti;
      }
      tj = v;
    }
    const bool owner = ti < nt;
    f4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = acc0;
    for (int m0 = 0; m0 < a.n_elite; m0 += CH) {
      const int nm = min(CH, a.n_elite - m0);
      if (!one_chunk) {
        stage_rows(m0, nm);
        __syncthreads();
      }
      if (owner) {
        const int ii = ti * 16 + (lane & 15), jj = tj * 16 + (lane & 15);
        const float mi = ii < D ? cen[ii] : 0.0f, mj = jj < D ? cen[jj] : 0.0f;
        for (int s4 = 0; s4 < nm; s4 += 8) {
          const int ma = s4 + (lane >> 4), mb = ma + 4;
          const float av0 = (ma < nm && ii < D) ? w[m0 + ma] * (stage[ma * D + ii] - mi) : 0.0f;
          const float bv0 = (ma < nm && jj < D) ? stage[ma * D + jj] - mj : 0.0f;
          const float av1 = (mb < nm && ii < D) ? w[m0 + mb] * (stage[mb * D + ii] - mi) : 0.0f;
          const float bv1 = (mb < nm && jj < D) ? stage[mb * D + jj] - mj : 0.0f;
          acc0 = mfma(av0, bv0, acc0);
          acc1 = mfma(av1, bv1, acc1);
        }
      }
      if (!one_chunk) __syncthreads();
    }
    if (owner) {
      const f4 acc = acc0 + acc1;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = ti * 16 + 4 * (lane >> 4) + r, j = tj * 16 + (lane & 15);
        if (i < D && j < D && i >= j) {
          float v;
          if (a.rule == 1)
            v = fmaf(cmu, acc[r] * inv_sw,
                     fmaf(c1r, pcN[i] * pcN[j], (1.0f - c1r - cmu) * cov[i * D + j]));
          else
            v = (1.0f - a.sigma) * cov[i * D + j] + a.sigma * (acc[r] * inv_sw);
          A[i * D + j] = v;
          A[j * D + i] = v;
        }
      }
    }
    __syncthreads();
    for (int e = tid; e < D * D; e += T) cov[e] = A[e];
    for (int d = tid; d < D; d += T) {
      mu[d] = muN[d];
      if (a.rule == 1) a.pc[prob * a.pc_stride + d] = pcN[d];
      a.best_xi[prob * a.best_stride + d] = xb[static_cast<int64_t>(e0) * D + d];
    }
    if (tid == 0) a.best_cost[prob] = delta;
    __syncthreads();
    PRIEST_CEM_MARK(5);
  } else {
    for (int e = tid; e < D * D; e += T) A[e] = cov[e];
    __syncthreads();
  }
  // 5. factor Sigma' + eps I (first wave)
  if (tid < 64) {
    float tr = 0.0f;
    for (int d = tid; d < D; d += 64) tr += A[d * D + d];
    tr = wave_sum(tr);
    const float eps = a.cov_jitter * tr / static_cast<float>(D);
    for (int d = tid; d < D; d += 64) A[d * D + d] += eps;
    const bool ok = cholesky_wave<DM>(A, D, tid, red);
    if (tid == 0 && a.status) {
      bool fin = ok;
      if (!a.chol_only) fin = fin && (a.best_cost[prob] == a.best_cost[prob]);
      if (!fin) a.status[prob] = PRIEST_ERR_NONFINITE;
    }
  }
  __syncthreads();
  PRIEST_CEM_MARK(6);
  for (int e = tid; e < D * D; e += T) {
    const int i = e / D, j = e - i * D;
    L[e] = (j <= i) ? A[e] : 0.0f;
  }
  PRIEST_CEM_MARK(7);
}

template <int IPT, int DM>
__global__ __launch_bounds__(kCemThreads) void cem_kernel(CemArgs a) {
  cem_block<IPT, DM>(a, blockIdx.x);
}

// Descriptor table: block t handles task t with its own arguments.
template <int IPT, int DM>
__global__ __launch_bounds__(kCemThreads) void cem_task_kernel(const CemArgs* tasks) {
  cem_block<IPT, DM>(tasks[blockIdx.x], 0);
}

}  // namespace

size_t cem_lds_bytes(int N, int D, int n_elite) {
  return cem_layout(D, N, n_elite).total;
}

template <int DM>
static void launch_dm(const CemArgs& a, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
  if (a.N <= kCemThreads * 2) hipLaunchKernelGGL((cem_kernel<2, DM>), grid, block, lds, s, a);
  else if (a.N <= kCemThreads * 4) hipLaunchKernelGGL((cem_kernel<4, DM>), grid, block, lds, s, a);
  else hipLaunchKernelGGL((cem_kernel<16, DM>), grid, block, lds, s, a);
}

template <int DM>
static void launch_task_dm(const CemTaskLaunch& t, size_t lds, hipStream_t s) {
  const dim3 grid(t.n_tasks), block(kCemThreads);
  if (t.max_N <= kCemThreads * 2) hipLaunchKernelGGL((cem_task_kernel<2, DM>), grid, block, lds, s, t.tasks);
  else if (t.max_N <= kCemThreads * 4) hipLaunchKernelGGL((cem_task_kernel<4, DM>), grid, block, lds, s, t.tasks);
  else hipLaunchKernelGGL((cem_task_kernel<16, DM>), grid, block, lds, s, t.tasks);
}

hipError_t launch_cem_tasks(const CemTaskLaunch& t, hipStream_t s) {
  const size_t lds = cem_layout(t.D, t.max_N, t.max_elite).total;
  if (t.D <= 24) launch_task_dm<24>(t, lds, s);
  else if (t.D <= 36) launch_task_dm<36>(t, lds, s);
  else launch_task_dm<48>(t, lds, s);
  return hipGetLastError();
}

// D-PRIEST pick: the group with the lowest final cost (NaN ranks last, ties
// go to the lower group index) and a copy of its best trajectory.
__global__ void pick_best_kernel(int G, int D, const float* xi, const float* cost, float* best_xi,
                                 float* best_cost, int32_t* best_group) {
  __shared__ int sb;
  if (threadIdx.x == 0) {
    int b = 0;
    float bc = cost[0];
    if (bc != bc) bc = INFINITY;
    for (int g = 1; g < G; ++g) {
      float c = cost[g];
      if (c != c) c = INFINITY;
      if (c < bc) {
        bc = c;
        b = g;
      }
    }
    sb = b;
    best_cost[0] = cost[b];
    best_group[0] = b;
  }
  __syncthreads();
  for (int d = threadIdx.x; d < D; d += blockDim.x) best_xi[d] = xi[static_cast<int64_t>(sb) * D + d];
}

hipError_t launch_pick_best(int G, int D, const float* xi, const float* cost, float* best_xi,
                            float* best_cost, int32_t* best_group, hipStream_t s) {
  hipLaunchKernelGGL(pick_best_kernel, dim3(1), dim3(64), 0, s, G, D, xi, cost, best_xi, best_cost,
                     best_group);
  return hipGetLastError();
}

hipError_t launch_cem(const CemArgs& a, int n_problems, hipStream_t s) {
  const size_t lds = cem_layout(a.D, a.n_proj, a.n_elite).total;
  const dim3 grid(n_problems), block(kCemThreads);
  // covariance factor rows padded to 24 / 36 / 48 (identity padding)
  if (a.D <= 24) launch_dm<24>(a, grid, block, lds, s);
  else if (a.D <= 36) launch_dm<36>(a, grid, block, lds, s);
  else launch_dm<48>(a, grid, block, lds, s);
  return hipGetLastError();
}

}  // namespace priest
