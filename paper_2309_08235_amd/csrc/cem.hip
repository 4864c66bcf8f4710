// Selection, refit and covariance factorisation of the sampling loop (Alg. 1,
// eqs. (9a)-(9c)) on gfx950: one 1024-thread block per problem.
//
//   1. ConstraintEliteSet: the n_proj samples with the lowest residual r,
//      ordered by (r, index) - a bitonic sort of 64-bit keys in LDS;
//   2. EliteSet: the n_elite lowest c_aug = c1 + r among them, ties kept in
//      the order of step 1;
//   3. weights c_m = exp(-(c_aug_m - delta)/gamma), delta = min c_aug;
//   4. mu' = (1-sigma) mu + sigma sum w xi_bar / sum w,
//      Sigma' = (1-sigma) Sigma + sigma sum w (xi_bar - mu')(xi_bar - mu')^T / sum w;
//   5. L = chol(Sigma' + eps I), eps = cov_jitter tr(Sigma')/D, for the next draw.
// Every sum runs in a fixed order, so results are bitwise reproducible.
#include "priest_internal.h"

namespace priest {
namespace {

__host__ __device__ inline int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

__host__ __device__ inline size_t align16(size_t n) { return (n + 15) & ~static_cast<size_t>(15); }

struct CemLayout {
  size_t keys, proj, elite, w, red, mu, A, total;
};

__host__ __device__ inline CemLayout cem_layout(int N, int D, int n_proj, int n_elite) {
  CemLayout l{};
  size_t o = 0;
  l.keys = o;  o += align16(sizeof(uint64_t) * pow2_at_least(N > 1 ? N : 2));
  l.proj = o;  o += align16(sizeof(int) * (n_proj > 0 ? n_proj : 1));
  l.elite = o; o += align16(sizeof(int) * (n_elite > 0 ? n_elite : 1));
  l.w = o;     o += align16(sizeof(float) * (n_elite > 0 ? n_elite : 1));
  l.red = o;   o += align16(sizeof(float) * kCemThreads);
  l.mu = o;    o += align16(sizeof(float) * D);
  l.A = o;     o += align16(sizeof(float) * D * D);
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

__device__ void bitonic_sort(uint64_t* k, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < (n >> 1); i += blockDim.x) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const uint64_t x = k[lo], y = k[hi];
        if ((x > y) == asc) { k[lo] = y; k[hi] = x; }
      }
      __syncthreads();
    }
  }
}

// Deterministic block sum of v over threads (fixed tree).
__device__ float block_sum(float v, float* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const float r = red[0];
  __syncthreads();
  return r;
}

// In-place lower Cholesky of the D x D matrix A in LDS (right-looking).
// Returns false if a pivot is not positive and finite.
__device__ bool cholesky_lds(float* A, int D, float* red) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < D; ++j) {
    if (threadIdx.x == 0) {
      const float ajj = A[j * D + j];
      if (!(ajj > 0.0f) || !(ajj < 3.0e38f)) { bad = 1; A[j * D + j] = 1.0f; }
      else A[j * D + j] = sqrtf(ajj);
    }
    __syncthreads();
    const float ljj = A[j * D + j];
    for (int i = j + 1 + threadIdx.x; i < D; i += blockDim.x) A[i * D + j] /= ljj;
    __syncthreads();
    const int m = D - j - 1;
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
      const int i = j + 1 + e / m, c = j + 1 + e % m;
      if (c <= i) A[i * D + c] = fmaf(-A[i * D + j], A[c * D + j], A[i * D + c]);
    }
    __syncthreads();
  }
  (void)red;
  return bad == 0;
}

__global__ __launch_bounds__(kCemThreads) void cem_kernel(CemArgs a) {
  extern __shared__ float4 sm4[];
  char* sm = reinterpret_cast<char*>(sm4);
  const int prob = blockIdx.x;
  const int D = a.D, N = a.N, tid = threadIdx.x, T = blockDim.x;
  const CemLayout l = cem_layout(N, D, a.n_proj, a.n_elite);
  uint64_t* keys = reinterpret_cast<uint64_t*>(sm + l.keys);
  int* proj = reinterpret_cast<int*>(sm + l.proj);
  int* elite = reinterpret_cast<int*>(sm + l.elite);
  float* w = reinterpret_cast<float*>(sm + l.w);
  float* red = reinterpret_cast<float*>(sm + l.red);
  float* muN = reinterpret_cast<float*>(sm + l.mu);
  float* A = reinterpret_cast<float*>(sm + l.A);
  float* mu = a.mu + prob * a.mu_stride;
  float* cov = a.cov + prob * a.cov_stride;
  float* L = a.L + prob * a.L_stride;

  if (!a.chol_only) {
    const float* r = a.resid + prob * a.n_stride;
    const float* c1 = a.c1 + prob * a.n_stride;
    const float* xb = a.xb + prob * a.xb_stride;
    // 1. lowest residuals
    const int n1 = pow2_at_least(N > 1 ? N : 2);
    for (int i = tid; i < n1; i += T)
      keys[i] = (i < N) ? ((static_cast<uint64_t>(ordered_bits(r[i])) << 32) | static_cast<uint32_t>(i))
                        : ~0ull;
    __syncthreads();
    bitonic_sort(keys, n1);
    for (int i = tid; i < a.n_proj; i += T) {
      proj[i] = static_cast<int>(keys[i] & 0xffffffffu);
      if (a.proj_idx) a.proj_idx[prob * a.n_proj + i] = proj[i];
    }
    __syncthreads();
    // 2. lowest c_aug within them; ties keep the order of step 1
    const int n2 = pow2_at_least(a.n_proj > 1 ? a.n_proj : 2);
    for (int i = tid; i < n2; i += T) {
      if (i < a.n_proj) {
        const int s = proj[i];
        keys[i] = (static_cast<uint64_t>(ordered_bits(c1[s] + r[s])) << 32) | static_cast<uint32_t>(i);
      } else {
        keys[i] = ~0ull;
      }
    }
    __syncthreads();
    bitonic_sort(keys, n2);
    for (int m = tid; m < a.n_elite; m += T) {
      elite[m] = proj[keys[m] & 0xffffffffu];
      if (a.elite_idx) a.elite_idx[prob * a.n_elite + m] = elite[m];
    }
    __syncthreads();
    // 3. weights
    const int e0 = elite[0];
    const float delta = c1[e0] + r[e0];
    float part = 0.0f;
    for (int m = tid; m < a.n_elite; m += T) {
      const int s = elite[m];
      const float wm = expf(-((c1[s] + r[s]) - delta) / a.gamma);
      w[m] = wm;
    }
    __syncthreads();
    // fixed-order partial sums: thread t sums m = t, t+T, ...
    for (int m = tid; m < a.n_elite; m += T) part += w[m];
    const float sw = block_sum(part, red);
    const float inv_sw = 1.0f / sw;
    // 4a. mean
    for (int d = tid; d < D; d += T) {
      float s = 0.0f;
      for (int m = 0; m < a.n_elite; ++m) s = fmaf(w[m], xb[static_cast<int64_t>(elite[m]) * D + d], s);
      muN[d] = (1.0f - a.sigma) * mu[d] + a.sigma * (s * inv_sw);
    }
    __syncthreads();
    // 4b. covariance about the new mean (lower triangle, then mirrored)
    for (int e = tid; e < D * D; e += T) {
      const int i = e / D, j = e - i * D;
      if (j > i) continue;
      float s = 0.0f;
      const float mi = muN[i], mj = muN[j];
      for (int m = 0; m < a.n_elite; ++m) {
        const float* x = xb + static_cast<int64_t>(elite[m]) * D;
        s = fmaf(w[m] * (x[i] - mi), x[j] - mj, s);
      }
      const float v = (1.0f - a.sigma) * cov[e] + a.sigma * (s * inv_sw);
      A[i * D + j] = v;
      A[j * D + i] = v;
    }
    __syncthreads();
    for (int e = tid; e < D * D; e += T) cov[e] = A[e];
    for (int d = tid; d < D; d += T) {
      mu[d] = muN[d];
      a.best_xi[prob * a.best_stride + d] = xb[static_cast<int64_t>(e0) * D + d];
    }
    if (tid == 0) a.best_cost[prob] = delta;
    __syncthreads();
  } else {
    for (int e = tid; e < D * D; e += T) A[e] = cov[e];
    __syncthreads();
  }
  // 5. factor Sigma' + eps I
  float tr = 0.0f;
  for (int d = tid; d < D; d += T) tr += A[d * D + d];
  const float eps = a.cov_jitter * block_sum(tr, red) / static_cast<float>(D);
  for (int d = tid; d < D; d += T) A[d * D + d] += eps;
  __syncthreads();
  const bool ok = cholesky_lds(A, D, red);
  for (int e = tid; e < D * D; e += T) {
    const int i = e / D, j = e - i * D;
    L[e] = (j <= i) ? A[e] : 0.0f;
  }
  if (tid == 0 && a.status) {
    bool fin = ok;
    if (!a.chol_only) fin = fin && (a.best_cost[prob] == a.best_cost[prob]);
    if (!fin) a.status[prob] = PRIEST_ERR_NONFINITE;
  }
}

}  // namespace

size_t cem_lds_bytes(int N, int D, int n_elite) {
  return cem_layout(N, D, N, n_elite).total;
}

hipError_t launch_cem(const CemArgs& a, int n_problems, hipStream_t s) {
  const size_t lds = cem_layout(a.N, a.D, a.n_proj, a.n_elite).total;
  hipLaunchKernelGGL(cem_kernel, dim3(n_problems), dim3(kCemThreads), lds, s, a);
  return hipGetLastError();
}

}  // namespace priest
