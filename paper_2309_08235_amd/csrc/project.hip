// Fused projection sweep for gfx950.
//
// One block owns a tile of S samples of one problem for the whole projection:
// the samples' coefficient vectors (xi, xi_bar, lambda), the basis rows and
// the obstacle table stay in LDS across all iterations, so HBM is touched only
// to load the tile and write the result.  Per iteration (Appendix, eqs.
// (15a)-(15g), rewritten for per-sample batching):
//
//   phase 1  (sample, t) items: p, v, a = rows of [P; Pdot; Pddot] xi_bar;
//            closed-form alpha/beta/d of every obstacle as a push-out
//            delta_o = Delta * max(0, 1/n - 1) (n = scaled distance), summed
//            over obstacles; velocity / acceleration push-outs
//            delta = w * min(0, w_max/|w| - 1)            -> LDS
//   phase 2  right-hand side g = P^T S_o + Pdot^T delta_v + Pddot^T delta_a
//            (= F^T (e^{k+1} - F xi_bar^k), obstacle sum taken first)
//   phase 3  multiplier lambda += rho g (eq. (15e)) and the QP of eq. (15g)
//            through the fixed KKT block:
//              k = 0 : xi_bar = Pi xi + c0 + M11 (lambda + rho g)
//              k > 0 : xi_bar += M11 (xi - xi_bar + lambda + rho g)
//            The k > 0 form equals M11 eta + M12 b whenever A xi_bar = b,
//            which holds after the first step, and avoids cancelling
//            n_obs |p| against rho F^T F xi_bar in FP32.
//
// After the last iteration one more phase 1 evaluates r(xi_bar) and the
// smoothness cost c1 = sum_t |a_t|^2 with fixed-order (deterministic) sums.
#include "priest_internal.h"

namespace priest {
namespace {

struct Layout {  // offsets into dynamic LDS, in floats
  int W, obs, ab, M11, Pi, c0, X, Xb, Lam, U, Delta, G, mu, L, Z, total;
};

__host__ __device__ inline int round4(int n) { return (n + 3) & ~3; }

__host__ __device__ inline Layout layout(int dims, int nv, int K, int M, int S, int G, int mode) {
  Layout l{};
  int o = 0;
  const int D = dims * nv;
  l.W = o;   o += round4(K * 3 * nv);
  l.obs = o; o += round4(M * 8);
  l.ab = o;  o += round4(M * 2);
  l.M11 = o; o += round4(nv * nv);
  l.Pi = o;  o += round4(nv * nv);
  l.c0 = o;  o += round4(D);
  l.X = o;   o += round4(S * D);
  l.Xb = o;  o += round4(S * D);
  l.Lam = o; o += round4(S * D);
  l.U = o;   o += round4(S * D);
  // scratch: delta (phase 1/2) and partial sums (phase 2); the sampler's mu,
  // L and z alias it before the first iteration
  const int delta = round4(S * K * 3 * dims);
  const int part = round4(G * S * D);
  int scratch = delta + part;
  const int samp = round4(D) + round4(D * D) + round4(S * round4(D));
  if (mode != kFromInput && samp > scratch) scratch = samp;
  l.Delta = o;
  l.G = o + delta;
  l.mu = o;
  l.L = o + round4(D);
  l.Z = o + round4(D) + round4(D * D);
  o += scratch;
  l.total = o;
  return l;
}

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// Push-out of one obstacle at one instant (eqs. (15a)-(15c) -> (13)):
// target - position = Delta * (max(1,n)/n - 1), n^2 = (dx^2+dy^2)/a^2 + dz^2/b^2.
// A zero offset takes the canonical direction (+x in 2D, +z in 3D).
template <int DIMS>
__device__ __forceinline__ bool obstacle_push(const float* o, const float* ab, float tt,
                                              const float p[DIMS], float d[DIMS]) {
  // o = (cx, cy, cz, vx, vy, vz, 1/a^2, 1/b^2)
  d[0] = p[0] - fmaf(o[3], tt, o[0]);
  d[1] = p[1] - fmaf(o[4], tt, o[1]);
  float q = (d[0] * d[0] + d[1] * d[1]) * o[6];
  if (DIMS == 3) {
    d[2] = p[2] - fmaf(o[5], tt, o[2]);
    q = fmaf(d[2] * d[2], o[7], q);
  }
  if (!(q < 1.0f)) return false;
  if (q > 0.0f) {
    const float f = rsq(q) - 1.0f;
#pragma unroll
    for (int ax = 0; ax < DIMS; ++ax) d[ax] *= f;
  } else {
#pragma unroll
    for (int ax = 0; ax < DIMS; ++ax) d[ax] = 0.0f;
    if (DIMS == 3) d[DIMS - 1] = ab[1];
    else d[0] = ab[0];
  }
  return true;
}

// Push-out of a norm bound |w| <= wmax (eqs. (11a)/(11b)).
template <int DIMS>
__device__ __forceinline__ float bound_push(const float w[DIMS], float wmax, float d[DIMS]) {
  float ww = 0.0f;
#pragma unroll
  for (int ax = 0; ax < DIMS; ++ax) ww = fmaf(w[ax], w[ax], ww);
  float f = 0.0f;
  if (ww > wmax * wmax) f = wmax * rsq(ww) - 1.0f;
#pragma unroll
  for (int ax = 0; ax < DIMS; ++ax) d[ax] = w[ax] * f;
  return ww * f * f;
}

template <int DIMS, int NVT>
__device__ __forceinline__ void eval_row(const float* w, const float* xb, int nv_rt,
                                         float p[DIMS], float v[DIMS], float acc[DIMS]) {
  const int nv = NVT ? NVT : nv_rt;
#pragma unroll
  for (int ax = 0; ax < DIMS; ++ax) {
    float sp = 0.0f, sv = 0.0f, sa = 0.0f;
    const float* x = xb + ax * nv;
#pragma unroll
    for (int c = 0; c < (NVT ? NVT : kMaxNV); ++c) {
      if (!NVT && c >= nv) break;
      const float xc = x[c];
      sp = fmaf(w[c], xc, sp);
      sv = fmaf(w[nv + c], xc, sv);
      sa = fmaf(w[2 * nv + c], xc, sa);
    }
    p[ax] = sp; v[ax] = sv; acc[ax] = sa;
  }
}

template <int DIMS, int NVT>
__global__ __launch_bounds__(kProjectThreads) void project_kernel(ProjArgs a) {
  extern __shared__ float4 sm4[];
  float* sm = reinterpret_cast<float*>(sm4);
  const int nv = NVT ? NVT : a.nv;
  const int K = a.K, M = a.M, S = a.S, G = a.G;
  const int D = DIMS * nv;
  const Layout l = layout(DIMS, nv, K, M, S, G, a.mode);
  const int prob = blockIdx.x / a.blocks_per_problem;
  const int tile = blockIdx.x - prob * a.blocks_per_problem;
  const int s0 = tile * S;
  const int ns = min(S, a.N - s0);
  const int tid = threadIdx.x, T = blockDim.x;

  float* sW = sm + l.W;
  float* sObs = sm + l.obs;
  float* sAB = sm + l.ab;
  float* sM11 = sm + l.M11;
  float* sPi = sm + l.Pi;
  float* sC0 = sm + l.c0;
  float* sX = sm + l.X;
  float* sXb = sm + l.Xb;
  float* sLam = sm + l.Lam;
  float* sU = sm + l.U;
  float* sDelta = sm + l.Delta;
  float* sG = sm + l.G;

  // ---- constants -----------------------------------------------------------
  for (int i = tid; i < K * 3 * nv; i += T) sW[i] = a.W[i];
  const float* obs = a.obs + prob * a.obs_stride;
  for (int j = tid; j < M; j += T) {
    const float* o = obs + 8 * j;
    float* so = sObs + 8 * j;
    so[0] = o[0]; so[1] = o[1]; so[2] = (DIMS == 3) ? o[2] : 0.0f;
    so[3] = o[3]; so[4] = o[4]; so[5] = (DIMS == 3) ? o[5] : 0.0f;
    const float ra = o[6], rb = (DIMS == 3) ? o[7] : o[6];
    so[6] = 1.0f / (ra * ra);
    so[7] = 1.0f / (rb * rb);
    sAB[2 * j] = ra;
    sAB[2 * j + 1] = rb;
  }
  for (int i = tid; i < nv * nv; i += T) { sM11[i] = a.M11[i]; sPi[i] = a.Pi[i]; }
  const float* bc = a.bc + prob * a.bc_stride;
  for (int i = tid; i < D; i += T) {
    const int ax = i / nv, c = i - ax * nv;
    float s = 0.0f;
#pragma unroll
    for (int r = 0; r < 6; ++r) s = fmaf(a.M12[c * 6 + r], bc[ax * 6 + r], s);
    sC0[i] = s;
  }

  // ---- samples -------------------------------------------------------------
  if (a.mode == kFromInput) {
    const float* src = a.xi_in + prob * a.xi_in_stride + static_cast<int64_t>(s0) * D;
    for (int i = tid; i < ns * D; i += T) sX[i] = src[i];
  } else {
    float* sMu = sm + l.mu;
    float* sL = sm + l.L;
    float* sZ = sm + l.Z;
    const int D4 = round4(D);
    const float* mu = a.mu + prob * a.mu_stride;
    const float* L = a.L + prob * a.L_stride;
    for (int i = tid; i < D; i += T) sMu[i] = mu[i];
    for (int i = tid; i < D * D; i += T) sL[i] = L[i];
    if (a.mode == kFromNoise) {
      const float* z = a.noise + prob * a.noise_stride + static_cast<int64_t>(s0) * D;
      for (int i = tid; i < ns * D; i += T) {
        const int s = i / D;
        sZ[s * D4 + (i - s * D)] = z[i];
      }
    } else {
      const int nq = D4 / 4;
      const uint32_t stream = a.stream_base + static_cast<uint32_t>(prob);
      for (int i = tid; i < ns * nq; i += T) {
        const int s = i / nq, q = i - s * nq;
        float z[4];
        philox_normals4(a.seed, static_cast<uint32_t>(s0 + s), static_cast<uint32_t>(q),
                        static_cast<uint32_t>(a.iter), stream, z);
        *reinterpret_cast<float4*>(sZ + s * D4 + 4 * q) = make_float4(z[0], z[1], z[2], z[3]);
      }
    }
    __syncthreads();
    for (int i = tid; i < ns * D; i += T) {
      const int s = i / D, d = i - s * D;
      const float* z = sZ + s * D4;
      const float* Lr = sL + d * D;
      float x = sMu[d];
      for (int e = 0; e <= d; ++e) x = fmaf(Lr[e], z[e], x);
      sX[i] = x;
    }
    __syncthreads();
    if (a.xi_src) {
      float* dst = a.xi_src + prob * a.xi_src_stride + static_cast<int64_t>(s0) * D;
      for (int i = tid; i < ns * D; i += T) dst[i] = sX[i];
    }
  }
  __syncthreads();
  for (int i = tid; i < ns * D; i += T) { sXb[i] = sX[i]; sLam[i] = 0.0f; }
  __syncthreads();

  const float rho = a.rho;
  const float vmax = a.vmax, amax = a.amax;
  const int nitems = ns * K;
  const int SD = S * D;

  // ---- projection iterations -------------------------------------------------
  for (int k = 0; k < a.n_iter; ++k) {
    // phase 1: per (sample, t) push-outs
    for (int it = tid; it < nitems; it += T) {
      const int s = it / K, t = it - s * K;
      float p[DIMS], v[DIMS], ac[DIMS];
      eval_row<DIMS, NVT>(sW + t * 3 * nv, sXb + s * D, nv, p, v, ac);
      const float tt = a.dt * static_cast<float>(t);
      float so[DIMS];
#pragma unroll
      for (int ax = 0; ax < DIMS; ++ax) so[ax] = 0.0f;
#pragma unroll 2
      for (int j = 0; j < M; ++j) {
        float d[DIMS];
        if (obstacle_push<DIMS>(sObs + 8 * j, sAB + 2 * j, tt, p, d)) {
#pragma unroll
          for (int ax = 0; ax < DIMS; ++ax) so[ax] += d[ax];
        }
      }
      float dv[DIMS], da[DIMS];
      bound_push<DIMS>(v, vmax, dv);
      bound_push<DIMS>(ac, amax, da);
      float* out = sDelta + it * 3 * DIMS;
#pragma unroll
      for (int ax = 0; ax < DIMS; ++ax) {
        out[ax] = so[ax];
        out[DIMS + ax] = dv[ax];
        out[2 * DIMS + ax] = da[ax];
      }
    }
    __syncthreads();
    // phase 2: g = W^T delta, time range split into G groups
    for (int idx = tid; idx < G * SD; idx += T) {
      const int gi = idx / SD, o = idx - gi * SD;
      const int s = o / D, r = o - s * D;
      const int ax = r / nv, c = r - ax * nv;
      if (s < ns) {
        float acc = 0.0f;
        for (int t = gi; t < K; t += G) {
          const float* w = sW + t * 3 * nv;
          const float* dl = sDelta + (s * K + t) * 3 * DIMS;
          acc = fmaf(w[c], dl[ax], acc);
          acc = fmaf(w[nv + c], dl[DIMS + ax], acc);
          acc = fmaf(w[2 * nv + c], dl[2 * DIMS + ax], acc);
        }
        sG[gi * SD + o] = acc;
      }
    }
    __syncthreads();
    // phase 3a: multiplier update and QP right-hand side increment
    for (int o = tid; o < ns * D; o += T) {
      float g = 0.0f;
      for (int gi = 0; gi < G; ++gi) g += sG[gi * SD + o];
      const float lam = fmaf(rho, g, sLam[o]);
      sLam[o] = lam;
      const float u = (k == 0) ? fmaf(rho, g, lam) : fmaf(rho, g, (sX[o] - sXb[o]) + lam);
      sU[o] = u;
    }
    __syncthreads();
    // phase 3b: xi_bar through the fixed KKT block
    for (int o = tid; o < ns * D; o += T) {
      const int s = o / D, r = o - s * D;
      const int ax = r / nv, c = r - ax * nv;
      const float* u = sU + s * D + ax * nv;
      const float* m = sM11 + c * nv;
      float acc = 0.0f;
      for (int e = 0; e < nv; ++e) acc = fmaf(m[e], u[e], acc);
      if (k == 0) {
        const float* x = sX + s * D + ax * nv;
        const float* pi = sPi + c * nv;
        float base = sC0[r];
        for (int e = 0; e < nv; ++e) base = fmaf(pi[e], x[e], base);
        sXb[o] = base + acc;
      } else {
        sXb[o] += acc;
      }
    }
    __syncthreads();
  }

  // ---- residual and smoothness cost of the returned iterate ------------------
  for (int it = tid; it < nitems; it += T) {
    const int s = it / K, t = it - s * K;
    float p[DIMS], v[DIMS], ac[DIMS];
    eval_row<DIMS, NVT>(sW + t * 3 * nv, sXb + s * D, nv, p, v, ac);
    const float tt = a.dt * static_cast<float>(t);
    float r2 = 0.0f;
    for (int j = 0; j < M; ++j) {
      float d[DIMS];
      if (obstacle_push<DIMS>(sObs + 8 * j, sAB + 2 * j, tt, p, d)) {
#pragma unroll
        for (int ax = 0; ax < DIMS; ++ax) r2 = fmaf(d[ax], d[ax], r2);
      }
    }
    float dv[DIMS], da[DIMS];
    r2 += bound_push<DIMS>(v, vmax, dv);
    r2 += bound_push<DIMS>(ac, amax, da);
    float cc = 0.0f;
#pragma unroll
    for (int ax = 0; ax < DIMS; ++ax) cc = fmaf(ac[ax], ac[ax], cc);
    sDelta[2 * it] = r2;
    sDelta[2 * it + 1] = cc;
  }
  __syncthreads();
  const int64_t nbase = prob * a.n_stride + s0;
  for (int s = tid; s < ns; s += T) {
    float r2 = 0.0f, cc = 0.0f;
    for (int t = 0; t < K; ++t) {
      r2 += sDelta[2 * (s * K + t)];
      cc += sDelta[2 * (s * K + t) + 1];
    }
    const float r = sqrtf(r2);
    if (a.resid) a.resid[nbase + s] = r;
    if (a.c1) a.c1[nbase + s] = cc;
    const int64_t dense = static_cast<int64_t>(prob) * a.N + s0 + s;
    if (a.resid2) a.resid2[dense] = r;
    if (a.c12) a.c12[dense] = cc;
  }
  float* dst = a.xi_out + prob * a.xi_out_stride + static_cast<int64_t>(s0) * D;
  for (int i = tid; i < ns * D; i += T) dst[i] = sXb[i];
  if (a.xi_out2) {
    float* dst2 = a.xi_out2 + (static_cast<int64_t>(prob) * a.N + s0) * D;
    for (int i = tid; i < ns * D; i += T) dst2[i] = sXb[i];
  }
}

// Per-row push-outs e(xi) - F xi, [N][M + 2][K][dims] (parity hook).
template <int DIMS>
__global__ void offsets_kernel(ProjArgs a, const float* xi, float* out) {
  const int nv = a.nv, K = a.K, M = a.M;
  const int D = DIMS * nv;
  const int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= a.N * K) return;
  const int s = it / K, t = it - s * K;
  float p[DIMS], v[DIMS], ac[DIMS];
  eval_row<DIMS, 0>(a.W + t * 3 * nv, xi + static_cast<int64_t>(s) * D, nv, p, v, ac);
  const float tt = a.dt * static_cast<float>(t);
  float* o = out + static_cast<int64_t>(s) * (M + 2) * K * DIMS;
  for (int j = 0; j < M; ++j) {
    const float* src = a.obs + 8 * j;
    const float ra = src[6], rb = (DIMS == 3) ? src[7] : src[6];
    const float ob[8] = {src[0], src[1], DIMS == 3 ? src[2] : 0.0f, src[3], src[4],
                         DIMS == 3 ? src[5] : 0.0f, 1.0f / (ra * ra), 1.0f / (rb * rb)};
    const float ab[2] = {ra, rb};
    float d[DIMS];
    if (!obstacle_push<DIMS>(ob, ab, tt, p, d))
      for (int ax = 0; ax < DIMS; ++ax) d[ax] = 0.0f;
    for (int ax = 0; ax < DIMS; ++ax) o[(j * K + t) * DIMS + ax] = d[ax];
  }
  float dv[DIMS], da[DIMS];
  bound_push<DIMS>(v, a.vmax, dv);
  bound_push<DIMS>(ac, a.amax, da);
  for (int ax = 0; ax < DIMS; ++ax) {
    o[(M * K + t) * DIMS + ax] = dv[ax];
    o[((M + 1) * K + t) * DIMS + ax] = da[ax];
  }
}

__global__ void normals_kernel(uint64_t seed, uint32_t stream, int iter, int N, int D, float* z) {
  const int nq = (D + 3) / 4;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * nq) return;
  const int s = i / nq, q = i - s * nq;
  float w[4];
  philox_normals4(seed, static_cast<uint32_t>(s), static_cast<uint32_t>(q),
                  static_cast<uint32_t>(iter), stream, w);
  for (int k = 0; k < 4; ++k)
    if (4 * q + k < D) z[static_cast<int64_t>(s) * D + 4 * q + k] = w[k];
}

}  // namespace

size_t project_lds_bytes(const ProjArgs& a) {
  return sizeof(float) * static_cast<size_t>(layout(a.dims, a.nv, a.K, a.M, a.S, a.G, a.mode).total);
}

int project_pick_tile(int dims, int nv, int K, int M, int N, int n_problems, int* S, int* G) {
  // Smallest tile whose (sample, t) items fill the block, so that single
  // problems still spread over all compute units; more samples per block only
  // when the batch alone fills the chip several times over.
  const int T = kProjectThreads;
  int s = (T + K - 1) / K;
  if (s < 1) s = 1;
  const long long blocks = static_cast<long long>(n_problems) * ((N + s - 1) / s);
  if (blocks > 8LL * 256) {
    while (s * 2 * K <= 4 * T && s * 2 <= 16) s *= 2;
  }
  if (s > N) s = N;
  const int D = dims * nv;
  int g = T / (s * D);
  if (g < 1) g = 1;
  *S = s;
  *G = g;
  (void)M;
  return 0;
}

hipError_t launch_project(const ProjArgs& a, int n_problems, hipStream_t s) {
  const size_t lds = project_lds_bytes(a);
  const dim3 grid(static_cast<unsigned>(n_problems * a.blocks_per_problem));
  const dim3 block(kProjectThreads);
  if (a.dims == 2) {
    if (a.nv == 11) {
      hipLaunchKernelGGL((project_kernel<2, 11>), grid, block, lds, s, a);
    } else {
      hipLaunchKernelGGL((project_kernel<2, 0>), grid, block, lds, s, a);
    }
  } else {
    if (a.nv == 11) {
      hipLaunchKernelGGL((project_kernel<3, 11>), grid, block, lds, s, a);
    } else {
      hipLaunchKernelGGL((project_kernel<3, 0>), grid, block, lds, s, a);
    }
  }
  return hipGetLastError();
}

hipError_t launch_debug_offsets(const ProjArgs& a, const float* xi, float* out, hipStream_t s) {
  const int n = a.N * a.K;
  const dim3 grid((n + 127) / 128), block(128);
  if (a.dims == 2) {
    hipLaunchKernelGGL(offsets_kernel<2>, grid, block, 0, s, a, xi, out);
  } else {
    hipLaunchKernelGGL(offsets_kernel<3>, grid, block, 0, s, a, xi, out);
  }
  return hipGetLastError();
}

hipError_t launch_debug_normals(uint64_t seed, uint32_t stream_id, int iter, int N, int D,
                                float* z, hipStream_t s) {
  const int n = N * ((D + 3) / 4);
  hipLaunchKernelGGL(normals_kernel, dim3((n + 255) / 256), dim3(256), 0, s, seed, stream_id,
                     iter, N, D, z);
  return hipGetLastError();
}

}  // namespace priest
