// Unfused projection: the plain form the fused kernel is compared against.
//
// The same projection iteration (Appendix eqs. (15a)-(15g)) as three kernels
// per iteration, every intermediate going through HBM, no MFMA, no culling:
//   forward : p, v, a of every (sample, t)                 -> pva  [N][3][dims][K]
//   push    : push-outs of every (sample, t), all obstacles -> delta [N][3][dims][K]
//             (and |delta|^2 summed per item on the final pass)
//   update  : g = W^T delta per (sample, axis), lambda += rho g, QP step through
//             the fixed KKT block (the same k = 0 full form / k > 0 increment
//             form as the fused kernel)
// followed after the last iteration by forward + push and a per-sample sum of
// the residual and c1.  The obstacle loop of `push` is the elementwise pass
// whose HBM throughput the benchmark reports.  Intermediates are laid out per
// sample as [row type][axis][t], so consecutive threads (consecutive t) and
// the update's lanes touch consecutive addresses.
#include <algorithm>

#include "priest_internal.h"

namespace priest {
namespace {

// Obstacle record of the push kernel (2D circles / 3D spheres and
// ellipsoids): centre, velocity, a, a^2, 1/a^2, 1/b^2.
struct ORec {
  float cx, cy, cz, vx, vy, vz, a, a2, ia2, ib2;
};

// One thread per (sample, t); the basis rows are staged in LDS (row stride
// 3 n_coeff floats: an odd stride for odd n_coeff, so lanes of consecutive t
// hit distinct banks).
__global__ void uf_forward(const float* __restrict__ W, const float* __restrict__ xb, int N, int K,
                           int nv, int dims, float* __restrict__ pva) {
  extern __shared__ float sW[];
  for (int j = threadIdx.x; j < K * 3 * nv; j += blockDim.x) sW[j] = W[j];
  __syncthreads();
  // grid-stride over (sample, t) items so the staging is amortised
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N * K; i += gridDim.x * blockDim.x) {
    const int s = i / K, t = i - s * K;
    const float* w = sW + t * 3 * nv;
    const float* x = xb + static_cast<int64_t>(s) * dims * nv;
    float* o = pva + static_cast<int64_t>(s) * 3 * dims * K + t;
    for (int d = 0; d < 3; ++d)
      for (int ax = 0; ax < dims; ++ax) {
        float acc = 0.0f;
        for (int c = 0; c < nv; ++c) acc = fmaf(w[d * nv + c], x[ax * nv + c], acc);
        o[(d * dims + ax) * K] = acc;
      }
  }
}

template <int DIMS, bool LAST>
__global__ void uf_push(const float* __restrict__ pva, const float* __restrict__ obs, int N, int K,
                        int M, float dt, float vmax, float amax, Box box,
                        float* __restrict__ delta, float* __restrict__ r2out) {
  extern __shared__ ORec orec[];
  for (int j = threadIdx.x; j < M; j += blockDim.x) {
    const float* o = obs + 8 * j;
    const float a = o[6], b = (DIMS == 3) ? o[7] : o[6];
    orec[j] = ORec{o[0], o[1], DIMS == 3 ? o[2] : 0.0f, o[3], o[4], DIMS == 3 ? o[5] : 0.0f,
                   a, a * a, 1.0f / (a * a), 1.0f / (b * b)};
  }
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * K) return;
  const int sm = i / K, t = i - sm * K;
  const float tt = dt * static_cast<float>(t);
  const float* in = pva + static_cast<int64_t>(sm) * 3 * DIMS * K + t;
  float p[DIMS], w[2][DIMS];
  for (int x = 0; x < DIMS; ++x) {
    p[x] = in[x * K];
    w[0][x] = in[(DIMS + x) * K];
    w[1][x] = in[(2 * DIMS + x) * K];
  }
  float S[DIMS];
  for (int x = 0; x < DIMS; ++x) S[x] = 0.0f;
  float r2 = 0.0f;
  for (int j = 0; j < M; ++j) {
    const ORec o = orec[j];
    float d[DIMS];
    d[0] = p[0] - fmaf(o.vx, tt, o.cx);
    d[1] = p[1] - fmaf(o.vy, tt, o.cy);
    if constexpr (DIMS == 3) d[2] = p[2] - fmaf(o.vz, tt, o.cz);
    const float h = fmaf(d[1], d[1], d[0] * d[0]);
    float q, f, len2;
    if constexpr (DIMS == 2) {
      q = h;
      len2 = h;
      f = fmaf(o.a, __builtin_amdgcn_rsqf(fmaxf(q, 1.0e-30f)), -1.0f);
      if (LAST) f = (q < o.a2) ? f : 0.0f;
    } else {
      q = fmaf(d[2] * d[2], o.ib2, h * o.ia2);
      len2 = fmaf(d[2], d[2], h);
      f = __builtin_amdgcn_rsqf(fmaxf(q, 1.0e-30f)) - 1.0f;
      if (LAST) f = (q < 1.0f) ? f : 0.0f;
    }
    f = fmaxf(f, 0.0f);
    for (int x = 0; x < DIMS; ++x) S[x] = fmaf(d[x], f, S[x]);
    if (LAST) r2 = fmaf(len2 * f, f, r2);
    if (q == 0.0f) {  // canonical direction of a zero offset
      if constexpr (DIMS == 2) {
        S[0] += o.a;
        if (LAST) r2 += o.a2;
      } else {
        const float bb = __builtin_amdgcn_rsqf(o.ib2);
        S[2] += bb;
        if (LAST) r2 = fmaf(bb, bb, r2);
      }
    }
  }
  if (box.on)  // workspace bounds: clamp(p, lo, hi) - p on the position rows
    for (int x = 0; x < DIMS; ++x) {
      const float e = fminf(fmaxf(p[x], box.lo[x]), box.hi[x]) - p[x];
      S[x] += e;
      if (LAST) r2 = fmaf(e, e, r2);
    }
  float* out = delta + static_cast<int64_t>(sm) * 3 * DIMS * K + t;
  for (int x = 0; x < DIMS; ++x) out[x * K] = S[x];
  for (int k = 0; k < 2; ++k) {
    const float wm = k == 0 ? vmax : amax;
    float ww = 0.0f;
    for (int x = 0; x < DIMS; ++x) ww = fmaf(w[k][x], w[k][x], ww);
    float f = 0.0f;
    if (ww > wm * wm) f = fmaf(wm, __builtin_amdgcn_rsqf(ww), -1.0f);
    for (int x = 0; x < DIMS; ++x) out[((k + 1) * DIMS + x) * K] = w[k][x] * f;
    if (LAST) r2 += ww * f * f;
  }
  if (LAST) r2out[i] = r2;
}

// One wave per (sample, axis): lanes split the K time steps of
// g = W^T delta, a wave reduction sums them, then lane r < n_coeff applies
// lambda += rho g and row r of the QP step through the fixed KKT block.
// Loops run to the compile-time bound kMaxNV with n_coeff guards so the
// per-lane vectors stay in registers.
__global__ void uf_update(const float* __restrict__ W, const float* __restrict__ M11,
                          const float* __restrict__ Pi, const float* __restrict__ M12,
                          const float* __restrict__ bc, const float* __restrict__ delta,
                          const float* __restrict__ xi, float* __restrict__ xb,
                          float* __restrict__ lam, int N, int K, int nv, int dims, float rho,
                          int first) {
  extern __shared__ float sW[];
  for (int j = threadIdx.x; j < K * 3 * nv; j += blockDim.x) sW[j] = W[j];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wstride = (gridDim.x * blockDim.x) >> 6;
  // whole waves stride over (sample, axis) rows, so the staging is amortised
  for (int wv = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; wv < N * dims; wv += wstride) {
  const int s = wv / dims, ax = wv - s * dims;
  float g[kMaxNV];
#pragma unroll
  for (int c = 0; c < kMaxNV; ++c) g[c] = 0.0f;
  const float* dl = delta + static_cast<int64_t>(s) * 3 * dims * K;
  for (int t = lane; t < K; t += 64)
    for (int d = 0; d < 3; ++d) {
      const float v = dl[(d * dims + ax) * K + t];
      const float* w = sW + (t * 3 + d) * nv;
#pragma unroll
      for (int c = 0; c < kMaxNV; ++c)
        if (c < nv) g[c] = fmaf(w[c], v, g[c]);
    }
#pragma unroll
  for (int c = 0; c < kMaxNV; ++c)
    if (c < nv)
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) g[c] += __shfl_xor(g[c], m, 64);
  const int64_t base = static_cast<int64_t>(s) * dims * nv + ax * nv;
  float u[kMaxNV], x0[kMaxNV];
  float lr = 0.0f, xr = 0.0f;
#pragma unroll
  for (int c = 0; c < kMaxNV; ++c) {
    u[c] = 0.0f;
    x0[c] = 0.0f;
    if (c < nv) {
      x0[c] = xi[base + c];
      const float xo = xb[base + c];
      const float l = lam[base + c] + rho * g[c];
      u[c] = first ? l + rho * g[c] : (x0[c] - xo) + l + rho * g[c];
      if (c == lane) {
        lr = l;
        xr = xo;
      }
    }
  }
  if (lane < nv) {
    const int r = lane;
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < kMaxNV; ++c)
      if (c < nv) acc = fmaf(M11[r * nv + c], u[c], acc);
    float nx;
    if (first) {
      float h = 0.0f;
#pragma unroll
      for (int c = 0; c < kMaxNV; ++c)
        if (c < nv) h = fmaf(Pi[r * nv + c], x0[c], h);
      float c0 = 0.0f;
      for (int e = 0; e < 6; ++e) c0 = fmaf(M12[r * 6 + e], bc[ax * 6 + e], c0);
      nx = (h + c0) + acc;
    } else {
      nx = xr + acc;
    }
    lam[base + r] = lr;
    xb[base + r] = nx;
  }
  }
}

__global__ void uf_finish(const float* __restrict__ r2, const float* __restrict__ pva, int N, int K,
                          int dims, float* __restrict__ resid, float* __restrict__ c1) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  float rr = 0.0f, cc = 0.0f;
  for (int t = 0; t < K; ++t) {
    rr += r2[static_cast<int64_t>(s) * K + t];
    const float* a = pva + static_cast<int64_t>(s) * 3 * dims * K + 2 * dims * K + t;
    for (int x = 0; x < dims; ++x) cc = fmaf(a[x * K], a[x * K], cc);
  }
  if (resid) resid[s] = sqrtf(rr);
  if (c1) c1[s] = cc;
}

__global__ void uf_init(const float* __restrict__ xi, float* __restrict__ xb,
                        float* __restrict__ lam, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  xb[i] = xi[i];
  lam[i] = 0.0f;
}

__global__ void uf_copy(const float* __restrict__ src, float* __restrict__ dst, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace

UnfusedLayout unfused_layout(int N, int K, int dims, int nv) {
  auto al = [](size_t n) { return (n + 255) & ~static_cast<size_t>(255); };
  UnfusedLayout l{};
  size_t o = 0;
  const size_t items = static_cast<size_t>(N) * K;
  l.pva = o;   o += al(sizeof(float) * items * 3 * dims);
  l.delta = o; o += al(sizeof(float) * items * 3 * dims);
  l.r2 = o;    o += al(sizeof(float) * items);
  l.xb = o;    o += al(sizeof(float) * static_cast<size_t>(N) * dims * nv);
  l.lam = o;   o += al(sizeof(float) * static_cast<size_t>(N) * dims * nv);
  l.total = o;
  return l;
}

hipError_t launch_unfused(const ProjArgs& a, const float* xi_in, float* xi_out, float* resid,
                          float* c1, char* ws, hipStream_t s) {
  const int N = a.N, K = a.K, nv = a.nv, dims = a.dims, M = a.M;
  const UnfusedLayout l = unfused_layout(N, K, dims, nv);
  float* pva = reinterpret_cast<float*>(ws + l.pva);
  float* delta = reinterpret_cast<float*>(ws + l.delta);
  float* r2 = reinterpret_cast<float*>(ws + l.r2);
  float* xb = reinterpret_cast<float*>(ws + l.xb);
  float* lam = reinterpret_cast<float*>(ws + l.lam);
  const int64_t nD = static_cast<int64_t>(N) * dims * nv;
  const int items = N * K;
  const dim3 b256(256), b1024(1024);
  // forward and update stage W in LDS: at most 8 blocks per CU, grid-stride beyond
  const dim3 g_items((items + 255) / 256), g_axes((N * dims + 15) / 16);
  const dim3 g_fwd(std::min<unsigned>(g_items.x, 2048u)), g_upd(std::min<unsigned>(g_axes.x, 512u));
  const size_t ldsW = sizeof(float) * K * 3 * nv;
  const dim3 g_nD(static_cast<unsigned>((nD + 255) / 256)), g_N((N + 255) / 256);
  const size_t lds = sizeof(ORec) * (M > 0 ? M : 1);
  hipLaunchKernelGGL(uf_init, g_nD, b256, 0, s, xi_in, xb, lam, nD);
  auto push = [&](bool last) {
    if (dims == 2) {
      if (last) hipLaunchKernelGGL((uf_push<2, true>), g_items, b256, lds, s, pva, a.obs, N, K, M, a.dt, a.vmax, a.amax, a.box, delta, r2);
      else hipLaunchKernelGGL((uf_push<2, false>), g_items, b256, lds, s, pva, a.obs, N, K, M, a.dt, a.vmax, a.amax, a.box, delta, r2);
    } else {
      if (last) hipLaunchKernelGGL((uf_push<3, true>), g_items, b256, lds, s, pva, a.obs, N, K, M, a.dt, a.vmax, a.amax, a.box, delta, r2);
      else hipLaunchKernelGGL((uf_push<3, false>), g_items, b256, lds, s, pva, a.obs, N, K, M, a.dt, a.vmax, a.amax, a.box, delta, r2);
    }
  };
  for (int k = 0; k < a.n_iter; ++k) {
    hipLaunchKernelGGL(uf_forward, g_fwd, b256, ldsW, s, a.W, xb, N, K, nv, dims, pva);
    push(false);
    hipLaunchKernelGGL(uf_update, g_upd, b1024, ldsW, s, a.W, a.M11, a.Pi, a.M12, a.bc, delta, xi_in,
                       xb, lam, N, K, nv, dims, a.rho, k == 0 ? 1 : 0);
  }
  hipLaunchKernelGGL(uf_forward, g_fwd, b256, ldsW, s, a.W, xb, N, K, nv, dims, pva);
  push(true);
  hipLaunchKernelGGL(uf_finish, g_N, b256, 0, s, r2, pva, N, K, dims, resid, c1);
  hipLaunchKernelGGL(uf_copy, g_nD, b256, 0, s, xb, xi_out, nD);
  return hipGetLastError();
}

}  // namespace priest
