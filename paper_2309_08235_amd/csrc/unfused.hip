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
#include <type_traits>

#include "priest_internal.h"

namespace priest {
namespace {

// Obstacle record of the push kernel (2D circles / 3D spheres and
// ellipsoids): centre, velocity, a, a^2, 1/a^2, 1/b^2.
struct ORec {
  float cx, cy, cz, vx, vy, vz, a, a2, ia2, ib2;
};

// One thread per time step t (blockIdx.y picks a chunk of kFwdT steps); a
// block runs through `spb` consecutive samples.  The thread keeps its three
// basis rows in registers (entries c >= n_coeff zeroed), and a sample's
// coefficients are block-uniform (staged in LDS as zero-padded rows of 16
// and read as four 16-byte broadcasts per axis), so each sample costs
// 3 dims coalesced row stores.
constexpr int kFwdT = 128;
constexpr int kFwdMaxSpb = 16;

__global__ __launch_bounds__(kFwdT) void uf_forward(const float* __restrict__ W,
                                                    const float* __restrict__ xb, int N, int K,
                                                    int nv, int dims, int spb,
                                                    float* __restrict__ pva) {
  const int t = blockIdx.y * kFwdT + threadIdx.x;
  const bool live = t < K;
  const int tc = live ? t : K - 1;
  float w[3][kMaxNV];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int c = 0; c < kMaxNV; ++c)
      w[d][c] = W[(tc * 3 + d) * nv + (c < nv ? c : nv - 1)] * (c < nv ? 1.0f : 0.0f);
  const int s0 = blockIdx.x * spb;
  const int s1 = min(N, s0 + spb);
  static_assert(kMaxNV == 16, "coefficient rows are staged as four float4");
  __shared__ float4 sx[kFwdMaxSpb * 3 * 4];  // [sample][axis][16], zero-padded
  for (int j = threadIdx.x; j < (s1 - s0) * dims * 16; j += kFwdT) {
    const int k = j / (dims * 16), rem = j - k * dims * 16, ax = rem >> 4, c = rem & 15;
    reinterpret_cast<float*>(sx)[j] =
        c < nv ? xb[static_cast<int64_t>(s0 + k) * dims * nv + ax * nv + c] : 0.0f;
  }
  __syncthreads();
  for (int s = s0; s < s1; ++s) {
    const float4* x = sx + (s - s0) * dims * 4;
    float* o = pva + static_cast<int64_t>(s) * 3 * dims * K + t;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      if (ax >= dims) break;
      float xv[kMaxNV];
#pragma unroll
      for (int c4 = 0; c4 < 4; ++c4) {
        const float4 v = x[ax * 4 + c4];
        xv[4 * c4] = v.x;
        xv[4 * c4 + 1] = v.y;
        xv[4 * c4 + 2] = v.z;
        xv[4 * c4 + 3] = v.w;
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        float acc = 0.0f;
#pragma unroll
        for (int c = 0; c < kMaxNV; ++c) acc = fmaf(w[d][c], xv[c], acc);
        if (live) o[(d * dims + ax) * K] = acc;
      }
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

// A group of `tpr` consecutive lanes (a power of two up to 64) per
// (sample, axis) row: g = W^T delta over the row's 3K entries, lambda +=
// rho g, and the QP step through the fixed KKT block.  The group streams
// its three K-long delta rows in VW-wide loads, lane `sub` taking vectors
// sub, sub + tpr, ... (consecutive lanes read consecutive addresses), and an
// xor butterfly inside the group sums g; every lane of the group then
// forms the step and lane 0 stores it.  W, M11 and Pi are staged in LDS with
// rows zero-padded to 16 entries, so the per-row loops run to 16 without
// conditions and entries c >= n_coeff stay zero.  tpr grows for small
// batches so that enough lanes stream.
constexpr int kUpdT = 128;

template <int VW>
__global__ __launch_bounds__(kUpdT) void uf_update(const float* __restrict__ W,
                                                   const float* __restrict__ M11,
                                                   const float* __restrict__ Pi,
                                                   const float* __restrict__ M12,
                                                   const float* __restrict__ bc,
                                                   const float* __restrict__ delta,
                                                   const float* __restrict__ xi,
                                                   float* __restrict__ xb, float* __restrict__ lam,
                                                   int N, int K, int nv, int dims, float rho,
                                                   int first, int tpr) {
  static_assert(kMaxNV == 16, "LDS rows are padded to 16 entries");
  extern __shared__ float4 sm4[];
  float* sW = reinterpret_cast<float*>(sm4);  // [3K][16]
  float* sM = sW + 3 * K * 16;                 // M11 [16][16]
  float* sP = sM + 256;                        // Pi  [16][16]
  for (int j = threadIdx.x; j < 3 * K * 16; j += kUpdT) {
    const int row = j >> 4, c = j & 15;
    sW[j] = c < nv ? W[row * nv + c] : 0.0f;
  }
  for (int j = threadIdx.x; j < 256; j += kUpdT) {
    const int row = j >> 4, c = j & 15;
    const bool in = row < nv && c < nv;
    sM[j] = in ? M11[row * nv + c] : 0.0f;
    sP[j] = in ? Pi[row * nv + c] : 0.0f;
  }
  __syncthreads();
  const int tid = blockIdx.x * kUpdT + threadIdx.x;
  const int rowi = tid / tpr, sub = tid - rowi * tpr;
  if (rowi >= N * dims) return;  // whole groups leave together (tpr divides 64)
  const int s = rowi / dims, ax = rowi - s * dims;
  float g[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) g[c] = 0.0f;
  const float* dl = delta + static_cast<int64_t>(s) * 3 * dims * K;
  using VT = typename std::conditional<VW == 4, float4, typename std::conditional<VW == 2, float2, float>::type>::type;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const VT* row = reinterpret_cast<const VT*>(dl + (d * dims + ax) * K);
#pragma unroll 4
    for (int q = sub; q < K / VW; q += tpr) {
      const VT v = row[q];
      const float* vv = reinterpret_cast<const float*>(&v);
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        const float4* w4 = reinterpret_cast<const float4*>(sW + ((q * VW + e) * 3 + d) * 16);
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) {
          const float4 w = w4[c4];
          g[4 * c4 + 0] = fmaf(w.x, vv[e], g[4 * c4 + 0]);
          g[4 * c4 + 1] = fmaf(w.y, vv[e], g[4 * c4 + 1]);
          g[4 * c4 + 2] = fmaf(w.z, vv[e], g[4 * c4 + 2]);
          g[4 * c4 + 3] = fmaf(w.w, vv[e], g[4 * c4 + 3]);
        }
      }
    }
  }
  for (int m = 1; m < tpr; m <<= 1)
#pragma unroll
    for (int c = 0; c < 16; ++c) g[c] += __shfl_xor(g[c], m, 64);
  auto cl = [nv](int c) { return c < nv ? c : nv - 1; };
  const int64_t base = static_cast<int64_t>(s) * dims * nv + ax * nv;
  float u[16], x0[16], xo[16], l[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const bool in = c < nv;
    x0[c] = in ? xi[base + cl(c)] : 0.0f;
    xo[c] = xb[base + cl(c)];
    l[c] = lam[base + cl(c)] + rho * g[c];
    u[c] = in ? (first ? l[c] + rho * g[c] : (x0[c] - xo[c]) + l[c] + rho * g[c]) : 0.0f;
  }
  float c0[16];
  if (first) {
    float bcv[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) bcv[e] = bc[ax * 6 + e];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      float a = 0.0f;
#pragma unroll
      for (int e = 0; e < 6; ++e) a = fmaf(M12[cl(r) * 6 + e], bcv[e], a);
      c0[r] = a;
    }
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < 16; ++c) acc = fmaf(sM[r * 16 + c], u[c], acc);
    float nx;
    if (first) {
      float h = 0.0f;
#pragma unroll
      for (int c = 0; c < 16; ++c) h = fmaf(sP[r * 16 + c], x0[c], h);
      nx = (h + c0[r]) + acc;
    } else {
      nx = xo[r] + acc;
    }
    if (r < nv && sub == 0) {
      lam[base + r] = l[r];
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
  const dim3 b256(256);
  const dim3 g_items((items + 255) / 256);
  // forward: blocks of kFwdT time steps over spb samples, about 2048+ blocks
  const int spb = std::max(1, std::min(kFwdMaxSpb, N / 2048));
  const dim3 g_fwd((N + spb - 1) / spb, (K + kFwdT - 1) / kFwdT), b_fwd(kFwdT);
  // update: tpr lanes per (sample, axis) row, raised only until about 64k
  // lanes stream (at most 16 per row: at N = 64000, 2D, one lane per row
  // takes 98 us, two 102 us and four 109 us; at N = 1000 sixteen take 14 us
  // against 52 us for one); W, M11 and Pi padded in LDS
  int tpr = 1;
  while (tpr < 16 && static_cast<int64_t>(N) * dims * tpr < (64 << 10)) tpr *= 2;
  const dim3 g_upd(static_cast<unsigned>((static_cast<int64_t>(N) * dims * tpr + kUpdT - 1) / kUpdT));
  const dim3 b_upd(kUpdT);
  const size_t lds_upd = sizeof(float) * (3 * K * 16 + 2 * 256);
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
    hipLaunchKernelGGL(uf_forward, g_fwd, b_fwd, 0, s, a.W, xb, N, K, nv, dims, spb, pva);
    push(false);
    if (K % 4 == 0)
      hipLaunchKernelGGL(uf_update<4>, g_upd, b_upd, lds_upd, s, a.W, a.M11, a.Pi, a.M12, a.bc, delta,
                         xi_in, xb, lam, N, K, nv, dims, a.rho, k == 0 ? 1 : 0, tpr);
    else if (K % 2 == 0)
      hipLaunchKernelGGL(uf_update<2>, g_upd, b_upd, lds_upd, s, a.W, a.M11, a.Pi, a.M12, a.bc, delta,
                         xi_in, xb, lam, N, K, nv, dims, a.rho, k == 0 ? 1 : 0, tpr);
    else
      hipLaunchKernelGGL(uf_update<1>, g_upd, b_upd, lds_upd, s, a.W, a.M11, a.Pi, a.M12, a.bc, delta,
                         xi_in, xb, lam, N, K, nv, dims, a.rho, k == 0 ? 1 : 0, tpr);
  }
  hipLaunchKernelGGL(uf_forward, g_fwd, b_fwd, 0, s, a.W, xb, N, K, nv, dims, spb, pva);
  push(true);
  hipLaunchKernelGGL(uf_finish, g_N, b256, 0, s, r2, pva, N, K, dims, resid, c1);
  hipLaunchKernelGGL(uf_copy, g_nD, b256, 0, s, xb, xi_out, nD);
  return hipGetLastError();
}

}  // namespace priest
