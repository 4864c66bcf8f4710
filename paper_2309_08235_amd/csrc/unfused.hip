// Unfused projection: the plain form the fused kernel is compared against.
//
// The same projection iteration (Appendix eqs. (15a)-(15g)) as three kernels
// per iteration, every intermediate going through HBM, no MFMA, no culling:
//   forward : p, v, a of every (sample, t)                 -> pva
//   push    : push-outs of every (sample, t), all obstacles -> delta
//             (and |delta|^2 per item on the final pass)
//   update  : g = W^T delta per (sample, axis), lambda += rho g, QP step through
//             the fixed KKT block (the same k = 0 full form / k > 0 increment
//             form as the fused kernel)
// followed after the last iteration by forward + push and a per-sample sum of
// the residual and c1.
//
// Intermediates are stored in tiles of 64 samples, sample-fastest inside a
// tile: [tile][row type][t][sample in tile][axis] (r2: [tile][t][sample in
// tile]), so that every pass streams consecutive addresses across
// consecutive lanes and each wave walks one contiguous region: forward and
// push take one sample per lane at a fixed t, and the update takes one
// (sample, axis) row per lane (or per group of lanes for small batches) and
// walks (row type, t), the same offset for every lane.  The operands a wave
// applies are then the same for all its lanes and come through scalar
// loads: W's rows (padded to 16 and ordered by (row type, t) in the
// workspace), M11 and Pi, and the obstacles placed at the wave's step
// (centre + velocity t dt, written per step into the workspace once per call).
#include <algorithm>
#include <type_traits>

#include "priest_internal.h"

namespace priest {
namespace {


constexpr float kUfTiny = 1.0e-36f;
// Added to the canonical component of every offset (x in 2D, z in 3D): below
// half an ulp of any offset above about 2e-8, so those are unchanged; an
// offset of exactly zero becomes 1e-15 along the canonical axis, whose
// push-out is the semi-axis up to rounding (1e-30 / b^2 stays above the clamp
// for semi-axes up to 1000).
constexpr float kUfNudge = 1.0e-15f;

constexpr int kUfTile = 64;  // samples per tile of the intermediates

// pva / delta index of (row type d, step t, sample s, axis x).
__device__ __forceinline__ int64_t soa(int d, int t, int s, int x, int K, int dims) {
  const int tile = s / kUfTile, si = s - tile * kUfTile;
  return ((static_cast<int64_t>(tile) * 3 * K + d * K + t) * kUfTile + si) * dims + x;
}

// One thread per sample and chunk of kFwdTC steps.  Blocks go to the 8 XCDs
// in turn, so block b works on group 8 (b / 8 / n_chunk) + b % 8 of 256
// samples, chunk (b / 8) % n_chunk: all chunks of a group run on one XCD
// close together and read its coefficients through that XCD's L2.  The
// sample's coefficients in registers; the chunk's W rows, staged in LDS as
// rows of 16 (zero-padded), are the same for every lane of a wave.
constexpr int kFwdTC = 10;

template <int DIMS, int NVP>
__global__ __launch_bounds__(256) void uf_forward(const float* __restrict__ W,
                                                  const float* __restrict__ xb, int N, int K,
                                                  int nv, int n_chunk, float* __restrict__ pva) {
  static_assert(kMaxNV == 16, "W rows are staged as four float4");
  __shared__ float4 sw[kFwdTC * 3 * 4];
  const int kb = blockIdx.x >> 3;
  const int grp = (kb / n_chunk) * 8 + (blockIdx.x & 7), chunk = kb - (kb / n_chunk) * n_chunk;
  if (grp * 256 >= N) return;
  const int t0 = chunk * kFwdTC, nt = min(kFwdTC, K - t0);
  for (int j = threadIdx.x; j < nt * 3 * 16; j += blockDim.x) {
    const int row = j >> 4, c = j & 15;
    reinterpret_cast<float*>(sw)[j] = c < nv ? W[(t0 * 3 + row) * nv + c] : 0.0f;
  }
  __syncthreads();
  const int s = grp * 256 + threadIdx.x;
  if (s >= N) return;
  float x[DIMS][kMaxNV];
  const float* xs = xb + static_cast<int64_t>(s) * DIMS * nv;
#pragma unroll
  for (int ax = 0; ax < DIMS; ++ax)
#pragma unroll
    for (int c = 0; c < kMaxNV; ++c) x[ax][c] = c < nv ? xs[ax * nv + c] : 0.0f;
#pragma unroll 2
  for (int tl = 0; tl < nt; ++tl) {
    const int t = t0 + tl;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      float acc[DIMS];
#pragma unroll
      for (int ax = 0; ax < DIMS; ++ax) acc[ax] = 0.0f;
#pragma unroll
      for (int c4 = 0; c4 < NVP / 4; ++c4) {  // (NVP: coefficients rounded up to float4s)
        const float4 w = sw[(tl * 3 + d) * 4 + c4];
        const float wc[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int h = 0; h < 4; ++h)
#pragma unroll
          for (int ax = 0; ax < DIMS; ++ax) acc[ax] = fmaf(wc[h], x[ax][4 * c4 + h], acc[ax]);
      }
      float* o = pva + soa(d, t, s, 0, K, DIMS);
      if constexpr (DIMS == 2) {
        *reinterpret_cast<float2*>(o) = make_float2(acc[0], acc[1]);
      } else {
#pragma unroll
        for (int ax = 0; ax < DIMS; ++ax) o[ax] = acc[ax];
      }
    }
  }
}

// One thread per item (t, sample), consecutive samples in consecutive lanes.
// Once per call: W's rows padded to 16 in (row type, t) order, and every
// obstacle at every step, (centre + velocity t dt, a), then the shape terms
// (a^2, 1/a^2, 1/b^2, 0) per obstacle.
__global__ void uf_prep(const float* __restrict__ W, const float* __restrict__ obs, int K, int nv,
                        int M, int dims, float dt, float* __restrict__ w16,
                        float4* __restrict__ cen) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3 * K * 16) {
    const int e = i >> 4, c = i & 15, d = e / K, t = e - d * K;
    w16[i] = c < nv ? W[(t * 3 + d) * nv + c] : 0.0f;
  }
  if (i < K * M) {
    const int t = i / M, j = i - t * M;
    const float* o = obs + 8 * j;
    const float tt = dt * static_cast<float>(t);
    cen[i] = make_float4(fmaf(o[3], tt, o[0]), fmaf(o[4], tt, o[1]),
                         dims == 3 ? fmaf(o[5], tt, o[2]) : 0.0f, o[6]);
  }
  if (i < M) {
    const float* o = obs + 8 * i;
    const float a = o[6], b = dims == 3 ? o[7] : o[6];
    cen[static_cast<int64_t>(K) * M + i] = make_float4(a * a, 1.0f / (a * a), 1.0f / (b * b), 0.0f);
  }
}

// One thread per item; a wave's 64 lanes share one step t (one tile row),
// so its obstacles come from that step's row of `cen` through scalar loads.
template <int DIMS, bool LAST>
__global__ __launch_bounds__(256) void uf_push(const float* __restrict__ pva,
                                               const float4* __restrict__ cen, int N, int K, int M,
                                               float vmax, float amax, Box box,
                                               float* __restrict__ delta,
                                               float* __restrict__ r2out) {
  // item i = (tile, t, sample in tile), the order of the intermediates
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per_tile = static_cast<int64_t>(K) * kUfTile;
  const int tile = static_cast<int>(i / per_tile);
  const int rem = static_cast<int>(i - tile * per_tile);
  const int t = __builtin_amdgcn_readfirstlane(rem / kUfTile);  // the same in the whole wave
  const int s = tile * kUfTile + (rem - (rem / kUfTile) * kUfTile);
  const float4* oc = cen + static_cast<int64_t>(t) * M;
  const float4* shp = cen + static_cast<int64_t>(K) * M;
  if (s >= N) return;

  float w[3][DIMS];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float* in = pva + soa(d, t, s, 0, K, DIMS);
    if constexpr (DIMS == 2) {
      const float2 v = *reinterpret_cast<const float2*>(in);
      w[d][0] = v.x;
      w[d][1] = v.y;
    } else {
#pragma unroll
      for (int x = 0; x < DIMS; ++x) w[d][x] = in[x];
    }
  }
  const float* p = w[0];
  float S[DIMS];
#pragma unroll
  for (int x = 0; x < DIMS; ++x) S[x] = 0.0f;
  float r2 = 0.0f;
#pragma unroll 4
  for (int j = 0; j < M; ++j) {
    const float4 c = oc[j];
    float d[DIMS];
    d[0] = p[0] - c.x;
    d[1] = p[1] - c.y;
    if constexpr (DIMS == 3) d[2] = p[2] - c.z;
    d[DIMS == 2 ? 0 : 2] += kUfNudge;
    const float h = fmaf(d[1], d[1], d[0] * d[0]);
    float q, f, len2;
    if constexpr (DIMS == 2) {
      q = h;
      len2 = h;
      f = fmaf(c.w, __builtin_amdgcn_rsqf(fmaxf(q, kUfTiny)), -1.0f);
      if (LAST) f = (q < shp[j].x) ? f : 0.0f;
    } else {
      const float4 sh = shp[j];
      q = fmaf(d[2] * d[2], sh.z, h * sh.y);
      len2 = fmaf(d[2], d[2], h);
      f = __builtin_amdgcn_rsqf(fmaxf(q, kUfTiny)) - 1.0f;
      if (LAST) f = (q < 1.0f) ? f : 0.0f;
    }
    f = fmaxf(f, 0.0f);
#pragma unroll
    for (int x = 0; x < DIMS; ++x) S[x] = fmaf(d[x], f, S[x]);
    if (LAST) r2 = fmaf(len2 * f, f, r2);
  }
  if (box.on)  // workspace bounds: clamp(p, lo, hi) - p on the position rows
#pragma unroll
    for (int x = 0; x < DIMS; ++x) {
      const float e = fminf(fmaxf(p[x], box.lo[x]), box.hi[x]) - p[x];
      S[x] += e;
      if (LAST) r2 = fmaf(e, e, r2);
    }
  float dl[3][DIMS];
#pragma unroll
  for (int x = 0; x < DIMS; ++x) dl[0][x] = S[x];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float wm = k == 0 ? vmax : amax;
    float ww = 0.0f;
#pragma unroll
    for (int x = 0; x < DIMS; ++x) ww = fmaf(w[k + 1][x], w[k + 1][x], ww);
    float f = 0.0f;
    if (ww > wm * wm) f = fmaf(wm, __builtin_amdgcn_rsqf(ww), -1.0f);
#pragma unroll
    for (int x = 0; x < DIMS; ++x) dl[k + 1][x] = w[k + 1][x] * f;
    if (LAST) r2 = fmaf(ww * f, f, r2);
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float* out = delta + soa(d, t, s, 0, K, DIMS);
    if constexpr (DIMS == 2) {
      *reinterpret_cast<float2*>(out) = make_float2(dl[d][0], dl[d][1]);
    } else {
#pragma unroll
      for (int x = 0; x < DIMS; ++x) out[x] = dl[d][x];
    }
  }
  if (LAST) r2out[i] = r2;  // [tile][t][sample in tile]
}

// A group of `tpr` consecutive lanes (a power of two up to 16) per (sample,
// axis) row: g = W^T delta over the row's 3K entries, lane `sub` of the
// group taking entries sub, sub + tpr, ... (with one lane per row, each load
// is coalesced across the wave), an xor butterfly summing the group's
// partials; then lambda += rho g and the QP step through the fixed KKT
// block, stored by the group's lane 0.  tpr grows for small batches so that
// enough lanes stream.
constexpr int kUpdT = 256;

// The QP step of one (sample s, axis ax) row from its g: lambda += rho g and
// xi_bar through the fixed KKT block (k = 0 full form, k > 0 increment form).
__device__ __forceinline__ void uf_row_step(const float g[kMaxNV], int s, int ax, int nv, int dims,
                                            float rho, int first, const float* __restrict__ M11,
                                            const float* __restrict__ Pi,
                                            const float* __restrict__ M12,
                                            const float* __restrict__ bc,
                                            const float* __restrict__ xi, float* __restrict__ xb,
                                            float* __restrict__ lam) {
  auto cl = [nv](int c) { return c < nv ? c : nv - 1; };
  const int64_t base = static_cast<int64_t>(s) * dims * nv + ax * nv;
  float u[kMaxNV], x0[kMaxNV], xo[kMaxNV], l[kMaxNV];
#pragma unroll
  for (int c = 0; c < kMaxNV; ++c) {
    const bool in = c < nv;
    x0[c] = in ? xi[base + cl(c)] : 0.0f;
    xo[c] = in ? xb[base + cl(c)] : 0.0f;
    l[c] = in ? lam[base + cl(c)] + rho * g[c] : 0.0f;
    u[c] = in ? (first ? l[c] + rho * g[c] : (x0[c] - xo[c]) + l[c] + rho * g[c]) : 0.0f;
  }
  float bcv[6];
  if (first)
#pragma unroll
    for (int e = 0; e < 6; ++e) bcv[e] = bc[ax * 6 + e];
  // (guarded bodies rather than breaks, so that the loops unroll: xo and l
  // stay in registers)
#pragma unroll
  for (int r = 0; r < kMaxNV; ++r) {
    if (r < nv) {
      float acc = 0.0f;
#pragma unroll
      for (int c = 0; c < kMaxNV; ++c)
        if (c < nv) acc = fmaf(M11[r * nv + c], u[c], acc);
      float nx;
      if (first) {
        float h = 0.0f, c0 = 0.0f;
#pragma unroll
        for (int c = 0; c < kMaxNV; ++c)
          if (c < nv) h = fmaf(Pi[r * nv + c], x0[c], h);
#pragma unroll
        for (int e = 0; e < 6; ++e) c0 = fmaf(M12[r * 6 + e], bcv[e], c0);
        nx = (h + c0) + acc;
      } else {
        nx = xo[r] + acc;
      }
      lam[base + r] = l[r];
      xb[base + r] = nx;
    }
  }
}

// Large batches: one block per `tiles` tiles of 64 samples (2 in 2D, 1 in
// 3D: 256 or 192 rows (sample, axis)) x kUpdParts parts of the row's 3K
// entries (part p taking entries p, p + kUpdParts, ..., so that the block's
// waves sweep the tile's region together), so that a launch is about one
// round of resident blocks.  A wave holds 64 consecutive rows of one part, so
// each entry is a 256-byte load across the wave and the same W row for every
// lane (an LDS broadcast); the parts' partial g are summed through LDS in part
// order and the first part's lanes take the QP step.  NVP: coefficients per
// row rounded up to whole float4s of W (12 covers the usual 11; the padding
// columns of W are zero, so they add nothing).
constexpr int kUpdParts = 4;

template <int NVP>
__global__ __launch_bounds__(1024, 8) void uf_update_tile(
    const float4* __restrict__ w16, const float* __restrict__ delta, float* __restrict__ gout,
    int N, int K, int dims, int tiles) {
  extern __shared__ float4 swe[];  // [3K][16] W rows, then the partials [parts - 1][block rows][16]
  const int E = 3 * K, trows = kUfTile * dims, rows = tiles * trows;
  for (int j = threadIdx.x; j < E * 4; j += blockDim.x) swe[j] = w16[j];
  __syncthreads();
  float* red = reinterpret_cast<float*>(swe + E * 4);
  // (rows is a multiple of 64: every wave lies in one part)
  const int part = threadIdx.x / rows, rl = threadIdx.x - part * rows;
  const int tile = blockIdx.x * tiles + rl / trows, rt = rl - (rl / trows) * trows;
  static_assert(NVP % 4 == 0 && NVP <= kMaxNV, "whole float4s of W");
  const int ne = (E - part + kUpdParts - 1) / kUpdParts;  // this part's entries
  float g[NVP];
#pragma unroll
  for (int c = 0; c < NVP; ++c) g[c] = 0.0f;
  // (a tile past the last sample, up to the layout's even tile count, only
  // reads workspace and stores nothing)
  const float* dl = delta + static_cast<int64_t>(tile) * E * trows + part * trows + rt;
  const int64_t estride = static_cast<int64_t>(kUpdParts) * trows;
  constexpr int kU = 8;  // loads in flight per lane (two blocks per CU)
  for (int i0 = 0; i0 < ne; i0 += kU) {
    float v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u;
      v[u] = i < ne ? dl[i * estride] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = min(i0 + u, ne - 1) * kUpdParts + part;  // (v = 0 past the end)
#pragma unroll
      for (int c4 = 0; c4 < NVP / 4; ++c4) {
        const float4 w = swe[e * 4 + c4];
        g[4 * c4 + 0] = fmaf(w.x, v[u], g[4 * c4 + 0]);
        g[4 * c4 + 1] = fmaf(w.y, v[u], g[4 * c4 + 1]);
        g[4 * c4 + 2] = fmaf(w.z, v[u], g[4 * c4 + 2]);
        g[4 * c4 + 3] = fmaf(w.w, v[u], g[4 * c4 + 3]);
      }
    }
  }
  if (part > 0)
#pragma unroll
    for (int c = 0; c < NVP; ++c) red[((part - 1) * rows + rl) * NVP + c] = g[c];
  __syncthreads();
  if (part > 0) return;
  for (int q = 1; q < kUpdParts; ++q)
#pragma unroll
    for (int c = 0; c < NVP; ++c) g[c] += red[((q - 1) * rows + rl) * NVP + c];
  const int r = tile * trows + rt;
  if (r >= N * dims) return;
  float4* gr = reinterpret_cast<float4*>(gout + static_cast<int64_t>(r) * kMaxNV);
#pragma unroll
  for (int c4 = 0; c4 < NVP / 4; ++c4)
    gr[c4] = make_float4(g[4 * c4], g[4 * c4 + 1], g[4 * c4 + 2], g[4 * c4 + 3]);
}

// The QP step of every (sample, axis) row from the g the streaming pass wrote:
// 16 lanes per row, lane c forming entry c of the multiplier, of u and of the
// new xi_bar (the same operations, in the same order, as uf_row_step), the
// row's u shared through LDS.  Every old xi_bar and multiplier entry of a
// row is read before the barrier, every new one written after it.
__global__ __launch_bounds__(256) void uf_qp(const float* __restrict__ gin,
                                             const float* __restrict__ M11,
                                             const float* __restrict__ Pi,
                                             const float* __restrict__ M12,
                                             const float* __restrict__ bc,
                                             const float* __restrict__ xi, float* __restrict__ xb,
                                             float* __restrict__ lam, int N, int nv, int dims,
                                             float rho, int first) {
  __shared__ float su[256];  // u of the block's 16 rows
  __shared__ float sm11[kMaxNV * kMaxNV];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (threadIdx.x < nv * nv) sm11[threadIdx.x] = M11[threadIdx.x];
  const int r = t >> 4, c = t & 15;
  const bool live = r < N * dims && c < nv;
  const int ax = r % dims;
  const int64_t base = static_cast<int64_t>(r) * nv;  // row (sample r / dims, axis ax)
  float l = 0.0f, u = 0.0f, xo = 0.0f;
  if (live) {
    const float gc = gin[static_cast<int64_t>(r) * kMaxNV + c];
    l = lam[base + c] + rho * gc;
    xo = xb[base + c];
    u = first ? l + rho * gc : (xi[base + c] - xo) + l + rho * gc;
  }
  su[threadIdx.x] = u;
  __syncthreads();
  if (!live) return;
  const float* ur = su + (threadIdx.x & ~15);
  float acc = 0.0f;
  for (int k = 0; k < nv; ++k) acc = fmaf(sm11[c * nv + k], ur[k], acc);
  float nx;
  if (first) {
    float h = 0.0f, c0 = 0.0f;
    for (int k = 0; k < nv; ++k) h = fmaf(Pi[c * nv + k], xi[base + k], h);
#pragma unroll
    for (int e = 0; e < 6; ++e) c0 = fmaf(M12[c * 6 + e], bc[ax * 6 + e], c0);
    nx = (h + c0) + acc;
  } else {
    nx = xo + acc;
  }
  lam[base + c] = l;
  xb[base + c] = nx;
}

// Small batches: a group of `tpr` consecutive lanes (a power of two up to
// 16) per (sample, axis) row, lane `sub` taking entries sub, sub + tpr, ...,
// an xor butterfly summing the group's partials, W's rows from an LDS copy.
__global__ __launch_bounds__(kUpdT) void uf_update(const float4* __restrict__ w16,
                                                   const float* __restrict__ M11,
                                                   const float* __restrict__ Pi,
                                                   const float* __restrict__ M12,
                                                   const float* __restrict__ bc,
                                                   const float* __restrict__ delta,
                                                   const float* __restrict__ xi,
                                                   float* __restrict__ xb, float* __restrict__ lam,
                                                   int N, int K, int nv, int dims, float rho,
                                                   int first, int tpr) {
  extern __shared__ float4 swe[];  // [3K][16]: entry e = d K + t holds W's row (t, d)
  for (int j = threadIdx.x; j < 3 * K * 4; j += kUpdT) swe[j] = w16[j];
  __syncthreads();
  const int tid = blockIdx.x * kUpdT + threadIdx.x;
  const int row = tid / tpr, sub = tid - row * tpr;
  if (row >= N * dims) return;  // whole groups leave together (tpr divides 64)
  const int s = row / dims, ax = row - s * dims;
  float g[kMaxNV];
#pragma unroll
  for (int c = 0; c < kMaxNV; ++c) g[c] = 0.0f;
  const float* dl = delta + soa(0, 0, s, ax, K, dims);  // entry (d, t) at + (d K + t) 64 dims
  const int64_t step = static_cast<int64_t>(kUfTile) * dims;
  const int E = 3 * K;
  constexpr int kU = 16;  // loads in flight per lane
  for (int e0 = sub; e0 < E; e0 += kU * tpr) {
    float v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = e0 + u * tpr;
      v[u] = e < E ? dl[e * step] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int e = min(e0 + u * tpr, E - 1);  // (v = 0 past the end)
#pragma unroll
      for (int c4 = 0; c4 < 4; ++c4) {
        const float4 w = swe[e * 4 + c4];
        g[4 * c4 + 0] = fmaf(w.x, v[u], g[4 * c4 + 0]);
        g[4 * c4 + 1] = fmaf(w.y, v[u], g[4 * c4 + 1]);
        g[4 * c4 + 2] = fmaf(w.z, v[u], g[4 * c4 + 2]);
        g[4 * c4 + 3] = fmaf(w.w, v[u], g[4 * c4 + 3]);
      }
    }
  }
  for (int m = 1; m < tpr; m <<= 1)
#pragma unroll
    for (int c = 0; c < kMaxNV; ++c) g[c] += __shfl_xor(g[c], m, 64);
  if (sub != 0) return;
  uf_row_step(g, s, ax, nv, dims, rho, first, M11, Pi, M12, bc, xi, xb, lam);
}

__global__ void uf_finish(const float* __restrict__ r2, const float* __restrict__ pva, int N, int K,
                          int dims, float* __restrict__ resid, float* __restrict__ c1) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  float rr = 0.0f, cc = 0.0f;
  const int tile = s / kUfTile, si = s - tile * kUfTile;
  for (int t = 0; t < K; ++t) {
    rr += r2[(static_cast<int64_t>(tile) * K + t) * kUfTile + si];
    const float* a = pva + soa(2, t, s, 0, K, dims);
    for (int x = 0; x < dims; ++x) cc = fmaf(a[x], a[x], cc);
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

UnfusedLayout unfused_layout(int N, int K, int dims, int nv, int M) {
  auto al = [](size_t n) { return (n + 255) & ~static_cast<size_t>(255); };
  UnfusedLayout l{};
  size_t o = 0;
  // tiles rounded up to even: a 2D update block reads two whole tiles
  const size_t tiles = static_cast<size_t>(((N + kUfTile - 1) / kUfTile + 1) / 2 * 2);
  const size_t items = tiles * kUfTile * K;
  l.pva = o;   o += al(sizeof(float) * items * 3 * dims);
  l.delta = o; o += al(sizeof(float) * items * 3 * dims);
  l.r2 = o;    o += al(sizeof(float) * items);
  l.xb = o;    o += al(sizeof(float) * static_cast<size_t>(N) * dims * nv);
  l.lam = o;   o += al(sizeof(float) * static_cast<size_t>(N) * dims * nv);
  l.w16 = o;   o += al(sizeof(float) * 3 * K * 16);
  l.cen = o;   o += al(sizeof(float) * 4 * (static_cast<size_t>(K) + 1) * M);
  l.g = o;     o += al(sizeof(float) * kMaxNV * static_cast<size_t>(N) * dims);
  l.total = o;
  return l;
}

hipError_t launch_unfused(const ProjArgs& a, const float* xi_in, float* xi_out, float* resid,
                          float* c1, char* ws, hipStream_t s) {
  const int N = a.N, K = a.K, nv = a.nv, dims = a.dims, M = a.M;
  const UnfusedLayout l = unfused_layout(N, K, dims, nv, M);
  float* pva = reinterpret_cast<float*>(ws + l.pva);
  float* delta = reinterpret_cast<float*>(ws + l.delta);
  float* r2 = reinterpret_cast<float*>(ws + l.r2);
  float* xb = reinterpret_cast<float*>(ws + l.xb);
  float* lam = reinterpret_cast<float*>(ws + l.lam);
  float* w16 = reinterpret_cast<float*>(ws + l.w16);
  float4* cen = reinterpret_cast<float4*>(ws + l.cen);
  float* gbuf = reinterpret_cast<float*>(ws + l.g);
  const int64_t nD = static_cast<int64_t>(N) * dims * nv;
  const int64_t items = static_cast<int64_t>((N + kUfTile - 1) / kUfTile) * kUfTile * K;
  const dim3 b256(256);
  const dim3 g_items(static_cast<unsigned>((items + 255) / 256));
  const int n_chunk = (K + kFwdTC - 1) / kFwdTC, n_grp = (N + 255) / 256;
  const dim3 g_fwd(static_cast<unsigned>(((n_grp + 7) / 8) * 8 * n_chunk));
  // update: tpr lanes per (sample, axis) row, raised until about 64k lanes
  // stream
  int tpr = 1;
  while (tpr < 16 && static_cast<int64_t>(N) * dims * tpr < (64 << 10)) tpr *= 2;
  const dim3 g_upd(static_cast<unsigned>((static_cast<int64_t>(N) * dims * tpr + kUpdT - 1) / kUpdT));
  const int ut = dims == 2 ? 2 : 1;  // tiles per update block: 1024 / 768 threads
  const int n_tiles = (N + kUfTile - 1) / kUfTile;
  const dim3 g_tiles(static_cast<unsigned>((n_tiles + ut - 1) / ut));
  const size_t lds_tile =
      sizeof(float) * (3 * K * 16 + (kUpdParts - 1) * ut * kUfTile * dims * kMaxNV);
  const dim3 g_nD(static_cast<unsigned>((nD + 255) / 256)), g_N((N + 255) / 256);
  const size_t lds_upd = sizeof(float) * 3 * K * 16;
  const int n_prep = std::max(3 * K * 16, K * M);
  hipLaunchKernelGGL(uf_prep, dim3((n_prep + 255) / 256), b256, 0, s, a.W, a.obs, K, nv, M, dims,
                     a.dt, w16, cen);
  hipLaunchKernelGGL(uf_init, g_nD, b256, 0, s, xi_in, xb, lam, nD);
  auto forward = [&]() {
    if (dims == 2) {
      if (nv <= 12) hipLaunchKernelGGL((uf_forward<2, 12>), g_fwd, b256, 0, s, a.W, xb, N, K, nv, n_chunk, pva);
      else hipLaunchKernelGGL((uf_forward<2, 16>), g_fwd, b256, 0, s, a.W, xb, N, K, nv, n_chunk, pva);
    } else {
      if (nv <= 12) hipLaunchKernelGGL((uf_forward<3, 12>), g_fwd, b256, 0, s, a.W, xb, N, K, nv, n_chunk, pva);
      else hipLaunchKernelGGL((uf_forward<3, 16>), g_fwd, b256, 0, s, a.W, xb, N, K, nv, n_chunk, pva);
    }
  };
  auto push = [&](bool last) {
    if (dims == 2) {
      if (last) hipLaunchKernelGGL((uf_push<2, true>), g_items, b256, 0, s, pva, cen, N, K, M, a.vmax, a.amax, a.box, delta, r2);
      else hipLaunchKernelGGL((uf_push<2, false>), g_items, b256, 0, s, pva, cen, N, K, M, a.vmax, a.amax, a.box, delta, r2);
    } else {
      if (last) hipLaunchKernelGGL((uf_push<3, true>), g_items, b256, 0, s, pva, cen, N, K, M, a.vmax, a.amax, a.box, delta, r2);
      else hipLaunchKernelGGL((uf_push<3, false>), g_items, b256, 0, s, pva, cen, N, K, M, a.vmax, a.amax, a.box, delta, r2);
    }
  };
  for (int k = 0; k < a.n_iter; ++k) {
    forward();
    push(false);
    if (tpr == 1) {
      // g = W^T delta per row, streamed; then the QP step per row
      hipLaunchKernelGGL(nv <= 12 ? uf_update_tile<12> : uf_update_tile<16>, g_tiles,
                         dim3(ut * kUfTile * dims * kUpdParts), lds_tile, s,
                         reinterpret_cast<const float4*>(w16), delta, gbuf, N, K, dims, ut);
      const dim3 g_rows(static_cast<unsigned>((static_cast<int64_t>(N) * dims * 16 + 255) / 256));
      hipLaunchKernelGGL(uf_qp, g_rows, b256, 0, s, gbuf, a.M11, a.Pi, a.M12, a.bc, xi_in, xb,
                         lam, N, nv, dims, a.rho, k == 0 ? 1 : 0);
    } else
      hipLaunchKernelGGL(uf_update, g_upd, dim3(kUpdT), lds_upd, s,
                         reinterpret_cast<const float4*>(w16), a.M11, a.Pi, a.M12, a.bc, delta,
                         xi_in, xb, lam, N, K, nv, dims, a.rho, k == 0 ? 1 : 0, tpr);
  }
  forward();
  push(true);
  hipLaunchKernelGGL(uf_finish, g_N, b256, 0, s, r2, pva, N, K, dims, resid, c1);
  hipLaunchKernelGGL(uf_copy, g_nD, b256, 0, s, xb, xi_out, nD);
  return hipGetLastError();
}

}  // namespace priest
