// Fused projection sweep for gfx950 (MFMA + VALU, state in registers).
//
// Work decomposition.  A block owns SPB samples of one problem for the whole
// projection and has one 64-lane wave per RT consecutive 16-step time blocks
// (K <= 256).  Sample coefficients live in registers in the layout of the
// 16x16 FP32 MFMA accumulator: column col = AS*sample + axis (AS axis slots
// per sample: 4, or 2 for 2D so that 8 samples share the 16 columns), row =
// coefficient (padded to 16), lane l holding rows 4*(l/16)..+3 of column
// l%16.  Per projection iteration (Appendix, eqs. (15a)-(15g), with the
// per-sample batching of Sec. III-A):
//
//   forward   p, v, a rows of each of the wave's time blocks = W xi_bar
//             (one MFMA 16x16x4 accumulation chain per row type over the
//             k-chunks, W = [P; Pdot; Pddot] rows as A)
//   transpose quad-local transpose through LDS: each lane then holds every
//             axis of 4/AS (sample, t) items per time block
//   push-out  closed-form alpha/beta/d of each obstacle as a push-out
//             Delta * max(0, 1/n - 1) (n = scaled distance), summed over the
//             obstacles that survive a wave-level bounding-box cull;
//             velocity / acceleration push-outs w * min(0, w_max/|w| - 1)
//   transpose back to the column layout
//   RHS       g_partial = W^T delta per 16-step block (MFMA, the sum over t
//             is the MFMA reduction); the partials of all blocks added in
//             time-block order through LDS (one barrier)
//   update    lambda += rho g (eq. (15e)); QP of eq. (15g) through the fixed
//             KKT block, redone identically by every wave (MFMA):
//               k = 0 : xi_bar = Pi xi + c0 + M11 (lambda + rho g)
//               k > 0 : xi_bar += M11 (xi - xi_bar + lambda + rho g)
//             The k > 0 form equals M11 eta + M12 b whenever A xi_bar = b,
//             which holds after the first step; it avoids cancelling
//             n_obs |p| against rho F^T F xi_bar in FP32.
//
// After the last iteration one more forward + push-out pass evaluates
// r(xi_bar) and c1 = sum_t |a_t|^2, summed per sample in fixed t order.
//
// Tile shapes (AS, RT), the persistent grid and the groups a wave draws
// change only which lanes, waves and blocks do the work: every sample goes
// through the same operations in the same order (per-column MFMA,
// per-16-step partials added in time-block order, culled obstacles
// contribute exact zeros), so every shape gives bit-identical results and the
// autotuner may pick any of them.
#include "priest_internal.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

namespace priest {
namespace {

using f4 = __attribute__((ext_vector_type(4))) float;

__host__ __device__ inline int round4(int n) { return (n + 3) & ~3; }

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// BF16 operands (mixed precision): round-to-nearest-even FP32 -> BF16 and the
// K = 16 BF16 MFMA with FP32 accumulation.  Lane l's four values are the same
// (row, k) slots the FP32 K = 4 MFMA uses across its four steps, so the
// register layouts carry over unchanged.
using s4 = __attribute__((ext_vector_type(4))) short;

__device__ __forceinline__ short to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<short>(u >> 16);
}
__device__ __forceinline__ float from_bf16(short h) {
  return __uint_as_float(static_cast<uint32_t>(static_cast<unsigned short>(h)) << 16);
}
__device__ __forceinline__ s4 pack_bf16(float a0, float a1, float a2, float a3) {
  return s4{to_bf16(a0), to_bf16(a1), to_bf16(a2), to_bf16(a3)};
}
__device__ __forceinline__ f4 mfma_bf16(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Orders this wave's LDS writes before its subsequent LDS reads by other lanes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Transpose buffers: each lane's float4 at 4 * (lane + lane / 8) floats, i.e.
// 16 bytes of padding after every 8 lanes.  The float4 writes (8 lanes per
// pass) then cover all 32 banks once, and so do the quad reads of the
// transposes (one slot of lane 4 q + x for the 8 quads q of a half-wave, x
// fixed): slot indices 4 q + x + q / 2 are distinct modulo 8.
constexpr int kXtRow = 288;            // one row type: 64 lanes x 4 + 8 x 4 padding
constexpr int kXtBlock = 3 * kXtRow;   // p, v, a (or their push-outs)
__device__ __forceinline__ int xt_at(int lane) { return 4 * (lane + (lane >> 3)); }

struct Layout {  // offsets into dynamic LDS, in floats
  int rec, xt, gp, fin, hist, cm, mu, L, z, xs, total;
};

// rec: obstacle records (three float4 arrays of M, structure of arrays); xt:
// per-wave transpose buffers (kXtBlock floats per 16-step block); gp: double-buffered partial right-hand sides
// (256 per block); fin: per-(t, sample) residual^2 and c1 of the final pass;
// cm: per-wave obstacle candidate masks (4 words per 64 obstacles); xs: the
// block's samples; mu/L/z: sampler staging.  NB = 16-step blocks of the
// launch, SPB = samples per block.
// MB: partial slots per buffer, a compile-time bound >= NB for the sum
// (slots NB..MB-1 hold zeros).
__host__ __device__ inline Layout layout(int dims, int nv, int M, int NB, int MB, int SPB, int mode) {
  Layout l{};
  const int D = dims * nv, D4 = round4(D);
  int o = 0;
  l.rec = o; o += 12 * M;
  l.xt = o;  o += NB * kXtBlock;
  l.gp = o;  o += 2 * MB * 256;
  l.fin = o; o += 2 * 16 * NB * SPB;
  l.hist = o; o += 2 * 16 * NB * SPB;
  l.cm = o;  o += NB * 4 * ((M + 63) / 64);
  l.xs = o;  o += SPB * D4;
  l.mu = o;
  l.L = o + D4;
  l.z = o + D4 + round4(D * D);
  if (mode != kFromInput) o += D4 + round4(D * D) + SPB * D4;
  l.total = o;
  return l;
}

// ---------------------------------------------------------------------------
// Push-outs of one (sample, t) item (eqs. (15a)-(15c), (11a)-(11b) -> (13)).
//
// Obstacle records (scene order), three float4 each:
//   R0 = (cx, cy, cz, cull)   cull = max(a, b) * 1.001 + 1e-4
//   R1 = (vx, vy, vz, |v|)
//   R2 = (a, a^2 (2D) or rsq(1/b^2) (3D), 1/a^2, 1/b^2)
// 2D uses circles of radius a (cz = vz = 0).  The push-out of obstacle j on a
// robot at p is Delta (max(1, n)/n - 1) with Delta = p - o_j(t) and n the
// scaled distance, i.e. f = max(0, a/|Delta| - 1) in 2D and
// f = max(0, 1/n - 1) in 3D; a zero offset takes the canonical direction
// (+x in 2D, +z in 3D).
//
// Culling: a wave tests all obstacles at once against the bounding box of its
// 64 item positions (centre at the middle of the wave's time window, radius
// cull + |v| * half-window) and loops only over the obstacles that may touch
// the box.  A skipped obstacle is farther than a * 1.001 + 1e-4 from every
// item, where the push-out is exactly 0, so culling does not change results.
// ---------------------------------------------------------------------------
constexpr float kTiny = 1.0e-36f;

// Obstacle candidates processed together in the push-out loop.
#ifndef PRIEST_CAND_UNROLL
#define PRIEST_CAND_UNROLL 1
#endif
constexpr int kCandUnroll = PRIEST_CAND_UNROLL;

// Wave-wide min / max: DPP within each row of 16 lanes (xor 1, xor 2,
// rotate 4, rotate 8), then the four row results combined as uniform values.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, 0xF,
                                                    0xF, false));
}
__device__ __forceinline__ float lane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ float wave_min(float v) {
  v = fminf(v, dpp<0xB1>(v));   // quad_perm [1,0,3,2]
  v = fminf(v, dpp<0x4E>(v));   // quad_perm [2,3,0,1]
  v = fminf(v, dpp<0x124>(v));  // row_ror:4
  v = fminf(v, dpp<0x128>(v));  // row_ror:8
  return fminf(fminf(lane_f(v, 0), lane_f(v, 16)), fminf(lane_f(v, 32), lane_f(v, 48)));
}
// Minimum / maximum over each row of 16 lanes, returned for all four rows.
__device__ __forceinline__ void row_min4(float v, float out[4]) {
  v = fminf(v, dpp<0xB1>(v));
  v = fminf(v, dpp<0x4E>(v));
  v = fminf(v, dpp<0x124>(v));
  v = fminf(v, dpp<0x128>(v));
#pragma unroll
  for (int q = 0; q < 4; ++q) out[q] = lane_f(v, 16 * q);
}
__device__ __forceinline__ void row_max4(float v, float out[4]) {
  v = fmaxf(v, dpp<0xB1>(v));
  v = fmaxf(v, dpp<0x4E>(v));
  v = fmaxf(v, dpp<0x124>(v));
  v = fmaxf(v, dpp<0x128>(v));
#pragma unroll
  for (int q = 0; q < 4; ++q) out[q] = lane_f(v, 16 * q);
}

struct Rec {  // one obstacle record held in (uniform) registers
  float cx, cy, cz, vx, vy, vz, a, a2, ia2, ib2;
  float mab;  // smaller semi-axis (3D; read only for clearance bounds)
  bool moving;
};

// Record of lane b broadcast to the wave; only the fields the push-out of a
// DIMS-dimensional, static or moving obstacle reads.
template <int DIMS>
__device__ __forceinline__ Rec rec_from_lane(const float4& R0, const float4& R1, const float4& R2,
                                             int b, bool moving) {
  Rec r;
  r.moving = moving;
  r.cx = lane_f(R0.x, b);
  r.cy = lane_f(R0.y, b);
  r.cz = (DIMS == 3) ? lane_f(R0.z, b) : 0.0f;
  r.vx = moving ? lane_f(R1.x, b) : 0.0f;
  r.vy = moving ? lane_f(R1.y, b) : 0.0f;
  r.vz = (moving && DIMS == 3) ? lane_f(R1.z, b) : 0.0f;
  r.a = (DIMS == 2) ? lane_f(R2.x, b) : 0.0f;
  r.a2 = (DIMS == 2) ? lane_f(R2.y, b) : 0.0f;
  r.ia2 = (DIMS == 3) ? lane_f(R2.z, b) : 0.0f;
  r.ib2 = (DIMS == 3) ? lane_f(R2.w, b) : 0.0f;
  return r;
}

__device__ __forceinline__ Rec rec_from_lds(const float4* rec, int M, int j) {
  const float4 R0 = rec[j], R1 = rec[M + j], R2 = rec[2 * M + j];
  Rec r;
  r.cx = R0.x; r.cy = R0.y; r.cz = R0.z;
  r.vx = R1.x; r.vy = R1.y; r.vz = R1.z;
  r.moving = R1.w != 0.0f;
  r.a = R2.x; r.a2 = R2.y; r.ia2 = R2.z; r.ib2 = R2.w;
  return r;
}

// Push-out of one obstacle on one item, accumulated into s.  LAST: exact
// hit test (so satisfied constraints give exactly 0) and r2 += |delta|^2.
// Returns true if the offset is exactly zero (the caller adds the canonical
// push-out for those lanes).
template <int DIMS, bool LAST>
__device__ __forceinline__ bool pair_push(const Rec& o, float tt, const float p[DIMS],
                                          float s[DIMS], float& r2) {
  float d[DIMS];
  if (o.moving) {
    d[0] = p[0] - fmaf(o.vx, tt, o.cx);
    d[1] = p[1] - fmaf(o.vy, tt, o.cy);
    if constexpr (DIMS == 3) d[2] = p[2] - fmaf(o.vz, tt, o.cz);
  } else {
    d[0] = p[0] - o.cx;
    d[1] = p[1] - o.cy;
    if constexpr (DIMS == 3) d[2] = p[2] - o.cz;
  }
  const float h = fmaf(d[1], d[1], d[0] * d[0]);
  float q, f, len2;
  if constexpr (DIMS == 2) {
    q = h;
    len2 = h;
    f = fmaf(o.a, rsq(fmaxf(q, kTiny)), -1.0f);
    if (LAST) f = (q < o.a2) ? f : 0.0f;
  } else {
    q = fmaf(d[2] * d[2], o.ib2, h * o.ia2);
    len2 = fmaf(d[2], d[2], h);
    f = rsq(fmaxf(q, kTiny)) - 1.0f;
    if (LAST) f = (q < 1.0f) ? f : 0.0f;
  }
  f = fmaxf(f, 0.0f);
#pragma unroll
  for (int x = 0; x < DIMS; ++x) s[x] = fmaf(d[x], f, s[x]);
  if (LAST) r2 = fmaf(len2 * f, f, r2);
  return q == 0.0f;
}

// The same push-out split in two so that the independent parts of several
// obstacles can interleave: pair_term computes the offset and the factor
// (MOVING: centre advanced to time t), pair_add accumulates them in the
// order the caller adds obstacles.  A zero offset gets its canonical push-out
// through kNudge.
template <int DIMS>
struct PairTerm {
  float d[DIMS];
  float f, len2;
  float sq;  // sqrt(q) from the same rsq (for clearance bounds; unused otherwise)
};

// Added to the canonical component of every offset (x in 2D, z in 3D): it is
// below half an ulp of any offset above about 2e-8, so those are unchanged,
// and it turns an offset of exactly zero into one of 1e-15 along the
// canonical axis, whose push-out is the semi-axis up to rounding, so the
// pair loop needs no test for that case.  Its square over b^2 (1e-30 / b^2)
// must stay above the clamp kTiny, which holds for semi-axes up to 1000.
constexpr float kNudge = 1.0e-15f;

template <int DIMS, bool LAST, bool MOVING>
__device__ __forceinline__ PairTerm<DIMS> pair_term(const Rec& o, float tt, const float p[DIMS]) {
  PairTerm<DIMS> r;
  if constexpr (MOVING) {
    r.d[0] = p[0] - fmaf(o.vx, tt, o.cx);
    r.d[1] = p[1] - fmaf(o.vy, tt, o.cy);
    if constexpr (DIMS == 3) r.d[2] = p[2] - fmaf(o.vz, tt, o.cz);
  } else {
    r.d[0] = p[0] - o.cx;
    r.d[1] = p[1] - o.cy;
    if constexpr (DIMS == 3) r.d[2] = p[2] - o.cz;
  }
  r.d[DIMS == 2 ? 0 : 2] += kNudge;
  const float h = fmaf(r.d[1], r.d[1], r.d[0] * r.d[0]);
  float q, f;
  if constexpr (DIMS == 2) {
    q = h;
    r.len2 = h;
    const float rq = rsq(fmaxf(q, kTiny));
    f = fmaf(o.a, rq, -1.0f);
    r.sq = q * rq;
    if (LAST) f = (q < o.a2) ? f : 0.0f;
  } else {
    q = fmaf(r.d[2] * r.d[2], o.ib2, h * o.ia2);
    r.len2 = fmaf(r.d[2], r.d[2], h);
    const float rq = rsq(fmaxf(q, kTiny));
    f = rq - 1.0f;
    r.sq = q * rq;
    if (LAST) f = (q < 1.0f) ? f : 0.0f;
  }
  r.f = fmaxf(f, 0.0f);
  return r;
}

// Lower bound on how far (Euclidean) the item may move before this pair's
// push-out, as the kernel computes it, can become nonzero: the push is zero
// while the scaled distance sqrt(q) (|d| / a in 2D) stays >= 1 + 1e-5, where
// the rounding of q, rsq and the factor cannot make f positive; the scaled
// distance changes by at most |move| / (smaller semi-axis); sqrt(q) from the
// rsq is taken 1e-6 low.  Negative inside that margin.
template <int DIMS>
__device__ __forceinline__ float pair_clearance(const Rec& o, const PairTerm<DIMS>& t) {
  if constexpr (DIMS == 2) return fmaf(t.sq, 0.999999f, -1.00001f * o.a);
  return fmaf(t.sq, 0.999999f, -1.00001f) * o.mab;
}

// ACC: also accumulate the squared push-out length into r2.
template <int DIMS, bool ACC>
__device__ __forceinline__ void pair_add(const Rec& o, const PairTerm<DIMS>& t, float s[DIMS],
                                         float& r2) {
  constexpr bool LAST = ACC;
#pragma unroll
  for (int x = 0; x < DIMS; ++x) s[x] = fmaf(t.d[x], t.f, s[x]);
  if (LAST) r2 = fmaf(t.len2 * t.f, t.f, r2);
}

// Record of lane b broadcast to the wave (velocity only if MOVING).
template <int DIMS, bool MOVING>
__device__ __forceinline__ Rec rec_of_lane(const float4& R0, const float4& R1, const float4& R2,
                                           int b) {
  Rec r;
  r.moving = MOVING;
  r.cx = lane_f(R0.x, b);
  r.cy = lane_f(R0.y, b);
  r.cz = (DIMS == 3) ? lane_f(R0.z, b) : 0.0f;
  r.vx = MOVING ? lane_f(R1.x, b) : 0.0f;
  r.vy = MOVING ? lane_f(R1.y, b) : 0.0f;
  r.vz = (MOVING && DIMS == 3) ? lane_f(R1.z, b) : 0.0f;
  r.a = (DIMS == 2) ? lane_f(R2.x, b) : 0.0f;
  r.a2 = lane_f(R2.y, b);
  r.ia2 = (DIMS == 3) ? lane_f(R2.z, b) : 0.0f;
  r.ib2 = (DIMS == 3) ? lane_f(R2.w, b) : 0.0f;
  // (3D keeps b = rsq(1/b^2) in place of a^2)
  r.mab = (DIMS == 3) ? fminf(lane_f(R2.x, b), r.a2) : r.a;
  return r;
}

// Record j read from the LDS table by every lane of the wave (j the same in
// all of them: a broadcast), with only the fields the push-out of a
// DIMS-dimensional, static or moving obstacle reads: the same values as
// rec_of_lane.
template <int DIMS, bool MOVING>
__device__ __forceinline__ Rec rec_at(const float4* rec, int M, int j) {
  const float4 R0 = rec[j], R2 = rec[2 * M + j];
  Rec r;
  r.moving = MOVING;
  r.cx = R0.x;
  r.cy = R0.y;
  r.cz = (DIMS == 3) ? R0.z : 0.0f;
  r.vx = r.vy = r.vz = 0.0f;
  if constexpr (MOVING) {
    const float4 R1 = rec[M + j];
    r.vx = R1.x;
    r.vy = R1.y;
    r.vz = (DIMS == 3) ? R1.z : 0.0f;
  }
  r.a = (DIMS == 2) ? R2.x : 0.0f;
  r.a2 = R2.y;
  r.ia2 = (DIMS == 3) ? R2.z : 0.0f;
  r.ib2 = (DIMS == 3) ? R2.w : 0.0f;
  r.mab = (DIMS == 3) ? fminf(R2.x, R2.y) : R2.x;
  return r;
}

// Canonical push-out of a zero offset (+x by a in 2D, +z by b in 3D).
template <int DIMS, bool LAST>
__device__ __forceinline__ void zero_push(const Rec& o, float s[DIMS], float& r2) {
  if constexpr (DIMS == 2) {
    s[0] += o.a;
    if (LAST) r2 += o.a2;
  } else {
    const float b = rsq(o.ib2);
    s[2] += b;
    if (LAST) r2 = fmaf(b, b, r2);
  }
}

// Push-out of a norm bound |w| <= wmax (eqs. (11a)-(11b)): d = w (wmax/|w| - 1)
// when violated, else 0; r2 += |d|^2 as one explicit fma (ww f) f + r2, so
// that every kernel rounds it the same way.
template <int DIMS>
__device__ __forceinline__ void bound_push(const float w[DIMS], float wmax, float d[DIMS], float& r2) {
  float ww = 0.0f;
#pragma unroll
  for (int x = 0; x < DIMS; ++x) ww = fmaf(w[x], w[x], ww);
  float f = 0.0f;
  if (ww > wmax * wmax) f = fmaf(wmax, rsq(ww), -1.0f);
#pragma unroll
  for (int x = 0; x < DIMS; ++x) d[x] = w[x] * f;
  r2 = fmaf(ww * f, f, r2);
}

// Weighted trajectory cost of one (sample, step) item: acceleration,
// regularised curvature, distance to the start-goal segment (clamped
// projection; s = start, u = goal - start, iuu = 1 / |u|^2 or 0) and the
// squared steering angle of a car-like robot (2D).
template <int DIMS>
__device__ __forceinline__ float weighted_cost(const float p[DIMS], const float v[DIMS],
                                               const float ac[DIMS], const CostArgs& k,
                                               const float s[DIMS], const float u[DIMS], float iuu) {
  float c = 0.0f;
  if (k.w_acc != 0.0f) {
    float aa = 0.0f;
#pragma unroll
    for (int x = 0; x < DIMS; ++x) aa = fmaf(ac[x], ac[x], aa);
    c = fmaf(k.w_acc, aa, c);
  }
  if (k.w_curv != 0.0f || k.w_steer != 0.0f) {
    float vv = k.eps;
#pragma unroll
    for (int x = 0; x < DIMS; ++x) vv = fmaf(v[x], v[x], vv);
    const float inv = 1.0f / (vv * sqrtf(vv));  // (|v|^2 + eps)^(-3/2)
    float cr2, crs = 0.0f;
    if constexpr (DIMS == 2) {
      crs = v[0] * ac[1] - v[1] * ac[0];
      cr2 = crs * crs;
    } else {
      const float c0 = v[1] * ac[2] - v[2] * ac[1];
      const float c1 = v[2] * ac[0] - v[0] * ac[2];
      const float c2 = v[0] * ac[1] - v[1] * ac[0];
      cr2 = c0 * c0 + c1 * c1 + c2 * c2;
    }
    if (k.w_curv != 0.0f) c = fmaf(k.w_curv, cr2 * inv * inv, c);
    if constexpr (DIMS == 2) {
      if (k.w_steer != 0.0f) {
        const float d = atanf(k.wheelbase * crs * inv);
        c = fmaf(k.w_steer, d * d, c);
      }
    }
  }
  if (k.w_path != 0.0f) {
    float rel[DIMS], ru = 0.0f;
#pragma unroll
    for (int x = 0; x < DIMS; ++x) {
      rel[x] = p[x] - s[x];
      ru = fmaf(rel[x], u[x], ru);
    }
    const float lam = fminf(fmaxf(ru * iuu, 0.0f), 1.0f);
    float qq = 0.0f;
#pragma unroll
    for (int x = 0; x < DIMS; ++x) {
      const float q = fmaf(-lam, u[x], rel[x]);
      qq = fmaf(q, q, qq);
    }
    c = fmaf(k.w_path, sqrtf(qq), c);
  }
  return c;
}

// Record table of one scene (any number of threads).
template <int DIMS, bool TRAJ = false>
__device__ void build_records(const float* obs, int M, int t, int nt, float4* rec, int K = 0) {
  // TRAJ: rows of K positions then (a, b); the record holds the centre and
  // radius of a sphere around the whole path (R1 = (radius, 0, 0, 0)), which
  // the cull test treats as a static obstacle grown by that radius
  const int width = TRAJ ? K * DIMS + 2 : 8;
  for (int j = t; j < M; j += nt) {
    const float* o = obs + static_cast<int64_t>(width) * j;
    const float a = o[width - 2], b = (DIMS == 3) ? o[width - 1] : o[width - 2];
    float c[3] = {o[0], o[1], DIMS == 3 ? o[2] : 0.0f}, v[3] = {0.0f, 0.0f, 0.0f};
    float sp = 0.0f;
    if constexpr (TRAJ) {
      float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
      for (int k = 0; k < K; ++k)
        for (int x = 0; x < DIMS; ++x) {
          lo[x] = fminf(lo[x], o[k * DIMS + x]);
          hi[x] = fmaxf(hi[x], o[k * DIMS + x]);
        }
      for (int x = 0; x < DIMS; ++x) c[x] = 0.5f * (lo[x] + hi[x]);
      for (int k = 0; k < K; ++k) {
        float d2 = 0.0f;
        for (int x = 0; x < DIMS; ++x) {
          const float e = o[k * DIMS + x] - c[x];
          d2 = fmaf(e, e, d2);
        }
        sp = fmaxf(sp, d2);
      }
      sp = sqrtf(sp) * 1.0001f + 1.0e-5f;  // rounding margin of the bound
      rec[j] = make_float4(c[0], c[1], c[2], fmaxf(a, b) * 1.001f + 1.0e-4f);
      rec[M + j] = make_float4(sp, 0.0f, 0.0f, 0.0f);
    } else {
      v[0] = o[3];
      v[1] = o[4];
      v[2] = (DIMS == 3) ? o[5] : 0.0f;
      sp = sqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      rec[j] = make_float4(c[0], c[1], c[2], fmaxf(a, b) * 1.001f + 1.0e-4f);
      rec[M + j] = make_float4(v[0], v[1], v[2], sp);
    }
    // 3D keeps rsq(1/b^2), the canonical zero-offset push-out, in place of a^2
    const float ib2 = 1.0f / (b * b);
    rec[2 * M + j] = make_float4(a, (DIMS == 3) ? rsq(ib2) : a * a, 1.0f / (a * a), ib2);
  }
}

// Coefficient held at row slot 4 q + r of the MFMA layouts (coefficient rows
// of xi_bar, lambda, g and the KKT blocks): slots r = 0..2 of the four q carry
// coefficients 0..11 and slot r = 3 carries 12..15, so for n_coeff <= 12 the
// k-chunk r = 3 of every product over coefficients is zero and is skipped.
__device__ __forceinline__ int coef_of(int q, int r) { return r < 3 ? 3 * q + r : 12 + q; }

// Groups of 64 obstacles whose candidate masks stay in (scalar) registers;
// the masks of further groups live in LDS.
constexpr int kRegGroups = 2;

// Per-wave memory of the last obstacle cull: every item's position when the
// candidate sets were built, the displacement (squared) up to which they stay
// valid, and the candidate and moving bits of the first kRegGroups groups of
// 64 obstacles (wave-uniform).  Masks of later groups live in LDS (4 words
// per group).
template <int NI, int DIMS, int REG = kRegGroups>
struct CullCache {
  float pref[NI][DIMS];
  float lim2;
  bool valid;
  uint32_t nok;    // valid items of the wave (wave-uniform)
  uint32_t pairs;  // (item, obstacle) pairs evaluated by the wave so far
  bool rebuilt;    // the last call built new candidate sets
  unsigned long long cm[REG > 0 ? REG : 1], mv[REG > 0 ? REG : 1];
};

// Growth of the candidate radius that lets a candidate set be reused: an
// obstacle is a candidate if it may come within (1 + kSlack) * cull of the
// wave's box, and the set is reused while no item has moved farther than
// kSlack * (smallest cull radius) from where it was when the set was built.
// A skipped obstacle then stays farther than its cull radius from every item,
// where its push-out is exactly zero.
#ifndef PRIEST_CULL_SLACK
#define PRIEST_CULL_SLACK 0.25f
#endif
constexpr float kSlack = PRIEST_CULL_SLACK;

// Obstacle push-outs of this lane's NI items, summed over obstacles, with
// wave-level culling.  tmid / thalf: centre and half-width of the wave's time
// window.  Candidates are added in one canonical order: per group of 64, the
// static obstacles by index, then the moving ones by index.
template <int DIMS, bool LAST, int NI, bool HIST = false, bool TRAJ = false, int REG = kRegGroups>
__device__ __forceinline__ void obstacle_pushes(const float4* rec, int M, const float tt[NI],
                                                const float tmid[4], const float thalf[4],
                                                const bool ok[NI],
                                                const float p[NI][DIMS], float S[NI][DIMS],
                                                float r2[NI], int lane, CullCache<NI, DIMS, REG>& cc,
                                                uint32_t* wm, const float* opath = nullptr,
                                                const int* tstep = nullptr, int K = 0) {
  // records of the first group, issued before anything waits on LDS
  const float4 zr = make_float4(0, 0, 0, 0);
  // (lanes past the scene load the last record: only lanes of obstacles are
  // ever read, and unconditional loads keep the compiler from putting each one
  // under a branch of its own)
  auto clampj = [M](int j) { return j < M ? j : M - 1; };
  float4 G0 = zr, G1 = zr, G2 = zr;
  if (M > 0) {
    const int l0 = clampj(lane);
    G0 = rec[l0];
    G1 = rec[M + l0];
    G2 = rec[2 * M + l0];
  }
  // reuse the candidate sets if every item is still within the slack
  bool reuse = false;
  if (cc.valid) {
    bool far = false;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      float d2 = 0.0f;
#pragma unroll
      for (int x = 0; x < DIMS; ++x) {
        const float e = p[i][x] - cc.pref[i][x];
        d2 = fmaf(e, e, d2);
      }
      far = far || (ok[i] && !(d2 <= cc.lim2));
    }
    reuse = __ballot(far) == 0ull;
  }
  cc.rebuilt = !reuse;
  if (!reuse) {
    // one box per row of 16 lanes (the items of 4 time steps): an obstacle is
    // a candidate if it may come near any of the four
    float lo[DIMS][4], hi[DIMS][4];
#pragma unroll
    for (int x = 0; x < DIMS; ++x) {
      float mn = INFINITY, mx = -INFINITY;
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        mn = fminf(mn, ok[i] ? p[i][x] : INFINITY);
        mx = fmaxf(mx, ok[i] ? p[i][x] : -INFINITY);
      }
      row_min4(mn, lo[x]);
      row_max4(mx, hi[x]);
    }
    float cmin = INFINITY;
    auto cull_group = [&](int g, float4 R0, float4 R1, unsigned long long& mask,
                          unsigned long long& moving) {
      const int j = 64 * g + lane;
      bool cand = false, mv = false;
      if (j < M) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          // (paths: the sphere around the whole path, grown by its radius)
          const float oc[3] = {TRAJ ? R0.x : fmaf(R1.x, tmid[q], R0.x),
                               TRAJ ? R0.y : fmaf(R1.y, tmid[q], R0.y),
                               TRAJ ? R0.z : fmaf(R1.z, tmid[q], R0.z)};
          float d2 = 0.0f;
#pragma unroll
          for (int x = 0; x < DIMS; ++x) {
            const float e = fmaxf(fmaxf(lo[x][q] - oc[x], oc[x] - hi[x][q]), 0.0f);
            d2 = fmaf(e, e, d2);
          }
          const float rr = TRAJ ? fmaf(R0.w, 1.0f + kSlack, R1.x)
                                : fmaf(R1.w, thalf[q], R0.w * (1.0f + kSlack));
          cand = cand || (d2 < rr * rr);
        }
        mv = !TRAJ && R1.w != 0.0f;
        cmin = fminf(cmin, R0.w);
      }
      mask = __ballot(cand);
      moving = __ballot(cand && mv);
    };
#pragma unroll
    for (int g = 0; g < REG; ++g) {
      cc.cm[g] = 0ull;
      cc.mv[g] = 0ull;
      if (64 * g < M) {
        const int j = 64 * g + lane;
        const float4 R0 = g == 0 ? G0 : rec[clampj(j)];
        const float4 R1 = g == 0 ? G1 : rec[M + clampj(j)];
        cull_group(g, R0, R1, cc.cm[g], cc.mv[g]);
      }
    }
    for (int g = REG; 64 * g < M; ++g) {
      const int j = 64 * g + lane;
      unsigned long long mask, moving;
      cull_group(g, rec[clampj(j)], rec[M + clampj(j)], mask, moving);
      if (lane == 0) {
        wm[4 * g + 0] = static_cast<uint32_t>(mask);
        wm[4 * g + 1] = static_cast<uint32_t>(mask >> 32);
        wm[4 * g + 2] = static_cast<uint32_t>(moving);
        wm[4 * g + 3] = static_cast<uint32_t>(moving >> 32);
      }
    }
    const float lim = kSlack * wave_min(cmin);
    cc.lim2 = lim * lim;
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int x = 0; x < DIMS; ++x) cc.pref[i][x] = p[i][x];
    cc.valid = true;
    if (M > 64 * REG) wave_lds_sync();
  }
  uint32_t ncand = 0;
  // the candidates of one group, kCandUnroll at a time (their offsets and
  // factors are independent), added in the canonical order, the tail one at a
  // time; R0..R2 hold the group's records, obstacle 64 g + lane in this lane
  auto group = [&](int base, unsigned long long cmask, unsigned long long mvmask, float4 R0,
                   float4 R1, float4 R2) {
    if constexpr (TRAJ) {
      // obstacle positions at each item's own time step, read from the path
      unsigned long long mask = cmask;
      while (mask) {
        const int b = __builtin_ctzll(mask);
        mask &= mask - 1;
        Rec o = rec_of_lane<DIMS, false>(R0, R1, R2, b);
        const float* path = opath + static_cast<int64_t>(base + b) * (K * DIMS + 2);
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          const float* pt = path + min(tstep[i], K - 1) * DIMS;
          o.cx = pt[0];
          o.cy = pt[1];
          if constexpr (DIMS == 3) o.cz = pt[2];
          pair_add<DIMS, LAST || HIST>(o, pair_term<DIMS, LAST, false>(o, tt[i], p[i]), S[i], r2[i]);
        }
      }
      return;
    }
    auto run = [&](unsigned long long mask, auto moving_tag) {
      constexpr bool MV = decltype(moving_tag)::value;
      while (mask) {
        if (__builtin_popcountll(mask) >= kCandUnroll) {
          Rec o[kCandUnroll];
#pragma unroll
          for (int u = 0; u < kCandUnroll; ++u) {
            o[u] = rec_of_lane<DIMS, MV>(R0, R1, R2, __builtin_ctzll(mask));
            mask &= mask - 1;
          }
          PairTerm<DIMS> tm[kCandUnroll][NI];
#pragma unroll
          for (int u = 0; u < kCandUnroll; ++u)
#pragma unroll
            for (int i = 0; i < NI; ++i) tm[u][i] = pair_term<DIMS, LAST, MV>(o[u], tt[i], p[i]);
#pragma unroll
          for (int u = 0; u < kCandUnroll; ++u)
#pragma unroll
            for (int i = 0; i < NI; ++i) pair_add<DIMS, LAST || HIST>(o[u], tm[u][i], S[i], r2[i]);
        } else {
          const Rec o0 = rec_of_lane<DIMS, MV>(R0, R1, R2, __builtin_ctzll(mask));
          mask &= mask - 1;
#pragma unroll
          for (int i = 0; i < NI; ++i)
            pair_add<DIMS, LAST || HIST>(o0, pair_term<DIMS, LAST, MV>(o0, tt[i], p[i]), S[i], r2[i]);
        }
      }
    };
    run(cmask & ~mvmask, std::false_type{});
    run(mvmask, std::true_type{});
  };
#pragma unroll
  for (int g = 0; g < REG; ++g) {
    const unsigned long long cmask = cc.cm[g];
    ncand += static_cast<uint32_t>(__builtin_popcountll(cmask));
    if (!cmask) continue;
    if (g == 0) {
      group(0, cmask, cc.mv[0], G0, G1, G2);
    } else {
      const int j = 64 * g + lane;
      group(64 * g, cmask, cc.mv[g], rec[clampj(j)], rec[M + clampj(j)], rec[2 * M + clampj(j)]);
    }
  }
  for (int g = REG; 64 * g < M; ++g) {
    const uint4 m4 = *reinterpret_cast<const uint4*>(wm + 4 * g);
    // (readfirstlane returns int: widen through uint32_t, not sign-extended)
    auto u64 = [](uint32_t lo, uint32_t hi) {
      return static_cast<unsigned long long>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(lo))) |
             (static_cast<unsigned long long>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(hi)))
              << 32);
    };
    const unsigned long long cmask = u64(m4.x, m4.y);
    ncand += static_cast<uint32_t>(__builtin_popcountll(cmask));
    if (!cmask) continue;
    const int j = 64 * g + lane;
    group(64 * g, cmask, u64(m4.z, m4.w), rec[clampj(j)], rec[M + clampj(j)],
          rec[2 * M + clampj(j)]);
  }
  cc.pairs += ncand * cc.nok;
#pragma unroll
  for (int i = 0; i < NI; ++i)
    if (!ok[i]) {
#pragma unroll
      for (int x = 0; x < DIMS; ++x) S[i][x] = 0.0f;
      r2[i] = 0.0f;
    }
}

template <int DIMS, bool LAST, int NI, bool HIST = false, bool TRAJ = false, int REG = kRegGroups>
__device__ __forceinline__ void item_push(const float4* rec, int M, const float tt[NI],
                                          const float tmid[4], const float thalf[4],
                                          const bool ok[NI], const float p[NI][DIMS],
                                          const float v[NI][DIMS], const float ac[NI][DIMS],
                                          float vmax, float amax, const Box& box,
                                          float S[NI][DIMS], float dv[NI][DIMS], float da[NI][DIMS],
                                          float r2[NI], int lane, CullCache<NI, DIMS, REG>& cc,
                                          uint32_t* wm, const float* opath = nullptr,
                                          const int* tstep = nullptr, int K = 0) {
#pragma unroll
  for (int i = 0; i < NI; ++i) {
#pragma unroll
    for (int x = 0; x < DIMS; ++x) { S[i][x] = 0.0f; dv[i][x] = 0.0f; da[i][x] = 0.0f; }
    r2[i] = 0.0f;
  }
  obstacle_pushes<DIMS, LAST, NI, HIST, TRAJ, REG>(rec, M, tt, tmid, thalf, ok, p, S, r2, lane, cc,
                                                    wm, opath, tstep, K);
#pragma unroll
  for (int i = 0; i < NI; ++i)
    if (ok[i]) {
      bound_push<DIMS>(v[i], vmax, dv[i], r2[i]);
      bound_push<DIMS>(ac[i], amax, da[i], r2[i]);
    }
  // workspace bounds: rows -P and P of G, whose targets min(tau, G xi_bar)
  // add clamp(p, lo, hi) - p to the position rows
  if (box.on) {
#pragma unroll
    for (int i = 0; i < NI; ++i)
      if (ok[i]) {
#pragma unroll
        for (int x = 0; x < DIMS; ++x) {
          const float e = fminf(fmaxf(p[i][x], box.lo[x]), box.hi[x]) - p[i][x];
          S[i][x] += e;
          r2[i] = fmaf(e, e, r2[i]);
        }
      }
  }
}

// One block's work: whole projections of tiles first, first + stride, ...
// below `total` (LOOP), or of tile `first` only; tile t holds samples
// [SPB*j, SPB*j + SPB) of problem t / blocks_per_problem, j its index within
// the problem.  The problem constants (W rows, M11, Pi) are loaded once per
// block.  AS: MFMA column slots per sample (4, or 2 in 2D); RT: 16-step time
// blocks per wave; MAXT: the launch bound.
template <int DIMS, int AS, int RT, int MAXT, bool BF16, bool LOOP, bool HIST = false,
          bool TRAJ = false>
__device__ __forceinline__ void project_block(const ProjArgs& a, int first, int stride, int total) {
  static_assert(AS == 4 || AS == 8 || (AS == 2 && DIMS == 2), "2 axis slots only hold 2D samples");
  constexpr int SPB = 16 / AS;           // samples per block
  // items per lane per time block; with 8 slots per sample only the lanes of
  // slots 0..3 carry an item (a wave holds 2 samples x 16 steps)
  constexpr int IPR = AS <= 4 ? 4 / AS : 1;
  constexpr int NI = RT * IPR;           // items per lane
  constexpr int MB = (MAXT / 64) * RT;   // 16-step block slots (power of two)
  extern __shared__ float4 sm4[];
  float* sm = reinterpret_cast<float*>(sm4);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, TW = blockDim.x >> 6;
  const int NB = TW * RT;
  const int nv = a.nv, K = a.K, M = a.M, D = DIMS * nv, D4 = round4(D);
  const Layout l = layout(DIMS, nv, M, NB, MB, SPB, a.mode);
  {
    // partial slots NB..MB-1 of both buffers stay zero (every reader passes
    // the barrier after the first tile's staging first)
    float* gz = sm + l.gp;
    for (int i = tid; i < (MB - NB) * 256; i += blockDim.x) {
      gz[NB * 256 + i] = 0.0f;
      gz[(MB + NB) * 256 + i] = 0.0f;
    }
  }
  // MFMA column layout: q = row group, col = AS*cs + cx
  const int q = lane >> 4, col = lane & 15, cs = col / AS, cx = col % AS;
  // items after the transpose: sample cs, step t0 + 16 rt + 4q + IPR cx + i
  const int t0 = 16 * RT * w;
  float tt[NI];
  int t_item[NI];
#pragma unroll
  for (int n = 0; n < NI; ++n) {
    t_item[n] = t0 + 16 * (n / IPR) + 4 * q + IPR * cx + (n % IPR);
    tt[n] = a.dt * static_cast<float>(t_item[n]);
  }
  // time window of each row of 16 lanes: steps t0 + 16 rt + 4 q + 0..3
  float tmid[4], thalf[4];
#pragma unroll
  for (int qq = 0; qq < 4; ++qq) {
    thalf[qq] = a.dt * (8.0f * (RT - 1) + 1.5f);
    tmid[qq] = a.dt * (static_cast<float>(t0 + 4 * qq) + 8.0f * (RT - 1) + 1.5f);
  }

  float4* rec = reinterpret_cast<float4*>(sm + l.rec);
  float* xs = sm + l.xs;

  // ---- per-lane MFMA operands and sample state -------------------------------
  float Af[RT][3][4], Ab[RT][3][4], Am[4], Ap[4];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int tf = t0 + 16 * rt + col, cf = coef_of(q, r);
        Af[rt][d][r] = (tf < K && cf < nv) ? a.W[(tf * 3 + d) * nv + cf] : 0.0f;
        const int tb = t0 + 16 * rt + 4 * q + r, cb = coef_of(col >> 2, col & 3);
        Ab[rt][d][r] = (tb < K && cb < nv) ? a.W[(tb * 3 + d) * nv + cb] : 0.0f;
      }
  const int crow = coef_of(col >> 2, col & 3);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ck = coef_of(q, r);
    const bool ok = (crow < nv) && (ck < nv);
    Am[r] = ok ? a.M11[crow * nv + ck] : 0.0f;
    Ap[r] = ok ? a.Pi[crow * nv + ck] : 0.0f;
  }
  const bool chunk3 = nv > 12;  // slot r = 3 holds coefficients 12..15
  const float rho = a.rho;
  f4 xb;
  // mixed precision: W^T rows as BF16, M11 as a BF16 hi/lo pair
  s4 Abf[RT][3], Mhi, Mlo;
  if constexpr (BF16) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int d = 0; d < 3; ++d)
        Abf[rt][d] = pack_bf16(Ab[rt][d][0], Ab[rt][d][1], Ab[rt][d][2], Ab[rt][d][3]);
    Mhi = pack_bf16(Am[0], Am[1], Am[2], Am[3]);
    Mlo = pack_bf16(Am[0] - from_bf16(Mhi[0]), Am[1] - from_bf16(Mhi[1]),
                    Am[2] - from_bf16(Mhi[2]), Am[3] - from_bf16(Mhi[3]));
  }
  float* xt = sm + l.xt + w * RT * kXtBlock;
  uint32_t* wm = reinterpret_cast<uint32_t*>(sm + l.cm) + w * 4 * ((M + 63) / 64);

  // Forward rows of this wave's time blocks, transposed to the item layout.
  auto forward = [&](float p[NI][DIMS], float v[NI][DIMS], float ac[NI][DIMS]) {
    const f4 z = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      // one accumulation chain per row type over k-chunks 0, 1, 2[, 3]; the
      // three chains interleave, so each product waits on nothing
      f4 Y0 = mfma(Af[rt][0][0], xb[0], z), Y1 = mfma(Af[rt][1][0], xb[0], z),
         Y2 = mfma(Af[rt][2][0], xb[0], z);
#pragma unroll
      for (int c = 1; c < 3; ++c) {
        Y0 = mfma(Af[rt][0][c], xb[c], Y0);
        Y1 = mfma(Af[rt][1][c], xb[c], Y1);
        Y2 = mfma(Af[rt][2][c], xb[c], Y2);
      }
      if (chunk3) {
        Y0 = mfma(Af[rt][0][3], xb[3], Y0);
        Y1 = mfma(Af[rt][1][3], xb[3], Y1);
        Y2 = mfma(Af[rt][2][3], xb[3], Y2);
      }
      float* x0 = xt + rt * kXtBlock + xt_at(lane);
      *reinterpret_cast<f4*>(x0) = Y0;
      *reinterpret_cast<f4*>(x0 + kXtRow) = Y1;
      *reinterpret_cast<f4*>(x0 + 2 * kXtRow) = Y2;
    }
    wave_lds_sync();
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int i = 0; i < IPR; ++i)
#pragma unroll
        for (int x = 0; x < DIMS; ++x) {
          const int src = rt * kXtBlock + xt_at(lane - cx + x) + IPR * cx + i;
          p[rt * IPR + i][x] = xt[src];
          v[rt * IPR + i][x] = xt[kXtRow + src];
          ac[rt * IPR + i][x] = xt[2 * kXtRow + src];
        }
    wave_lds_sync();
  };

  int cur_prob = -1;
  auto tile_body = [&](int t) {
    const int prob = t / a.blocks_per_problem;
    const int s0 = (t - prob * a.blocks_per_problem) * SPB;
    const int ns = min(SPB, a.N - s0);
    bool item_ok[NI];
#pragma unroll
    for (int n = 0; n < NI; ++n) item_ok[n] = (t_item[n] < K) && (cs < ns) && (AS <= 4 || cx < 4);
    // ---- scene records, samples ---------------------------------------------
    // (every reader of the previous tile's records passed the barrier that
    // precedes its epilogue)
    if (prob != cur_prob)
      build_records<DIMS, TRAJ>(a.obs + prob * a.obs_stride, M, tid, blockDim.x, rec, K);
    const float* opath = a.obs + prob * a.obs_stride;
    cur_prob = prob;
    if (a.mode == kFromInput) {
      const float* src = a.xi_in + prob * a.xi_in_stride + static_cast<int64_t>(s0) * D;
      for (int i = tid; i < ns * D; i += blockDim.x) xs[(i / D) * D4 + i % D] = src[i];
    } else {
      float* sMu = sm + l.mu;
      float* sL = sm + l.L;
      float* sZ = sm + l.z;
      const float* mu = a.mu + prob * a.mu_stride;
      const float* Lm = a.L + prob * a.L_stride;
      for (int i = tid; i < D; i += blockDim.x) sMu[i] = mu[i];
      for (int i = tid; i < D * D; i += blockDim.x) sL[i] = Lm[i];
      if (a.mode == kFromNoise) {
        const float* z = a.noise + prob * a.noise_stride + static_cast<int64_t>(s0) * D;
        for (int i = tid; i < ns * D; i += blockDim.x) sZ[(i / D) * D4 + i % D] = z[i];
      } else {
        const int nq = D4 / 4;
        const uint32_t stream = a.stream_base + static_cast<uint32_t>(prob);
        for (int i = tid; i < ns * nq; i += blockDim.x) {
          const int s = i / nq, qq = i - s * nq;
          float z[4];
          philox_normals4(a.seed, static_cast<uint32_t>(s0 + s), static_cast<uint32_t>(qq),
                          static_cast<uint32_t>(a.iter), stream, z);
          *reinterpret_cast<float4*>(sZ + s * D4 + 4 * qq) = make_float4(z[0], z[1], z[2], z[3]);
        }
      }
      __syncthreads();
      for (int i = tid; i < ns * D; i += blockDim.x) {
        const int s = i / D, d = i - s * D;
        const float* zz = sZ + s * D4;
        const float* Lr = sL + d * D;
        float x = sMu[d];
        for (int e = 0; e <= d; ++e) x = fmaf(Lr[e], zz[e], x);
        xs[s * D4 + d] = x;
      }
      __syncthreads();
      if (a.xi_src) {
        float* dst = a.xi_src + prob * a.xi_src_stride + static_cast<int64_t>(s0) * D;
        for (int i = tid; i < ns * D; i += blockDim.x) dst[i] = xs[(i / D) * D4 + i % D];
      }
    }
    __syncthreads();

    const bool colok = (cx < DIMS) && (cs < ns);
    const float* bc = a.bc + prob * a.bc_stride;
    f4 xi, c0v;
  #pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = coef_of(q, r);
      const bool ok = colok && (c < nv);
      xi[r] = ok ? xs[cs * D4 + cx * nv + c] : 0.0f;
      float s = 0.0f;
      if (ok)
        for (int i = 0; i < 6; ++i) s = fmaf(a.M12[c * 6 + i], bc[cx * 6 + i], s);
      c0v[r] = s;
    }
    xb = xi;
    f4 lam = {0.0f, 0.0f, 0.0f, 0.0f};
    CullCache<NI, DIMS> cull;
    cull.valid = false;
    cull.pairs = 0;
    cull.nok = 0;
#pragma unroll
    for (int n = 0; n < NI; ++n) cull.nok += static_cast<uint32_t>(__builtin_popcountll(__ballot(item_ok[n])));

    {
      // waves of mid-trajectory time blocks carry the most obstacle
      // candidates (the samples spread most there) and set the pace at every
      // barrier: they get issue priority over the wave that shares their SIMD
      // (C2 plan: 203.8 -> 199.3 us per launch; full launches unchanged)
      const int d2 = abs(2 * w - (TW - 1));
      const int pr = d2 >= 6 ? 0 : 3 - d2 / 2;
      if (pr == 3) __builtin_amdgcn_s_setprio(3);
      else if (pr == 2) __builtin_amdgcn_s_setprio(2);
      else if (pr == 1) __builtin_amdgcn_s_setprio(1);
      else __builtin_amdgcn_s_setprio(0);
    }
    // ---- projection iterations ---------------------------------------------------
    for (int k = 0; k < a.n_iter; ++k) {
      float p[NI][DIMS], v[NI][DIMS], ac[NI][DIMS];
      forward(p, v, ac);
      float S[NI][DIMS], dv[NI][DIMS], da[NI][DIMS], r2[NI];
      item_push<DIMS, false, NI, HIST, TRAJ>(rec, M, tt, tmid, thalf, item_ok, p, v, ac, a.vmax, a.amax,
                                             a.box, S, dv, da, r2, lane, cull, wm, opath, t_item, K);
      if constexpr (HIST) {
        // squared push-outs of this iteration per (t, sample), summed per
        // sample after the barrier below (double-buffered by iteration)
        float* hb = sm + l.hist + (k & 1) * 16 * NB * SPB;
  #pragma unroll
        for (int n = 0; n < NI; ++n)
          if (AS <= 4 || cx < 4) hb[t_item[n] * SPB + cs] = item_ok[n] ? r2[n] : 0.0f;
      }
      // back to the column layout: slot AS*i + x of the lane's f4 holds axis x
      // of item i
  #pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        f4 T0 = {0.0f, 0.0f, 0.0f, 0.0f}, T1 = T0, T2 = T0;
  #pragma unroll
        for (int i = 0; i < IPR; ++i)
  #pragma unroll
          for (int x = 0; x < DIMS; ++x) {
            T0[AS * i + x] = S[rt * IPR + i][x];
            T1[AS * i + x] = dv[rt * IPR + i][x];
            T2[AS * i + x] = da[rt * IPR + i][x];
          }
        float* x0 = xt + rt * kXtBlock + xt_at(lane);
        *reinterpret_cast<f4*>(x0) = T0;
        *reinterpret_cast<f4*>(x0 + kXtRow) = T1;
        *reinterpret_cast<f4*>(x0 + 2 * kXtRow) = T2;
      }
      wave_lds_sync();
      float B[RT][3][4];
  #pragma unroll
      for (int rt = 0; rt < RT; ++rt)
  #pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int src = rt * kXtBlock + xt_at(lane - cx + r / IPR) + AS * (r % IPR) + cx;
          // (8 slots: columns 4..7 of a sample are padding and stay zero)
          const bool pad = (AS == 8) && (cx >= 4);
          B[rt][0][r] = pad ? 0.0f : xt[src];
          B[rt][1][r] = pad ? 0.0f : xt[kXtRow + src];
          B[rt][2][r] = pad ? 0.0f : xt[2 * kXtRow + src];
        }
      const f4 zb = {0.0f, 0.0f, 0.0f, 0.0f};
      const bool lowp = BF16 && (k < a.bf16_iters);
      float* gp = sm + l.gp + (k & 1) * MB * 256;
      if (lowp) {
        // right-hand side with BF16 operands, FP32 accumulation: one K = 16
        // MFMA per row type covers a whole 16-step block
  #pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          f4 g = zb;
  #pragma unroll
          for (int d = 0; d < 3; ++d)
            g = mfma_bf16(Abf[rt][d], pack_bf16(B[rt][d][0], B[rt][d][1], B[rt][d][2], B[rt][d][3]), g);
          *reinterpret_cast<f4*>(gp + (w * RT + rt) * 256 + lane * 4) = g;
        }
      } else {
        f4 G[RT];
  #pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          // two accumulation chains over the three row types and four
          // k-chunks, added once at the end: one chain is faster for a lone
          // small launch, but its dependent products stall full launches
          // (N = 64000: 8.2 against 6.0 ms)
          constexpr int NCH = 2;
          f4 acc[NCH];
  #pragma unroll
          for (int c = 0; c < NCH; ++c) acc[c] = zb;
  #pragma unroll
          for (int d = 0; d < 3; ++d)
  #pragma unroll
            for (int r = 0; r < 4; ++r) acc[(4 * d + r) % NCH] = mfma(Ab[rt][d][r], B[rt][d][r], acc[(4 * d + r) % NCH]);
          f4 gs = acc[0];
  #pragma unroll
          for (int c = 1; c < NCH; ++c) gs = gs + acc[c];
          G[rt] = gs;
        }
        // issue the LDS reads before the MFMAs that consume them
        __builtin_amdgcn_sched_group_barrier(0x100, 12 * RT, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 12 * RT, 0);
  #pragma unroll
        for (int rt = 0; rt < RT; ++rt)
          *reinterpret_cast<f4*>(gp + (w * RT + rt) * 256 + lane * 4) = G[rt];
      }
      __syncthreads();
      // g = +0 + the block partials added one by one in time-block order
      // (slots NB..MB-1 hold +0, which leaves the sum unchanged).  No partial
      // is -0 (its MFMA chains start at +0), so neither is any sum, and a
      // partial of exact zeros leaves the sum as it is: the whole-horizon
      // shape adds only its nonzero partials and gets the same bits.
      f4 g = {0.0f, 0.0f, 0.0f, 0.0f};
  #pragma unroll
      for (int b = 0; b < MB; ++b) g = g + *reinterpret_cast<const f4*>(gp + b * 256 + lane * 4);
      if constexpr (HIST) {
        // ||F xi_bar^k - e^{k+1}|| per sample, summed over t in order
        if (tid < ns) {
          const float* hb = sm + l.hist + (k & 1) * 16 * NB * SPB;
          float h = 0.0f;
          for (int t = 0; t < K; ++t) h += hb[t * SPB + tid];
          a.resid_hist[static_cast<int64_t>(k) * a.N + s0 + tid] = sqrtf(h);
        }
      }
      lam += rho * g;
      const f4 z = {0.0f, 0.0f, 0.0f, 0.0f};
      if (k == 0) {
        const f4 u = lam + rho * g;
        const f4 h0 = mfma(Ap[1], xi[1], mfma(Ap[0], xi[0], c0v));
        f4 h1 = mfma(Ap[2], xi[2], z);
        const f4 h2 = mfma(Am[1], u[1], mfma(Am[0], u[0], z));
        f4 h3 = mfma(Am[2], u[2], z);
        if (chunk3) {
          h1 = mfma(Ap[3], xi[3], h1);
          h3 = mfma(Am[3], u[3], h3);
        }
        xb = (h0 + h1) + (h2 + h3);
      } else if (lowp) {
        // KKT product with BF16 hi/lo splits of M11 and u (three K = 16 MFMAs)
        const f4 u = (xi - xb) + lam + rho * g;
        const s4 uh = pack_bf16(u[0], u[1], u[2], u[3]);
        const s4 ul = pack_bf16(u[0] - from_bf16(uh[0]), u[1] - from_bf16(uh[1]),
                                u[2] - from_bf16(uh[2]), u[3] - from_bf16(uh[3]));
        // (the two small cross terms first, then the leading one, all into
        // one accumulator)
        xb = xb + mfma_bf16(Mhi, uh, mfma_bf16(Mlo, uh, mfma_bf16(Mhi, ul, z)));
      } else {
        // accumulated straight into xi_bar: one chain, no VALU sums
        const f4 u = (xi - xb) + lam + rho * g;
        xb = mfma(Am[2], u[2], mfma(Am[1], u[1], mfma(Am[0], u[0], xb)));
        if (chunk3) xb = mfma(Am[3], u[3], xb);
      }
    }

    // ---- residual and smoothness cost of the returned iterate -----------------------
    {
      float p[NI][DIMS], v[NI][DIMS], ac[NI][DIMS];
      forward(p, v, ac);
      float S[NI][DIMS], dv[NI][DIMS], da[NI][DIMS], r2[NI];
      item_push<DIMS, true, NI, false, TRAJ>(rec, M, tt, tmid, thalf, item_ok, p, v, ac, a.vmax, a.amax,
                                             a.box, S, dv, da, r2, lane, cull, wm, opath, t_item, K);
      float* fin = sm + l.fin;
      // segment of the path-following term: start p0 -> goal pf of this problem
      float sg[DIMS], ug[DIMS], iuu = 0.0f;
      if (a.cost.kind != 0) {
        float uu = 0.0f;
  #pragma unroll
        for (int x = 0; x < DIMS; ++x) {
          sg[x] = bc[x * 6 + 0];
          ug[x] = bc[x * 6 + 3] - sg[x];
          uu = fmaf(ug[x], ug[x], uu);
        }
        iuu = uu > 0.0f ? 1.0f / uu : 0.0f;
      }
  #pragma unroll
      for (int n = 0; n < NI; ++n) {
        float cc = 0.0f;
        if (a.cost.kind == 0) {
  #pragma unroll
          for (int x = 0; x < DIMS; ++x) cc = fmaf(ac[n][x], ac[n][x], cc);
        } else {
          cc = weighted_cost<DIMS>(p[n], v[n], ac[n], a.cost, sg, ug, iuu);
        }
        float* f = fin + 2 * (t_item[n] * SPB + cs);
        if (AS <= 4 || cx < 4) {  // lanes without items own no slot
          f[0] = item_ok[n] ? r2[n] : 0.0f;
          f[1] = item_ok[n] ? cc : 0.0f;
        }
      }
    }
    __syncthreads();
    if (tid < ns) {
      const int s = tid;
      float r2 = 0.0f, cc = 0.0f;
      for (int t = 0; t < K; ++t) {
        const float* f = sm + l.fin + 2 * (t * SPB + s);
        r2 += f[0];
        cc += f[1];
      }
      const float r = sqrtf(r2);
      const int64_t nb = prob * a.n_stride + s0 + s;
      const int64_t dense = static_cast<int64_t>(prob) * a.N + s0 + s;
      if (a.resid) a.resid[nb] = r;
      if (a.c1) a.c1[nb] = cc;
      if (a.resid2) a.resid2[dense] = r;
      if (a.c12) a.c12[dense] = cc;
    }
    if (a.pair_count && lane == 0) atomicAdd(a.pair_count, static_cast<unsigned long long>(cull.pairs));
    if (w == 0 && colok) {
      float* dst = a.xi_out + prob * a.xi_out_stride + static_cast<int64_t>(s0 + cs) * D + cx * nv;
      float* dst2 = a.xi_out2 ? a.xi_out2 + (static_cast<int64_t>(prob) * a.N + s0 + cs) * D + cx * nv
                              : nullptr;
  #pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = coef_of(q, r);
        if (c < nv) {
          dst[c] = xb[r];
          if (dst2) dst2[c] = xb[r];
        }
      }
    }
  };
  if constexpr (LOOP) {
    for (int t = first; t < total; t += stride) tile_body(t);
  } else {
    if (first < total) tile_body(first);
  }
}

// Uniform batch of `total` tiles (problem = tile / blocks_per_problem).  With
// a grid smaller than `total` (persistent launch) every block loops over
// tiles with stride gridDim.x.  When the grid is a multiple of the 8 XCDs,
// logical block ids are laid out so that each XCD (which receives every 8th
// hardware block) walks a contiguous range of tiles, keeping a problem's
// scene in one L2.
template <int DIMS, int AS, int RT, int MAXT, bool BF16, bool LOOP>
__global__ __launch_bounds__(MAXT) void project_kernel(ProjArgs a, int total) {
  const int G = gridDim.x;
  int lb = blockIdx.x;
  if ((G & 7) == 0) lb = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  project_block<DIMS, AS, RT, MAXT, BF16, LOOP>(a, lb, G, total);
}

// The default shape with the per-iteration residual history (HIST, one
// problem) and/or obstacles given by their paths (TRAJ); one block per tile.
template <int DIMS, int MAXT, bool BF16, bool HIST, bool TRAJ>
__global__ __launch_bounds__(MAXT) void project_special_kernel(ProjArgs a, int total) {
  project_block<DIMS, 4, 1, MAXT, BF16, false, HIST, TRAJ>(a, blockIdx.x, 1, total);
}

// Descriptor table (heterogeneous requests sharing n_steps): task t owns
// blocks [prefix[t], prefix[t+1]); every field of its ProjArgs is its own.
// Serving uses the default tile shape (4 axis slots, one time block per wave).
template <int DIMS, int MAXT, bool BF16>
__global__ __launch_bounds__(MAXT) void project_task_kernel(const ProjArgs* tasks,
                                                            const int* prefix, int n_tasks) {
  int lo = 0, hi = n_tasks;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= static_cast<int>(blockIdx.x)) lo = mid;
    else hi = mid;
  }
  project_block<DIMS, 4, 1, MAXT, BF16, false>(tasks[lo], static_cast<int>(blockIdx.x) - prefix[lo], 1,
                                              tasks[lo].blocks_per_problem);
}

// ---------------------------------------------------------------------------
// Whole-horizon tile shape (row_tiles = 0).  A wave owns 16/AS samples for
// every time step: per projection iteration it walks the 16-step time blocks
// of the horizon one after another, so the sum of the right-hand side over
// time stays inside the wave and no iteration needs a block barrier, a
// cross-wave partial sum or a KKT step repeated by every wave.  The waves of
// a block share only read-only tables in LDS (obstacle records and the W
// operands of every time block), so on a SIMD they drift out of step and
// the matrix core of one wave overlaps the vector work of another.
//
// Forward rows are computed with the sample coefficients as the MFMA A
// operand and the W rows as B (D = xi_bar W^T): lane l then holds time step
// l % 16 of columns 4 (l / 16) + 0..3, i.e. every axis of its (sample, t)
// items, with no transpose.  The right-hand side needs the time steps
// spread over lane groups (they are the reduction index), so the push-outs
// go back to the column layout through one LDS pass per time block: each
// item lane writes its four column values to four planes, and each column
// lane reads its four time steps from one plane with a 16-byte read.
//
// Each time block keeps its obstacle candidate cache (the grown boxes of
// the item positions it was built from and the candidate masks) in the
// wave's LDS region between iterations, so the block loop is not unrolled.
//
// Rows that cannot push are not evaluated.  Between two iterations the
// coefficients change by Delta, which moves row type d of any step by at
// most S_d max|Delta| (S_d: the largest absolute row sum of W's rows of that
// type).  Each wave keeps, per time block and row type, a budget: the margin
// found at the last evaluation (the distance of the items to the cache's
// grown boxes, or of |v|, |a| to v_max, a_max) over S_d, less the rounding
// of two MFMA evaluations, less the max|Delta| of every iteration since.
// While it is positive the row type's push-outs are exactly zero on every
// valid item, as a full evaluation would find: its forward MFMAs, bound
// checks and right-hand side are skipped.  A position budget is the smaller
// of the items' margin to the grown boxes and their clearance to every
// candidate obstacle (pair_clearance, over sqrt(dims)), and exists only
// while no position push-out is nonzero; when it runs out the items are
// checked against the grown boxes, and the cache is rebuilt only if one has
// left its box.
//
// The arithmetic per sample is that of the time-split shape: the same
// product chains per 16-step block (operands swapped in the forward rows,
// the same products in the same order), the per-block partial right-hand
// sides added in the same time-block order, the same push-out,
// multiplier and KKT steps, and the residual and cost summed in t order.
// ---------------------------------------------------------------------------
constexpr int kWaveMaxBlocks = 8;  // 16-step time blocks (n_steps <= 128)
constexpr int kPlane = 68;         // floats per transpose plane: 64 lanes + 4 (conflict-free reads)
constexpr int kWtabV4 = 3;         // float4 per lane and time block in the W table

struct WaveLayout {  // offsets into dynamic LDS, in floats
  int rec, wtab, wave, wave_floats, cache, cstride, mul, ctr, total;
};

// rec: obstacle records; wtab: per time block and lane the 12 forward-row B
// operands (rows P, Pdot, Pddot x 4 coefficient chunks; the right-hand side
// reads its A operands from them); wave: per wave 12
// transpose planes (3 quantities x 4 column residues), which also stage the
// wave's samples before it iterates (2 SPW D4 <= 768 floats), then per time
// block its candidate cache: words 0..31 the box of each row of 16 lanes grown
// by the reuse slack (low corner, high corner as float4), then 4 mask words
// per obstacle group (static, moving; 64 bits each); mul: the problem's mean
// and Cholesky factor (when the kernel draws the samples); ctr: the tile's
// group counter.
__host__ __device__ inline WaveLayout wave_layout(int dims, int nv, int M, int NB, int WPB,
                                                  int mode) {
  WaveLayout l{};
  const int D = dims * nv, D4 = round4(D), G = (M + 63) / 64;
  int o = 0;
  l.rec = o;  o += 12 * M;
  l.wtab = o; o += NB * kWtabV4 * 64 * 4;
  l.cache = 12 * kPlane;
  l.cstride = 32 + 4 * G;
  l.wave_floats = round4(l.cache + NB * l.cstride);
  l.wave = o; o += WPB * l.wave_floats;
  l.mul = o;
  if (mode != kFromInput) o += D4 + round4(D * D);
  l.ctr = o;  o += 4;
  l.total = o;
  return l;
}
static_assert(2 * 8 * ((3 * kMaxNV + 3) & ~3) <= 12 * kPlane, "a wave's samples fit its planes");

// Wave-wide maximum / minimum of floats that are >= +0 (or +inf / NaN),
// compared as their bit patterns, which orders them as floats (NaN above
// +inf): integer max / min with DPP operands within each row (xor 1, xor 2,
// half-row mirror, row mirror), then the rows combined through row
// broadcasts (lane 15 into rows 1 and 3, lane 31 into rows 2 and 3).
// (Lanes of rows that a broadcast leaves unwritten hold undefined values
// afterwards; lane 63, the only one read, takes its operands from written
// lanes only: lanes 15 and 47 after the row steps, lane 31 after the first
// broadcast.)
// Ballot of a per-lane condition: the 64-bit lane mask, taken from the
// condition itself (no round trip through an int).
__device__ __forceinline__ unsigned long long wballot(bool c) {
  return __builtin_amdgcn_ballot_w64(c);
}

template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ uint32_t dppu(uint32_t v) {
  return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(v), CTRL, ROWS, 0xF, true));
}
template <bool MAX>
__device__ __forceinline__ float wave_reduce_nn(float x) {
  auto op = [](uint32_t a, uint32_t b) { return MAX ? (a > b ? a : b) : (a < b ? a : b); };
  uint32_t v = __float_as_uint(x);
  v = op(v, dppu<0xB1>(v));
  v = op(v, dppu<0x4E>(v));
  v = op(v, dppu<0x141>(v));
  v = op(v, dppu<0x140>(v));
  v = op(v, dppu<0x142, 0xA>(v));
  v = op(v, dppu<0x143, 0xC>(v));
  return __uint_as_float(static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 63)));
}

// Minimum / maximum over each row of 16 lanes, left in every lane of the row.
__device__ __forceinline__ float row16_min(float v) {
  v = fminf(v, dpp<0xB1>(v));
  v = fminf(v, dpp<0x4E>(v));
  v = fminf(v, dpp<0x124>(v));
  return fminf(v, dpp<0x128>(v));
}
__device__ __forceinline__ float row16_max(float v) {
  v = fmaxf(v, dpp<0xB1>(v));
  v = fmaxf(v, dpp<0x4E>(v));
  v = fmaxf(v, dpp<0x124>(v));
  return fmaxf(v, dpp<0x128>(v));
}

// Builds the candidate cache of one 16-step block of the whole-horizon
// shape.  Each row of 16 lanes (one or two samples over the block's steps)
// gets the bounding box of its valid items; an obstacle is a candidate if its
// sphere, grown by sqrt(DIMS) * slack and by |v| * (half window) for a moving
// obstacle (centre taken at the window's middle), comes near any row's box.
// While every valid item lies in its row's box grown by `slack` per axis, it
// is at most sqrt(DIMS) * slack from the box, so a skipped obstacle stays
// farther than its cull radius (a * 1.001 + 1e-4 beyond the surface) from
// every item, where the push-out is exactly zero.  Writes the grown boxes and
// the masks; returns the candidate count.
template <int DIMS, int NI>
__device__ __forceinline__ uint32_t wave_block_cull(const float4* rec, int M, const float p[NI][DIMS],
                                                    const bool ok[NI], float tmid, float thalf,
                                                    float slack, int lane, uint32_t* cw) {
  float lo[DIMS], hi[DIMS];
#pragma unroll
  for (int x = 0; x < DIMS; ++x) {
    float mn = INFINITY, mx = -INFINITY;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      mn = fminf(mn, ok[i] ? p[i][x] : INFINITY);
      mx = fmaxf(mx, ok[i] ? p[i][x] : -INFINITY);
    }
    lo[x] = row16_min(mn);
    hi[x] = row16_max(mx);
  }
  if ((lane & 15) == 0) {
    float* bx = reinterpret_cast<float*>(cw) + 8 * (lane >> 4);
    *reinterpret_cast<float4*>(bx) = make_float4(lo[0] - slack, lo[1] - slack,
                                                 DIMS == 3 ? lo[DIMS - 1] - slack : 0.0f, 0.0f);
    *reinterpret_cast<float4*>(bx + 4) = make_float4(hi[0] + slack, hi[1] + slack,
                                                     DIMS == 3 ? hi[DIMS - 1] + slack : 0.0f, 0.0f);
  }
  float blo[DIMS][4], bhi[DIMS][4];
#pragma unroll
  for (int x = 0; x < DIMS; ++x)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      blo[x][q] = lane_f(lo[x], 16 * q);
      bhi[x][q] = lane_f(hi[x], 16 * q);
    }
  uint32_t* masks = cw + 32;
  const float grow = (DIMS == 3 ? 1.7320508f : 1.4142136f) * slack * 1.0001f;
  uint32_t ncand = 0;
  for (int g = 0; 64 * g < M; ++g) {
    const int j = 64 * g + lane;
    const int jc = j < M ? j : M - 1;
    const float4 R0 = rec[jc], R1 = rec[M + jc];
    const float oc[3] = {fmaf(R1.x, tmid, R0.x), fmaf(R1.y, tmid, R0.y), fmaf(R1.z, tmid, R0.z)};
    const float rr = fmaf(R1.w, thalf, R0.w + grow);
    bool cand = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float d2 = 0.0f;
#pragma unroll
      for (int x = 0; x < DIMS; ++x) {
        const float e = fmaxf(fmaxf(blo[x][q] - oc[x], oc[x] - bhi[x][q]), 0.0f);
        d2 = fmaf(e, e, d2);
      }
      cand = cand || (d2 < rr * rr);
    }
    cand = cand && (j < M);
    const unsigned long long mask = wballot(cand), moving = wballot(cand && R1.w != 0.0f);
    if (lane == 0) {
      *reinterpret_cast<uint4*>(masks + 4 * g) =
          make_uint4(static_cast<uint32_t>(mask), static_cast<uint32_t>(mask >> 32),
                     static_cast<uint32_t>(moving), static_cast<uint32_t>(moving >> 32));
    }
    ncand += static_cast<uint32_t>(__builtin_popcountll(mask));
  }
  wave_lds_sync();
  return ncand;
}

// Push-outs of this lane's items in one 16-step block of the whole-horizon
// shape (the per-pair and per-bound arithmetic of item_push, in the same
// canonical obstacle order) for the row types in `comp` (bit 0: obstacles
// and workspace bounds on the positions, bit 1: velocity, bit 2:
// acceleration); the push-outs of the other row types are zero on every
// valid item and are left at zero.  Position push-outs use the block's
// candidate cache.  With `test`, every valid item is first checked against
// its row's grown box: the cache is rebuilt if one is outside (or there is no
// cache yet, ncand = ~0), and pmargin (per lane) receives the smallest
// distance per axis from its valid items to its row's grown box (slack after
// a rebuild); lclear (per lane) takes the smallest clearance of its valid
// items to the candidates (pair_clearance; not in the final pass).  Items
// that are not valid
// still get finite push-outs, which the caller masks where they matter
// (steps past the horizon meet zero W rows in the right-hand side; columns of
// absent samples are never written out).  Returns which row types have a
// nonzero push-out on some valid item; wwv / wwa receive the largest |v|^2 /
// |a|^2 over the valid items when that row type has none (not in the final
// pass).
template <int DIMS, bool LAST, int NI>
__device__ __forceinline__ uint32_t wave_block_push(const float4* rec, int M, float tt, float tmid,
                                                    float thalf, float slack, uint32_t comp,
                                                    bool test, const bool ok[NI],
                                                    const float p[NI][DIMS], const float v[NI][DIMS],
                                                    const float ac[NI][DIMS], float vmax, float amax,
                                                    const Box& box, float S[NI][DIMS],
                                                    float dv[NI][DIMS], float da[NI][DIMS],
                                                    float r2[NI], int lane, uint32_t* cw,
                                                    uint32_t& ncand, uint32_t nok, uint32_t& pairs,
                                                    float& wwv, float& wwa, float& pmargin,
                                                    float& lclear) {
  // (dv / da are written below whenever their row type has a nonzero
  // push-out, the only case in which they are read)
#pragma unroll
  for (int i = 0; i < NI; ++i) {
#pragma unroll
    for (int x = 0; x < DIMS; ++x) S[i][x] = 0.0f;
    r2[i] = 0.0f;
  }
  if (comp & 1u) {
    if (test) {
      bool rebuild = ncand == ~0u;
      if (!rebuild) {
        const float* bx = reinterpret_cast<const float*>(cw) + 8 * (lane >> 4);
        const float4 glo = *reinterpret_cast<const float4*>(bx);
        const float4 ghi = *reinterpret_cast<const float4*>(bx + 4);
        const float gl[3] = {glo.x, glo.y, glo.z}, gh[3] = {ghi.x, ghi.y, ghi.z};
        // smallest signed distance of a valid item to its box, NaN if any is
        // (IEEE minimum: NaN-propagating), so an item is outside or not a
        // number exactly when the margin is not >= 0
        float mu = INFINITY;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          float mi = INFINITY;
#pragma unroll
          for (int x = 0; x < DIMS; ++x) {
            const int xx = (DIMS == 3 || x < 2) ? x : 2;
            mi = __builtin_elementwise_minimum(
                mi, __builtin_elementwise_minimum(p[i][x] - gl[xx], gh[xx] - p[i][x]));
          }
          mu = ok[i] ? __builtin_elementwise_minimum(mu, mi) : mu;
        }
        rebuild = wballot(!(mu >= 0.0f)) != 0ull;
        // (every valid distance is >= 0 here; the mask turns -0 into +0)
        if (!rebuild) pmargin = __uint_as_float(__float_as_uint(mu) & 0x7fffffffu);
      }
      if (rebuild) {
        ncand = wave_block_cull<DIMS, NI>(rec, M, p, ok, tmid, thalf, slack, lane, cw);
        pmargin = slack;
      }
    }
    if (ncand) {
      const uint32_t* masks = cw + 32;
      pairs += ncand * nok;
      float tt_[NI];
#pragma unroll
      for (int i = 0; i < NI; ++i) tt_[i] = tt;
      for (int g = 0; 64 * g < M; ++g) {
        const uint4 m4 = *reinterpret_cast<const uint4*>(masks + 4 * g);
        auto u64 = [](uint32_t lo, uint32_t hi) {
          return static_cast<unsigned long long>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(lo))) |
                 (static_cast<unsigned long long>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(hi))) << 32);
        };
        const unsigned long long cmask = u64(m4.x, m4.y);
        if (!cmask) continue;
        const unsigned long long mvmask = u64(m4.z, m4.w);
        unsigned long long ms = cmask & ~mvmask;
        while (ms) {
          const Rec o = rec_at<DIMS, false>(rec, M, 64 * g + __builtin_ctzll(ms));
          ms &= ms - 1;
#pragma unroll
          for (int i = 0; i < NI; ++i) {
            const PairTerm<DIMS> pt = pair_term<DIMS, LAST, false>(o, tt_[i], p[i]);
            pair_add<DIMS, LAST>(o, pt, S[i], r2[i]);
            if (!LAST) lclear = fminf(lclear, ok[i] ? pair_clearance<DIMS>(o, pt) : INFINITY);
          }
        }
        unsigned long long mm = mvmask;
        while (mm) {
          const Rec o = rec_at<DIMS, true>(rec, M, 64 * g + __builtin_ctzll(mm));
          mm &= mm - 1;
#pragma unroll
          for (int i = 0; i < NI; ++i) {
            const PairTerm<DIMS> pt = pair_term<DIMS, LAST, true>(o, tt_[i], p[i]);
            pair_add<DIMS, LAST>(o, pt, S[i], r2[i]);
            if (!LAST) lclear = fminf(lclear, ok[i] ? pair_clearance<DIMS>(o, pt) : INFINITY);
          }
        }
      }
    }
  }
  // velocity / acceleration bounds: the push-outs of a row type are computed
  // only when some valid item exceeds its bound (r2 += |d|^2 as the explicit
  // fma of bound_push; with f = 0 it leaves r2 unchanged, so items without a
  // violation need no update)
  uint32_t nz = 0;
  auto bounds = [&](const float (*w)[DIMS], float wmax, float (*d)[DIMS], uint32_t bit, float& wwm) {
    float ww[NI];
    bool any = false;
    float m = 0.0f;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      ww[i] = 0.0f;
#pragma unroll
      for (int x = 0; x < DIMS; ++x) ww[i] = fmaf(w[i][x], w[i][x], ww[i]);
      any = any | (ok[i] & (ww[i] > wmax * wmax));
      m = ok[i] ? fmaxf(m, ww[i]) : m;
    }
    if (wballot(any) == 0ull) {
      if (!LAST) wwm = wave_reduce_nn<true>(m);
    } else {
      nz |= bit;
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        float f = 0.0f;
        if (ww[i] > wmax * wmax) f = fmaf(wmax, rsq(ww[i]), -1.0f);
#pragma unroll
        for (int x = 0; x < DIMS; ++x) d[i][x] = w[i][x] * f;
        if (LAST) r2[i] = fmaf(ww[i] * f, f, r2[i]);
      }
    }
  };
  if (comp & 2u) bounds(v, vmax, dv, 2u, wwv);
  if (comp & 4u) bounds(ac, amax, da, 4u, wwa);
  if ((comp & 1u) && box.on) {
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int x = 0; x < DIMS; ++x) {
        const float e = fminf(fmaxf(p[i][x], box.lo[x]), box.hi[x]) - p[i][x];
        S[i][x] += e;
        if (LAST) r2[i] = fmaf(e, e, r2[i]);
      }
  }
  if ((comp & 1u) && (ncand || box.on)) {
    bool any = false;
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int x = 0; x < DIMS; ++x) any = any || (ok[i] && S[i][x] != 0.0f);
    if (wballot(any) != 0ull) nz |= 1u;
  }
  return nz;
}

template <int DIMS, int AS, bool BF16, bool GQ>
__device__ __forceinline__ void project_wave_block(const ProjArgs& a, int first, int stride, int total) {
  static_assert(AS == 4 || (AS == 2 && DIMS == 2), "2 axis slots only hold 2D samples");
  constexpr int SPW = 16 / AS;  // samples per wave
  constexpr int NI = 4 / AS;    // items per lane and time block
  extern __shared__ float4 sm4[];
  float* sm = reinterpret_cast<float*>(sm4);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, WPB = blockDim.x >> 6;
  const int nv = a.nv, K = a.K, M = a.M, D = DIMS * nv, D4 = round4(D);
  const int NB = (K + 15) >> 4, SPB = a.S;  // samples per block: SPW per group, 1 or 4 groups per wave
  const WaveLayout l = wave_layout(DIMS, nv, M, NB, WPB, a.mode);
  // column layout (MFMA state): col = AS * cs + cx, coefficient rows 4 q + r;
  // item layout (forward rows, push-outs): step ti of columns 4 q + 0..3
  const int q = lane >> 4, col = lane & 15, cs = col / AS, cx = col % AS, ti = lane & 15;
  float4* rec = reinterpret_cast<float4*>(sm + l.rec);
  const float4* wtab = reinterpret_cast<const float4*>(sm + l.wtab);
  float* wr = sm + l.wave + w * l.wave_floats;
  uint32_t* cwords = reinterpret_cast<uint32_t*>(wr + l.cache);
  const int cstride = l.cstride;  // cache words per time block

  // forward B operands of every time block, once per block: lane ll, row
  // type d, coefficient chunk h -> W[16 tb + ll % 16][d][coefficient of
  // chunk h, row ll / 16] (zero past the horizon and the coefficients)
  {
    float4* wt = reinterpret_cast<float4*>(sm + l.wtab);
    for (int e = tid; e < NB * kWtabV4 * 64; e += blockDim.x) {
      const int ll = e & 63, d = (e >> 6) % kWtabV4, tb = (e >> 6) / kWtabV4;
      const int t = 16 * tb + (ll & 15);
      float v[4];
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int c = coef_of(ll >> 4, h);
        v[h] = (t < K && c < nv) ? a.W[(t * 3 + d) * nv + c] : 0.0f;
      }
      wt[e] = make_float4(v[0], v[1], v[2], v[3]);
    }
  }
  // the right-hand-side A operand of this lane (time rows 4 q + 0..3 of a
  // block, coefficient row of column `col`) is the forward operand of lane
  // 16 (col / 4) + 4 q + jj, chunk col % 4: its float offsets in a table row
  const float* wtf = reinterpret_cast<const float*>(wtab);
  const int rhs_off = (16 * (col >> 2) + 4 * q) * 4 + (col & 3);
  float Am[4];
  const int crow = coef_of(col >> 2, col & 3);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ck = coef_of(q, r);
    Am[r] = (crow < nv && ck < nv) ? a.M11[crow * nv + ck] : 0.0f;
  }
  s4 Mhi, Mlo;
  if constexpr (BF16) {
    Mhi = pack_bf16(Am[0], Am[1], Am[2], Am[3]);
    Mlo = pack_bf16(Am[0] - from_bf16(Mhi[0]), Am[1] - from_bf16(Mhi[1]),
                    Am[2] - from_bf16(Mhi[2]), Am[3] - from_bf16(Mhi[3]));
  }
  const bool chunk3 = nv > 12;
  const float rho = a.rho;
  const f4 zf = {0.0f, 0.0f, 0.0f, 0.0f};
  // half the time window of a 16-step block
  const float thalf = a.dt * 7.5f;

  // The tile's groups of SPW samples are drawn by the block's waves from a
  // counter in LDS: a wave that finishes a group early takes the next one
  // instead of idling until the slowest wave of the block is done.  With GQ
  // the waves of every block draw (problem, group) pairs from one counter in
  // global memory for the whole launch (total = the number of pairs), with
  // the problems' obstacle records in global memory too, so no block waits
  // for its waves before the end of the launch.
  int* ctr = reinterpret_cast<int*>(sm + l.ctr);
  float* sMu = sm + l.mul;
  float* sL = sMu + D4;
  const int gpp = (a.N + SPW - 1) / SPW;  // groups per problem
  // (the W table is complete before any wave reads it; without GQ the first
  // barrier of the tile loop does this)
  if constexpr (GQ) __syncthreads();
  [[maybe_unused]] int cur_prob = -1;
  for (int tile = first; GQ ? tile == first : tile < total; tile += stride) {
    int prob = 0, s0 = 0, ns = a.N, ngroups = 0;
    if constexpr (!GQ) {
      prob = tile / a.blocks_per_problem;
      s0 = (tile - prob * a.blocks_per_problem) * SPB;
      ns = min(SPB, a.N - s0);
      ngroups = (ns + SPW - 1) / SPW;
      // (every wave is done with the previous tile: records, mean, factor and
      // counter may change)
      __syncthreads();
      if (prob != cur_prob) {
        build_records<DIMS>(a.obs + prob * a.obs_stride, M, tid, blockDim.x, rec);
        if (a.mode != kFromInput) {
          const float* mu = a.mu + prob * a.mu_stride;
          const float* Lm = a.L + prob * a.L_stride;
          for (int i = tid; i < D; i += blockDim.x) sMu[i] = mu[i];
          for (int i = tid; i < D * D; i += blockDim.x) sL[i] = Lm[i];
        }
      }
      cur_prob = prob;
      if (tid == 0) *ctr = 0;
      __syncthreads();
    }
    for (;;) {
      int gi = 0;
      if (lane == 0) gi = atomicAdd(GQ ? a.gq : ctr, 1);
      gi = __builtin_amdgcn_readfirstlane(gi);
      if constexpr (GQ) {
        if (gi >= total) break;
        prob = gi / gpp;
        gi -= prob * gpp;
      } else {
        if (gi >= ngroups) break;
      }
      // this problem's obstacle records, mean and factor
      const float4* recp = GQ ? reinterpret_cast<const float4*>(a.grec + prob * a.grec_stride) : rec;
      const float* muP = GQ ? a.mu + prob * a.mu_stride : sMu;
      const float* LP = GQ ? a.L + prob * a.L_stride : sL;
      const float* bc = a.bc + prob * a.bc_stride;
      const int gs0 = s0 + gi * SPW;  // the group's first sample
      const int nsw = min(SPW, ns - gi * SPW);
      // the group's samples, staged in this wave's planes
      float* xs = wr;
      if (a.mode == kFromInput) {
        const float* src = a.xi_in + prob * a.xi_in_stride + static_cast<int64_t>(gs0) * D;
        for (int i = lane; i < nsw * D; i += 64) xs[(i / D) * D4 + i % D] = src[i];
      } else {
        float* sZ = xs + SPW * D4;
        if (a.mode == kFromNoise) {
          const float* z = a.noise + prob * a.noise_stride + static_cast<int64_t>(gs0) * D;
          for (int i = lane; i < nsw * D; i += 64) sZ[(i / D) * D4 + i % D] = z[i];
        } else {
          const int nq = D4 / 4;
          const uint32_t stream_id = a.stream_base + static_cast<uint32_t>(prob);
          for (int i = lane; i < nsw * nq; i += 64) {
            const int s = i / nq, qq = i - s * nq;
            float z[4];
            philox_normals4(a.seed, static_cast<uint32_t>(gs0 + s), static_cast<uint32_t>(qq),
                            static_cast<uint32_t>(a.iter), stream_id, z);
            *reinterpret_cast<float4*>(sZ + s * D4 + 4 * qq) = make_float4(z[0], z[1], z[2], z[3]);
          }
        }
        wave_lds_sync();
        for (int i = lane; i < nsw * D; i += 64) {
          const int s = i / D, d = i - s * D;
          const float* zz = sZ + s * D4;
          const float* Lr = LP + d * D;
          float x = muP[d];
          for (int e = 0; e <= d; ++e) x = fmaf(Lr[e], zz[e], x);
          xs[s * D4 + d] = x;
        }
        wave_lds_sync();
        if (a.xi_src) {
          float* dst = a.xi_src + prob * a.xi_src_stride + static_cast<int64_t>(gs0) * D;
          for (int i = lane; i < nsw * D; i += 64) dst[i] = xs[(i / D) * D4 + i % D];
        }
      }
      wave_lds_sync();
      const bool colok = (cx < DIMS) && (cs < nsw);
      f4 xi;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = coef_of(q, r);
        xi[r] = (colok && c < nv) ? xs[cs * D4 + cx * nv + c] : 0.0f;
      }
      // (the samples are read: the planes become transpose buffers)
      wave_lds_sync();

      // planes of padding columns (axis slots >= DIMS) are read as zeros; no
      // time block has a candidate cache yet
      if constexpr (AS == 4) {
#pragma unroll
        for (int x = DIMS; x < 4; ++x)
#pragma unroll
          for (int d = 0; d < 3; ++d) wr[(d * 4 + x) * kPlane + lane] = 0.0f;
      }
      wave_lds_sync();
      // reuse slack of the candidate masks: the smallest cull radius of the scene
      float slack = INFINITY;
      for (int j = lane; j < M; j += 64) slack = fminf(slack, recp[j].w);
      slack = M > 0 ? wave_min(slack) : 1.0f;

      f4 xb = xi;
      f4 lam = {0.0f, 0.0f, 0.0f, 0.0f};
      uint32_t pairs = 0;

      // Displacement budgets.  Lane tb < NB holds, for time block tb, how much
      // more the coefficients may move (summed max |change| over this wave's
      // valid columns) before its positions may leave the grown boxes of its
      // candidate cache (Bp) or its velocities / accelerations may exceed
      // their bounds (Bv, Ba), and the block's candidate count (ncl).  A row
      // type whose budget is left is not evaluated: its push-outs are zero on
      // every valid item; with no budget left the positions are tested against
      // the grown boxes and the cache is rebuilt only if an item is outside.
      // The budgets come from the last evaluation: a change
      // Delta moves row type d by at most S_d max|Delta| (bscale), and the
      // MFMA rounding of the two evaluations, at most 3e-6 S_d X with X a bound
      // on max |xi_bar|, is taken off with margin (1e-5 X); the factor 0.99899
      // covers the rounding of the budget arithmetic.
      float Bp = -1.0f, Bv = -1.0f, Ba = -1.0f;
      uint32_t ncl = ~0u;  // no cache yet
      const uint32_t blocks = (1u << NB) - 1u;
      uint32_t mP = blocks, mV = blocks, mA = blocks;  // blocks to evaluate
      float X;
      {
        float m = 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) m = fmaxf(m, fabsf(xi[r]));
        X = wave_reduce_nn<true>(colok ? m : 0.0f) * 1.000002f;
      }
      auto budget = [&](float A) { return fmaf(A, 0.99899f, -1.0e-5f * X); };
      auto bound_budget = [&](float wmax, float wwm, float scale) {
        // (v_sqrt_f32 is within 1 ulp)
        return budget((wmax * 0.999999f - __builtin_amdgcn_sqrtf(wwm) * 1.000001f) * scale);
      };

      // One time block: forward rows of the row types in `comp` (bit 0:
      // positions, 1: velocities, 2: accelerations) of columns 4 q + 0..3 at
      // step 16 tb + ti (item layout), then the push-outs of this lane's items.
      auto block_items = [&](int tb, uint32_t comp, bool test, uint32_t& ncand, auto last_tag,
                             float p[NI][DIMS], float v[NI][DIMS], float ac[NI][DIMS],
                             float S[NI][DIMS], float dv[NI][DIMS], float da[NI][DIMS], float r2[NI],
                             bool ok[NI], float& wwv, float& wwa, float& pm, float& lcl) {
        constexpr bool LAST = decltype(last_tag)::value;
        const float4* wt = wtab + tb * kWtabV4 * 64 + lane;
        f4 Y0 = zf, Y1 = zf, Y2 = zf;
        if (comp == 7u) {
          const float4 w0 = wt[0], w1 = wt[64], w2 = wt[128];
          Y0 = mfma(xb[0], w0.x, zf);
          Y1 = mfma(xb[0], w1.x, zf);
          Y2 = mfma(xb[0], w2.x, zf);
          Y0 = mfma(xb[1], w0.y, Y0);
          Y1 = mfma(xb[1], w1.y, Y1);
          Y2 = mfma(xb[1], w2.y, Y2);
          Y0 = mfma(xb[2], w0.z, Y0);
          Y1 = mfma(xb[2], w1.z, Y1);
          Y2 = mfma(xb[2], w2.z, Y2);
          if (chunk3) {
            Y0 = mfma(xb[3], w0.w, Y0);
            Y1 = mfma(xb[3], w1.w, Y1);
            Y2 = mfma(xb[3], w2.w, Y2);
          }
        } else {
          // the same chains, one row type at a time
          auto chain = [&](const float4 w) {
            f4 Y = mfma(xb[0], w.x, zf);
            Y = mfma(xb[1], w.y, Y);
            Y = mfma(xb[2], w.z, Y);
            if (chunk3) Y = mfma(xb[3], w.w, Y);
            return Y;
          };
          if (comp & 1u) Y0 = chain(wt[0]);
          if (comp & 2u) Y1 = chain(wt[64]);
          if (comp & 4u) Y2 = chain(wt[128]);
        }
        const int t = 16 * tb + ti;
        uint32_t nok = 0;
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          ok[i] = (t < K) && ((4 * q) / AS + i < nsw);
          nok += static_cast<uint32_t>(__builtin_popcountll(wballot(ok[i])));
#pragma unroll
          for (int x = 0; x < DIMS; ++x) {
            p[i][x] = Y0[AS * i + x];
            v[i][x] = Y1[AS * i + x];
            ac[i][x] = Y2[AS * i + x];
          }
        }
        const float tmid = a.dt * (static_cast<float>(16 * tb) + 7.5f);
        return wave_block_push<DIMS, LAST, NI>(recp, M, a.dt * static_cast<float>(t), tmid, thalf, slack,
                                               comp, test, ok, p, v, ac, a.vmax, a.amax, a.box, S,
                                               dv, da, r2, lane, cwords + tb * cstride, ncand, nok,
                                               pairs, wwv, wwa, pm, lcl);
      };

      // ---- projection iterations ---------------------------------------------------
      for (int k = 0; k < a.n_iter; ++k) {
        const bool lowp = BF16 && (k < a.bf16_iters);
        // right-hand side: the nonzero block partials added to +0 in time-block
        // order, the sum of the time-split shape (an all-zero partial leaves it
        // unchanged)
        f4 g = zf;
        // (the blocks with a row type to evaluate, in ascending order; the
        // others add nothing)
        uint32_t todo = a.box.on ? blocks : (mP | mV | mA);
        while (todo) {
          const int tb = __builtin_ctz(todo);
          todo &= todo - 1u;
          const uint32_t bit = 1u << tb;
          uint32_t ncand = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(ncl), tb));
          const bool test = (mP & bit) != 0u;
          uint32_t comp = ((mV & bit) ? 2u : 0u) | ((mA & bit) ? 4u : 0u);
          // (while the position budget lasts, every valid item is inside its
          // grown box and clear of every candidate: no obstacle can push)
          if (test || a.box.on) comp |= 1u;
          if (comp) {
            float p[NI][DIMS], v[NI][DIMS], ac[NI][DIMS], S[NI][DIMS], dv[NI][DIMS], da[NI][DIMS], r2[NI];
            bool ok[NI];
            float wwv = 0.0f, wwa = 0.0f, pm = 0.0f, lcl = INFINITY;
            const uint32_t nz = block_items(tb, comp, test, ncand, std::false_type{}, p, v, ac, S, dv,
                                            da, r2, ok, wwv, wwa, pm, lcl);
            // new budgets of the row types evaluated here; the position budget
            // is the smaller of the grown-box margin (per axis) and the
            // candidates' clearance (Euclidean, over sqrt(dims)), or none while
            // some position push-out is nonzero
            if (test) {
              float bp = -1.0f;
              if (!(nz & 1u)) {
                // (one reduction of both: rounding is monotone, so the smallest
                // scaled clearance is the smallest clearance scaled)
                float lm = pm;
                if (ncand) {
                  const float c = fmaxf(lcl, 0.0f) * (DIMS == 3 ? 0.57735026f : 0.70710678f);
                  lm = fminf(lm, __uint_as_float(__float_as_uint(c) & 0x7fffffffu));
                }
                const float m = wave_reduce_nn<false>(lm);
                if (m > 0.0f) bp = budget(m * a.bscale[0]);
              }
              Bp = lane == tb ? bp : Bp;
              ncl = lane == tb ? ncand : ncl;
            }
            if (comp & 2u) {
              const float bv = (nz & 2u) ? -1.0f : bound_budget(a.vmax, wwv, a.bscale[1]);
              Bv = lane == tb ? bv : Bv;
            }
            if (comp & 4u) {
              const float ba = (nz & 4u) ? -1.0f : bound_budget(a.amax, wwa, a.bscale[2]);
              Ba = lane == tb ? ba : Ba;
            }
            // Right-hand side of the row types with a nonzero push-out.  The
            // products of an all-zero row type are exact zeros, and an
            // accumulator that starts at +0 is unchanged by adding them, so
            // skipping them leaves the partial bit for bit as in the full chains.
            if (nz) {
              f4 part;
              const float (*src[3])[DIMS] = {S, dv, da};
#pragma unroll
              for (int d = 0; d < 3; ++d)
                if (nz & (1u << d)) {
#pragma unroll
                  for (int i = 0; i < NI; ++i)
#pragma unroll
                    for (int x = 0; x < DIMS; ++x) wr[(d * 4 + AS * i + x) * kPlane + lane] = src[d][i][x];
                }
              wave_lds_sync();
              f4 B[3];
              float4 wa[3];
#pragma unroll
              for (int d = 0; d < 3; ++d)
                if (nz & (1u << d)) {
                  B[d] = *reinterpret_cast<const f4*>(wr + (d * 4 + (col & 3)) * kPlane + 16 * (col >> 2) + 4 * q);
                  const float* wr0 = wtf + (tb * kWtabV4 + d) * 256 + rhs_off;
                  wa[d] = make_float4(wr0[0], wr0[4], wr0[8], wr0[12]);
                }
              wave_lds_sync();
              if (lowp) {
                f4 gg = zf;
#pragma unroll
                for (int d = 0; d < 3; ++d)
                  if (nz & (1u << d)) {
                    const float4 A4 = wa[d];
                    gg = mfma_bf16(pack_bf16(A4.x, A4.y, A4.z, A4.w),
                                   pack_bf16(B[d][0], B[d][1], B[d][2], B[d][3]), gg);
                  }
                part = gg;
              } else {
                // the two accumulation chains of the time-split shape
                f4 acc0 = zf, acc1 = zf;
#pragma unroll
                for (int d = 0; d < 3; ++d)
                  if (nz & (1u << d)) {
                    const float4 A4 = wa[d];
                    acc0 = mfma(A4.x, B[d][0], acc0);
                    acc1 = mfma(A4.y, B[d][1], acc1);
                    acc0 = mfma(A4.z, B[d][2], acc0);
                    acc1 = mfma(A4.w, B[d][3], acc1);
                  }
                part = acc0 + acc1;
              }
              g = g + part;
            }
          }
        }
        lam += rho * g;
        const f4 xold = xb;
        if (k == 0) {
          // Pi and c0 = M12 b enter the first step only
          float Ap[4];
          f4 c0v;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int c = coef_of(q, r);
            Ap[r] = (crow < nv && c < nv) ? a.Pi[crow * nv + c] : 0.0f;
            float sacc = 0.0f;
            if (colok && c < nv)
              for (int i = 0; i < 6; ++i) sacc = fmaf(a.M12[c * 6 + i], bc[cx * 6 + i], sacc);
            c0v[r] = sacc;
          }
          const f4 u = lam + rho * g;
          const f4 h0 = mfma(Ap[1], xi[1], mfma(Ap[0], xi[0], c0v));
          f4 h1 = mfma(Ap[2], xi[2], zf);
          const f4 h2 = mfma(Am[1], u[1], mfma(Am[0], u[0], zf));
          f4 h3 = mfma(Am[2], u[2], zf);
          if (chunk3) {
            h1 = mfma(Ap[3], xi[3], h1);
            h3 = mfma(Am[3], u[3], h3);
          }
          xb = (h0 + h1) + (h2 + h3);
        } else if (lowp) {
          const f4 u = (xi - xb) + lam + rho * g;
          const s4 uh = pack_bf16(u[0], u[1], u[2], u[3]);
          const s4 ul = pack_bf16(u[0] - from_bf16(uh[0]), u[1] - from_bf16(uh[1]),
                                  u[2] - from_bf16(uh[2]), u[3] - from_bf16(uh[3]));
          xb = xb + mfma_bf16(Mhi, uh, mfma_bf16(Mlo, uh, mfma_bf16(Mhi, ul, zf)));
        } else {
          const f4 u = (xi - xb) + lam + rho * g;
          xb = mfma(Am[2], u[2], mfma(Am[1], u[1], mfma(Am[0], u[0], xb)));
          if (chunk3) xb = mfma(Am[3], u[3], xb);
        }
        // every block's budgets shrink by the largest coefficient change of
        // the wave's valid columns (rounded up)
        {
          float m = 0.0f;
#pragma unroll
          for (int r = 0; r < 4; ++r) m = fmaxf(m, fabsf(xb[r] - xold[r]));
          const float dl = wave_reduce_nn<true>(colok ? m : 0.0f) * 1.000002f;
          X += dl;
          Bp -= dl;
          Bv -= dl;
          Ba -= dl;
          const bool inb = lane < NB;
          mP = static_cast<uint32_t>(wballot(inb && !(Bp >= 0.0f)));
          mV = static_cast<uint32_t>(wballot(inb && !(Bv >= 0.0f)));
          mA = static_cast<uint32_t>(wballot(inb && !(Ba >= 0.0f)));
        }
      }

      // ---- residual and cost of the returned iterate, summed in t order --------------
      float sg[DIMS], ug[DIMS], iuu = 0.0f;
      if (a.cost.kind != 0) {
        float uu = 0.0f;
#pragma unroll
        for (int x = 0; x < DIMS; ++x) {
          sg[x] = bc[x * 6 + 0];
          ug[x] = bc[x * 6 + 3] - sg[x];
          uu = fmaf(ug[x], ug[x], uu);
        }
        iuu = uu > 0.0f ? 1.0f / uu : 0.0f;
      }
      float racc = 0.0f, cacc = 0.0f;
      for (int tb = 0; tb < NB; ++tb) {
        float p[NI][DIMS], v[NI][DIMS], ac[NI][DIMS], S[NI][DIMS], dv[NI][DIMS], da[NI][DIMS], r2[NI];
        bool ok[NI];
        uint32_t ncand = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(ncl), tb));
        float wwv = 0.0f, wwa = 0.0f, pm = 0.0f, lcl = INFINITY;
        block_items(tb, 7u, (mP >> tb) & 1u, ncand, std::true_type{}, p, v, ac, S, dv, da, r2, ok, wwv,
                    wwa, pm, lcl);
        // per-(t, sample) residual^2 and cost through this wave's planes
#pragma unroll
        for (int i = 0; i < NI; ++i) {
          float cc = 0.0f;
          if (a.cost.kind == 0) {
#pragma unroll
            for (int x = 0; x < DIMS; ++x) cc = fmaf(ac[i][x], ac[i][x], cc);
          } else {
            cc = weighted_cost<DIMS>(p[i], v[i], ac[i], a.cost, sg, ug, iuu);
          }
          float* f = wr + 2 * (ti * SPW + (4 * q) / AS + i);
          f[0] = ok[i] ? r2[i] : 0.0f;
          f[1] = ok[i] ? cc : 0.0f;
        }
        wave_lds_sync();
        if (lane < nsw) {
          const int nt = min(16, K - 16 * tb);
          for (int t = 0; t < nt; ++t) {
            const float* f = wr + 2 * (t * SPW + lane);
            racc += f[0];
            cacc += f[1];
          }
        }
        wave_lds_sync();
      }
      if (lane < nsw) {
        const int s = gs0 + lane;
        const float r = sqrtf(racc);
        const int64_t nb = prob * a.n_stride + s;
        const int64_t dense = static_cast<int64_t>(prob) * a.N + s;
        if (a.resid) a.resid[nb] = r;
        if (a.c1) a.c1[nb] = cacc;
        if (a.resid2) a.resid2[dense] = r;
        if (a.c12) a.c12[dense] = cacc;
      }
      if (a.pair_count && lane == 0) atomicAdd(a.pair_count, static_cast<unsigned long long>(pairs));
      if (colok) {
        float* dst = a.xi_out + prob * a.xi_out_stride + static_cast<int64_t>(gs0 + cs) * D + cx * nv;
        float* dst2 = a.xi_out2 ? a.xi_out2 + (static_cast<int64_t>(prob) * a.N + gs0 + cs) * D + cx * nv
                                : nullptr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int c = coef_of(q, r);
          if (c < nv) {
            dst[c] = xb[r];
            if (dst2) dst2[c] = xb[r];
          }
        }
      }
    }
  }
}

// Whole-horizon shape: one block of blockDim / 64 waves per tile of a.S
// samples of one problem (one or four groups of 16 / AS samples per wave,
// drawn by the waves from the tile's counter).  XCD-aware block order as
// project_kernel.
template <int DIMS, int AS, bool BF16, bool GQ>
__global__ __launch_bounds__(1024) void project_wave_kernel(ProjArgs a, int total) {
  const int G = gridDim.x;
  int lb = blockIdx.x;
  if ((G & 7) == 0) lb = (blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  project_wave_block<DIMS, AS, BF16, GQ>(a, lb, G, total);
}

// Before a launch that draws (problem, group) pairs from global memory: each
// problem's obstacle records (one block per problem), and the counter set to
// zero.
template <int DIMS>
__global__ void wave_records_kernel(ProjArgs a) {
  const int prob = blockIdx.x;
  build_records<DIMS>(a.obs + prob * a.obs_stride, a.M, threadIdx.x, blockDim.x,
                      reinterpret_cast<float4*>(a.grec + prob * a.grec_stride));
  if (prob == 0 && threadIdx.x == 0) *a.gq = 0;
}

// Per-row push-outs e(xi) - F xi, [N][M + 2][K][dims] (parity hook): one
// thread per (sample, t), the same record table and per-pair push-out
// arithmetic as the projection kernel, one obstacle at a time.
template <int DIMS>
__global__ void offsets_kernel(ProjArgs a, const float* xi, float* out) {
  __shared__ float4 rec[3 * PRIEST_MAX_OBS];
  const int nv = a.nv, K = a.K, M = a.M;
  const int D = DIMS * nv;
  if (a.traj) build_records<DIMS, true>(a.obs, M, threadIdx.x, blockDim.x, rec, K);
  else build_records<DIMS>(a.obs, M, threadIdx.x, blockDim.x, rec);
  __syncthreads();
  const int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= a.N * K) return;
  const int s = it / K, t = it - s * K;
  float p[DIMS], v[DIMS], ac[DIMS];
  for (int x = 0; x < DIMS; ++x) {
    float sp = 0.0f, sv = 0.0f, sa = 0.0f;
    for (int c = 0; c < nv; ++c) {
      const float xc = xi[static_cast<int64_t>(s) * D + x * nv + c];
      sp = fmaf(a.W[(t * 3 + 0) * nv + c], xc, sp);
      sv = fmaf(a.W[(t * 3 + 1) * nv + c], xc, sv);
      sa = fmaf(a.W[(t * 3 + 2) * nv + c], xc, sa);
    }
    p[x] = sp; v[x] = sv; ac[x] = sa;
  }
  const float tt = a.dt * static_cast<float>(t);
  float* o = out + static_cast<int64_t>(s) * (M + 2) * K * DIMS;
  for (int j = 0; j < M; ++j) {
    Rec r = rec_from_lds(rec, M, j);
    if (a.traj) {  // the obstacle's position at step t, from its path
      const float* pt = a.obs + static_cast<int64_t>(j) * (K * DIMS + 2) + t * DIMS;
      r.cx = pt[0];
      r.cy = pt[1];
      r.cz = (DIMS == 3) ? pt[2] : 0.0f;
      r.vx = r.vy = r.vz = 0.0f;
      r.moving = false;
    }
    float S[DIMS], r2 = 0.0f;
    for (int x = 0; x < DIMS; ++x) S[x] = 0.0f;
    if (pair_push<DIMS, false>(r, tt, p, S, r2)) zero_push<DIMS, false>(r, S, r2);
    for (int x = 0; x < DIMS; ++x) o[(j * K + t) * DIMS + x] = S[x];
  }
  float dv[DIMS], da[DIMS];
  float r2b = 0.0f;
  bound_push<DIMS>(v, a.vmax, dv, r2b);
  bound_push<DIMS>(ac, a.amax, da, r2b);
  for (int x = 0; x < DIMS; ++x) {
    o[(M * K + t) * DIMS + x] = dv[x];
    o[((M + 1) * K + t) * DIMS + x] = da[x];
  }
}

__global__ void normals_kernel(uint64_t seed, uint32_t stream, int iter, int N, int D, float* z) {
  const int nq = (D + 3) / 4;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * nq) return;
  const int s = i / nq, qq = i - s * nq;
  float w[4];
  philox_normals4(seed, static_cast<uint32_t>(s), static_cast<uint32_t>(qq),
                  static_cast<uint32_t>(iter), stream, w);
  for (int k = 0; k < 4; ++k)
    if (4 * qq + k < D) z[static_cast<int64_t>(s) * D + 4 * qq + k] = w[k];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
int waves_for(int K, int RT) { return (K + 16 * RT - 1) / (16 * RT); }

// Partial slots of the sum tree: (launch bound / 64) * RT, the bound being
// 512 threads up to 8 waves and 1024 above.
int partial_slots(int K, int RT) { return (waves_for(K, RT) <= 8 ? 8 : 16) * RT; }

// Resident blocks per CU of one kernel instance for a block size and LDS
// size, cached (the query is not free and launches repeat).
struct OccKey {
  const void* fn;
  int threads;
  size_t lds;
};

int resident_blocks(const void* fn, int threads, size_t lds) {
  static std::mutex mu;
  static OccKey keys[64];
  static int vals[64];
  static int n = 0;
  std::lock_guard<std::mutex> lock(mu);
  for (int i = 0; i < n; ++i)
    if (keys[i].fn == fn && keys[i].threads == threads && keys[i].lds == lds) return vals[i];
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  int dev = 0, cus = 0, smem_cu = 0, thr_cu = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  // the query does not always bound the count by the block's dynamic LDS and
  // threads: cap it by the CU's LDS and thread slots
  if (lds > 0 &&
      hipDeviceGetAttribute(&smem_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
          hipSuccess &&
      smem_cu > 0)
    per_cu = std::max(1, std::min(per_cu, static_cast<int>(static_cast<size_t>(smem_cu) / lds)));
  if (hipDeviceGetAttribute(&thr_cu, hipDeviceAttributeMaxThreadsPerMultiProcessor, dev) ==
          hipSuccess &&
      thr_cu > 0)
    per_cu = std::max(1, std::min(per_cu, thr_cu / threads));
  const int v = per_cu * cus;
  if (n < 64) {
    keys[n] = OccKey{fn, threads, lds};
    vals[n] = v;
    ++n;
  }
  return v;
}

// Launch events: when set, the runtime stamps the kernel's own start and end
// into them (no marker commands of their own on the stream).
struct KEvents {
  hipEvent_t start, stop;
};

template <typename F, typename... A>
void launch_k(F kernel, dim3 g, dim3 b, size_t lds, hipStream_t s, KEvents ev, A... args) {
  hipExtLaunchKernelGGL(kernel, g, b, static_cast<std::uint32_t>(lds), s, ev.start, ev.stop, 0u,
                        args...);
}

template <int DIMS, int AS, int RT, int MAXT, bool BF16>
hipError_t launch_shape(const ProjArgs& a, int total, int threads, size_t lds, hipStream_t s,
                        KEvents ev) {
  if (a.persistent) {
    const void* fn = reinterpret_cast<const void*>(&project_kernel<DIMS, AS, RT, MAXT, BF16, true>);
    const int grid = std::min(total, resident_blocks(fn, threads, lds));
    launch_k(project_kernel<DIMS, AS, RT, MAXT, BF16, true>, dim3(grid), dim3(threads), lds, s, ev,
             a, total);
  } else {
    launch_k(project_kernel<DIMS, AS, RT, MAXT, BF16, false>, dim3(total), dim3(threads), lds, s,
             ev, a, total);
  }
  return hipGetLastError();
}

template <int DIMS, int AS, bool BF16>
hipError_t launch_wave_shape(const ProjArgs& a, int total, int threads, size_t lds, hipStream_t s,
                             KEvents ev) {
  if (a.persistent && a.gq && a.grec && !a.traj) {
    // one counter over every (problem, group) pair of the launch, drawn by
    // the waves of a grid of resident blocks
    const int P = total / a.blocks_per_problem;
    const int pairs = P * ((a.N + 16 / AS - 1) / (16 / AS));
    hipLaunchKernelGGL(wave_records_kernel<DIMS>, dim3(P), dim3(256), 0, s, a);
    const void* fn = reinterpret_cast<const void*>(&project_wave_kernel<DIMS, AS, BF16, true>);
    const int wpb = threads / 64;
    const int grid = std::max(1, std::min((pairs + wpb - 1) / wpb, resident_blocks(fn, threads, lds)));
    launch_k(project_wave_kernel<DIMS, AS, BF16, true>, dim3(grid), dim3(threads), lds, s, ev, a,
             pairs);
  } else {
    launch_k(project_wave_kernel<DIMS, AS, BF16, false>, dim3(total), dim3(threads), lds, s, ev, a,
             total);
  }
  return hipGetLastError();
}

template <int DIMS, bool BF16>
hipError_t launch_dims(const ProjArgs& a, int total, int threads, size_t lds, hipStream_t s,
                       KEvents ev) {
  if (a.row_tiles == 0) {  // whole-horizon shape (n_steps <= 128, checked by the caller)
    if constexpr (DIMS == 2)
      if (a.axis_slots == 2) return launch_wave_shape<DIMS, 2, BF16>(a, total, threads, lds, s, ev);
    return launch_wave_shape<DIMS, 4, BF16>(a, total, threads, lds, s, ev);
  }
  if (a.resid_hist || a.traj) {  // default shape only (checked by the caller)
    const dim3 g(total), b(threads);
    if (threads <= 512) {
      if (a.resid_hist && a.traj) launch_k(project_special_kernel<DIMS, 512, BF16, true, true>, g, b, lds, s, ev, a, total);
      else if (a.traj) launch_k(project_special_kernel<DIMS, 512, BF16, false, true>, g, b, lds, s, ev, a, total);
      else launch_k(project_special_kernel<DIMS, 512, BF16, true, false>, g, b, lds, s, ev, a, total);
    } else {
      if (a.resid_hist && a.traj) launch_k(project_special_kernel<DIMS, 1024, BF16, true, true>, g, b, lds, s, ev, a, total);
      else if (a.traj) launch_k(project_special_kernel<DIMS, 1024, BF16, false, true>, g, b, lds, s, ev, a, total);
      else launch_k(project_special_kernel<DIMS, 1024, BF16, true, false>, g, b, lds, s, ev, a, total);
    }
    return hipGetLastError();
  }
  if (a.row_tiles == 2) {
    if constexpr (DIMS == 2)
      if (a.axis_slots == 2) return launch_shape<DIMS, 2, 2, 512, BF16>(a, total, threads, lds, s, ev);
    return launch_shape<DIMS, 4, 2, 512, BF16>(a, total, threads, lds, s, ev);
  }
  if (threads <= 512) {
    if constexpr (DIMS == 2)
      if (a.axis_slots == 2) return launch_shape<DIMS, 2, 1, 512, BF16>(a, total, threads, lds, s, ev);
    if (a.axis_slots == 8) return launch_shape<DIMS, 8, 1, 512, BF16>(a, total, threads, lds, s, ev);
    return launch_shape<DIMS, 4, 1, 512, BF16>(a, total, threads, lds, s, ev);
  }
  if constexpr (DIMS == 2)
    if (a.axis_slots == 2) return launch_shape<DIMS, 2, 1, 1024, BF16>(a, total, threads, lds, s, ev);
  if (a.axis_slots == 8) return launch_shape<DIMS, 8, 1, 1024, BF16>(a, total, threads, lds, s, ev);
  return launch_shape<DIMS, 4, 1, 1024, BF16>(a, total, threads, lds, s, ev);
}

}  // namespace

bool tiling_valid(int dims, int axis_slots, int row_tiles, int K) {
  if (axis_slots == 8) return row_tiles == 1;  // 2 samples per block, more blocks for small N
  if (row_tiles == 0)  // one wave per sample group over the whole horizon
    return (axis_slots == 4 || (axis_slots == 2 && dims == 2)) && K <= 16 * kWaveMaxBlocks;
  return (axis_slots == 4 || (axis_slots == 2 && dims == 2)) && (row_tiles == 1 || row_tiles == 2);
}

// Largest dynamic LDS a block may use on the current device (cached).
size_t device_lds_limit() {
  static std::mutex mu;
  static size_t lim[64] = {};
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev < 0 || dev >= 64) dev = 0;
  std::lock_guard<std::mutex> lock(mu);
  if (!lim[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      v = 64 << 10;
    lim[dev] = static_cast<size_t>(v);
  }
  return lim[dev];
}

size_t wave_lds_bytes(const ProjArgs& a, int wpb) {
  return sizeof(float) *
         static_cast<size_t>(wave_layout(a.dims, a.nv, a.M, (a.K + 15) / 16, wpb, a.mode).total);
}

// Waves per block of the whole-horizon shape: the most (16, 12, 8 or 4)
// whose LDS (the block's W table and records, a region per wave) fits.
int wave_block_waves(const ProjArgs& a) {
  const size_t limit = device_lds_limit();
  for (int wpb : {16, 12, 8})
    if (wave_lds_bytes(a, wpb) <= limit) return wpb;
  return 4;
}

// Whole-horizon shape: a block covers one group of 16 / axis_slots samples
// per wave, or kWaveGroups groups per wave that its waves draw from a
// counter (the third tiling field).
constexpr int kWaveGroups = 4;

int samples_per_block(const ProjArgs& a) {
  if (a.row_tiles == 0) return wave_block_waves(a) * (16 / a.axis_slots) * (a.persistent ? kWaveGroups : 1);
  return 16 / a.axis_slots;
}

int project_threads(int K, int row_tiles) { return 64 * waves_for(K, row_tiles); }

size_t project_lds_bytes(const ProjArgs& a) {
  if (a.row_tiles == 0) return wave_lds_bytes(a, wave_block_waves(a));
  const int NB = waves_for(a.K, a.row_tiles) * a.row_tiles;
  return sizeof(float) *
         static_cast<size_t>(layout(a.dims, a.nv, a.M, NB, partial_slots(a.K, a.row_tiles),
                                    16 / a.axis_slots, a.mode).total);
}

void set_default_tiling(ProjArgs& a) {
  a.axis_slots = 4;
  a.row_tiles = 1;
  a.persistent = 0;
  a.S = samples_per_block(a);
}

hipError_t launch_project(const ProjArgs& a, int n_problems, hipStream_t s, hipEvent_t start,
                          hipEvent_t stop) {
  if (!tiling_valid(a.dims, a.axis_slots, a.row_tiles, a.K) || a.S != samples_per_block(a) ||
      a.blocks_per_problem != (a.N + a.S - 1) / a.S)
    return hipErrorInvalidValue;
  if ((a.resid_hist || a.traj) && (a.axis_slots != 4 || a.row_tiles != 1 || a.persistent))
    return hipErrorInvalidValue;
  if (a.resid_hist && n_problems != 1) return hipErrorInvalidValue;
  const size_t lds = project_lds_bytes(a);
  const int threads = a.row_tiles == 0 ? 64 * wave_block_waves(a) : project_threads(a.K, a.row_tiles);
  const int total = n_problems * a.blocks_per_problem;
  if (total <= 0) return hipSuccess;
  const bool bf = a.bf16_iters > 0;
  const KEvents ev{start, stop};
  if (a.dims == 2) return bf ? launch_dims<2, true>(a, total, threads, lds, s, ev)
                             : launch_dims<2, false>(a, total, threads, lds, s, ev);
  return bf ? launch_dims<3, true>(a, total, threads, lds, s, ev)
            : launch_dims<3, false>(a, total, threads, lds, s, ev);
}

hipError_t launch_project_tasks(const ProjTaskLaunch& t, hipStream_t s) {
  const dim3 grid(static_cast<unsigned>(t.n_blocks));
  const dim3 block(project_threads(t.K, 1));
  const size_t lds = t.lds_bytes;
  const bool bf = t.bf16;
  if (block.x <= 512) {
    if (t.dims == 2) {
      if (bf) hipLaunchKernelGGL((project_task_kernel<2, 512, true>), grid, block, lds, s, t.tasks, t.prefix, t.n_tasks);
      else hipLaunchKernelGGL((project_task_kernel<2, 512, false>), grid, block, lds, s, t.tasks, t.prefix, t.n_tasks);
    } else {
      if (bf) hipLaunchKernelGGL((project_task_kernel<3, 512, true>), grid, block, lds, s, t.tasks, t.prefix, t.n_tasks);
      else hipLaunchKernelGGL((project_task_kernel<3, 512, false>), grid, block, lds, s, t.tasks, t.prefix, t.n_tasks);
    }
  } else {
    if (t.dims == 2) {
      if (bf) hipLaunchKernelGGL((project_task_kernel<2, 1024, true>), grid, block, lds, s, t.tasks, t.prefix, t.n_tasks);
      else hipLaunchKernelGGL((project_task_kernel<2, 1024, false>), grid, block, lds, s, t.tasks, t.prefix, t.n_tasks);
    } else {
      if (bf) hipLaunchKernelGGL((project_task_kernel<3, 1024, true>), grid, block, lds, s, t.tasks, t.prefix, t.n_tasks);
      else hipLaunchKernelGGL((project_task_kernel<3, 1024, false>), grid, block, lds, s, t.tasks, t.prefix, t.n_tasks);
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
