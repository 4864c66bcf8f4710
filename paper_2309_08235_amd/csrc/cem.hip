// Selection, refit and covariance factorisation of the sampling loop (Alg. 1,
// eqs. (9a)-(9c)) on gfx950: one 512-thread block per problem.
//
//   1. ConstraintEliteSet: the n_proj samples with the lowest residual r,
//      ordered by (r, index) over the order-preserving bit patterns of r
//      (ties keep index order);
//   2. EliteSet: the n_elite lowest c_aug = c1 + r among them, ties kept in
//      the order of step 1.
//   When the ordered set of step 1 is an output, both steps sort packed
//   64-bit keys (order-preserving key bits above the position) with a
//   bitonic network in LDS; otherwise (N <= 2048, n_elite <= 512) they are
//   radix selects of the boundary keys and a ranking of the n_elite
//   survivors by counting, which select and order exactly the same samples.
//   3. weights c_m = exp(-(c_aug_m - delta)/gamma), delta = min c_aug;
//   4. mu' = (1-sigma) mu + sigma sum w xi_bar / sum w,
//      Sigma' = (1-sigma) Sigma + sigma sum w (xi_bar - mu')(xi_bar - mu')^T / sum w;
//   5. L = chol(Sigma' + eps I), eps = cov_jitter tr(Sigma')/D, for the next
//      draw: one wave, lane i holds row i in registers.
// Every sum runs in a fixed order, so results are bitwise reproducible.
#include "priest_internal.h"

namespace priest {
namespace {

constexpr int kStageFloats = 4096;  // elite rows staged in LDS per chunk

__host__ __device__ inline size_t align16(size_t n) { return (n + 15) & ~static_cast<size_t>(15); }

struct CemLayout {
  size_t proj, elite, w, red, mu, pc, A, mu0, cov0, pc0, stage, total;
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
  l.mu0 = o;   o += align16(sizeof(float) * D);
  l.cov0 = o;  o += align16(sizeof(float) * D * D);
  l.pc0 = o;   o += align16(sizeof(float) * D);
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

// Lower Cholesky factor L of A + eps I, A the D x D matrix in LDS, by one
// wave, rows padded to DM with the identity; lane i keeps row i in registers.
// Column j of L is broadcast lane by lane with readlane (lane c holds
// L[c][j], which the update of entry c of every row needs), so the
// factorisation reads LDS only to load A.  Writes L (zeros above the
// diagonal) row by row to `L`; A is left unchanged.  Returns false if a pivot
// is not positive and finite (it is replaced by 1).
template <int DM>
__device__ __forceinline__ bool cholesky_wave(const float* A, float eps, int D, int lane, float* L) {
  // (every lane loads a clamped, in-range entry and scales it by zero where
  // it pads: with a select the compiler puts each load under its own branch,
  // one LDS round trip after another)
  float row[DM];
  const int lr = lane < D ? lane : D - 1;
  const float inrow = lane < D ? 1.0f : 0.0f;
#pragma unroll
  for (int c = 0; c < DM; ++c) {
    const float v = A[lr * D + (c < D ? c : D - 1)];
    const float m = (c < D) ? inrow : 0.0f;
    row[c] = v * m + (lane == c ? (m != 0.0f ? eps : 1.0f) : 0.0f);
  }
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
      if (c < D) L[lane * D + c] = c <= lane ? row[c] : 0.0f;
  }
  return !bad;
}

using f4 = __attribute__((ext_vector_type(4))) float;

__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Ascending sort of n packed keys (key bits << 32 | position) in LDS by a
// bitonic network over the next power of two (padding keys sort last).  The
// positions make every key distinct, so the order is that of a stable sort
// of the key bits.  Every thread of the block calls it; a[] holds at least
// the next power of two >= n entries.
__device__ __forceinline__ void bitonic_sort_keys(unsigned long long* a, int n) {
  const int tid = threadIdx.x;
  int m = 1;
  while (m < n) m <<= 1;
  for (int i = n + tid; i < m; i += kCemThreads) a[i] = ~0ull;
  __syncthreads();
  for (int k = 2; k <= m; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < (m >> 1); i += kCemThreads) {
        const int lo = 2 * i - (i & (j - 1)), hi = lo + j;
        const unsigned long long x = a[lo], y = a[hi];
        const bool up = (lo & k) == 0;
        if ((x > y) == up) {
          a[lo] = y;
          a[hi] = x;
        }
      }
      __syncthreads();
    }
  }
}

// ---- selection without a full sort ------------------------------------------
// Used when the ordered constraint-elite set is not asked for: the two
// selections of steps 1 and 2 as exact radix selects (the k-th smallest key,
// 8 bits per pass from the top), then the n_elite survivors ranked by
// counting.  Selects exactly the samples, in exactly the order, of the two
// stable sorts: step 1 keeps the lowest (r key, index), step 2 the lowest
// (c_aug key, r key, index).

constexpr int kFastElite = kCemThreads;  // largest n_elite of the fast selection
static_assert(kCemThreads == 512, "index-order scans assume 8 waves");

// Exclusive sum over the lanes of a wave of values below 2^12, bit-sliced:
// one ballot per bit, no LDS.
__device__ __forceinline__ uint32_t wave_excl_sum12(uint32_t v, int lane) {
  const unsigned long long lt = (1ull << lane) - 1ull;
  uint32_t s = 0;
#pragma unroll
  for (int b = 0; b < 12; ++b)
    s += static_cast<uint32_t>(__builtin_popcountll(__ballot((v >> b) & 1u) & lt)) << b;
  return s;
}

// The k-th smallest (0-based) of the keys with valid[j] set, over the block
// (k below their count, at most 4095 of them), 8 bits per pass from the top.
// On return the keys whose bits under vmask are below v are the `less`
// smallest, and `eq` keys match v under vmask, the k-th among them; vmask is
// all ones unless the k-th key is the largest of its group after an earlier
// pass (then the group is taken whole and the remaining passes are skipped).
// hist: 4 x 256 zeroed LDS counters, bc: 12 LDS words.
template <int IPT>
__device__ __forceinline__ void radix_select(const uint32_t (&key)[IPT], const bool (&valid)[IPT],
                                             uint32_t k, uint32_t* hist, uint32_t* bc, uint32_t& v,
                                             uint32_t& vmask, uint32_t& less, uint32_t& eq) {
  const int tid = threadIdx.x, lane = tid & 63;
  uint32_t prefix = 0, mask = 0, kk = k;
  less = 0;
  eq = 0;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int shift = 24 - 8 * p;
    uint32_t* h = hist + 256 * p;
#pragma unroll
    for (int j = 0; j < IPT; ++j)
      if (valid[j] && (key[j] & mask) == prefix) atomicAdd(h + ((key[j] >> shift) & 255u), 1u);
    __syncthreads();
    if (tid < 64) {
      uint32_t c[4], sum = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c[q] = h[4 * lane + q];
        sum += c[q];
      }
      uint32_t cum = wave_excl_sum12(sum, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (kk >= cum && kk < cum + c[q]) {
          bc[3 * p] = 4 * lane + q;
          bc[3 * p + 1] = cum;
          bc[3 * p + 2] = c[q];
        }
        cum += c[q];
      }
    }
    __syncthreads();
    const uint32_t bin = bc[3 * p], before = bc[3 * p + 1];
    eq = bc[3 * p + 2];
    prefix |= bin << shift;
    mask |= 255u << shift;
    kk -= before;
    less += before;
    if (kk + 1 == eq) break;
  }
  v = prefix;
  vmask = mask;
}

// Exclusive count of the set flags in index order (item j of thread t is
// sample j * 512 + t).  wc: 8 * IPT LDS words.
template <int IPT>
__device__ __forceinline__ void index_scan(const bool (&f)[IPT], uint32_t (&pre)[IPT], uint32_t* wc) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const unsigned long long b = __ballot(f[j]);
    pre[j] = static_cast<uint32_t>(__builtin_popcountll(b & lt));
    if (lane == 0) wc[8 * j + wv] = static_cast<uint32_t>(__builtin_popcountll(b));
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    uint32_t off = 0;
    for (int x = 0; x < 8 * j + wv; ++x) off += wc[x];
    pre[j] += off;
  }
}

// LDS of the fast selection (words): 2 x 4 x 256 histogram counters, 24
// broadcast words, 8 * IPT scan counts, one slot counter, and four lists of
// kFastElite entries (c_aug keys, r keys, indices, ranks).  The counters, the
// slot counter and the ranks must be zero on entry.
template <int IPT>
constexpr int fast_select_words() { return 2048 + 24 + 8 * IPT + 1 + 4 * kFastElite; }

// Steps 1 and 2 for N <= 512 * IPT samples: elite[0..n_elite) receives the
// sample indices in rank order.  vr / vc: this thread's r and c1 (sample
// j * 512 + tid); s_r: r of every sample (LDS); gk2: N LDS words of scratch.
template <int IPT>
__device__ __forceinline__ void select_fast(const float (&vr)[IPT], const float (&vc)[IPT], int N,
                                            int n_proj, int n_elite, const float* s_r, uint32_t* ws,
                                            uint32_t* gk2, int* elite) {
  const int tid = threadIdx.x;
  uint32_t* hist = ws;
  uint32_t* bc = ws + 2048;
  uint32_t* wc = bc + 24;
  uint32_t* cnt = wc + 8 * IPT;
  uint32_t* lk2 = cnt + 1;
  uint32_t* lk1 = lk2 + kFastElite;
  int* li = reinterpret_cast<int*>(lk1 + kFastElite);
  uint32_t* lrank = reinterpret_cast<uint32_t*>(li + kFastElite);
  bool valid[IPT];
  uint32_t k1[IPT];
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    valid[j] = tid + j * kCemThreads < N;
    k1[j] = valid[j] ? ordered_bits(vr[j]) : ~0u;
  }
  // step 1: the n_proj lowest (r key, index)
  uint32_t v1, m1, less1, eq1;
  radix_select<IPT>(k1, valid, static_cast<uint32_t>(n_proj - 1), hist, bc, v1, m1, less1, eq1);
  const uint32_t t1 = static_cast<uint32_t>(n_proj) - less1;  // members among the keys equal to v1
  bool mem[IPT];
  if (eq1 == t1) {
#pragma unroll
    for (int j = 0; j < IPT; ++j) mem[j] = valid[j] && (k1[j] & m1) <= v1;
  } else {
    // (only after all four passes: m1 is all ones)
    bool tie[IPT];
    uint32_t pre[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) tie[j] = valid[j] && k1[j] == v1;
    index_scan<IPT>(tie, pre, wc);
#pragma unroll
    for (int j = 0; j < IPT; ++j) mem[j] = valid[j] && (k1[j] < v1 || (tie[j] && pre[j] < t1));
  }
  // step 2: the n_elite lowest (c_aug key, r key, index) among them
  uint32_t k2[IPT];
#pragma unroll
  for (int j = 0; j < IPT; ++j) k2[j] = mem[j] ? ordered_bits(vc[j] + vr[j]) : ~0u;
  uint32_t v2, m2, less2, eq2;
  radix_select<IPT>(k2, mem, static_cast<uint32_t>(n_elite - 1), hist + 1024, bc + 12,
                    v2, m2, less2, eq2);
  const uint32_t t2 = static_cast<uint32_t>(n_elite) - less2;
  bool sel[IPT];
  if (eq2 == t2) {
#pragma unroll
    for (int j = 0; j < IPT; ++j) sel[j] = mem[j] && (k2[j] & m2) <= v2;
  } else {
    // more c_aug ties at the boundary than places left: rank the tied
    // samples by (r key, index)
#pragma unroll
    for (int j = 0; j < IPT; ++j)
      if (valid[j]) gk2[tid + j * kCemThreads] = k2[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      sel[j] = mem[j] && k2[j] < v2;
      if (mem[j] && k2[j] == v2) {
        const int i = tid + j * kCemThreads;
        uint32_t rank = 0;
        for (int x = 0; x < N; ++x) {
          const uint32_t kx = ordered_bits(s_r[x]);
          rank += static_cast<uint32_t>(gk2[x] == v2) &
                  (static_cast<uint32_t>(kx < k1[j]) | (static_cast<uint32_t>(kx == k1[j]) & static_cast<uint32_t>(x < i)));
        }
        sel[j] = rank < t2;
      }
    }
  }
  // the n_elite survivors, in slots of arbitrary order ...
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    if (sel[j]) {
      const uint32_t slot = atomicAdd(cnt, 1u);
      if (slot < static_cast<uint32_t>(n_elite)) {
        lk2[slot] = k2[j];
        lk1[slot] = k1[j];
        li[slot] = tid + j * kCemThreads;
      }
    }
  }
  __syncthreads();
  // ... ranked by counting: Q threads per survivor, each over a share of the
  // others
  // (all three fields read and compared without short-circuits: a lazy read
  // of the tie fields becomes a branch and an LDS round trip per comparison)
  const int Q = kCemThreads / n_elite;
  const int am = tid % n_elite, q = tid / n_elite;
  if (q < Q) {
    const unsigned long long ak = (static_cast<unsigned long long>(lk2[am]) << 32) | lk1[am];
    const int ai = li[am];
    uint32_t rk = 0;
#pragma unroll 4
    for (int b = q * n_elite / Q; b < (q + 1) * n_elite / Q; ++b) {
      const unsigned long long bk = (static_cast<unsigned long long>(lk2[b]) << 32) | lk1[b];
      const int bi = li[b];
      rk += static_cast<uint32_t>(bk < ak) | (static_cast<uint32_t>(bk == ak) & static_cast<uint32_t>(bi < ai));
    }
    atomicAdd(lrank + am, rk);
  }
  __syncthreads();
  for (int m = tid; m < n_elite; m += kCemThreads) {
    const uint32_t rk = lrank[m];
    if (rk < static_cast<uint32_t>(n_elite)) elite[rk] = li[m];
  }
}

// One block's work: selection, refit and factorisation for problem `prob`
// of `a`.  Shared by the uniform-batch kernel and the descriptor-table kernel.
template <int IPT, int DM>
__device__ __forceinline__ void cem_block(const CemArgs& a, int prob) {
  // packed sort keys of the ordered selection; their low words double as the
  // fast selection's scratch
  __shared__ unsigned long long skv[kCemThreads * IPT];
  uint32_t* skey = reinterpret_cast<uint32_t*>(skv);
  // r and c1 of every sample, read from HBM once (up to 2048 samples; larger
  // problems gather them from HBM)
  constexpr bool kPre = IPT <= 4;
  __shared__ float s_r[kPre ? kCemThreads * IPT : 1], s_c1[kPre ? kCemThreads * IPT : 1];
  __shared__ uint32_t s_fast[kPre ? fast_select_words<IPT>() : 1];
  extern __shared__ float4 sm4[];
  char* sm = reinterpret_cast<char*>(sm4);
  const int D = a.D, N = a.N, tid = threadIdx.x;
  constexpr int T = kCemThreads;  // (every launch of the refit uses this block size)
  const CemLayout l = cem_layout(D, a.n_proj, a.n_elite);
  int* proj = reinterpret_cast<int*>(sm + l.proj);
  int* elite = reinterpret_cast<int*>(sm + l.elite);
  float* w = reinterpret_cast<float*>(sm + l.w);
  float* red = reinterpret_cast<float*>(sm + l.red);
  float* muN = reinterpret_cast<float*>(sm + l.mu);
  float* pcN = reinterpret_cast<float*>(sm + l.pc);
  float* A = reinterpret_cast<float*>(sm + l.A);
  float* mu0 = reinterpret_cast<float*>(sm + l.mu0);
  float* cov0 = reinterpret_cast<float*>(sm + l.cov0);
  float* pc0 = reinterpret_cast<float*>(sm + l.pc0);
  float* mu = a.mu + prob * a.mu_stride;
  float* cov = a.cov + prob * a.cov_stride;
  float* L = a.L + prob * a.L_stride;

  bool best_ok = true;  // the best c_aug is not NaN
  // (the factorisation that starts a plan also starts its status word)
  if (a.chol_only && a.status && tid == 0) a.status[prob] = PRIEST_OK;
  if (!a.chol_only) {
    const float* xb = a.xb + prob * a.xb_stride;
    // everything the refit reads besides the elite rows, loaded in one batch
    // so that the block waits on HBM once: r, c1, mu, Sigma (and the
    // evolution path)
    const float* r = a.resid + prob * a.n_stride;
    const float* c1 = a.c1 + prob * a.n_stride;
    constexpr int kCovPer = (DM * DM + kCemThreads - 1) / kCemThreads;
    float vr[IPT], vc[IPT], vcov[kCovPer];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const int i = tid + k * kCemThreads;
      vr[k] = i < N ? r[i] : 0.0f;
      vc[k] = (kPre && i < N) ? c1[i] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kCovPer; ++k) {
      const int i = tid + k * kCemThreads;
      vcov[k] = i < D * D ? cov[i] : 0.0f;
    }
    const float vmu = tid < D ? mu[tid] : 0.0f;
    const float vpc = (a.rule == 1 && !a.first && tid < D) ? a.pc[prob * a.pc_stride + tid] : 0.0f;
#pragma unroll
    for (int k = 0; k < kCovPer; ++k) {
      const int i = tid + k * kCemThreads;
      if (i < D * D) cov0[i] = vcov[k];
    }
    if (tid < D) {
      mu0[tid] = vmu;
      pc0[tid] = vpc;
    }
    // 1. lowest residuals
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
      const int i = tid + k * kCemThreads;
      if (i < N) {
        if constexpr (kPre) {
          s_r[i] = vr[k];
          s_c1[i] = vc[k];
        }
        skv[i] = (static_cast<unsigned long long>(ordered_bits(vr[k])) << 32) | static_cast<uint32_t>(i);
      }
    }
    if constexpr (kPre) {
      r = s_r;
      c1 = s_c1;
    }
    // the ordered constraint-elite set is produced only when asked for;
    // otherwise both selections run as radix selects
    const bool fast = kPre && !a.proj_idx && a.n_elite <= kFastElite;
    if (fast) {
      // (zero counters, ranks and a valid elite list before anyone counts)
      for (int i = tid; i < fast_select_words<IPT>(); i += T) s_fast[i] = 0u;
      for (int m = tid; m < a.n_elite; m += T) elite[m] = 0;
    }
    __syncthreads();
    if (fast) {
      if constexpr (kPre) select_fast<IPT>(vr, vc, N, a.n_proj, a.n_elite, s_r, s_fast, skey, elite);
      __syncthreads();
    } else {
      bitonic_sort_keys(skv, N);
      for (int i = tid; i < a.n_proj; i += T) {
        const int s = static_cast<int>(static_cast<uint32_t>(skv[i]));
        proj[i] = s;
        if (a.proj_idx) a.proj_idx[prob * a.n_proj + i] = s;
      }
      __syncthreads();
      // 2. lowest c_aug within them; ties keep the order of step 1
      for (int i = tid; i < a.n_proj; i += T) {
        const int s = proj[i];
        skv[i] = (static_cast<unsigned long long>(ordered_bits(c1[s] + r[s])) << 32) |
                 static_cast<uint32_t>(i);
      }
      __syncthreads();
      bitonic_sort_keys(skv, a.n_proj);
      for (int m = tid; m < a.n_elite; m += T) elite[m] = proj[static_cast<uint32_t>(skv[m])];
      __syncthreads();
    }
    if (a.elite_idx)
      for (int m = tid; m < a.n_elite; m += T) a.elite_idx[prob * a.n_elite + m] = elite[m];
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
    // 4. mean and covariance from elite rows staged in LDS, CH rows at a time
    float* stage = reinterpret_cast<float*>(sm + l.stage);
    const int CH = kStageFloats / D;
    const bool one_chunk = a.n_elite <= CH;
    // (eight loads per thread in flight before the first store)
    auto stage_rows = [&](int m0, int nm) {
      constexpr int kG = 8;
      for (int b = 0; b < nm * D; b += kG * kCemThreads) {
        float v[kG];
#pragma unroll
        for (int u = 0; u < kG; ++u) {
          const int i = b + u * kCemThreads + tid;
          const int m = i / D;
          v[u] = i < nm * D ? xb[static_cast<int64_t>(elite[m0 + m]) * D + (i - m * D)] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kG; ++u) {
          const int i = b + u * kCemThreads + tid;
          if (i < nm * D) stage[i] = v[u];
        }
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
#pragma unroll 5
        for (int m = part; m < nm; m += 4) macc = fmaf(w[m0 + m], stage[m * D + md], macc);
      }
      if (!one_chunk) __syncthreads();
    }
    if (part < 4) A[tid] = macc;
    __syncthreads();
    if (tid < D) {
      const float sm4 = (A[tid] + A[D + tid]) + (A[2 * D + tid] + A[3 * D + tid]);
      const float mw = sm4 * inv_sw;
      muN[tid] = (1.0f - a.sigma) * mu0[tid] + a.sigma * mw;
      if (a.rule == 1) {
        pcN[tid] = fmaf(sqrtf(cc * (2.0f - cc) * mu_eff), mw - mu0[tid], (1.0f - cc) * pc0[tid]);
      }
    }
    __syncthreads();
    // covariance about the new mean, sum_m w_m (x_m - mu')(x_m - mu')^T (rule
    // 1: about the current mean), on MFMA 16x16x4: wave v computes
    // lower-triangle tile v of the ceil(D/16)^2 tiles, elites four at a time
    // (two accumulation chains, added at the end)
    const float* cen = (a.rule == 1) ? mu0 : muN;
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
        const bool iok = ii < D, jok = jj < D;
        const int ic = iok ? ii : 0, jc = jok ? jj : 0;
        const float mi = cen[ic], mj = cen[jc];
        // four groups of eight elites per step: every load of a step is
        // issued before its products.  Positions past the chunk load a
        // clamped, in-range (finite) row and are scaled by zero: a select
        // here lets the compiler move each load under its own branch, one
        // LDS round trip after another.
        constexpr int kU = 4;
        for (int s0 = 0; s0 < nm; s0 += 8 * kU) {
          float av[kU][2], bv[kU][2];
#pragma unroll
          for (int u = 0; u < kU; ++u)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int m = s0 + 8 * u + 4 * h + (lane >> 4);
              const bool ok = m < nm;
              const int mc = ok ? m : 0;
              const float wm = w[m0 + mc], xi_ = stage[mc * D + ic], xj_ = stage[mc * D + jc];
              av[u][h] = (wm * (xi_ - mi)) * ((ok && iok) ? 1.0f : 0.0f);
              bv[u][h] = (xj_ - mj) * ((ok && jok) ? 1.0f : 0.0f);
            }
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            acc0 = mfma(av[u][0], bv[u][0], acc0);
            acc1 = mfma(av[u][1], bv[u][1], acc1);
          }
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
                     fmaf(c1r, pcN[i] * pcN[j], (1.0f - c1r - cmu) * cov0[i * D + j]));
          else
            v = (1.0f - a.sigma) * cov0[i * D + j] + a.sigma * (acc[r] * inv_sw);
          A[i * D + j] = v;
          A[j * D + i] = v;
        }
      }
    }
    __syncthreads();
    // the outputs other than L, written by the other waves while the first
    // one factors
    if (tid >= 64) {
      const int t2 = tid - 64, T2 = T - 64;
      for (int e = t2; e < D * D; e += T2) cov[e] = A[e];
      for (int d = t2; d < D; d += T2) {
        mu[d] = muN[d];
        if (a.rule == 1) a.pc[prob * a.pc_stride + d] = pcN[d];
        // (elite 0's row is still staged when all elites fit one chunk)
        a.best_xi[prob * a.best_stride + d] = one_chunk ? stage[d] : xb[static_cast<int64_t>(e0) * D + d];
      }
      if (t2 == 0) a.best_cost[prob] = delta;
    }
    best_ok = delta == delta;
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
    const bool ok = cholesky_wave<DM>(A, eps, D, tid, L);
    if (tid == 0 && a.status && !(ok && best_ok)) a.status[prob] = PRIEST_ERR_NONFINITE;
  }
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
