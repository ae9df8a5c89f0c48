// Learned merge proposal (an extension outside the paper's method).
//
// Per coarsening level:
//   1. k_rate_cand: the rating of Eq. 2 with the validity test of Sec. III-A,
//      keeping each node's 8 best valid candidates by (hist, id) together
//      with c(n, m) = |in(n) n in(m)|;
//   2. symmetric candidate sets C(n) = topK(n) u {m : n in topK(m)}: both
//      orientations of every kept pair are sorted by (n, m) and deduplicated;
//   3. k_cand_score: exact integer features of the unordered pair, their
//      8-bit codes and the fixed-point network (two 64-unit ReLU layers on
//      MFMA, a 64-term integer dot product for the output);
//   4. k_cand_best / k_cand_pick: pair(n) = argmax over C(n) of (score, id).
// The network's values are integers carried in BF16 (|w| <= 255, codes and
// activations in 0..255) and every partial sum stays below 2^24 in magnitude,
// so the FP32 accumulation of v_mfma_f32_32x32x8_bf16 is exact in any order
// and the scores are bit-identical for (n, m) and (m, n).
#include <mutex>

#include "learned.hpp"

namespace hgp {

// ---------------------------------------------------------------------------
// 1. top-8 valid candidates per node
// ---------------------------------------------------------------------------
constexpr int CAND_NT = 512;
constexpr int CAND_LDS_BYTES = 128 * 1024;
static_assert((CAND_NT / 64) * kCandK == 64, "block merge assumes one entry per lane of wave 0");

// Inserts (key, c) into a descending register list if it beats the last entry.
__device__ __forceinline__ void cand_insert(uint64_t (&kk)[kCandK], int32_t (&kc)[kCandK], uint64_t key,
                                            int32_t c) {
  kk[kCandK - 1] = key;
  kc[kCandK - 1] = c;
#pragma unroll
  for (int j = kCandK - 1; j > 0; --j) {
    if (kk[j] > kk[j - 1]) {
      const uint64_t tk = kk[j];
      kk[j] = kk[j - 1];
      kk[j - 1] = tk;
      const int32_t tc = kc[j];
      kc[j] = kc[j - 1];
      kc[j - 1] = tc;
    }
  }
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t x = __shfl_xor(v, o, 64);
    v = x > v ? x : v;
  }
  return v;
}

// One workgroup per node n.  The neighbour histogram is the dense LDS window
// of the plain rating (hist in the low bits, c in the high bits of one 32-bit
// counter, or a 64-bit pair).  Each thread keeps the 8 largest keys
// hist << 32 | m of valid candidates it scans; a key is tested against Omega
// and Delta only when it would enter the thread's list.  Keys are unique (one
// thread owns each m), so the merge extracts maxima without ties.
// Output: ck[n*8 + r] = r-th best key (0 past the end), cc[n*8 + r] = c,
// ccnt[n] = number of valid candidates kept (at most `keep`).
__global__ __launch_bounds__(CAND_NT) void k_rate_cand(
    int32_t N, const int32_t *__restrict__ ioff, const uint32_t *__restrict__ inc, const int32_t *__restrict__ hoff,
    const uint32_t *__restrict__ hpin, const int32_t *__restrict__ hw, const int32_t *__restrict__ size,
    const int32_t *__restrict__ indeg, const int32_t *__restrict__ total, const int32_t *__restrict__ maxin,
    int32_t omega, int32_t delta, int32_t words, int32_t keep, uint64_t *__restrict__ ck, int32_t *__restrict__ cc,
    int32_t *__restrict__ ccnt, unsigned long long *__restrict__ units) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ uint64_t wk[CAND_NT / 64][kCandK];
  __shared__ int32_t wc[CAND_NT / 64][kCandK];
  __shared__ int32_t tbl[CAND_NT / 64 * 192];
  __shared__ int2 rng_s[CAND_NT / 64];
  __shared__ uint64_t selk[kCandK];
  __shared__ int32_t selc[kCandK];
  __shared__ int32_t selcnt;
  const int n = xcd_node((int)blockIdx.x, N);
  if (n < 0) return;
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = lane_id();
  uint64_t kk[kCandK];
  int32_t kc[kCandK];
#pragma unroll
  for (int j = 0; j < kCandK; ++j) {
    kk[j] = 0;
    kc[j] = 0;
  }
  int64_t streamed = 0;
  const int64_t sn = size[n];
  const uint32_t din = (uint32_t)indeg[n];
  bool half = false;
  if (sn < omega) {
    const uint32_t tot = (uint32_t)total[n];
    const int hb = tot ? 32 - __clz(tot) : 0;
    const int cb = din ? 32 - __clz(din) : 0;
    const bool packed = hb + cb <= 32;
    // hist alone in 16-bit halves when it fits and no candidate can break
    // Delta (c is then counted afterwards for the kept candidates only)
    half = maxin && hb <= 16 && (int64_t)din + (int64_t)(*maxin) <= (int64_t)delta && inbound_slots(din) <= words;
    const uint64_t hmask = (hb >= 32) ? 0xffffffffull : ((1ull << hb) - 1ull);
    const int R = half ? 2 * words : (packed ? words : (words >> 1));
    const int i0 = ioff[n], i1 = ioff[n + 1];
    uint64_t *lds64 = reinterpret_cast<uint64_t *>(lds);
    // windows over the neighbours' id range only
    const int2 rg = neighbour_range<CAND_NT>(i0, i1, inc, hoff, hpin, rng_s);
    const uint32_t *clip = ((int64_t)rg.y - rg.x >= R) ? hpin : nullptr;  // several windows
    for (int lo = rg.x; lo <= rg.y; lo += R) {
      const int span = min(R, rg.y + 1 - lo);
      const int zw = half ? (span + 1) >> 1 : (packed ? span : 2 * span);
      for (int i = tid; i < zw; i += CAND_NT) lds[i] = 0u;
      __syncthreads();
      // counter layout: 0 = hist in 16-bit halves, 1 = packed 32-bit, 2 = 64-bit
      streamed += with_mode(half ? 0 : (packed ? 1 : 2), [&](auto mode) {
        constexpr int MODE = decltype(mode)::value;
        return stream_segments<CAND_NT / 64, kRateU, true, uint32_t>(
            i0, i1, inc, hoff, nullptr, hw, tbl, [&](int j) { return hpin[j]; },
            [&](uint32_t y, uint32_t info) {
              const int m = (int)(y & kIdMask);
              const uint32_t rel = (uint32_t)(m - lo);
              if ((m != n) & (rel < (uint32_t)span)) {
                const uint32_t we = info & kIdMask;
                const uint32_t both = (info & y) >> 31;
                if constexpr (MODE == 0)
                  atomicAdd(&lds[rel >> 1], we << ((rel & 1u) << 4));
                else if constexpr (MODE == 1)
                  atomicAdd(&lds[rel], we + (both << hb));
                else
                  atomicAdd((unsigned long long *)&lds64[rel],
                            (unsigned long long)we | ((unsigned long long)both << 32));
              }
            },
            clip, lo, lo + span);
      });
      __syncthreads();
      if (half) {
        // Delta holds for every candidate here, whatever c is
        for (int i = tid; i < zw; i += CAND_NT) {
          const uint32_t v = lds[i];
          if (!v) continue;
#pragma unroll
          for (int hh = 0; hh < 2; ++hh) {
            const uint64_t h = hh ? (v >> 16) : (v & 0xffffu);
            const int m = lo + 2 * i + hh;
            const uint64_t key = (h << 32) | (uint32_t)m;
            if (h && key > kk[kCandK - 1] && sn + size[m] <= omega) cand_insert(kk, kc, key, 0);
          }
        }
        __syncthreads();
        continue;
      }
      for (int i = tid; i < span; i += CAND_NT) {
        uint64_t h, c;
        if (packed) {
          const uint32_t v = lds[i];
          if (!v) continue;
          h = v & hmask;
          c = (hb >= 32) ? 0 : (v >> hb);
        } else {
          const uint64_t v = lds64[i];
          if (!v) continue;
          h = v & 0xffffffffull;
          c = v >> 32;
        }
        const int m = lo + i;
        const uint64_t key = (h << 32) | (uint32_t)m;
        if (key > kk[kCandK - 1]) {
          const int64_t un = (int64_t)din + indeg[m] - (int64_t)c;
          if (sn + size[m] <= omega && un <= delta) cand_insert(kk, kc, key, (int32_t)c);
        }
      }
      __syncthreads();
    }
  }
  add_wave_units(units, streamed);
  // per wave: 8 rounds of "largest head", popped by its owner lane
#pragma unroll
  for (int r = 0; r < kCandK; ++r) {
    const uint64_t best = wave_max_u64(kk[0]);
    if (best != 0 && kk[0] == best) {
      wk[w][r] = best;
      wc[w][r] = kc[0];
#pragma unroll
      for (int j = 0; j + 1 < kCandK; ++j) {
        kk[j] = kk[j + 1];
        kc[j] = kc[j + 1];
      }
      kk[kCandK - 1] = 0;
      kc[kCandK - 1] = 0;
    }
    if (best == 0 && l == 0) {
      wk[w][r] = 0;
      wc[w][r] = 0;
    }
  }
  __syncthreads();
  if (w == 0) {
    uint64_t e = wk[l / kCandK][l % kCandK];
    const int32_t ec = wc[l / kCandK][l % kCandK];
    int cnt = 0;
#pragma unroll
    for (int r = 0; r < kCandK; ++r) {
      const uint64_t best = wave_max_u64(e);
      if (best != 0 && e == best) {
        selk[r] = best;
        selc[r] = ec;
        e = 0;
      }
      if (best == 0 && l == 0) {
        selk[r] = 0;
        selc[r] = 0;
      }
      cnt += best != 0 ? 1 : 0;
    }
    if (l == 0) selcnt = cnt;
  }
  __syncthreads();
  // c(n, m) of the kept candidates (the window's LDS is free now)
  if (half) inbound_common<CAND_NT>(n, ioff, inc, lds, inbound_slots(din), selk, selc, selcnt);
  __syncthreads();
  if (tid < kCandK) {
    ck[(int64_t)n * kCandK + tid] = selk[tid];
    cc[(int64_t)n * kCandK + tid] = selc[tid];
  }
  if (tid == 0) ccnt[n] = selcnt < keep ? selcnt : keep;
}

// ---------------------------------------------------------------------------
// 2. symmetric candidate sets
// ---------------------------------------------------------------------------
// Both orientations of every kept pair: key n << idbits | m, value = slot of
// the pair in ck / cc.  off[n] = exclusive prefix of ccnt.  With kept (the
// device count of kept pairs), the entries from 2 *kept up to the bound
// Mb get the key of all ones over 2 idbits bits, which no pair has (n != m),
// so that they sort last.
__global__ void k_cand_mirror(const uint64_t *__restrict__ ck, const int32_t *__restrict__ ccnt,
                              const int32_t *__restrict__ off, int32_t N, int idbits, uint64_t *__restrict__ key,
                              uint32_t *__restrict__ val, const int32_t *__restrict__ kept, int64_t Mb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * kCandK) return;
  if (kept) {
    const int64_t M = 2 * (int64_t)*kept;
    const uint64_t pad = (1ull << (2 * idbits)) - 1ull;
    if (2 * t >= M && 2 * t < Mb) key[2 * t] = pad;
    if (2 * t + 1 >= M && 2 * t + 1 < Mb) key[2 * t + 1] = pad;
  }
  const int n = (int)(t / kCandK), j = (int)(t % kCandK);
  if (j >= ccnt[n]) return;
  const uint64_t m = ck[t] & 0xffffffffull;
  const int64_t p = 2 * ((int64_t)off[n] + j);
  key[p] = ((uint64_t)n << idbits) | m;
  key[p + 1] = (m << idbits) | (uint64_t)n;
  val[p] = (uint32_t)t;
  val[p + 1] = (uint32_t)t;
}

// First entry of each distinct key among the first M (2 *kept when kept is
// given; the entries up to the bound Mb are padding).
__global__ void k_cand_first(const uint64_t *__restrict__ key, int64_t Mb, const int32_t *__restrict__ kept,
                             int32_t *__restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t M = kept ? 2 * (int64_t)*kept : Mb;
  if (i < Mb) flag[i] = (i < M && (i == 0 || key[i] != key[i - 1])) ? 1 : 0;
}

__global__ void k_cand_compact(const uint64_t *__restrict__ key, const uint32_t *__restrict__ val, int64_t Mb,
                               const int32_t *__restrict__ kept, const int32_t *__restrict__ pos,
                               uint64_t *__restrict__ cnm, uint32_t *__restrict__ csrc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t M = kept ? 2 * (int64_t)*kept : Mb;
  if (i >= M) return;
  if (i == 0 || key[i] != key[i - 1]) {
    cnm[pos[i]] = key[i];
    csrc[pos[i]] = val[i];
  }
}

// coff[n] = first entry of node n (n = 0 .. N; coff[N] = C; C = *cdev if given,
// and then added to *units when that is non-null: the network's rows)
__global__ void k_cand_offsets(const uint64_t *__restrict__ cnm, int64_t C, const int32_t *__restrict__ cdev,
                               int32_t N, int idbits, int64_t *__restrict__ coff, unsigned long long *units) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n > N) return;
  if (n == 0 && cdev && units) atomicAdd(units, (unsigned long long)*cdev);
  const uint64_t x = (uint64_t)n << idbits;
  int64_t lo = 0, hi = cdev ? (int64_t)*cdev : C;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (cnm[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  coff[n] = lo;
}

// ---------------------------------------------------------------------------
// 3. features and the network
// ---------------------------------------------------------------------------
// 8 floor(log2(f+1)) + the three bits of f+1 below its leading one, <= 255.
__device__ __forceinline__ int32_t qlog_code(uint64_t f) {
  const uint64_t v = f + 1ull;
  const int e = 63 - __clzll((long long)v);
  const uint64_t t = e >= 3 ? (v >> (e - 3)) & 7ull : (v << (3 - e)) & 7ull;
  const int32_t code = 8 * e + (int32_t)t;
  return code < 255 ? code : 255;
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

// BF16 bits of an integer |v| <= 256 (exact: its float has no low mantissa bits).
__device__ __forceinline__ short bf16_of_int(int v) { return (short)(__float_as_uint((float)v) >> 16); }

__device__ __forceinline__ bf16x4 bf16x4_of(int a, int b, int c, int d) {
  bf16x4 r;
  r[0] = bf16_of_int(a);
  r[1] = bf16_of_int(b);
  r[2] = bf16_of_int(c);
  r[3] = bf16_of_int(d);
  return r;
}

constexpr int MLP_NT = 256;
constexpr int MLP_LD = 65;  // padded LDS row (words) of a wave's 32 x 64 activation tile

// Network parameters as laid out in hgp_mlp (int32): k, r1, r2, b3, w1[16*64],
// b1[64], w2[64*64], b2[64], w3[64].
struct MlpView {
  int32_t r1, r2, b3;
  const int32_t *w1, *b1, *w2, *b2, *w3;
};
__device__ __forceinline__ MlpView mlp_view(const int32_t *p) {
  MlpView v;
  v.r1 = p[1];
  v.r2 = p[2];
  v.b3 = p[3];
  v.w1 = p + 4;
  v.b1 = v.w1 + kMlpF * kMlpH;
  v.w2 = v.b1 + kMlpH;
  v.b2 = v.w2 + kMlpH * kMlpH;
  v.w3 = v.b2 + kMlpH;
  return v;
}

// Requantisation: clamp(round_half_even(v / 2^r), 0, 255) of an exact integer v.
__device__ __forceinline__ int requant(float v, float inv) {
  const float q = rintf(v * inv);
  return (int)fminf(fmaxf(q, 0.0f), 255.0f);
}

// Scores rows [0, n) of 16 codes each (codes(i, x) fills row i).  One wave
// per 32-row tile; tiles are strided over the grid.  MFMA operand layout of
// v_mfma_f32_32x32x8_bf16: lane l supplies A[l%32][4(l/32) + j] and
// B[4(l/32) + j][l%32], j = 0..3, and holds D[8(r/4) + 4(l/32) + r%4][l%32]
// in accumulator r = 0..15.
template <class Codes>
__device__ void mlp_tiles(int64_t n, const int32_t *__restrict__ params, Codes codes, int32_t *__restrict__ out,
                          int32_t *tile) {
  const MlpView P = mlp_view(params);
  const int l = lane_id();
  const int col = l & 31, half = l >> 5;
  bf16x4 B1[2][2], B2[2][8];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int k0 = 8 * s + 4 * half;
      const int c = 32 * t + col;
      B1[t][s] = bf16x4_of(P.w1[(k0 + 0) * kMlpH + c], P.w1[(k0 + 1) * kMlpH + c], P.w1[(k0 + 2) * kMlpH + c],
                           P.w1[(k0 + 3) * kMlpH + c]);
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k0 = 8 * s + 4 * half;
      const int c = 32 * t + col;
      B2[t][s] = bf16x4_of(P.w2[(k0 + 0) * kMlpH + c], P.w2[(k0 + 1) * kMlpH + c], P.w2[(k0 + 2) * kMlpH + c],
                           P.w2[(k0 + 3) * kMlpH + c]);
    }
  }
  const float bias1[2] = {(float)P.b1[col], (float)P.b1[32 + col]};
  const float bias2[2] = {(float)P.b2[col], (float)P.b2[32 + col]};
  const float inv1 = ldexpf(1.0f, -P.r1), inv2 = ldexpf(1.0f, -P.r2);
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t ntiles = (n + 31) / 32;
  for (int64_t tileno = wave; tileno < ntiles; tileno += waves) {
    const int64_t row0 = tileno * 32;
    const int64_t gi = row0 + col;
    int32_t x[kMlpF];
    if (gi < n) {
      codes(gi, x);
    } else {
#pragma unroll
      for (int f = 0; f < kMlpF; ++f) x[f] = 0;
    }
    bf16x4 A1[2];
    A1[0] = half ? bf16x4_of(x[4], x[5], x[6], x[7]) : bf16x4_of(x[0], x[1], x[2], x[3]);
    A1[1] = half ? bf16x4_of(x[12], x[13], x[14], x[15]) : bf16x4_of(x[8], x[9], x[10], x[11]);
    // layer 1
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      floatx16 acc = {};
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(A1[0], B1[t][0], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(A1[1], B1[t][1], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r >> 2) + 4 * half + (r & 3);
        tile[row * MLP_LD + 32 * t + col] = requant(acc[r] + bias1[t], inv1);
      }
    }
    wave_lds_sync();
    bf16x4 A2[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int k0 = 8 * s + 4 * half;
      const int32_t *src = tile + col * MLP_LD + k0;
      A2[s] = bf16x4_of(src[0], src[1], src[2], src[3]);
    }
    wave_lds_sync();
    // layer 2
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      floatx16 acc = {};
#pragma unroll
      for (int s = 0; s < 8; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(A2[s], B2[t][s], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r >> 2) + 4 * half + (r & 3);
        tile[row * MLP_LD + 32 * t + col] = requant(acc[r] + bias2[t], inv2);
      }
    }
    wave_lds_sync();
    // output unit: an exact integer dot product per row
    if (half == 0 && gi < n) {
      int32_t sc = P.b3;
      const int32_t *a = tile + col * MLP_LD;
#pragma unroll 8
      for (int j = 0; j < kMlpH; ++j) sc += a[j] * P.w3[j];
      out[gi] = sc;
    }
    wave_lds_sync();
  }
}

__global__ __launch_bounds__(MLP_NT) void k_mlp_score_codes(const int32_t *__restrict__ xq, int64_t n,
                                                            const int32_t *__restrict__ params,
                                                            int32_t *__restrict__ out) {
  __shared__ int32_t tiles[MLP_NT / 64][32 * MLP_LD];
  mlp_tiles(
      n, params,
      [&](int64_t i, int32_t(&x)[kMlpF]) {
#pragma unroll
        for (int f = 0; f < kMlpF; ++f) x[f] = xq[i * kMlpF + f];
      },
      out, tiles[threadIdx.x >> 6]);
}

// Features of entry i = (n, m) of the symmetric sets, canonical a < b:
// hist, c, size(a), size(b), |in(a) u in(b)|, |I(a)|, |I(b)|, level,
// Omega - size(a) - size(b), Delta - |in(a) u in(b)|, six zeros.
struct CandCodes {
  const uint64_t *cnm;
  const uint32_t *csrc;
  const uint64_t *ck;
  const int32_t *cc;
  const int32_t *size, *indeg, *ioff;
  int idbits, level;
  int32_t omega, delta;
  __device__ __forceinline__ void operator()(int64_t i, int32_t (&x)[kMlpF]) const {
    const uint64_t key = cnm[i];
    const uint32_t src = csrc[i];
    const int n = (int)(key >> idbits);
    const int m = (int)(key & ((1ull << idbits) - 1ull));
    const int a = n < m ? n : m, b = n < m ? m : n;
    const int64_t h = (int64_t)(ck[src] >> 32);
    const int64_t c = cc[src];
    const int64_t sa = size[a], sb = size[b];
    const int64_t uni = (int64_t)indeg[a] + indeg[b] - c;
    x[0] = qlog_code((uint64_t)h);
    x[1] = qlog_code((uint64_t)c);
    x[2] = qlog_code((uint64_t)sa);
    x[3] = qlog_code((uint64_t)sb);
    x[4] = qlog_code((uint64_t)uni);
    x[5] = qlog_code((uint64_t)(ioff[a + 1] - ioff[a]));
    x[6] = qlog_code((uint64_t)(ioff[b + 1] - ioff[b]));
    x[7] = qlog_code((uint64_t)level);
    x[8] = qlog_code((uint64_t)(omega - sa - sb));
    x[9] = qlog_code((uint64_t)(delta - uni));
#pragma unroll
    for (int f = kMlpNFeat; f < kMlpF; ++f) x[f] = 0;
  }
};

__global__ __launch_bounds__(MLP_NT) void k_cand_score(CandCodes cf, int64_t C, const int32_t *__restrict__ cdev,
                                                       const int32_t *__restrict__ params, int32_t *__restrict__ out) {
  __shared__ int32_t tiles[MLP_NT / 64][32 * MLP_LD];
  mlp_tiles(cdev ? (int64_t)*cdev : C, params, cf, out, tiles[threadIdx.x >> 6]);
}

// Codes only (for the level API): the same feature function, written out.
__global__ void k_cand_codes(CandCodes cf, int64_t C, int32_t *__restrict__ xq) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= C) return;
  int32_t x[kMlpF];
  cf(i, x);
#pragma unroll
  for (int f = 0; f < kMlpF; ++f) xq[i * kMlpF + f] = x[f];
}

// ---------------------------------------------------------------------------
// 4. selection
// ---------------------------------------------------------------------------
// pair(n) = argmax over C(n) of (score, id); the matching key is score + 2^31
// (order-preserving, in [0, 2^32)).  ppair / pscore: the plain pair (first
// kept candidate) and its hist.
// pair(n) = the candidate m maximising (score, id), as the packed key
// (score + 2^31) << 32 | m (scores stay far above -2^31, so a key is never 0,
// the value of a node without candidates).  One lane per candidate of the
// node-sorted array: a segmented maximum over the wave's runs of equal n and
// one atomicMax per run, so a node that is in the candidate sets of
// thousands of others costs a few hundred atomics, not a serial scan.
__global__ void k_cand_best(const uint64_t *__restrict__ cnm, const int32_t *__restrict__ cs, int64_t C,
                            const int32_t *__restrict__ cdev, int idbits, unsigned long long *__restrict__ best) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = i < (cdev ? (int64_t)*cdev : C);
  const uint64_t e = in ? cnm[i] : 0ull;
  const int64_t n = in ? (int64_t)(e >> idbits) : -1 - (int64_t)lane_id();  // lanes past C: runs of their own
  unsigned long long key =
      in ? ((unsigned long long)((int64_t)cs[i] + 2147483648LL) << 32) | (e & ((1ull << idbits) - 1ull)) : 0ull;
  const int l = lane_id();
  // the array is sorted by n, so equal n are contiguous lanes
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned long long k2 = __shfl_up(key, o, 64);
    const int64_t n2 = __shfl_up(n, o, 64);
    if (l >= o && n2 == n && k2 > key) key = k2;
  }
  const int64_t nn = __shfl_down(n, 1, 64);
  if (in && (l == 63 || nn != n)) atomicMax(&best[n], key);
}

// Unpacks the selection and records the plain pair (the first candidate of
// the rating).
__global__ void k_cand_pick(const unsigned long long *__restrict__ best, int32_t N, const uint64_t *__restrict__ ck,
                            const int32_t *__restrict__ ccnt, int32_t *__restrict__ pair, int64_t *__restrict__ score,
                            int32_t *__restrict__ ppair, int64_t *__restrict__ pscore) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const unsigned long long b = best[n];
  pair[n] = b ? (int32_t)(b & 0xffffffffull) : -1;
  score[n] = b ? (int64_t)(b >> 32) : 0;
  const uint64_t k0 = ck[n * kCandK];
  const bool any = ccnt[n] > 0;
  ppair[n] = any ? (int)(k0 & 0xffffffffull) : -1;
  pscore[n] = any ? (int64_t)(k0 >> 32) : 0;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

const int32_t *upload_mlp(DevBuf &buf, const hgp_mlp *q, hipStream_t s) {
  check_mlp(q);
  buf.reserve(sizeof(hgp_mlp));
  HGP_HIP(hipMemcpyAsync(buf.ptr, q, sizeof(hgp_mlp), hipMemcpyHostToDevice, s));
  return buf.as<int32_t>();
}

static int grid_for_tiles(int64_t rows) {
  const int64_t tiles = (rows + 31) / 32;
  const int64_t blocks = (tiles + MLP_NT / 64 - 1) / (MLP_NT / 64);
  return (int)std::min<int64_t>(std::max<int64_t>(blocks, 1), 4096);
}

void launch_mlp_score_codes(const int32_t *xq, int64_t n, const int32_t *params, int32_t *out, hipStream_t s) {
  if (n <= 0) return;
  KScope ks(HGP_K_MLP, s);
  add_units(HGP_K_MLP, n);
  k_mlp_score_codes<<<grid_for_tiles(n), MLP_NT, 0, s>>>(xq, n, params, out);
  HGP_LAUNCH_CHECK();
}

int64_t build_candidates(const LevelView &L, const int32_t *total, int32_t omega, int32_t delta, int keep,
                         CandBufs &B, DevBuf &scan_tmp, DevBuf &sort_tmp, hipStream_t s) {
  if (keep < 1 || keep > kCandK) throw Error(HGP_EINVAL, "candidates per node outside 1..8");
  const int32_t N = L.n;
  if (N <= 0) return 0;
  {
    // thread-safe one-time opt-in to the large dynamic LDS size
  static const bool attr_set = [] {
    HGP_HIP(hipFuncSetAttribute((const void *)k_rate_cand, hipFuncAttributeMaxDynamicSharedMemorySize, CAND_LDS_BYTES));
    return true;
  }();
  (void)attr_set;
    const int max_words = CAND_LDS_BYTES / 4;
    int words = N <= max_words / 2 ? 2 * N : max_words;
    words = (words + 1) & ~1;
    KScope ks(HGP_K_RATE, s);
    k_rate_cand<<<xcd_grid(N), CAND_NT, (size_t)words * 4, s>>>(N, L.ioff, L.inc, L.hoff, L.hpin, L.hw, L.size,
                                                                 L.indeg, total, L.maxin, omega, delta, words, keep,
                                                                 B.ck, B.cc, B.ccnt, units_ptr(HGP_K_RATE));
    HGP_LAUNCH_CHECK();
  }
  return candidate_sets(L, B, scan_tmp, sort_tmp, s);
}

int64_t candidate_sets(const LevelView &L, CandBufs &B, DevBuf &scan_tmp, DevBuf &sort_tmp, hipStream_t s) {
  const int32_t N = L.n;
  if (N <= 0) return 0;
  const int idbits = std::max(1, bits_for(N - 1));
  int64_t C = 0, M = 0;
  {
    KScope ks(HGP_K_MLP, s);
    scan_i32(B.ccnt, B.coff32, N, B.tot32, scan_tmp, s);
    HGP_HIP(hipMemcpyAsync(B.hbox, B.tot32, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HGP_HIP(hipStreamSynchronize(s));
    const int32_t kept = *reinterpret_cast<const int32_t *>(B.hbox);
    M = 2 * (int64_t)kept;
    if (M > 0) {
      k_cand_mirror<<<div_up((int64_t)N * kCandK, 256), 256, 0, s>>>(B.ck, B.ccnt, B.coff32, N, idbits, B.key,
                                                                      B.val, nullptr, M);
      HGP_LAUNCH_CHECK();
    }
  }
  if (M > 1) radix_sort_u64(B.key, B.key2, B.val, B.val2, M, 2 * idbits, sort_tmp, s);
  KScope ks(HGP_K_MLP, s);
  if (M > 0) {
    k_cand_first<<<div_up(M, 256), 256, 0, s>>>(B.key, M, nullptr, B.flag);
    HGP_LAUNCH_CHECK();
    scan_i32(B.flag, B.flag, M, B.tot32 + 1, scan_tmp, s);
    k_cand_compact<<<div_up(M, 256), 256, 0, s>>>(B.key, B.val, M, nullptr, B.flag, B.cnm, B.csrc);
    HGP_LAUNCH_CHECK();
    HGP_HIP(hipMemcpyAsync(B.hbox, B.tot32 + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HGP_HIP(hipStreamSynchronize(s));
    C = *reinterpret_cast<const int32_t *>(B.hbox);
  }
  k_cand_offsets<<<div_up((int64_t)N + 1, 256), 256, 0, s>>>(B.cnm, C, nullptr, N, idbits, B.coff, nullptr);
  HGP_LAUNCH_CHECK();
  B.cdev = nullptr;
  return C;
}

int64_t candidate_sets_dev(const LevelView &L, CandBufs &B, int keep, DevBuf &scan_tmp, DevBuf &sort_tmp,
                           hipStream_t s) {
  const int32_t N = L.n;
  B.cdev = nullptr;
  if (N <= 0) return 0;
  if (keep < 1 || keep > kCandK) throw Error(HGP_EINVAL, "candidates per node outside 1..8");
  const int idbits = std::max(1, bits_for(N - 1));
  const int64_t Mb = 2 * (int64_t)N * keep;  // every node keeps at most `keep` pairs
  {
    KScope ks(HGP_K_MLP, s);
    scan_i32(B.ccnt, B.coff32, N, B.tot32, scan_tmp, s);
    k_cand_mirror<<<div_up((int64_t)N * kCandK, 256), 256, 0, s>>>(B.ck, B.ccnt, B.coff32, N, idbits, B.key, B.val,
                                                                    B.tot32, Mb);
    HGP_LAUNCH_CHECK();
  }
  if (Mb > 1) radix_sort_u64(B.key, B.key2, B.val, B.val2, Mb, 2 * idbits, sort_tmp, s);
  KScope ks(HGP_K_MLP, s);
  k_cand_first<<<div_up(Mb, 256), 256, 0, s>>>(B.key, Mb, B.tot32, B.flag);
  HGP_LAUNCH_CHECK();
  scan_i32(B.flag, B.flag, Mb, B.tot32 + 1, scan_tmp, s);
  k_cand_compact<<<div_up(Mb, 256), 256, 0, s>>>(B.key, B.val, Mb, B.tot32, B.flag, B.cnm, B.csrc);
  HGP_LAUNCH_CHECK();
  k_cand_offsets<<<div_up((int64_t)N + 1, 256), 256, 0, s>>>(B.cnm, 0, B.tot32 + 1, N, idbits, B.coff,
                                                              units_ptr(HGP_K_MLP));
  HGP_LAUNCH_CHECK();
  B.cdev = B.tot32 + 1;
  return Mb;
}

void score_and_select(const LevelView &L, int32_t omega, int32_t delta, int level, const int32_t *params,
                      CandBufs &B, int64_t C, hipStream_t s) {
  const int32_t N = L.n;
  if (N <= 0) return;
  KScope ks(HGP_K_MLP, s);
  const int idbits = std::max(1, bits_for(N - 1));
  CandCodes cf{B.cnm, B.csrc, B.ck, B.cc, L.size, L.indeg, L.ioff, idbits, level, omega, delta};
  if (C > 0) {
    if (!B.cdev) add_units(HGP_K_MLP, C);
    k_cand_score<<<grid_for_tiles(C), MLP_NT, 0, s>>>(cf, C, B.cdev, params, B.cs);
    HGP_LAUNCH_CHECK();
  }
  fill_i64(reinterpret_cast<int64_t *>(B.best), N, 0, s);
  if (C > 0) {
    k_cand_best<<<div_up(C, 256), 256, 0, s>>>(B.cnm, B.cs, C, B.cdev, idbits, B.best);
    HGP_LAUNCH_CHECK();
  }
  k_cand_pick<<<div_up(N, 256), 256, 0, s>>>(B.best, N, B.ck, B.ccnt, B.pair, B.score, B.ppair, B.pscore);
  HGP_LAUNCH_CHECK();
}

int64_t learned_candidates(const LevelView &L, const int32_t *total, int32_t omega, int32_t delta, int level,
                           int keep, const int32_t *params, CandBufs &B, DevBuf &scan_tmp, DevBuf &sort_tmp,
                           hipStream_t s) {
  const int64_t C = build_candidates(L, total, omega, delta, keep, B, scan_tmp, sort_tmp, s);
  score_and_select(L, omega, delta, level, params, B, C, s);
  return C;
}

void launch_cand_codes(const LevelView &L, int32_t omega, int32_t delta, int level, const CandBufs &B, int64_t C,
                       int32_t *xq, hipStream_t s) {
  if (C <= 0) return;
  const int idbits = std::max(1, bits_for(L.n - 1));
  CandCodes cf{B.cnm, B.csrc, B.ck, B.cc, L.size, L.indeg, L.ioff, idbits, level, omega, delta};
  k_cand_codes<<<div_up(C, 256), 256, 0, s>>>(cf, C, xq);
  HGP_LAUNCH_CHECK();
}

__global__ void k_widen_scores(const int32_t *__restrict__ in, int64_t n, int64_t *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}

void launch_widen_scores(const int32_t *in, int64_t n, int64_t *out, hipStream_t s) {
  if (n <= 0) return;
  k_widen_scores<<<div_up(n, 256), 256, 0, s>>>(in, n, out);
  HGP_LAUNCH_CHECK();
}

// network score of the selected pair from its matching key (0 without pair)
__global__ void k_unkey(const int32_t *__restrict__ pair, const int64_t *__restrict__ key, int32_t n,
                        int64_t *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = pair[i] >= 0 ? key[i] - 2147483648LL : 0;
}

void launch_unkey(const int32_t *pair, const int64_t *key, int32_t n, int64_t *out, hipStream_t s) {
  if (n <= 0) return;
  k_unkey<<<div_up(n, 256), 256, 0, s>>>(pair, key, n, out);
  HGP_LAUNCH_CHECK();
}

__global__ void k_cand_ids(const uint64_t *__restrict__ cnm, int64_t C, int idbits, int32_t *__restrict__ ids) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < C) ids[i] = (int32_t)(cnm[i] & ((1ull << idbits) - 1ull));
}

void launch_cand_ids(const CandBufs &B, int64_t C, int32_t N, int32_t *ids, hipStream_t s) {
  if (C <= 0) return;
  const int idbits = std::max(1, bits_for(N - 1));
  k_cand_ids<<<div_up(C, 256), 256, 0, s>>>(B.cnm, C, idbits, ids);
  HGP_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// scoring without device allocation
// ---------------------------------------------------------------------------
// The scratch of hgp_mlp_score_device_noalloc: the integer network staged
// from host memory, then the int32 scores of up to HGP_NOALLOC_MAX_ROWS rows
// before they are widened.  One copy per device (each device that loads the
// library's code object holds its own), kept until the process ends.  Host
// code must not pass `scratch` itself to a kernel: its name on the host is a
// stand-in, not a device address.  noalloc_scratch_init looks the address up
// once per device, with that device current, and later calls use it.
constexpr size_t kNoAllocParamBytes = (sizeof(hgp_mlp) + 255) & ~size_t(255);
constexpr size_t kNoAllocBytes = kNoAllocParamBytes + (size_t)HGP_NOALLOC_MAX_ROWS * sizeof(int32_t);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

void *noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) throw Error(HGP_EUNSUPPORTED, "device id beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    HGP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(HGP_EDEVICE, "no device address for the scoring scratch");
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

void mlp_score_noalloc(void *scratch_dev, const hgp_mlp *q, const int32_t *xq, int64_t n, int64_t *score,
                       hipStream_t s) {
  if (!scratch_dev) throw Error(HGP_EINTERNAL, "scoring scratch not set up");
  if (n > HGP_NOALLOC_MAX_ROWS) throw Error(HGP_EUNSUPPORTED, "more rows than the allocation-free scratch holds");
  if (n <= 0) return;
  // every byte read below is written first: the network by the copy, the
  // int32 scores by the scoring kernel, so nothing needs clearing
  unsigned char *base = static_cast<unsigned char *>(scratch_dev);
  HGP_HIP(hipMemcpyAsync(base, q, sizeof(hgp_mlp), hipMemcpyHostToDevice, s));
  int32_t *tmp = reinterpret_cast<int32_t *>(base + kNoAllocParamBytes);
  launch_mlp_score_codes(xq, n, reinterpret_cast<const int32_t *>(base), tmp, s);
  launch_widen_scores(tmp, n, score, s);
}

}  // namespace hgp
