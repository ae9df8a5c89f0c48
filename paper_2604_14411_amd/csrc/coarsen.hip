// Coarsening kernels (Sec. III): canonical input, incidence transpose,
// constrained candidate rating (Eq. 2), pseudo-forest matching, contraction.
#include "coarsen.hpp"

namespace hgp {

constexpr int SEG_NT = 256;

// ---------------------------------------------------------------------------
// input validation + canonical level 0
// ---------------------------------------------------------------------------
__global__ void k_check_offsets(const int32_t *__restrict__ off, int32_t E, int32_t *err) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0 && off[0] != 0) atomicOr(err, kErrCsr);
  if (e < E) {
    const int32_t a = off[e], b = off[e + 1];
    if (b < a) atomicOr(err, kErrCsr);
    else if (b - a > kHugeCap) atomicOr(err, kErrBigHedge);
  }
}

__global__ void k_check_weights(const int32_t *__restrict__ hw, int32_t E, const int32_t *__restrict__ nw,
                                int32_t N, int32_t *err, unsigned long long *sums) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long a = 0, b = 0;
  if (i < E) {
    const int32_t x = hw ? hw[i] : 1;
    if (x < 1) atomicOr(err, kErrWeight);
    else a = (unsigned long long)x;
  }
  if (i < N) {
    const int32_t x = nw ? nw[i] : 1;
    if (x < 1) atomicOr(err, kErrWeight);
    else b = (unsigned long long)x;
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane_id() == 0) {
    if (a) atomicAdd(&sums[0], a);
    if (b) atomicAdd(&sums[1], b);
  }
}

// One workgroup per hedge: tag destinations, sort pins by id, reject
// out-of-range pins, duplicates and bad source counts.
// Bit 31 of a canonical pin marks the pins whose hedges count toward Delta
// for their part: destinations (inbound, Sec. II-A), sources (outbound) or
// every pin (incident); `role` is HGP_INBOUND / HGP_OUTBOUND / HGP_INCIDENT.
// Hedges above kSegCap pins sort their keys in global scratch (huge_keys at
// twice the hedge's pin offset: next_pow2(|e|) < 2|e| words).
__device__ __forceinline__ void canon_hedge(int e, int b, int len, const int32_t *__restrict__ pins,
                                            const int32_t *__restrict__ nsrc, int32_t N, int32_t role, int32_t *err,
                                            uint32_t *__restrict__ hpin, uint32_t *key) {
  const int ns = nsrc ? nsrc[e] : 1;
  if (threadIdx.x == 0 && (ns < 0 || ns > len)) atomicOr(err, kErrNsrc);
  const int np = next_pow2(len);
  for (int i = threadIdx.x; i < np; i += SEG_NT) {
    uint32_t k = 0xffffffffu;
    if (i < len) {
      const int32_t v = pins[b + i];
      if (v < 0 || v >= N) {
        atomicOr(err, kErrPin);
        k = 0xfffffffeu;
      } else {
        const bool dst = i >= ns;
        const uint32_t f = role == 0 ? (dst ? 1u : 0u) : role == 1 ? (dst ? 0u : 1u) : 1u;
        k = ((uint32_t)v << 1) | f;
      }
    }
    key[i] = k;
  }
  __syncthreads();
  block_bitonic_sort<uint32_t, SEG_NT>(key, np);
  for (int i = threadIdx.x; i < len; i += SEG_NT) {
    const uint32_t k = key[i];
    if (i + 1 < len && (key[i + 1] >> 1) == (k >> 1)) atomicOr(err, kErrDup);
    hpin[b + i] = (k >> 1) | ((k & 1u) << 31);
  }
}

__global__ __launch_bounds__(SEG_NT) void k_canon(const int32_t *__restrict__ off, const int32_t *__restrict__ pins,
                                                  const int32_t *__restrict__ nsrc, int32_t N, int32_t role,
                                                  int32_t *err, uint32_t *__restrict__ hpin,
                                                  uint32_t *__restrict__ huge_keys) {
  __shared__ uint32_t key[kSegCap];
  const int e = blockIdx.x;
  const int b = off[e];
  const int len = off[e + 1] - b;
  if (len <= 0) return;
  if (len <= kSegCap) {
    canon_hedge(e, b, len, pins, nsrc, N, role, err, hpin, key);
  } else if (huge_keys && len <= kHugeCap) {
    canon_hedge(e, b, len, pins, nsrc, N, role, err, hpin, huge_keys + 2 * (int64_t)b);
  } else if (threadIdx.x == 0) {
    atomicOr(err, kErrInternal);
  }
}

// ---------------------------------------------------------------------------
// incidence transpose: I(n) with the destination flag, |in(n)|, total(n)
// ---------------------------------------------------------------------------
// (node, hedge|dst) pairs in hedge order, then a stable radix sort by node:
// every I(n) comes out ascending by hedge id, with no contended atomics.
// Per pin j: its node id as the sort key and (hedge | dst) << 32 | j as the
// value, so the sort by node yields inc and perm together.
// (node, hedge|dst) pairs in hedge order, one wave per hedge.
__global__ void k_expand(const int32_t *__restrict__ hoff, const uint32_t *__restrict__ hpin, int32_t E,
                         uint32_t *__restrict__ key, uint64_t *__restrict__ val) {
  const int wid = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (wid >= E) return;
  for (int j = hoff[wid] + lane_id(); j < hoff[wid + 1]; j += 64) {
    const uint32_t x = hpin[j];
    key[j] = x & kIdMask;
    val[j] = ((uint64_t)((uint32_t)wid | (x & kDst)) << 32) | (uint32_t)j;
  }
}

// A wave takes 64 consecutive hedges: each lane writes the pins of its own
// hedge when it has at most kThreadSegMax of them (coarse levels: most
// hedges), then the wave writes the longer ones together, one at a time.
// Levels of long hedges use k_expand (a wave per hedge): with 64 long hedges
// per wave the loads in flight would be too few.
__global__ __launch_bounds__(256) void k_expand_lanes(const int32_t *__restrict__ hoff, const uint32_t *__restrict__ hpin,
                                                int32_t E, uint32_t *__restrict__ key, uint64_t *__restrict__ val) {
  const int64_t e0 = (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) << 6;
  if (e0 >= E) return;
  const int l = lane_id();
  const int64_t e = e0 + l;
  int b = 0, len = 0;
  if (e < E) {
    b = hoff[e];
    len = hoff[e + 1] - b;
  }
  const bool mine = len <= kThreadSegMax;
  if (mine) {
    for (int j = 0; j < len; ++j) {
      const uint32_t x = hpin[b + j];
      key[b + j] = x & kIdMask;
      val[b + j] = ((uint64_t)((uint32_t)e | (x & kDst)) << 32) | (uint32_t)(b + j);
    }
  }
  uint64_t rest = __ballot(!mine);
  while (rest) {
    const int i = __ffsll((long long)rest) - 1;
    rest &= rest - 1ull;
    const int hb = __shfl(b, i, 64), hl = __shfl(len, i, 64);
    const uint32_t he = (uint32_t)(e0 + i);
    for (int j = l; j < hl; j += 64) {
      const uint32_t x = hpin[hb + j];
      key[hb + j] = x & kIdMask;
      val[hb + j] = ((uint64_t)(he | (x & kDst)) << 32) | (uint32_t)(hb + j);
    }
  }
}

// ioff[v] = first position of node v in the sorted keys (P if none after).
__global__ void k_offsets_from_sorted(const uint32_t *__restrict__ key, int64_t P, int32_t N,
                                      int32_t *__restrict__ ioff) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j > P) return;
  const int64_t cur = j < P ? (int64_t)key[j] : (int64_t)N;
  const int64_t prev = j > 0 ? (int64_t)key[j - 1] : -1;
  for (int64_t v = prev + 1; v <= cur; ++v) ioff[v] = (int32_t)j;
}

__global__ void k_feasible(const int32_t *__restrict__ size, const int32_t *__restrict__ indeg, int32_t N,
                           int32_t omega, int32_t delta, int32_t *err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N && (size[i] > omega || indeg[i] > delta)) atomicOr(err, kErrInfeasible);
}

// ---------------------------------------------------------------------------
// rating + constrained selection (Eq. 2, Sec. III-A)
// ---------------------------------------------------------------------------
// One workgroup per node n.  The neighbour histogram lives in LDS as a dense
// array over an id window [lo, lo+R); windows are swept until all ids are
// covered.  Each counter packs hist (low hb bits) and c(n,m) = |in(n) n in(m)|
// (high bits) in 32 bits when they fit, else a 64-bit (c << 32 | hist) pair.
// A candidate is checked against Omega and Delta only when it would improve
// the thread's running best, with |in(n) u in(m)| = |in(n)|+|in(m)|-c.
// When |in(n)| + max_m |in(m)| <= Delta every candidate passes the Delta test
// whatever c is; then only hist is counted, in 16-bit halves of the LDS words
// when hist < 2^16 (hist(n,m) <= total(n)), so a window covers twice the ids.
template <int NT>
__global__ __launch_bounds__(NT) void k_rate(int32_t N, const int32_t *__restrict__ ioff,
                                             const uint32_t *__restrict__ inc, const int32_t *__restrict__ hoff,
                                             const uint32_t *__restrict__ hpin, const int32_t *__restrict__ hw,
                                             const int32_t *__restrict__ size, const int32_t *__restrict__ indeg,
                                             const int32_t *__restrict__ total, const int32_t *__restrict__ maxin,
                                             int32_t omega, int32_t delta, int32_t words,
                                             int32_t *__restrict__ pair, int64_t *__restrict__ score,
                                             unsigned long long *__restrict__ units) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ int64_t red_h[NT / 64];
  __shared__ int32_t red_m[NT / 64];
  __shared__ int32_t tbl[NT / 64 * 192];
  __shared__ int2 rng_s[NT / 64];
  const int n = xcd_node((int)blockIdx.x, N);
  if (n < 0) return;
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = lane_id();
  int best_m = -1;
  int64_t best_h = 0;
  int64_t streamed = 0;
  const int64_t sn = size[n];
  if (sn < omega) {
    const uint32_t tot = (uint32_t)total[n];
    const uint32_t din = (uint32_t)indeg[n];
    const int hb = tot ? 32 - __clz(tot) : 0;
    const int cb = din ? 32 - __clz(din) : 0;
    const bool packed = hb + cb <= 32;
    const bool half = hb <= 16 && (int64_t)din + (int64_t)(*maxin) <= (int64_t)delta;
    const uint64_t hmask = (hb >= 32) ? 0xffffffffull : ((1ull << hb) - 1ull);
    const int R = half ? 2 * words : (packed ? words : (words >> 1));
    const int i0 = ioff[n], i1 = ioff[n + 1];
    uint64_t *lds64 = reinterpret_cast<uint64_t *>(lds);
    // windows over the neighbours' id range only
    const int2 rg = neighbour_range<NT>(i0, i1, inc, hoff, hpin, rng_s);
    const uint32_t *clip = ((int64_t)rg.y - rg.x >= R) ? hpin : nullptr;  // several windows
    for (int lo = rg.x; lo <= rg.y; lo += R) {
      const int span = min(R, rg.y + 1 - lo);
      const int zw = half ? (span + 1) >> 1 : (packed ? span : 2 * span);
      for (int i = tid; i < zw; i += NT) lds[i] = 0u;
      __syncthreads();
      // counter layout: 0 = hist in 16-bit halves, 1 = packed 32-bit, 2 = 64-bit
      streamed += with_mode(half ? 0 : (packed ? 1 : 2), [&](auto mode) {
        constexpr int MODE = decltype(mode)::value;
        return stream_segments<NT / 64, kRateU, true, uint32_t>(
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
        for (int i = tid; i < zw; i += NT) {
          const uint32_t v = lds[i];
          if (!v) continue;
#pragma unroll
          for (int hh = 0; hh < 2; ++hh) {
            const int64_t h = hh ? (int64_t)(v >> 16) : (int64_t)(v & 0xffffu);
            const int m = lo + 2 * i + hh;
            if (h && (h > best_h || (h == best_h && m > best_m)) && sn + size[m] <= omega) {
              best_h = h;
              best_m = m;
            }
          }
        }
        __syncthreads();
        continue;
      }
      for (int i = tid; i < span; i += NT) {
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
        if ((int64_t)h > best_h || ((int64_t)h == best_h && m > best_m)) {
          const int64_t un = (int64_t)din + indeg[m] - (int64_t)c;
          if (sn + size[m] <= omega && un <= delta) {
            best_h = (int64_t)h;
            best_m = m;
          }
        }
      }
      __syncthreads();
    }
  }
  add_wave_units(units, streamed);
  // block argmax of (h, m)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t oh = __shfl_xor(best_h, o, 64);
    const int om = __shfl_xor(best_m, o, 64);
    if (oh > best_h || (oh == best_h && om > best_m)) {
      best_h = oh;
      best_m = om;
    }
  }
  if (l == 0) {
    red_h[w] = best_h;
    red_m[w] = best_m;
  }
  __syncthreads();
  if (tid == 0) {
    for (int q = 1; q < NT / 64; ++q)
      if (red_h[q] > best_h || (red_h[q] == best_h && red_m[q] > best_m)) {
        best_h = red_h[q];
        best_m = red_m[q];
      }
    pair[n] = best_m;
    score[n] = best_m < 0 ? 0 : best_h;
  }
}

// ---------------------------------------------------------------------------
// matching over the pairing pseudo-forest (Sec. III-A/B)
// ---------------------------------------------------------------------------
// best(p) as a packed (score << 32 | id) maximum over the nodes proposing p.
__global__ void k_best(const int32_t *__restrict__ pair, const int64_t *__restrict__ score, int32_t N,
                       unsigned long long *__restrict__ best) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int32_t p = pair[n];
  if (p >= 0) atomicMax(&best[p], ((unsigned long long)score[n] << 32) | (unsigned long long)n);
}

// up(n): true on a 2-cycle, false without candidate or when n is not the
// best proposer of pair(n), else the negation of up(pair(n)).  Each thread
// follows the chain of "best proposer" links to a node whose value is
// local; scores never decrease along the chain, so it ends (the walk is
// capped at N steps; hitting the cap flags an internal error).
__global__ void k_up(const int32_t *__restrict__ pair, const unsigned long long *__restrict__ best, int32_t N,
                     uint8_t *__restrict__ up, int32_t *err) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  int u = (int)n;
  uint32_t parity = 0;
  int r = -1;
  for (int64_t step = 0; step <= N; ++step) {
    const int p = pair[u];
    if (p < 0) {
      r = 0;
      break;
    }
    if (pair[p] == u) {
      r = 1;
      break;
    }
    if ((int)(best[p] & 0xffffffffull) != u) {
      r = 0;
      break;
    }
    parity ^= 1u;
    u = p;
  }
  if (r < 0) {
    atomicOr(err, kErrInternal);
    r = 0;
  }
  up[n] = (uint8_t)((uint32_t)r ^ parity);
}

// ---------------------------------------------------------------------------
// exact matching: the tree recursion over the pairing pseudo-forest
// ---------------------------------------------------------------------------
// Components hang from 2-cycles or from nodes without candidate; a node's
// children are its proposers other than its 2-cycle partner.  With f(v) the
// best matching weight in v's subtree and g(v) that with v left free:
//   g(v) = sum of f(c) over the children,
//   d(v) = max over the children of g(c) + score(c) - f(c) (by value, id),
//   f(v) = g(v) + max(0, d(v)), and v takes c*(v) when d(v) >= 0;
// a 2-cycle {a, b} is matched iff g(a) + g(b) + score(a) >= f(a) + f(b).
// Bottom-up without waiting: a thread starts at every leaf; at each node it
// adds f to the parent's g, offers (d-candidate, id) to the parent's packed
// maximum, and the last child to arrive (counter) carries on with the parent,
// whose sums are then complete.  Scores lie in [0, 2^31), so every
// d-candidate lies in (-2^31, 2^31) and packs as (value + 2^31) << 32 | id.
__global__ void k_dp_children(const int32_t *__restrict__ pair, const int64_t *__restrict__ score, int32_t N,
                              int32_t *__restrict__ nchild, int32_t *err) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int32_t p = pair[n];
  if (p < 0) return;
  const int64_t sc = score[n];
  if (sc < 0 || sc > 2147483647LL) atomicOr(err, kErrWeight);
  if (pair[p] != (int32_t)n) atomicAdd(&nchild[p], 1);
}

__global__ void k_dp_climb(const int32_t *__restrict__ pair, const int64_t *__restrict__ score, int32_t N,
                           const int32_t *__restrict__ nchild, int32_t *__restrict__ arrived,
                           unsigned long long *__restrict__ gsum, unsigned long long *__restrict__ dkey,
                           int64_t *__restrict__ f, int32_t *err) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N || nchild[n] != 0) return;
  int v = (int)n;
  for (int64_t step = 0; step <= N; ++step) {
    // every child of v has arrived: its sums are final (read at device scope)
    const int64_t gv = (int64_t)atomicAdd(&gsum[v], 0ull);
    const unsigned long long dk = atomicAdd(&dkey[v], 0ull);
    const int64_t d = dk ? (int64_t)(dk >> 32) - (int64_t(1) << 31) : 0;
    const int64_t fv = gv + (d > 0 ? d : 0);
    f[v] = fv;
    const int32_t p = pair[v];
    if (p < 0 || pair[p] == v) return;
    atomicAdd(&gsum[p], (unsigned long long)fv);
    const int64_t val = gv + score[v] - fv;
    atomicMax(&dkey[p], ((unsigned long long)(val + (int64_t(1) << 31)) << 32) | (unsigned long long)(uint32_t)v);
    __threadfence();
    if (atomicAdd(&arrived[p], 1) + 1 != nchild[p]) return;
    __threadfence();
    v = p;
  }
  atomicOr(err, kErrInternal);
}

// best(v) = c*(v) (flag bit 32 set) when d(v) >= 0, else 0; root(v) = 1 on a
// 2-cycle the recursion matches.
__global__ void k_dp_decide(const int32_t *__restrict__ pair, const int64_t *__restrict__ score, int32_t N,
                            const unsigned long long *__restrict__ gsum, const unsigned long long *__restrict__ dkey,
                            const int64_t *__restrict__ f, unsigned long long *__restrict__ best,
                            uint8_t *__restrict__ root) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const unsigned long long dk = dkey[n];
  const int64_t d = dk ? (int64_t)(dk >> 32) - (int64_t(1) << 31) : -1;
  best[n] = (dk && d >= 0) ? ((1ull << 32) | (dk & 0xffffffffull)) : 0ull;
  const int32_t p = pair[n];
  uint8_t r = 0;
  if (p >= 0 && pair[p] == (int32_t)n) {
    const int32_t a = min((int32_t)n, p), b = max((int32_t)n, p);
    r = ((int64_t)gsum[a] + (int64_t)gsum[b] + score[a] >= f[a] + f[b]) ? 1 : 0;
  }
  root[n] = r;
}

// up(n) as in k_up, with best = c* and a 2-cycle matched only when the
// recursion says so.
__global__ void k_up_exact(const int32_t *__restrict__ pair, const unsigned long long *__restrict__ best,
                           const uint8_t *__restrict__ root, int32_t N, uint8_t *__restrict__ up, int32_t *err) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  int u = (int)n;
  uint32_t parity = 0;
  int r = -1;
  for (int64_t step = 0; step <= N; ++step) {
    const int p = pair[u];
    if (p < 0) {
      r = 0;
      break;
    }
    if (pair[p] == u) {
      r = root[u];
      break;
    }
    const unsigned long long b = best[p];
    if (!b || (int)(b & 0xffffffffull) != u) {
      r = 0;
      break;
    }
    parity ^= 1u;
    u = p;
  }
  if (r < 0) {
    atomicOr(err, kErrInternal);
    r = 0;
  }
  up[n] = (uint8_t)((uint32_t)r ^ parity);
}

__global__ void k_match(const int32_t *__restrict__ pair, const unsigned long long *__restrict__ best,
                        const uint8_t *__restrict__ up, int32_t N, int32_t *__restrict__ match,
                        int32_t *__restrict__ rep) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  int m = (int)n;
  if (up[n]) {
    m = pair[n];
  } else {
    const unsigned long long b = best[n];
    if (b) {
      const int c = (int)(b & 0xffffffffull);
      if (up[c]) m = c;
    }
  }
  match[n] = m;
  rep[n] = (m >= n) ? 1 : 0;
}

__global__ void k_gamma(const int32_t *__restrict__ match, int32_t N, int32_t *__restrict__ gamma) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int m = match[n];
  if (m < n) gamma[n] = gamma[m];
}

// The whole matching of a small level in one workgroup (the coarse levels
// that merge a few pairs each): the phases of k_best, k_up, k_match, the
// scan of the representative flags and k_gamma, separated by barriers
// instead of launches, with the same results.  *n_next = the number of
// clusters.
constexpr int MATCH_SMALL_NT = 1024;
constexpr int kMatchSmallMax = 8192;

__global__ __launch_bounds__(MATCH_SMALL_NT) void k_match_small(const int32_t *__restrict__ pair,
                                                                const int64_t *__restrict__ score, int32_t N,
                                                                unsigned long long *best, uint8_t *up, int32_t *match,
                                                                int32_t *rep, int32_t *gamma, int32_t *n_next,
                                                                int32_t *err) {
  __shared__ int32_t tmp[MATCH_SMALL_NT / 64 + 1];
  const int tid = threadIdx.x;
  for (int n = tid; n < N; n += MATCH_SMALL_NT) best[n] = 0ull;
  __syncthreads();
  for (int n = tid; n < N; n += MATCH_SMALL_NT) {
    const int32_t p = pair[n];
    if (p >= 0) atomicMax(&best[p], ((unsigned long long)score[n] << 32) | (unsigned long long)n);
  }
  __syncthreads();
  for (int n = tid; n < N; n += MATCH_SMALL_NT) {
    int u = n;
    uint32_t parity = 0;
    int r = -1;
    for (int64_t step = 0; step <= N; ++step) {
      const int p = pair[u];
      if (p < 0) {
        r = 0;
        break;
      }
      if (pair[p] == u) {
        r = 1;
        break;
      }
      if ((int)(best[p] & 0xffffffffull) != u) {
        r = 0;
        break;
      }
      parity ^= 1u;
      u = p;
    }
    if (r < 0) {
      atomicOr(err, kErrInternal);
      r = 0;
    }
    up[n] = (uint8_t)((uint32_t)r ^ parity);
  }
  __syncthreads();
  for (int n = tid; n < N; n += MATCH_SMALL_NT) {
    int m = n;
    if (up[n]) {
      m = pair[n];
    } else {
      const unsigned long long b = best[n];
      if (b) {
        const int c = (int)(b & 0xffffffffull);
        if (up[c]) m = c;
      }
    }
    match[n] = m;
    rep[n] = (m >= n) ? 1 : 0;
    gamma[n] = rep[n];
  }
  __syncthreads();
  const int32_t total = block_exclusive_scan<int32_t, MATCH_SMALL_NT>(gamma, N, tmp);
  // representatives hold their rank now; the others take their partner's
  for (int n = tid; n < N; n += MATCH_SMALL_NT) {
    const int m = match[n];
    if (m < n) gamma[n] = gamma[m];
  }
  if (tid == 0) *n_next = total;
}

// ---------------------------------------------------------------------------
// contraction (Sec. III-B)
// ---------------------------------------------------------------------------
__global__ void k_cluster_size(const int32_t *__restrict__ match, const int32_t *__restrict__ gamma,
                               const int32_t *__restrict__ size, int32_t N, int32_t *__restrict__ csize) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int m = match[n];
  if (m >= n) csize[gamma[n]] = size[n] + (m != n ? size[m] : 0);
}

// One workgroup per hedge: map pins through `map`, sort (id << 1 | dst),
// keep the last key of every id run (its low bit is the OR of the run's
// destination flags), write the survivors at the hedge's old offset.
__device__ __forceinline__ void contract_block(int e, const int32_t *__restrict__ hoff,
                                               const uint32_t *__restrict__ hpin, const int32_t *__restrict__ map,
                                               uint32_t *__restrict__ out, int32_t *__restrict__ cnt, uint32_t *key,
                                               int32_t *pos, int32_t *tmp) {
  const int b = hoff[e];
  const int len = hoff[e + 1] - b;
  if (len <= 0) {
    if (threadIdx.x == 0) cnt[e] = 0;
    return;
  }
  const int np = next_pow2(len);
  for (int i = threadIdx.x; i < np; i += SEG_NT) {
    uint32_t k = 0xffffffffu;
    if (i < len) {
      const uint32_t x = hpin[b + i];
      k = ((uint32_t)map[x & kIdMask] << 1) | (x >> 31);
    }
    key[i] = k;
  }
  __syncthreads();
  block_bitonic_sort<uint32_t, SEG_NT>(key, np);
  for (int i = threadIdx.x; i < len; i += SEG_NT)
    pos[i] = (i + 1 == len || (key[i + 1] >> 1) != (key[i] >> 1)) ? 1 : 0;
  __syncthreads();
  const int kept = block_exclusive_scan<int32_t, SEG_NT>(pos, len, tmp);
  for (int i = threadIdx.x; i < len; i += SEG_NT) {
    const bool last = (i + 1 == len || (key[i + 1] >> 1) != (key[i] >> 1));
    if (last) {
      const uint32_t k = key[i];
      out[b + pos[i]] = (k >> 1) | ((k & 1u) << 31);
    }
  }
  if (threadIdx.x == 0) cnt[e] = kept;
}

// Workgroup per hedge, grid-stride over list[0 .. count): count from the
// device when list_n is set, else n_fixed.
// Hedges above kSegCap pins use the global scratch (keys at twice the pin
// offset in huge_i, run flags at the pin offset in huge_k).
__global__ __launch_bounds__(SEG_NT) void k_contract(const int32_t *__restrict__ hoff,
                                                     const uint32_t *__restrict__ hpin,
                                                     const int32_t *__restrict__ map, uint32_t *__restrict__ out,
                                                     int32_t *__restrict__ cnt, const int32_t *__restrict__ list,
                                                     const int32_t *__restrict__ list_n, int32_t n_fixed,
                                                     uint64_t *__restrict__ huge_k, int32_t *__restrict__ huge_i,
                                                     int32_t *err) {
  __shared__ uint32_t key[kSegCap];
  __shared__ int32_t pos[kSegCap];
  __shared__ int32_t tmp[SEG_NT / 64 + 1];
  const int count = list_n ? *list_n : n_fixed;
  for (int t = blockIdx.x; t < count; t += gridDim.x) {
    const int e = list[t];
    const int b = hoff[e], len = hoff[e + 1] - b;
    if (len <= kSegCap)
      contract_block(e, hoff, hpin, map, out, cnt, key, pos, tmp);
    else if (huge_k && len <= kHugeCap)
      contract_block(e, hoff, hpin, map, out, cnt, reinterpret_cast<uint32_t *>(huge_i) + 2 * (int64_t)b,
                     reinterpret_cast<int32_t *>(huge_k) + b, tmp);
    else if (threadIdx.x == 0)
      atomicOr(err, kErrInternal);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
void launch_check_offsets(const int32_t *off, int32_t E, int32_t *err, hipStream_t s) {
  k_check_offsets<<<div_up((int64_t)E + 1, 256), 256, 0, s>>>(off, E, err);
  HGP_LAUNCH_CHECK();
}

void launch_check_weights(const int32_t *hw, int32_t E, const int32_t *nw, int32_t N, int32_t *err,
                          unsigned long long *sums, hipStream_t s) {
  const int64_t m = E > N ? E : N;
  if (m <= 0) return;
  k_check_weights<<<div_up(m, 256), 256, 0, s>>>(hw, E, nw, N, err, sums);
  HGP_LAUNCH_CHECK();
}

void launch_canon(const int32_t *off, const int32_t *pins, const int32_t *nsrc, int32_t E, int32_t N, int32_t role, int32_t *err,
                  uint32_t *hpin, uint32_t *huge_keys, hipStream_t s) {
  if (E <= 0) return;
  k_canon<<<E, SEG_NT, 0, s>>>(off, pins, nsrc, N, role, err, hpin, huge_keys);
  HGP_LAUNCH_CHECK();
}

static int bits_of(int64_t x) {
  int b = 0;
  while (b < 62 && (int64_t(1) << b) <= x) ++b;
  return b;
}

// |in(n)| and total(n) = sum of w(e) over I(n) from the node-sorted
// incidences (node[i] = node of incidence i): one lane per incidence, a
// segmented sum over each workgroup's runs of equal nodes (within waves by
// shuffles, across the workgroup's waves through LDS) and one atomic add per
// run and workgroup, so a coarse cluster with a hundred thousand incidences
// costs about a hundred atomics (a wave per node left it on one wave, a
// wave-level sum still made it take one atomic per wave on one address).
// indeg and total are zeroed by the caller.
constexpr int NS_NT = 1024;
__global__ __launch_bounds__(NS_NT) void k_node_stats_seg(const uint32_t *__restrict__ node,
                                                          const uint32_t *__restrict__ inc,
                                                          const int32_t *__restrict__ hw, int64_t P,
                                                          int32_t *__restrict__ indeg, int32_t *__restrict__ total) {
  constexpr int NW = NS_NT / 64;
  __shared__ int64_t head_v[NW], tail_v[NW];
  __shared__ int32_t tail_s[NW], tail_d[NW], carry_s[NW], carry_d[NW];
  const int64_t i = (int64_t)blockIdx.x * NS_NT + threadIdx.x;
  const int l = lane_id(), w = (int)(threadIdx.x >> 6);
  const bool in = i < P;
  const uint32_t x = in ? inc[i] : 0u;
  const int64_t v = in ? (int64_t)node[i] : -1 - (int64_t)threadIdx.x;  // past P: runs of their own
  int32_t s = in ? hw[x & kIdMask] : 0;
  int32_t d = (int32_t)(x >> 31);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t s2 = __shfl_up(s, o, 64), d2 = __shfl_up(d, o, 64);
    const int64_t v2 = __shfl_up(v, o, 64);
    if (l >= o && v2 == v) {
      s += s2;
      d += d2;
    }
  }
  if (l == 0) head_v[w] = v;
  if (l == 63) {
    tail_v[w] = v;
    tail_s[w] = s;
    tail_d[w] = d;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // carry[q]: the part of wave q's first run held by earlier waves (the
    // nodes are sorted, so a run continues across waves only through whole
    // waves of one node)
    int32_t cs = 0, cd = 0;
    carry_s[0] = 0;
    carry_d[0] = 0;
    for (int q = 1; q < NW; ++q) {
      if (tail_v[q - 1] == head_v[q]) {
        const bool whole = head_v[q - 1] == tail_v[q - 1];
        cs = tail_s[q - 1] + (whole ? cs : 0);
        cd = tail_d[q - 1] + (whole ? cd : 0);
      } else {
        cs = 0;
        cd = 0;
      }
      carry_s[q] = cs;
      carry_d[q] = cd;
    }
  }
  __syncthreads();
  if (v == head_v[w]) {
    s += carry_s[w];
    d += carry_d[w];
  }
  // the last lane of each run within the workgroup adds the run's sums (the
  // shuffle runs on every lane: a lane masked off would leave its
  // neighbour's read undefined)
  const int64_t dn = __shfl_down(v, 1, 64);
  const int64_t vn = l < 63 ? dn : (w + 1 < NW ? head_v[w + 1] : -1 - (int64_t)NS_NT);
  if (in && vn != v) {
    atomicAdd(&total[v], s);
    if (d) atomicAdd(&indeg[v], d);
  }
}

void build_incidence(const int32_t *hoff, const uint32_t *hpin, int32_t E, int32_t N, int64_t P, const int32_t *hw,
                     int32_t *ioff, uint32_t *inc, uint32_t *perm, int32_t *indeg, int32_t *total, uint32_t *tkey,
                     uint32_t *tkey2, uint64_t *tval, uint64_t *tval2, DevBuf &sort_tmp, hipStream_t s) {
  KScope ks(5, s);
  if (E > 0 && P > 0) {
    // lanes take whole hedges when they are short on average (coarse levels)
    if (P <= (int64_t)kThreadSegMax * E)
      k_expand_lanes<<<div_up(E, 256), 256, 0, s>>>(hoff, hpin, E, tkey, tval);
    else
      k_expand<<<div_up((int64_t)E * 64, 256), 256, 0, s>>>(hoff, hpin, E, tkey, tval);
    HGP_LAUNCH_CHECK();
    radix_sort_u32_split(tkey, tkey2, tval, tval2, P, bits_of(N > 0 ? N - 1 : 0), inc, perm, sort_tmp, s);
  }
  k_offsets_from_sorted<<<div_up(P + 1, 256), 256, 0, s>>>(tkey, P, N, ioff);
  HGP_LAUNCH_CHECK();
  if (N > 0) {
    fill_i32(indeg, N, 0, s);
    fill_i32(total, N, 0, s);
    if (P > 0) {
      // tkey holds the sorted node of every incidence
      k_node_stats_seg<<<div_up(P, NS_NT), NS_NT, 0, s>>>(tkey, inc, hw, P, indeg, total);
      HGP_LAUNCH_CHECK();
    }
  }
}

void launch_feasible(const int32_t *size, const int32_t *indeg, int32_t N, int32_t omega, int32_t delta,
                     int32_t *err, hipStream_t s) {
  if (N <= 0) return;
  k_feasible<<<div_up(N, 256), 256, 0, s>>>(size, indeg, N, omega, delta, err);
  HGP_LAUNCH_CHECK();
}

constexpr int RATE_NT = 512;
constexpr int RATE_LDS_BYTES = 128 * 1024;

// max over the nodes of |in(n)| into *out (zeroed by the caller)
__global__ __launch_bounds__(256) void k_max_i32(const int32_t *__restrict__ a, int32_t n, int32_t *__restrict__ out) {
  __shared__ int32_t red[4];
  int32_t m = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) m = max(m, a[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
  if (lane_id() == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(out, max(max(red[0], red[1]), max(red[2], red[3])));
}

template <int NT>
static void launch_rate_nt(const LevelView &L, const int32_t *total, const int32_t *maxin, int32_t omega,
                           int32_t delta, int32_t *pair, int64_t *score, int words, hipStream_t s) {
  // thread-safe one-time opt-in to the large dynamic LDS size
  static const bool attr_set = [] {
    HGP_HIP(hipFuncSetAttribute((const void *)k_rate<NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                RATE_LDS_BYTES));
    return true;
  }();
  (void)attr_set;
  k_rate<NT><<<xcd_grid(L.n), NT, (size_t)words * 4, s>>>(L.n, L.ioff, L.inc, L.hoff, L.hpin, L.hw, L.size, L.indeg, total,
                                                maxin, omega, delta, words, pair, score, units_ptr(0));
  HGP_LAUNCH_CHECK();
}

void launch_max_i32(const int32_t *a, int32_t n, int32_t *out, hipStream_t s) {
  fill_i32(out, 1, 0, s);
  if (n <= 0) return;
  k_max_i32<<<std::min(div_up(n, 2048), 256), 256, 0, s>>>(a, n, out);
  HGP_LAUNCH_CHECK();
}

void launch_rate(const LevelView &L, const int32_t *total, int32_t omega, int32_t delta, int32_t *pair,
                 int64_t *score, int32_t *maxin, hipStream_t s, int tile) {
  if (L.n <= 0) return;
  // dense window: whole id range if it fits, else RATE_LDS_BYTES of counters
  const int max_words = RATE_LDS_BYTES / 4;
  int words = L.n <= max_words / 2 ? 2 * L.n : max_words;
  words = (words + 1) & ~1;
  KScope ks(0, s);
  fill_i32(maxin, 1, 0, s);
  k_max_i32<<<std::min(div_up(L.n, 2048), 256), 256, 0, s>>>(L.indeg, L.n, maxin);
  HGP_LAUNCH_CHECK();
  if (tile == 256)
    launch_rate_nt<256>(L, total, maxin, omega, delta, pair, score, words, s);
  else if (tile == 1024)
    launch_rate_nt<1024>(L, total, maxin, omega, delta, pair, score, words, s);
  else
    launch_rate_nt<RATE_NT>(L, total, maxin, omega, delta, pair, score, words, s);
}

void launch_match(const int32_t *pair, const int64_t *score, int32_t N, unsigned long long *best, uint8_t *up,
                  int32_t *match, int32_t *gamma, int32_t *rep, int32_t *n_next_dev, int32_t *err,
                  DevBuf &scan_tmp, hipStream_t s) {
  if (N <= 0) return;
  KScope ks(7, s);
  add_units(7, N);
  if (N <= kMatchSmallMax) {
    k_match_small<<<1, MATCH_SMALL_NT, 0, s>>>(pair, score, N, best, up, match, rep, gamma, n_next_dev, err);
    HGP_LAUNCH_CHECK();
    return;
  }
  fill_i64(reinterpret_cast<int64_t *>(best), N, 0, s);
  const int g = div_up(N, 256);
  k_best<<<g, 256, 0, s>>>(pair, score, N, best);
  HGP_LAUNCH_CHECK();
  k_up<<<g, 256, 0, s>>>(pair, best, N, up, err);
  HGP_LAUNCH_CHECK();
  k_match<<<g, 256, 0, s>>>(pair, best, up, N, match, rep);
  HGP_LAUNCH_CHECK();
  scan_i32(rep, gamma, N, n_next_dev, scan_tmp, s);
  k_gamma<<<g, 256, 0, s>>>(match, N, gamma);
  HGP_LAUNCH_CHECK();
}

void launch_match_exact(const int32_t *pair, const int64_t *score, int32_t N, const MatchScratch &m,
                        unsigned long long *best, uint8_t *up, int32_t *match, int32_t *gamma, int32_t *rep,
                        int32_t *n_next_dev, int32_t *err, DevBuf &scan_tmp, hipStream_t s) {
  if (N <= 0) return;
  KScope ks(7, s);
  add_units(7, N);
  fill_i32(m.nchild, N, 0, s);
  fill_i32(m.arrived, N, 0, s);
  fill_i64(reinterpret_cast<int64_t *>(m.gsum), N, 0, s);
  fill_i64(reinterpret_cast<int64_t *>(m.dkey), N, 0, s);
  const int g = div_up(N, 256);
  k_dp_children<<<g, 256, 0, s>>>(pair, score, N, m.nchild, err);
  HGP_LAUNCH_CHECK();
  k_dp_climb<<<g, 256, 0, s>>>(pair, score, N, m.nchild, m.arrived, m.gsum, m.dkey, m.f, err);
  HGP_LAUNCH_CHECK();
  k_dp_decide<<<g, 256, 0, s>>>(pair, score, N, m.gsum, m.dkey, m.f, best, m.root);
  HGP_LAUNCH_CHECK();
  k_up_exact<<<g, 256, 0, s>>>(pair, best, m.root, N, up, err);
  HGP_LAUNCH_CHECK();
  k_match<<<g, 256, 0, s>>>(pair, best, up, N, match, rep);
  HGP_LAUNCH_CHECK();
  scan_i32(rep, gamma, N, n_next_dev, scan_tmp, s);
  k_gamma<<<g, 256, 0, s>>>(match, N, gamma);
  HGP_LAUNCH_CHECK();
}

void launch_cluster_size(const int32_t *match, const int32_t *gamma, const int32_t *size, int32_t N, int32_t *csize,
                         hipStream_t s) {
  if (N <= 0) return;
  k_cluster_size<<<div_up(N, 256), 256, 0, s>>>(match, gamma, size, N, csize);
  HGP_LAUNCH_CHECK();
}

void launch_contract(const int32_t *hoff, const uint32_t *hpin, int32_t E, const int32_t *map, uint32_t *tmp_pins,
                     int32_t *cnt, int32_t *new_hoff, uint32_t *new_hpin, const BigHedges &big, DevBuf &scan_tmp,
                     int32_t *list_buf, int32_t *err, hipStream_t s) {
  if (E <= 0) {
    fill_i32(new_hoff, 1, 0, s);
    fill_i32(list_buf + 1, 1, 0, s);  // no long hedges (list_buf[E + 1])
    return;
  }
  KScope ks(4, s);
  launch_contract_split(hoff, hpin, E, map, tmp_pins, cnt, list_buf, s);
  int32_t *bl = list_buf + E + 1;
  const int grid = std::min(std::min(big.n, big.bound), 2048);
  if (grid > 0) {
    // this level's hedges above kWaveSegMax (the level-0 list is a superset)
    launch_mid_hedges(hoff, E, bl + 1, bl, s, kWaveSegMax, 0x7fffffff);
    k_contract<<<grid, SEG_NT, 0, s>>>(hoff, hpin, map, tmp_pins, cnt, bl + 1, bl, 0, big.huge_k, big.huge_i, err);
    HGP_LAUNCH_CHECK();
  } else {
    fill_i32(bl, 1, 0, s);  // the count the caller may read back
  }
  scan_i32(cnt, new_hoff, E, new_hoff + E, scan_tmp, s);
  launch_pack_split(hoff, new_hoff, E, tmp_pins, new_hpin, list_buf, s);
}

__global__ void k_check_range(const int32_t *__restrict__ a, int64_t n, int32_t lo, int32_t hi, int32_t *err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (a[i] < lo || a[i] >= hi)) atomicOr(err, kErrPin);
}

void launch_check_range(const int32_t *a, int64_t n, int32_t lo, int32_t hi, int32_t *err, hipStream_t s) {
  if (n <= 0) return;
  k_check_range<<<div_up(n, 256), 256, 0, s>>>(a, n, lo, hi, err);
  HGP_LAUNCH_CHECK();
}

// A canonical level: pin ids in [0, n), strictly ascending within a hedge.
__global__ void k_check_level(const int32_t *__restrict__ hoff, const uint32_t *__restrict__ hpin, int32_t E,
                              int32_t n, int32_t *err) {
  const int wid = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (wid >= E) return;
  const int b = hoff[wid], en = hoff[wid + 1];
  for (int j = b + lane_id(); j < en; j += 64) {
    const int v = (int)(hpin[j] & kIdMask);
    if (v >= n) atomicOr(err, kErrPin);
    if (j > b && (int)(hpin[j - 1] & kIdMask) >= v) atomicOr(err, kErrDup);
  }
}

void launch_check_level(const int32_t *hoff, const uint32_t *hpin, int32_t E, int32_t n, int32_t *err,
                        hipStream_t s) {
  if (E <= 0) return;
  k_check_level<<<div_up((int64_t)E * 64, 256), 256, 0, s>>>(hoff, hpin, E, n, err);
  HGP_LAUNCH_CHECK();
}

}  // namespace hgp
