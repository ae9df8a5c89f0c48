// Incremental coarsening for levels that merge few pairs (Sec. III-A
// selection, exact).
//
// When a level merges only a few pairs, the candidate sets of most nodes are
// unchanged: for nodes n, m that both stay unmerged, hist(n,m), c(n,m), their
// sizes and |in| do not change, hence neither does the validity of m for n.
// Each node therefore keeps the exact top-TK valid candidates of its last
// full rating (key = hist << 32 | id, with c(n,m) beside it) and kappa, the
// key of the best valid candidate left off the list (0 if none was left off).
// Invariant: every valid candidate not in the list has a key <= kappa.  The
// renumbering of a level preserves the order of unmerged nodes (new ids are
// ranks of the clusters' smallest members), so kappa carries over as
// (hist, new id) when its node stays unmerged; when it merged, only its hist
// is kept (id part all ones), a bound that still holds.
//
// At the next level:
//  - every new cluster c' gets a full rating; its histogram row gives
//    hist(n', c') and c(n', c') for every node n' (both are symmetric) and is
//    offered to the unmerged nodes;
//  - an unmerged node drops listed candidates that merged, renames the rest
//    through gamma (order-preserving on unmerged nodes), inserts offers with
//    keys above kappa, and if the list overflows TK the evicted key raises
//    kappa;
//  - the first `need` entries are the exact best valid candidates when the
//    need-th entry's key exceeds kappa, or when kappa is 0 (nothing hidden);
//    otherwise the node gets a full rating again.  The plain selection needs
//    the head only (need 1); the learned proposal needs its k best.
//
// Ratings use a dense LDS window over the node's neighbour id range; a range
// wider than the window is covered by several windows, each streaming only
// the pins inside it (binary search per hedge).
#include <algorithm>
#include <cstdlib>

#include "../../include/hgp.h"
#include "coarsen.hpp"
#include "tail.hpp"

namespace hgp {

__device__ __forceinline__ uint64_t cand_key(uint64_t h, uint32_t m) { return (h << 32) | (uint64_t)m; }

// Inserts (x, xc) into the descending list (k, kc) of length L; the entry
// pushed off the end is returned in x (0 if the list had room).
template <int L>
__device__ __forceinline__ void list_insert(uint64_t (&k)[L], int32_t (&kc)[L], uint64_t &x, int32_t &xc) {
#pragma unroll
  for (int z = 0; z < L; ++z) {
    if (x > k[z]) {
      const uint64_t t = k[z];
      const int32_t tc = kc[z];
      k[z] = x;
      kc[z] = xc;
      x = t;
      xc = tc;
    }
  }
}

// One pin of a rated node's hedge added to its window counter rel (layout
// MODE: 0 = hist in 16-bit halves, 1 = hist | c << hb in 32 bits, 2 = hist |
// c << 32 in 64 bits), weight we and co-destination bit both.  Every pin a
// rating streams lies in its window (the window spans the node's neighbour
// id range, or the segments were clipped to it), so no range test is needed;
// masked lanes add zero.  The node's own pin is counted too and its counter
// cleared afterwards (window_clear_self): its count, total(n) | indeg(n) <<
// hb, fits the layout by the same bounds as every other counter.
template <int MODE>
__device__ __forceinline__ void window_add(uint32_t *lds, uint64_t *lds64, uint32_t rel, uint32_t we, uint32_t both,
                                           int hb) {
  if constexpr (MODE == 0)
    atomicAdd(&lds[rel >> 1], we << ((rel & 1u) << 4));
  else if constexpr (MODE == 1)
    atomicAdd(&lds[rel], we + (both << hb));
  else
    atomicAdd((unsigned long long *)&lds64[rel], (unsigned long long)we | ((unsigned long long)both << 32));
}

// Clears the rated node's own counter (relative id rn) in a window of span
// ids after a stream (block-wide; the caller's barrier precedes it, one
// follows it).
__device__ __forceinline__ void window_clear_self(uint32_t *lds, uint64_t *lds64, int mode, int rn, int span) {
  if (threadIdx.x == 0 && (uint32_t)rn < (uint32_t)span) {
    if (mode == 0)
      lds[rn >> 1] &= ~(0xffffu << ((rn & 1) << 4));
    else if (mode == 1)
      lds[rn] = 0u;
    else
      lds64[rn] = 0ull;
  }
  __syncthreads();
}

// Groups of nodes with the same inbound hedges (the nodes of one position
// across the channels of a layered network) share the part of their
// histograms that those hedges give: hist(n, m) is the sum over n's inbound
// hedges plus the sum over its other (outbound) hedges, and c(n, m) counts
// inbound hedges only.  A workgroup rating such a group streams the inbound
// hedges once per window into a scratch slot of its own, and every member
// then reloads the window and adds only its outbound hedges.
constexpr int kGroupCap = 64;   // members per group at most
constexpr int kGroupWins = 4;   // windows of a shared histogram at most

// Block-wide set-up of group list[m0 .. m1): whether every member has the
// leader's inbound hedges (checked exactly: equal |in|, and each inbound hedge
// of a member found as an inbound hedge in the leader's incidence, which is
// sorted by hedge id), the union of the members' neighbour ranges, and the
// largest total(n).  The result is uniform across the block.
template <int NT>
__device__ bool group_setup(const int32_t *__restrict__ list, int64_t m0, int64_t m1,
                            const int32_t *__restrict__ ioff, const uint32_t *__restrict__ inc,
                            const int32_t *__restrict__ hoff, const uint32_t *__restrict__ hpin,
                            const int32_t *__restrict__ indeg, const int32_t *__restrict__ total, int2 *rng_s,
                            int *bad, int2 &range, uint32_t &max_total) {
  const int tid = threadIdx.x;
  const int leader = list[m0];
  const int li0 = ioff[leader], li1 = ioff[leader + 1];
  const int32_t ldin = indeg[leader];
  if (tid == 0) *bad = 0;
  __syncthreads();
  int lo = 0x7fffffff, hi = -1;
  uint32_t mt = 0;
  for (int64_t t = m0; t < m1; ++t) {
    const int v = list[t];
    mt = max(mt, (uint32_t)total[v]);
    if (t > m0) {
      if (tid == 0 && indeg[v] != ldin) *bad = 1;
      for (int i = ioff[v] + tid; i < ioff[v + 1]; i += NT) {
        const uint32_t x = inc[i];
        if (!(x & kDst)) continue;
        const uint32_t e = x & kIdMask;
        int a = li0, z = li1;
        while (a < z) {
          const int mid = (a + z) >> 1;
          if ((inc[mid] & kIdMask) < e) a = mid + 1;
          else z = mid;
        }
        if (a == li1 || (inc[a] & kIdMask) != e || !(inc[a] & kDst)) *bad = 1;
      }
    }
    const int2 r = neighbour_range<NT>(ioff[v], ioff[v + 1], inc, hoff, hpin, rng_s);
    lo = min(lo, r.x);
    hi = max(hi, r.y);
  }
  __syncthreads();
  range = make_int2(lo, hi);
  max_total = mt;
  return *bad == 0;
}

// Full rating with top-(TK+1) selection of the nodes in list[0 .. *count)
// (or of every node when list is null).  With pre non-null, node t's counters
// are row t of pre (N 64-bit counters hist | c << 32, from k_tail_hist)
// instead of a stream of its pins; nodes with a row slot then also write
// their validated counters to rows[slot * N + m] (rows may alias pre: slot t
// is row t).  words: LDS words of the window.
template <int NT>
__global__ __launch_bounds__(NT) void k_rate_topk(int32_t N, const int32_t *__restrict__ list,
                                                  const int64_t *__restrict__ count, const int32_t *__restrict__ ioff,
                                                  const uint32_t *__restrict__ inc, const int32_t *__restrict__ hoff,
                                                  const uint32_t *__restrict__ hpin, const int32_t *__restrict__ hw,
                                                  const int32_t *__restrict__ size, const int32_t *__restrict__ indeg,
                                                  const int32_t *__restrict__ total, const int32_t *__restrict__ maxin,
                                                  int32_t omega, int32_t delta,
                                                  const int32_t *__restrict__ row_slot, uint64_t *rows,
                                                  int32_t *__restrict__ pair, int64_t *__restrict__ score,
                                                  uint64_t *__restrict__ tk_key, int32_t *__restrict__ tk_c,
                                                  int32_t *__restrict__ tk_cnt, uint64_t *__restrict__ tk_kappa,
                                                  int32_t words, const uint64_t *pre,
                                                  unsigned long long *__restrict__ units) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ int32_t tbl[NT / 64 * 192];
  __shared__ int2 rng_s[NT / 64];
  __shared__ uint64_t red[NT / 64];
  __shared__ uint64_t found[kTopK + 1];
  __shared__ int32_t foundc[kTopK + 1];
  const int tid = threadIdx.x, w = tid >> 6, l = lane_id();
  uint64_t *lds64 = reinterpret_cast<uint64_t *>(lds);
  const int64_t cnt_nodes = list ? *count : (int64_t)N;
  int64_t streamed = 0;
  for (int64_t t = blockIdx.x; t < cnt_nodes; t += gridDim.x) {
    const int n = list ? list[t] : (int)t;
    const int64_t sn = size[n];
    const uint32_t tot = (uint32_t)total[n];
    const uint32_t din = (uint32_t)indeg[n];
    const int hb = tot ? 32 - __clz(tot) : 0;
    const int cb = din ? 32 - __clz(din) : 0;
    const bool packed = hb + cb <= 32;
    // hist alone in 16-bit halves when it fits and no candidate can break
    // Delta (then c is not needed to select; it is counted afterwards for
    // the listed candidates only)
    const bool half = !pre && maxin && hb <= 16 && (int64_t)din + (int64_t)(*maxin) <= (int64_t)delta &&
                      inbound_slots(din) <= words;
    const uint64_t hmask = (hb >= 32) ? 0xffffffffull : ((1ull << hb) - 1ull);
    // each thread keeps the TK+1 largest valid keys of its counters, descending
    uint64_t top[kTopK + 1];
    int32_t topc[kTopK + 1];
#pragma unroll
    for (int z = 0; z <= kTopK; ++z) {
      top[z] = 0ull;
      topc[z] = 0;
    }
    auto offer = [&](uint64_t h, uint64_t c, int m) {
      bool ok = false;
      if (h) {
        const int64_t un = (int64_t)din + indeg[m] - (int64_t)c;
        ok = sn + size[m] <= omega && un <= delta;
      }
      if (ok) {
        uint64_t x = cand_key(h, (uint32_t)m);
        int32_t xc = (int32_t)c;
        if (x > top[kTopK]) list_insert<kTopK + 1>(top, topc, x, xc);
      }
      return ok;
    };
    if (pre) {
      const uint64_t *row = pre + t * (int64_t)N;
      const int slot = row_slot ? row_slot[n] : -1;
      for (int i = tid; i < N; i += NT) {
        const uint64_t v = row[i];
        const bool ok = offer(v & 0xffffffffull, v >> 32, i);
        if (slot >= 0) rows[(int64_t)slot * N + i] = ok ? v : 0ull;
      }
    } else if (sn < omega) {
      const int i0 = ioff[n], i1 = ioff[n + 1];
      const int R = half ? 2 * words : (packed ? words : (words >> 1));
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
          return stream_segments<NT / 64, kRateU, true, uint32_t, true>(
              i0, i1, inc, hoff, nullptr, hw, tbl, [&](int j) { return hpin[j]; },
              [&](uint32_t y, uint32_t info, bool ok) {
                window_add<MODE>(lds, lds64, (y & kIdMask) - (uint32_t)lo, ok ? info & kIdMask : 0u,
                                 ok ? (info & y) >> 31 : 0u, hb);
              },
              clip, lo, lo + span);
        });
        __syncthreads();
        window_clear_self(lds, lds64, half ? 0 : (packed ? 1 : 2), n - lo, span);
        if (half) {
          // Delta holds for every candidate here, whatever c is
          for (int i = tid; i < zw; i += NT) {
            const uint32_t v = lds[i];
            if (!v) continue;
            offer(v & 0xffffu, 0, lo + 2 * i);
            offer(v >> 16, 0, lo + 2 * i + 1);
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
          offer(h, c, lo + i);
        }
        __syncthreads();
      }
    }
    // merge of the per-thread lists: TK+1 rounds of a block max over the
    // heads; keys are distinct (the id is in the low bits), so exactly one
    // thread owns each winner and drops it from its list
    int nf = 0;
    for (int r = 0; r <= kTopK; ++r) {
      uint64_t best = top[0];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const uint64_t x = __shfl_xor(best, o, 64);
        best = x > best ? x : best;
      }
      if (l == 0) red[w] = best;
      __syncthreads();
      if (tid == 0) {
        uint64_t b = red[0];
        for (int q = 1; q < NT / 64; ++q) b = red[q] > b ? red[q] : b;
        found[r] = b;
      }
      __syncthreads();
      const uint64_t win = found[r];
      if (win == 0) break;
      nf = r + 1;
      if (top[0] == win) {
        foundc[r] = topc[0];
#pragma unroll
        for (int z = 0; z < kTopK; ++z) {
          top[z] = top[z + 1];
          topc[z] = topc[z + 1];
        }
        top[kTopK] = 0ull;
        topc[kTopK] = 0;
      }
    }
    __syncthreads();
    if (half) {
      // c(n, m) of the listed candidates (the window's LDS is free now)
      inbound_common<NT>(n, ioff, inc, lds, inbound_slots(din), found, foundc, nf < kTopK ? nf : kTopK);
      __syncthreads();
    }
    if (tid == 0) {
      const int keep = nf < kTopK ? nf : kTopK;
      for (int q = 0; q < kTopK; ++q) {
        tk_key[(int64_t)n * kTopK + q] = q < keep ? found[q] : 0ull;
        tk_c[(int64_t)n * kTopK + q] = q < keep ? foundc[q] : 0;
      }
      tk_cnt[n] = keep;
      tk_kappa[n] = nf > kTopK ? found[kTopK] : 0ull;
      pair[n] = keep ? (int32_t)(found[0] & 0xffffffffull) : -1;
      score[n] = keep ? (int64_t)(found[0] >> 32) : 0;
    }
    __syncthreads();
  }
  add_wave_units(units, streamed);
}

// k_rate_topk over the groups list[goff[g] .. goff[g+1]) for g < *gcount
// (groups of equal inbound hedge sets, kGroupCap members at most; launched
// with GROUPED = true and pre null): every member's rating is that of
// k_rate_topk.  Members of a checked group share the windows of their
// inbound hedges through the workgroup's slot of gscratch (kGroupWins windows
// of `words` words).  A kernel of its own, so that k_rate_topk keeps its
// registers.
template <int NT, bool GROUPED>
__global__ __launch_bounds__(NT) void k_rate_topk_groups(int32_t N, const int32_t *__restrict__ list,
                                                  const int64_t *__restrict__ count, const int32_t *__restrict__ ioff,
                                                  const uint32_t *__restrict__ inc, const int32_t *__restrict__ hoff,
                                                  const uint32_t *__restrict__ hpin, const int32_t *__restrict__ hw,
                                                  const int32_t *__restrict__ size, const int32_t *__restrict__ indeg,
                                                  const int32_t *__restrict__ total, const int32_t *__restrict__ maxin,
                                                  int32_t omega, int32_t delta,
                                                  const int32_t *__restrict__ row_slot, uint64_t *rows,
                                                  int32_t *__restrict__ pair, int64_t *__restrict__ score,
                                                  uint64_t *__restrict__ tk_key, int32_t *__restrict__ tk_c,
                                                  int32_t *__restrict__ tk_cnt, uint64_t *__restrict__ tk_kappa,
                                                  int32_t words, const uint64_t *pre,
                                                  const int32_t *__restrict__ goff, const int32_t *__restrict__ gcount,
                                                  uint32_t *__restrict__ gscratch,
                                                  unsigned long long *__restrict__ units) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ int32_t tbl[NT / 64 * 192];
  __shared__ int2 rng_s[NT / 64];
  __shared__ int s_bad;
  __shared__ unsigned long long s_basecnt[kGroupWins];  // pin visits of the shared windows
  __shared__ uint64_t red[NT / 64];
  __shared__ uint64_t found[kTopK + 1];
  __shared__ int32_t foundc[kTopK + 1];
  const int tid = threadIdx.x, w = tid >> 6, l = lane_id();
  uint64_t *lds64 = reinterpret_cast<uint64_t *>(lds);
  const int64_t n_items = GROUPED ? (int64_t)*gcount : (list ? *count : (int64_t)N);
  int64_t streamed = 0;
  for (int64_t item = blockIdx.x; item < n_items; item += gridDim.x) {
  const int64_t m0 = GROUPED ? goff[item] : item, m1 = GROUPED ? goff[item + 1] : item + 1;
  bool shared = false;
  int2 grg = make_int2(0x7fffffff, -1);
  uint32_t gtot = 0, gdin = 0;
  if (GROUPED && m1 - m0 > 1) {
    if (tid < kGroupWins) s_basecnt[tid] = 0ull;  // group_setup's barriers publish it
    shared = group_setup<NT>(list, m0, m1, ioff, inc, hoff, hpin, indeg, total, rng_s, &s_bad, grg, gtot);
    gdin = (uint32_t)indeg[list[m0]];
    // the group's layout must hold every member's counters; more windows
    // than the scratch slot holds rate the members one by one
    const int hb = gtot ? 32 - __clz(gtot) : 0, cb = gdin ? 32 - __clz(gdin) : 0;
    const bool half = maxin && hb <= 16 && (int64_t)gdin + (int64_t)(*maxin) <= (int64_t)delta &&
                      inbound_slots(gdin) <= words;
    const int R = half ? 2 * words : (hb + cb <= 32 ? words : (words >> 1));
    if (grg.y >= grg.x && ((int64_t)grg.y - grg.x) / R + 1 > kGroupWins) shared = false;
  }
  bool have_base = false;  // the shared windows are in the scratch slot
  for (int64_t t = m0; t < m1; ++t) {
    const int n = list ? list[t] : (int)t;
    const int64_t sn = size[n];
    const uint32_t tot = shared ? gtot : (uint32_t)total[n];
    const uint32_t din = shared ? gdin : (uint32_t)indeg[n];
    const int hb = tot ? 32 - __clz(tot) : 0;
    const int cb = din ? 32 - __clz(din) : 0;
    const bool packed = hb + cb <= 32;
    // hist alone in 16-bit halves when it fits and no candidate can break
    // Delta (then c is not needed to select; it is counted afterwards for
    // the listed candidates only)
    const bool half = !pre && maxin && hb <= 16 && (int64_t)din + (int64_t)(*maxin) <= (int64_t)delta &&
                      inbound_slots(din) <= words;
    const uint64_t hmask = (hb >= 32) ? 0xffffffffull : ((1ull << hb) - 1ull);
    // each thread keeps the TK+1 largest valid keys of its counters, descending
    uint64_t top[kTopK + 1];
    int32_t topc[kTopK + 1];
#pragma unroll
    for (int z = 0; z <= kTopK; ++z) {
      top[z] = 0ull;
      topc[z] = 0;
    }
    auto offer = [&](uint64_t h, uint64_t c, int m) {
      bool ok = false;
      if (h) {
        const int64_t un = (int64_t)din + indeg[m] - (int64_t)c;
        ok = sn + size[m] <= omega && un <= delta;
      }
      if (ok) {
        uint64_t x = cand_key(h, (uint32_t)m);
        int32_t xc = (int32_t)c;
        if (x > top[kTopK]) list_insert<kTopK + 1>(top, topc, x, xc);
      }
      return ok;
    };
    if (pre) {
      const uint64_t *row = pre + t * (int64_t)N;
      const int slot = row_slot ? row_slot[n] : -1;
      for (int i = tid; i < N; i += NT) {
        const uint64_t v = row[i];
        const bool ok = offer(v & 0xffffffffull, v >> 32, i);
        if (slot >= 0) rows[(int64_t)slot * N + i] = ok ? v : 0ull;
      }
    } else if (sn < omega) {
      const int i0 = ioff[n], i1 = ioff[n + 1];
      const int R = half ? 2 * words : (packed ? words : (words >> 1));
      const int2 rg = shared ? grg : neighbour_range<NT>(i0, i1, inc, hoff, hpin, rng_s);
      const uint32_t *clip = ((int64_t)rg.y - rg.x >= R) ? hpin : nullptr;  // several windows
      int wi = 0;
      for (int lo = rg.x; lo <= rg.y; lo += R, ++wi) {
        const int span = min(R, rg.y + 1 - lo);
        const int zw = half ? (span + 1) >> 1 : (packed ? span : 2 * span);
        uint32_t *slot = shared ? gscratch + ((int64_t)blockIdx.x * kGroupWins + wi) * words : nullptr;
        if (GROUPED && have_base) {
          for (int i = tid; i < zw; i += NT) lds[i] = slot[i];
          // the method's pin visits for this member include the shared ones
          if (w == 0) streamed += (int64_t)s_basecnt[wi];
        } else {
          for (int i = tid; i < zw; i += NT) lds[i] = 0u;
        }
        __syncthreads();
        // counter layout: 0 = hist in 16-bit halves, 1 = packed 32-bit, 2 = 64-bit
        streamed += with_mode(half ? 0 : (packed ? 1 : 2), [&](auto mode) {
          constexpr int MODE = decltype(mode)::value;
          auto add = [&](uint32_t y, uint32_t info, bool ok) {
            window_add<MODE>(lds, lds64, (y & kIdMask) - (uint32_t)lo, ok ? info & kIdMask : 0u,
                             ok ? (info & y) >> 31 : 0u, hb);
          };
          auto ld = [&](int j) { return hpin[j]; };
          if (!GROUPED || !shared)
            return stream_segments<NT / 64, kRateU, true, uint32_t, true>(i0, i1, inc, hoff, nullptr, hw, tbl, ld,
                                                                           add, clip, lo, lo + span);
          int64_t s = 0;
          if (!have_base) {
            // the group's inbound hedges (this member's equal the leader's),
            // kept in the slot for the other members
            s = stream_segments<NT / 64, kRateU, true, uint32_t, true, 1>(i0, i1, inc, hoff, nullptr, hw, tbl, ld,
                                                                           add, clip, lo, lo + span);
            if (l == 0 && s) atomicAdd(&s_basecnt[wi], (unsigned long long)s);
            __syncthreads();
            for (int i = tid; i < zw; i += NT) slot[i] = lds[i];
            __syncthreads();
          }
          return s + stream_segments<NT / 64, kRateU, true, uint32_t, true, 2>(i0, i1, inc, hoff, nullptr, hw, tbl,
                                                                                ld, add, clip, lo, lo + span);
        });
        __syncthreads();
        window_clear_self(lds, lds64, half ? 0 : (packed ? 1 : 2), n - lo, span);
        if (half) {
          // Delta holds for every candidate here, whatever c is
          for (int i = tid; i < zw; i += NT) {
            const uint32_t v = lds[i];
            if (!v) continue;
            offer(v & 0xffffu, 0, lo + 2 * i);
            offer(v >> 16, 0, lo + 2 * i + 1);
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
          offer(h, c, lo + i);
        }
        __syncthreads();
      }
      if (GROUPED && shared) have_base = true;
    }
    // merge of the per-thread lists: TK+1 rounds of a block max over the
    // heads; keys are distinct (the id is in the low bits), so exactly one
    // thread owns each winner and drops it from its list
    int nf = 0;
    for (int r = 0; r <= kTopK; ++r) {
      uint64_t best = top[0];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const uint64_t x = __shfl_xor(best, o, 64);
        best = x > best ? x : best;
      }
      if (l == 0) red[w] = best;
      __syncthreads();
      if (tid == 0) {
        uint64_t b = red[0];
        for (int q = 1; q < NT / 64; ++q) b = red[q] > b ? red[q] : b;
        found[r] = b;
      }
      __syncthreads();
      const uint64_t win = found[r];
      if (win == 0) break;
      nf = r + 1;
      if (top[0] == win) {
        foundc[r] = topc[0];
#pragma unroll
        for (int z = 0; z < kTopK; ++z) {
          top[z] = top[z + 1];
          topc[z] = topc[z + 1];
        }
        top[kTopK] = 0ull;
        topc[kTopK] = 0;
      }
    }
    __syncthreads();
    if (half) {
      // c(n, m) of the listed candidates (the window's LDS is free now)
      inbound_common<NT>(n, ioff, inc, lds, inbound_slots(din), found, foundc, nf < kTopK ? nf : kTopK);
      __syncthreads();
    }
    if (tid == 0) {
      const int keep = nf < kTopK ? nf : kTopK;
      for (int q = 0; q < kTopK; ++q) {
        tk_key[(int64_t)n * kTopK + q] = q < keep ? found[q] : 0ull;
        tk_c[(int64_t)n * kTopK + q] = q < keep ? foundc[q] : 0;
      }
      tk_cnt[n] = keep;
      tk_kappa[n] = nf > kTopK ? found[kTopK] : 0ull;
      pair[n] = keep ? (int32_t)(found[0] & 0xffffffffull) : -1;
      score[n] = keep ? (int64_t)(found[0] >> 32) : 0;
    }
    __syncthreads();
  }
  }
  add_wave_units(units, streamed);
}

// Carry the lists of unmerged level-l nodes to level l+1 and offer the new
// clusters (one thread per level-l node).  rows[j * n_coarse + m] = hist |
// c << 32 of new cluster j and node m (0 if not a valid pair).  Nodes whose
// first `need` entries are not certain get rflag = 1 (rflag zeroed by the
// caller), from which the caller builds their list in id order.
// list[pos[i]] = i for the flagged i, given pos = the exclusive scan of the
// 0/1 flags and *total their sum; *count = *total.
__global__ void k_list_from_scan(const int32_t *__restrict__ pos, int32_t n, const int32_t *__restrict__ total,
                                 int32_t *__restrict__ list, int64_t *__restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t p = pos[i], q = i + 1 < n ? pos[i + 1] : *total;
  if (q > p) list[p] = (int32_t)i;
  if (i == 0) *count = *total;
}

// Nodes below a merged bound node searched for a representative.
constexpr int kBoundScan = 64;

__global__ void k_rate_update(int32_t n_fine, const int32_t *__restrict__ match, const int32_t *__restrict__ gamma,
                              const uint64_t *__restrict__ old_key, const int32_t *__restrict__ old_c,
                              const int32_t *__restrict__ old_cnt, const uint64_t *__restrict__ old_kappa,
                              int32_t n_new, const int32_t *__restrict__ newc, const uint64_t *__restrict__ rows,
                              int32_t n_coarse, const int32_t *__restrict__ csize,
                              const int32_t *__restrict__ cindeg, int32_t omega, int32_t delta, int32_t need,
                              uint64_t *__restrict__ tk_key,
                              int32_t *__restrict__ tk_c, int32_t *__restrict__ tk_cnt,
                              uint64_t *__restrict__ tk_kappa, int32_t *__restrict__ pair,
                              int64_t *__restrict__ score, int32_t *__restrict__ rflag,
                              int64_t *__restrict__ why) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= n_fine || match[n] != n) return;
  const int nc = gamma[n];
  uint64_t a[kTopK];
  int32_t ac[kTopK];
#pragma unroll
  for (int q = 0; q < kTopK; ++q) {
    a[q] = 0ull;
    ac[q] = 0;
  }
  // key bound of the candidates left off the list, in the new numbering
  // (an id part of all ones marks a hist-only bound: it stays as it is).
  // The hidden candidates that stay unmerged keep their keys; those with the
  // bound's hist h have old ids below the bound's node m9.  If m9 stays
  // unmerged its new id bounds theirs.  If it merged, every unmerged node
  // below m9 is a representative at most r, the largest representative
  // below m9, so new ids are at most gamma(r): (h, gamma(r)) still bounds
  // every hidden key, and (h, 0) does when no representative is below m9.
  // (Hidden candidates that merged are offered again as new clusters.)
  uint64_t kap = old_kappa[n];
  const uint32_t k9 = (uint32_t)(kap & 0xffffffffull);
  if (kap && k9 != 0xffffffffu) {
    const int m9 = (int)k9;  // a node of the finer level, 0 <= m9 < n_fine
    const uint64_t h = kap & 0xffffffff00000000ull;
    if (match[m9] == m9) {
      kap = h | (uint64_t)(uint32_t)gamma[m9];
    } else {
      if (why) atomicAdd((unsigned long long *)(why + 3), 1ull);
      // representatives: unmerged nodes and the smaller node of each pair
      int r = m9 - 1;
      for (int step = 0; step < kBoundScan && r >= 0 && match[r] < r; ++step) --r;
      if (r < 0) kap = h;
      else if (match[r] >= r) kap = h | (uint64_t)(uint32_t)gamma[r];
      else kap = h | 0xffffffffull;  // none found within the scan: hist-only bound
    }
  }
  const int c0 = old_cnt[n];
  // surviving old candidates, renamed (already in descending key order);
  // four at a time, each round of gathers issued before the next
  int k = 0;
  for (int q0 = 0; q0 < c0; q0 += 4) {
    uint64_t key[4];
    int32_t cm[4], mt[4], gm[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool in = q0 + u < c0;
      key[u] = in ? old_key[n * kTopK + q0 + u] : 0ull;
      cm[u] = in ? old_c[n * kTopK + q0 + u] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) mt[u] = q0 + u < c0 ? match[(int)(key[u] & 0xffffffffull)] : -1;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int m = (int)(key[u] & 0xffffffffull);
      gm[u] = (q0 + u < c0 && mt[u] == m) ? gamma[m] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int m = (int)(key[u] & 0xffffffffull);
      if (q0 + u >= c0 || mt[u] != m) continue;
      const uint64_t nk = (key[u] & 0xffffffff00000000ull) | (uint64_t)(uint32_t)gm[u];
#pragma unroll
      for (int z = 0; z < kTopK; ++z)
        if (z == k) {
          a[z] = nk;
          ac[z] = cm[u];
        }
      ++k;
    }
  }
  // offers from the new clusters (valid pairs with keys above kappa only), in
  // cluster order, four rows loaded at a time; the rows hold the raw
  // counters hist | c << 32 of every node against each new cluster
  const int64_t sn = csize[nc];
  const int64_t dn = cindeg[nc];
  for (int j0 = 0; j0 < n_new; j0 += 4) {
    uint64_t v[4];
    uint32_t id[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool in = j0 + u < n_new;
      v[u] = in ? rows[(int64_t)(j0 + u) * n_coarse + nc] : 0ull;
      id[u] = in ? (uint32_t)newc[j0 + u] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint64_t h = v[u] & 0xffffffffull;
      if (h == 0) continue;  // also the slots past n_new
      uint64_t x = cand_key(h, id[u]);
      if (x <= kap) continue;
      int32_t xc = (int32_t)(v[u] >> 32);
      if (sn + csize[id[u]] > omega || dn + cindeg[id[u]] - xc > delta) continue;  // not a valid pair
      list_insert<kTopK>(a, ac, x, xc);
      if (x > kap) kap = x;  // evicted (0 if the list had room)
    }
  }
  int cnt = 0;
#pragma unroll
  for (int z = 0; z < kTopK; ++z) {
    tk_key[(int64_t)nc * kTopK + z] = a[z];
    tk_c[(int64_t)nc * kTopK + z] = ac[z];
    cnt += a[z] ? 1 : 0;
  }
  tk_cnt[nc] = cnt;
  tk_kappa[nc] = kap;
  // the first `need` entries are certain only above every hidden
  // candidate's key (or when nothing is hidden)
  uint64_t kneed = 0;
#pragma unroll
  for (int z = 0; z < kTopK; ++z)
    if (z == need - 1) kneed = a[z];
  const bool certain = kap == 0 || (cnt >= need && kneed > kap);
  if (!certain) {
    rflag[nc] = 1;
    // diagnostics: why the node is re-rated (hist-only bound, short list,
    // need-th key not above the bound)
    if (why)
      atomicAdd((unsigned long long *)(why + ((kap & 0xffffffffull) == 0xffffffffull ? 0 : cnt < need ? 1 : 2)),
                1ull);
  } else {
    pair[nc] = cnt ? (int32_t)(a[0] & 0xffffffffull) : -1;
    score[nc] = cnt ? (int64_t)(a[0] >> 32) : 0;
  }
}

// New clusters of a matching: representatives a < match(a); newc[k] = gamma(a)
// in ascending order, row_slot[gamma(a)] = k, row_slot = -1 elsewhere.
__global__ void k_new_flags(const int32_t *__restrict__ match, int32_t n, int32_t *__restrict__ flag) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) flag[v] = match[v] > v ? 1 : 0;
}

__global__ void k_new_list(const int32_t *__restrict__ match, const int32_t *__restrict__ gamma,
                           const int32_t *__restrict__ off, int32_t n, int32_t *__restrict__ newc,
                           int32_t *__restrict__ row_slot) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && match[v] > v) {
    newc[off[v]] = gamma[v];
    row_slot[gamma[v]] = off[v];
  }
}

// Histogram rows of the listed nodes, each node's incidences split into
// `slices` parts streamed by different workgroups (a level that merges few
// pairs rates only a few clusters: one workgroup per row would leave the
// device idle).  Workgroup b handles slice b % slices of row b / slices,
// over LDS windows of its slice's neighbour id range, and adds its counters
// to acc[row * N + m] as hist | c << 32.
template <int NT>
__global__ __launch_bounds__(NT) void k_tail_hist(int32_t N, const int32_t *__restrict__ list, int32_t rows_n,
                                                  int32_t slices, const int32_t *__restrict__ ioff,
                                                  const uint32_t *__restrict__ inc, const int32_t *__restrict__ hoff,
                                                  const uint32_t *__restrict__ hpin, const int32_t *__restrict__ hw,
                                                  const int32_t *__restrict__ size, const int32_t *__restrict__ indeg,
                                                  const int32_t *__restrict__ total, int32_t omega, int32_t words,
                                                  unsigned long long *__restrict__ acc,
                                                  unsigned long long *__restrict__ units) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ int32_t tbl[NT / 64 * 192];
  __shared__ int2 rng_s[NT / 64];
  const int tid = threadIdx.x;
  const int r = (int)(blockIdx.x / slices), sl = (int)(blockIdx.x % slices);
  if (r >= rows_n) return;
  const int n = list[r];
  if (size[n] >= omega) return;
  const uint32_t tot = (uint32_t)total[n];
  const uint32_t din = (uint32_t)indeg[n];
  const int hb = tot ? 32 - __clz(tot) : 0;
  const int cb = din ? 32 - __clz(din) : 0;
  const bool packed = hb + cb <= 32;
  const uint64_t hmask = (hb >= 32) ? 0xffffffffull : ((1ull << hb) - 1ull);
  const int i0 = ioff[n], i1 = ioff[n + 1];
  const int chunk = (i1 - i0 + slices - 1) / slices;
  const int a = i0 + sl * chunk, z = min(i1, a + chunk);
  if (a >= z) return;
  uint64_t *lds64 = reinterpret_cast<uint64_t *>(lds);
  const int R = packed ? words : (words >> 1);
  const int2 rg = neighbour_range<NT>(a, z, inc, hoff, hpin, rng_s);
  const uint32_t *clip = ((int64_t)rg.y - rg.x >= R) ? hpin : nullptr;  // several windows
  unsigned long long *row = acc + (int64_t)r * N;
  int64_t streamed = 0;
  for (int lo = rg.x; lo <= rg.y; lo += R) {
    const int span = min(R, rg.y + 1 - lo);
    const int zw = packed ? span : 2 * span;
    for (int i = tid; i < zw; i += NT) lds[i] = 0u;
    __syncthreads();
    streamed += with_mode(packed ? 1 : 2, [&](auto mode) {
      constexpr int MODE = decltype(mode)::value;
      return stream_segments<NT / 64, kRateU, true, uint32_t, true>(
          a, z, inc, hoff, nullptr, hw, tbl, [&](int j) { return hpin[j]; },
          [&](uint32_t y, uint32_t info, bool ok) {
            window_add<MODE>(lds, lds64, (y & kIdMask) - (uint32_t)lo, ok ? info & kIdMask : 0u,
                             ok ? (info & y) >> 31 : 0u, hb);
          },
          clip, lo, lo + span);
    });
    __syncthreads();
    window_clear_self(lds, lds64, packed ? 1 : 2, n - lo, span);
    for (int i = tid; i < span; i += NT) {
      unsigned long long v;
      if (packed) {
        const uint32_t x = lds[i];
        v = x ? ((unsigned long long)(x & hmask) | ((unsigned long long)(hb >= 32 ? 0u : (x >> hb)) << 32)) : 0ull;
      } else {
        v = lds64[i];
      }
      if (v) atomicAdd(&row[lo + i], v);
    }
    __syncthreads();
  }
  add_wave_units(units, streamed);
}

// 1024-thread workgroups: a window of up to kTopKWideMaxWords words leaves
// room for one workgroup per CU, and 16 waves then hide the latency of the pin
// streams (4 waves per CU with 256 threads).  Their static LDS (12.5 KB of
// stream tables and reductions) and the window share the CU's 160 KB.
constexpr int TOPK_NT = 1024;
// The grouped rating runs 512-thread workgroups: its per-member selection
// keeps its lists in registers there (205 registers, none spilled, against
// 131 spilled at 1024 threads; rate_tail 1342 to 1329 ms on conv302k).
constexpr int GROUP_NT = 512;
constexpr int TOPK_GRID = 512;
constexpr int kTopKWideMaxWords = 37376;

static void topk_attr() {
  // thread-safe one-time opt-in to the large dynamic LDS size
  static const bool attr_set = [] {
    HGP_HIP(hipFuncSetAttribute((const void *)k_rate_topk<TOPK_NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                kTopKWideMaxWords * 4));
    HGP_HIP(hipFuncSetAttribute((const void *)k_rate_topk_groups<GROUP_NT, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, kTopKWideMaxWords * 4));
    HGP_HIP(hipFuncSetAttribute((const void *)k_tail_hist<TOPK_NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                kTopKWideMaxWords * 4));
    return true;
  }();
  (void)attr_set;
}

// LDS words of the window: the whole id range when it fits, else the maximum
static int topk_words(int32_t n) {
  const int64_t w = 2 * (int64_t)n;
  return (int)std::max<int64_t>(2, std::min<int64_t>(kTopKWideMaxWords, (w + 1) & ~int64_t(1)));
}

void launch_rate_topk(const LevelView &L, const int32_t *total, int32_t omega, int32_t delta, const int32_t *list,
                      const int64_t *count, int64_t grid_nodes, int32_t *pair, int64_t *score, TopK &tk,
                      hipStream_t s) {
  if (L.n <= 0 || grid_nodes <= 0) return;
  KScope ks(8, s);
  topk_attr();
  const int words = topk_words(L.n);
  const int grid = (int)std::min<int64_t>(TOPK_GRID, xcd_grid((int)std::min<int64_t>(grid_nodes, TOPK_GRID)));
  k_rate_topk<TOPK_NT><<<grid, TOPK_NT, (size_t)words * 4, s>>>(
      L.n, list, count, L.ioff, L.inc, L.hoff, L.hpin, L.hw, L.size, L.indeg, total, L.maxin, omega, delta, nullptr,
      nullptr,
      pair, score, tk.key, tk.c, tk.cnt, tk.kappa, words, nullptr, units_ptr(8));
  HGP_LAUNCH_CHECK();
}

// splitmix64's finaliser (a bijection of 64-bit words)
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// keys[t] = a 32-bit hash (masked by `mask`) of the set of inbound hedges of
// node list[t] (t < *count; one wave per entry), vals[t] = the node; entries
// from *count up to the bound get the key 0xffffffff, which no node's key
// has, so that they sort last.
__global__ void k_group_keys(const int32_t *__restrict__ list, const int64_t *__restrict__ count, int64_t bound,
                             const int32_t *__restrict__ ioff, const uint32_t *__restrict__ inc, uint32_t mask,
                             uint32_t *__restrict__ keys, uint32_t *__restrict__ vals) {
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int l = lane_id();
  if (t >= bound) return;  // uniform per wave
  const int64_t cnt = count ? *count : bound;
  if (t >= cnt) {
    if (l == 0) {
      keys[t] = 0xffffffffu;
      vals[t] = 0xffffffffu;
    }
    return;
  }
  const int n = list ? list[t] : (int)t;
  uint64_t h = 0;  // a sum of mixed hedge ids: independent of their order
  for (int i = ioff[n] + l; i < ioff[n + 1]; i += 64) {
    const uint32_t x = inc[i];
    if (x & kDst) h += mix64((uint64_t)(x & kIdMask) + 1ull);
  }
  h = wave_sum(h);
  if (l == 0) {
    const uint32_t k = (uint32_t)(mix64(h) >> 32) & mask;
    keys[t] = k == 0xffffffffu ? 0xfffffffeu : k;
    vals[t] = (uint32_t)n;
  }
}

// A group starts at every change of key and at every multiple of kGroupCap.
__device__ __forceinline__ bool group_start(const uint32_t *__restrict__ keys, int64_t i) {
  return i == 0 || keys[i] != keys[i - 1] || i % kGroupCap == 0;
}
__global__ void k_group_flags(const uint32_t *__restrict__ keys, int64_t bound, const int64_t *__restrict__ count,
                              int32_t *__restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= bound) return;
  const int64_t cnt = count ? *count : bound;
  flags[i] = (i < cnt && group_start(keys, i)) ? 1 : 0;
}
// goff[pos[i]] = i for the group starts; goff[*groups] = the entry count.
__global__ void k_group_offsets(const uint32_t *__restrict__ keys, const int32_t *__restrict__ pos, int64_t bound,
                                const int64_t *__restrict__ count, const int32_t *__restrict__ groups,
                                int32_t *__restrict__ goff) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= bound) return;
  const int64_t cnt = count ? *count : bound;
  if (i < cnt && group_start(keys, i)) goff[pos[i]] = (int32_t)i;
  if (i == 0) goff[*groups] = (int32_t)cnt;
}

static uint32_t group_hash_mask() {
  // tests narrow the key to force collisions, which the exact check catches
  const char *e = std::getenv("HGP_GROUP_HASH_BITS");
  const int b = e && e[0] ? std::atoi(e) : 32;
  return b >= 32 ? 0xffffffffu : (b <= 0 ? 0u : ((1u << b) - 1u));
}

int64_t group_scratch_words(int32_t n) { return (int64_t)TOPK_GRID * kGroupWins * topk_words(n); }

// stat[0] = the number of groups, stat[1] = the number of rated nodes
__global__ void k_group_stat(int32_t *__restrict__ stat, const int32_t *__restrict__ groups,
                             const int64_t *__restrict__ count, int32_t n) {
  if (threadIdx.x == 0) {
    stat[0] = *groups;
    stat[1] = count ? (int32_t)*count : n;
  }
}

void launch_group_order(const LevelView &L, const int32_t *list, const int64_t *count, int64_t bound,
                        const GroupBufs &G, hipStream_t s) {
  if (L.n <= 0 || bound <= 0) return;
  KScope ks(8, s);
  k_group_keys<<<div_up(bound * 64, 256), 256, 0, s>>>(list, count, bound, L.ioff, L.inc, group_hash_mask(), G.keys,
                                                       G.vals);
  HGP_LAUNCH_CHECK();
  radix_sort_u32(G.keys, G.alt, G.vals, G.valt, bound, 32, *G.tmp, s);
  k_group_flags<<<div_up(bound, 256), 256, 0, s>>>(G.keys, bound, count, G.pos);
  HGP_LAUNCH_CHECK();
  scan_i32(G.pos, G.pos, bound, G.groups, *G.scan_tmp, s);
  k_group_offsets<<<div_up(bound, 256), 256, 0, s>>>(G.keys, G.pos, bound, count, G.groups, G.goff);
  HGP_LAUNCH_CHECK();
}

void launch_rate_topk_grouped(const LevelView &L, const int32_t *total, int32_t omega, int32_t delta,
                              const int64_t *count, int64_t bound, int32_t *pair, int64_t *score, TopK &tk,
                              const GroupBufs &G, int32_t *stat, hipStream_t s) {
  if (L.n <= 0 || bound <= 0) return;
  KScope ks(8, s);
  topk_attr();
  const int words = topk_words(L.n);
  const int grid = (int)std::min<int64_t>(TOPK_GRID, xcd_grid((int)std::min<int64_t>(bound, TOPK_GRID)));
  k_rate_topk_groups<GROUP_NT, true><<<grid, GROUP_NT, (size_t)words * 4, s>>>(
      L.n, reinterpret_cast<const int32_t *>(G.vals), nullptr, L.ioff, L.inc, L.hoff, L.hpin, L.hw, L.size, L.indeg,
      total, L.maxin, omega, delta, nullptr, nullptr, pair, score, tk.key, tk.c, tk.cnt, tk.kappa, words, nullptr,
      G.goff, G.groups, G.scratch, units_ptr(8));
  HGP_LAUNCH_CHECK();
  if (stat) {
    k_group_stat<<<1, 64, 0, s>>>(stat, G.groups, count, (int32_t)bound);
    HGP_LAUNCH_CHECK();
  }
}

uint64_t *launch_rate_topk_rows(const LevelView &L, const int32_t *total, int32_t omega, int32_t delta,
                                const int32_t *list, const int64_t *count, int32_t n_rows, const int32_t *row_slot,
                                int32_t *pair, int64_t *score, TopK &tk, DevBuf &acc, hipStream_t s) {
  if (L.n <= 0 || n_rows <= 0) return nullptr;
  KScope ks(8, s);
  topk_attr();
  const int words = topk_words(L.n);
  // about TOPK_GRID workgroups over the rows, at most 256 slices per row
  const int slices =
      (int)std::max<int64_t>(1, std::min<int64_t>(256, (TOPK_GRID + n_rows - 1) / n_rows));
  const int64_t cells = (int64_t)n_rows * L.n;
  acc.reserve((size_t)cells * 8);
  unsigned long long *a = acc.as<unsigned long long>();
  fill_i64(reinterpret_cast<int64_t *>(a), cells, 0, s);
  k_tail_hist<TOPK_NT><<<n_rows * slices, TOPK_NT, (size_t)words * 4, s>>>(
      L.n, list, n_rows, slices, L.ioff, L.inc, L.hoff, L.hpin, L.hw, L.size, L.indeg, total, omega, words, a,
      units_ptr(8));
  HGP_LAUNCH_CHECK();
  // the rows stay raw counters: k_rate_update tests each offer's validity
  // itself, so they are not written back validated (a dense row set is
  // gigabytes at the early levels)
  uint64_t *rows = reinterpret_cast<uint64_t *>(a);
  const int grid = std::min(TOPK_GRID, xcd_grid(std::min(n_rows, TOPK_GRID)));
  k_rate_topk<TOPK_NT><<<grid, TOPK_NT, (size_t)words * 4, s>>>(
      L.n, list, count, L.ioff, L.inc, L.hoff, L.hpin, L.hw, L.size, L.indeg, total, L.maxin, omega, delta, nullptr,
      nullptr,
      pair, score, tk.key, tk.c, tk.cnt, tk.kappa, words, rows, units_ptr(8));
  HGP_LAUNCH_CHECK();
  return rows;
}

void launch_rate_update(int32_t n_fine, const int32_t *match, const int32_t *gamma, const TopK &old_tk,
                        int32_t n_new, const int32_t *newc, const uint64_t *rows, int32_t n_coarse,
                        const int32_t *csize, const int32_t *cindeg, int32_t omega, int32_t delta, int32_t need,
                        TopK &tk, int32_t *pair, int64_t *score, int32_t *rflag, int32_t *rerate,
                        int64_t *rerate_cnt, DevBuf &scan_tmp, hipStream_t s, int64_t *why) {
  fill_i64(rerate_cnt, 1, 0, s);
  if (n_fine <= 0 || n_coarse <= 0) return;
  KScope ks(8, s);
  fill_i32(rflag, n_coarse, 0, s);
  k_rate_update<<<div_up(n_fine, 256), 256, 0, s>>>(n_fine, match, gamma, old_tk.key, old_tk.c, old_tk.cnt,
                                                    old_tk.kappa, n_new, newc, rows, n_coarse, csize, cindeg, omega,
                                                    delta, need, tk.key, tk.c,
                                                    tk.cnt, tk.kappa, pair, score, rflag, why);
  HGP_LAUNCH_CHECK();
  // the re-rated nodes in id order: nearby ids share hedges, and the rating
  // gives each XCD a contiguous part of the list
  int32_t *total = reinterpret_cast<int32_t *>(rerate_cnt + 1);
  scan_i32(rflag, rflag, n_coarse, total, scan_tmp, s);
  k_list_from_scan<<<div_up(n_coarse, 256), 256, 0, s>>>(rflag, n_coarse, total, rerate, rerate_cnt);
  HGP_LAUNCH_CHECK();
}

void launch_new_clusters(const int32_t *match, const int32_t *gamma, int32_t n_fine, int32_t n_coarse,
                         int32_t *flag_tmp, int32_t *newc, int32_t *row_slot, DevBuf &scan_tmp, hipStream_t s) {
  fill_i32(row_slot, n_coarse, -1, s);
  if (n_fine <= 0) return;
  k_new_flags<<<div_up(n_fine, 256), 256, 0, s>>>(match, n_fine, flag_tmp);
  HGP_LAUNCH_CHECK();
  scan_i32(flag_tmp, flag_tmp, n_fine, nullptr, scan_tmp, s);
  k_new_list<<<div_up(n_fine, 256), 256, 0, s>>>(match, gamma, flag_tmp, n_fine, newc, row_slot);
  HGP_LAUNCH_CHECK();
}

// Candidate lists of the learned proposal (stride kCandOut per node) from the
// top-K lists: the first min(cnt, keep) entries (certain by construction), 0
// past them.
constexpr int kCandOut = 8;
static_assert(kCandOut <= kTopK, "the lists hold every candidate slot of the learned proposal");

__global__ void k_cand_from_lists(int32_t n, int32_t keep, const uint64_t *__restrict__ tk_key,
                                  const int32_t *__restrict__ tk_c, const int32_t *__restrict__ tk_cnt,
                                  uint64_t *__restrict__ ck, int32_t *__restrict__ cc, int32_t *__restrict__ ccnt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * kCandOut) return;
  const int64_t v = t / kCandOut;
  const int r = (int)(t % kCandOut);
  const int c = tk_cnt[v];
  const int k = c < keep ? c : keep;
  const int64_t src = v * kTopK + r;
  ck[t] = r < k ? tk_key[src] : 0ull;
  cc[t] = r < k ? tk_c[src] : 0;
  if (r == 0) ccnt[v] = k;
}

void launch_cand_from_lists(int32_t n, int32_t keep, const TopK &tk, uint64_t *ck, int32_t *cc, int32_t *ccnt,
                            hipStream_t s) {
  if (n <= 0) return;
  if (keep < 1 || keep > kCandOut) throw Error(HGP_EINVAL, "candidates per node outside 1..8");
  k_cand_from_lists<<<div_up((int64_t)n * kCandOut, 256), 256, 0, s>>>(n, keep, tk.key, tk.c, tk.cnt, ck, cc, ccnt);
  HGP_LAUNCH_CHECK();
}

}  // namespace hgp
