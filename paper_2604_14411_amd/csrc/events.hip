// In-sequence gains and sequence validity (Sec. IV-B), without contended
// atomics.
//
// Gains.  For the moving pins of hedge e, every move i of node v (p_s -> p_d)
// gives a source event on (p_s, i) and a destination event on (p_d, i).
// Sorted by (part, position), a prefix within each part gives
// pins_{i-1}(p, e) = pins_0(p, e) + earlier arrivals - earlier departures,
// and the exact change of Eq. 1 caused by move i on hedge e is
//   +w(e) if pins_{i-1}(p_s, e) = 1   (p_s leaves the hedge)
//   -w(e) if pins_{i-1}(p_d, e) = 0   (p_d joins the hedge).
// The two terms are stored per pin (contrib[j] = (source term, destination
// term)); g'(i) is then the sum over the incidences of v, read through the
// incidence -> pin permutation of the transpose.
//
// Validity.  Destination pins do the same on pins_in(p, e) and emit an
// inbound-count event (p, i, -1) on a 1 -> 0 transition of p_s and (p, i, +1)
// on a 0 -> 1 transition of p_d.  With the size events (p_s, i) and (p_d, i)
// of every move, all events are sorted by (part, position); prefix sums give
// each part's size and inbound count after every position, and a change of
// validity between consecutive positions of a part adds +-1 to viol there.
#include "coarsen.hpp"

namespace hgp {

constexpr int kClsEvents = 3;        // timing class of these kernels (sequence evaluation)
constexpr int kClsSort = 6;          // timing class of sorts
constexpr int EVW_NT = 128;          // two waves per workgroup
constexpr int EVW_MAX_MOVING = 256;  // moving pins of a hedge handled by one wave
constexpr int EVW_PT_STAGE = 256;    // part-table entries staged in LDS per wave
constexpr int EVW_U = 4;             // 64-pin chunks loaded together
constexpr int EVB_NT = 256;          // workgroup kernel for the remaining hedges
constexpr int EVB_GRID = 512;
static_assert(kSegCap <= 4096, "slot field of the workgroup event keys is 12 bits");

// Sorts a wave's nev (<= 64 * KPL) event keys held in LDS, in registers, and
// writes them back with the exclusive prefix of their count deltas within
// their part (key >> pshift): pins in the low 16 bits, pins_in in the high 16
// bits (both signed).  The first event of every part is found by a max-scan
// of part-start indices, so no event searches for it.  `at_starts` runs
// between the two phases, when evk is sorted and pre holds the raw prefix:
// whatever it subtracts from pre at a part's first event is added to every
// event of that part.
template <int KPL, class K, class AtStarts>
__device__ __forceinline__ void ev_wave_sort_scan(int nev, int pshift, K *evk, int32_t *pre, AtStarts at_starts) {
  const int l = lane_id();
  K k[KPL];
#pragma unroll
  for (int j = 0; j < KPL; ++j) {
    const int i = l * KPL + j;
    k[j] = i < nev ? evk[i] : ~K(0);
  }
  wave_bitonic_sort<KPL>(k);
  const K prev_last = __shfl_up(k[KPL - 1], 1, 64);
  int32_t d[KPL];
  int st[KPL];
  int32_t run = 0;
  int cur = -1;  // latest part start seen in this lane
#pragma unroll
  for (int j = 0; j < KPL; ++j) {
    const int i = l * KPL + j;
    int32_t x = 0;
    if (i < nev) {
      const int sgn = (k[j] & K(2)) ? 1 : -1;
      x = sgn + ((k[j] & K(1)) ? sgn * 65536 : 0);
    }
    d[j] = run;
    run += x;
    const K pk = j == 0 ? prev_last : k[j - 1];
    if (i == 0 || (k[j] >> pshift) != (pk >> pshift)) cur = i;
    st[j] = cur;
  }
  const int32_t base = wave_exclusive_scan(run);
  int carry = cur;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(carry, o, 64);
    if (l >= o) carry = max(carry, t);
  }
  int cin = __shfl_up(carry, 1, 64);
  if (l == 0) cin = 0;
#pragma unroll
  for (int j = 0; j < KPL; ++j) {
    const int i = l * KPL + j;
    if (st[j] < 0) st[j] = cin;
    if (i < nev) {
      evk[i] = k[j];
      pre[i] = base + d[j];
    }
  }
  wave_lds_sync();
  at_starts();
  wave_lds_sync();
  int32_t at_start[KPL];
#pragma unroll
  for (int j = 0; j < KPL; ++j) at_start[j] = (l * KPL + j < nev) ? pre[st[j]] : 0;
  wave_lds_sync();
#pragma unroll
  for (int j = 0; j < KPL; ++j) {
    const int i = l * KPL + j;
    if (i < nev) pre[i] = base + d[j] - at_start[j];
  }
}

// Splits a prefix difference of packed deltas into (pins, pins_in).
__device__ __forceinline__ int2 unpack_delta(int32_t pd) {
  const int32_t p = (int32_t)(int16_t)(pd & 0xffff);
  return make_int2(p, (pd - p) >> 16);
}

// Part table of a hedge staged in LDS (parts ascending; counts packed as
// pins | pins_in << 16, both <= kSegCap).
__device__ __forceinline__ int2 pt_lookup_lds(const int32_t *sp, const uint32_t *sc, int len, int p) {
  int lo = 0, hi = len;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (sp[mid] < p) lo = mid + 1;
    else hi = mid;
  }
  if (lo < len && sp[lo] == p) return make_int2((int)(sc[lo] & 0xffffu), (int)(sc[lo] >> 16));
  return make_int2(0, 0);
}

// One wave per hedge with at most EVW_MAX_MOVING moving pins; other hedges
// with moving pins are queued in heavy[] for k_ev_block.
// Key of a pin event: part << (qbits + 11) | position << 11 | slot << 2 |
// role << 1 | dst, slot = index of the moving pin (< 512), role 1 = destination.
// The inbound-count events of hedge e go to its own region evpad[2 hoff[e] ..)
// (at most one per pin event, i.e. 2 |e|) and their number to evcnt[e]; a
// scan of evcnt then packs them (k_ev_compact), so no counter is shared.
template <class KP>
__global__ __launch_bounds__(EVW_NT) void k_ev_wave(
    const int32_t *__restrict__ hoff, const uint32_t *__restrict__ hpin, int32_t E, const int32_t *__restrict__ hw,
    const int32_t *__restrict__ rho, const int32_t *__restrict__ dest, const int32_t *__restrict__ pos,
    const int32_t *__restrict__ pt, const uint32_t *__restrict__ ptc, const int32_t *__restrict__ lam, int qbits,
    int2 *__restrict__ contrib, KP *__restrict__ evpad, int64_t *__restrict__ evcnt,
    int64_t *__restrict__ scal, int32_t *__restrict__ heavy) {
  __shared__ uint64_t evk_s[EVW_NT / 64][2 * EVW_MAX_MOVING];
  __shared__ int32_t pre_s[EVW_NT / 64][2 * EVW_MAX_MOVING];
  __shared__ int16_t li_s[EVW_NT / 64][EVW_MAX_MOVING];
  __shared__ int32_t sp_s[EVW_NT / 64][EVW_PT_STAGE];
  __shared__ uint32_t sc_s[EVW_NT / 64][EVW_PT_STAGE];
  const int w = threadIdx.x >> 6, l = lane_id();
  const int e = (int)(blockIdx.x * (EVW_NT / 64) + w);
  if (e >= E) return;
  const int b = hoff[e], len = hoff[e + 1] - b;
  const int32_t we = hw[e];
  const int plen = lam[e];
  const int pshift = qbits + 11;
  const uint64_t qmask = (1ull << qbits) - 1ull;
  uint64_t *evk = evk_s[w];
  int32_t *pre = pre_s[w];
  int16_t *li = li_s[w];
  const uint64_t lt = (l == 0) ? 0ull : ((~0ull) >> (64 - l));
  // one pass over the pins, EVW_U chunks of 64 at a time: all pin loads of a
  // batch are issued before the position gathers, and those before the part
  // gathers of the moving pins
  int m = 0;
  for (int c = 0; c < len && m <= EVW_MAX_MOVING; c += 64 * EVW_U) {
    uint32_t x[EVW_U];
    int q[EVW_U];
#pragma unroll
    for (int u = 0; u < EVW_U; ++u) {
      const int i = c + 64 * u + l;
      x[u] = i < len ? hpin[b + i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < EVW_U; ++u) {
      const int i = c + 64 * u + l;
      q[u] = i < len ? pos[x[u] & kIdMask] : 0;
    }
    int32_t ps[EVW_U], pd[EVW_U];
#pragma unroll
    for (int u = 0; u < EVW_U; ++u) {
      ps[u] = 0;
      pd[u] = 0;
      if (q[u] > 0) {
        ps[u] = rho[x[u] & kIdMask];
        pd[u] = dest[x[u] & kIdMask];
      }
    }
#pragma unroll
    for (int u = 0; u < EVW_U; ++u) {
      const uint64_t mask = __ballot(q[u] > 0);
      const int slot = m + __popcll(mask & lt);
      if (q[u] > 0 && slot < EVW_MAX_MOVING) {
        const uint64_t tail = ((uint64_t)q[u] << 11) | ((uint64_t)slot << 2) | (uint64_t)(x[u] >> 31);
        li[slot] = (int16_t)(c + 64 * u + l);
        evk[2 * slot] = ((uint64_t)(uint32_t)ps[u] << pshift) | tail;
        evk[2 * slot + 1] = ((uint64_t)(uint32_t)pd[u] << pshift) | tail | 2ull;
      }
      m += __popcll(mask);
    }
  }
  if (m == 0) {
    if (l == 0) evcnt[e] = 0;
    return;
  }
  if (m > EVW_MAX_MOVING) {
    if (l == 0) heavy[atomicAdd((unsigned long long *)&scal[SC_HEAVY], 1ull)] = e;
    return;
  }
  wave_lds_sync();
  const int nev = 2 * m;
  // the hedge's part table in LDS (parts ascending; pins | pins_in << 16)
  const bool staged = plen <= EVW_PT_STAGE;
  int32_t *sp = sp_s[w];
  uint32_t *sc = sc_s[w];
  if (staged) {
    for (int i = l; i < plen; i += 64) {
      sp[i] = pt[b + i];
      sc[i] = ptc[b + i];
    }
  }
  if (nev <= 64) ev_wave_sort_scan<1>(nev, pshift, evk, pre, [] {});
  else if (nev <= 128) ev_wave_sort_scan<2>(nev, pshift, evk, pre, [] {});
  else if (nev <= 256) ev_wave_sort_scan<4>(nev, pshift, evk, pre, [] {});
  else ev_wave_sort_scan<8>(nev, pshift, evk, pre, [] {});
  wave_lds_sync();
  uint32_t evbits = 0;  // bit t: event l + 64 t changes an inbound count
  int nout = 0;
  for (int t = 0; t * 64 < nev; ++t) {
    const int i = l + 64 * t;
    if (i >= nev) continue;
    const uint64_t k = evk[i];
    const int part = (int)(k >> pshift);
    const int2 before = unpack_delta(pre[i]);
    const int2 c0 = staged ? pt_lookup_lds(sp, sc, plen, part) : pt_lookup(pt, ptc, b, plen, part);
    const bool dst_role = (k & 2ull) != 0;
    int2 *cp = &contrib[b + li[(int)((k >> 2) & 511ull)]];
    if (dst_role) cp->y = (c0.x + before.x == 0) ? -we : 0;
    else cp->x = (c0.x + before.x == 1) ? we : 0;
    if (k & 1ull) {
      const int bin = c0.y + before.y;
      if ((!dst_role && bin == 1) || (dst_role && bin == 0)) {
        evbits |= 1u << t;
        ++nout;
      }
    }
  }
  const int off = wave_exclusive_scan(nout);
  if (l == 63) evcnt[e] = off + nout;
  const int vshift = qbits + 2;
  int64_t o = 2 * (int64_t)b + off;
  for (int t = 0; evbits; ++t, evbits >>= 1) {
    if (!(evbits & 1u)) continue;
    const uint64_t k = evk[l + 64 * t];
    const uint64_t q = (k >> 11) & qmask;
    evpad[o++] = (KP)(((k >> pshift) << vshift) | (q << 2) | ((k >> 1) & 1ull));
  }
}

// 32-bit variant of k_ev_wave, for part ids below 2^22 and positions below
// 2^24 (the register sort dominates the kernel, and 32-bit keys halve its
// work).  The hedge's moving pins are first sorted by position (key
// position << 8 | slot); a pin's rank r in that order replaces its position
// in the event keys: part << 10 | r << 2 | role << 1 | dst.  The counts
// pins_0 / pins_in_0 of the hedge's part table enter the prefixes at the
// first event of each part (a search of the sorted events per table entry),
// so neither the table nor per-event lookups take LDS.  KP: the word of the
// padded event regions (32-bit when the packed keys fit).
constexpr int EVN_PBITS = 22;
constexpr int EVN_QBITS = 24;
constexpr int EVN_PT_REG = 4;  // 64-entry chunks of the part table prefetched into registers

template <class KP>
__global__ __launch_bounds__(EVW_NT) void k_ev_wave32(
    const int32_t *__restrict__ hoff, const uint32_t *__restrict__ hpin, int32_t E, const int32_t *__restrict__ hw,
    const int32_t *__restrict__ rho, const int32_t *__restrict__ dest, const int32_t *__restrict__ pos,
    const int32_t *__restrict__ pt, const uint32_t *__restrict__ ptc, const int32_t *__restrict__ lam, int qbits,
    int2 *__restrict__ contrib, KP *__restrict__ evpad, int64_t *__restrict__ evcnt,
    int64_t *__restrict__ scal, int32_t *__restrict__ heavy) {
  __shared__ uint32_t evk_s[EVW_NT / 64][2 * EVW_MAX_MOVING];
  __shared__ int32_t pre_s[EVW_NT / 64][2 * EVW_MAX_MOVING];
  __shared__ uint32_t qs_s[EVW_NT / 64][EVW_MAX_MOVING];   // position << 8 | slot, then in rank order
  __shared__ int16_t li_s[EVW_NT / 64][EVW_MAX_MOVING];
  const int w = threadIdx.x >> 6, l = lane_id();
  const int e = (int)(blockIdx.x * (EVW_NT / 64) + w);
  if (e >= E) return;
  const int b = hoff[e], len = hoff[e + 1] - b;
  const int32_t we = hw[e];
  const int plen = lam[e];
  uint32_t *evk = evk_s[w];
  int32_t *pre = pre_s[w];
  uint32_t *qs = qs_s[w];
  int16_t *li = li_s[w];
  const uint64_t lt = (l == 0) ? 0ull : ((~0ull) >> (64 - l));
  // one pass over the pins, as in k_ev_wave; the events carry the slot's
  // rank once the positions are sorted
  int m = 0;
  for (int c = 0; c < len && m <= EVW_MAX_MOVING; c += 64 * EVW_U) {
    uint32_t x[EVW_U];
    int q[EVW_U];
#pragma unroll
    for (int u = 0; u < EVW_U; ++u) {
      const int i = c + 64 * u + l;
      x[u] = i < len ? hpin[b + i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < EVW_U; ++u) {
      const int i = c + 64 * u + l;
      q[u] = i < len ? pos[x[u] & kIdMask] : 0;
    }
    int32_t ps[EVW_U], pd[EVW_U];
#pragma unroll
    for (int u = 0; u < EVW_U; ++u) {
      ps[u] = 0;
      pd[u] = 0;
      if (q[u] > 0) {
        ps[u] = rho[x[u] & kIdMask];
        pd[u] = dest[x[u] & kIdMask];
      }
    }
#pragma unroll
    for (int u = 0; u < EVW_U; ++u) {
      const uint64_t mask = __ballot(q[u] > 0);
      const int slot = m + __popcll(mask & lt);
      if (q[u] > 0 && slot < EVW_MAX_MOVING) {
        const uint32_t dbit = x[u] >> 31;
        li[slot] = (int16_t)(c + 64 * u + l);
        qs[slot] = ((uint32_t)q[u] << 8) | (uint32_t)slot;
        evk[2 * slot] = ((uint32_t)ps[u] << 10) | dbit;
        evk[2 * slot + 1] = ((uint32_t)pd[u] << 10) | dbit | 2u;
      }
      m += __popcll(mask);
    }
  }
  if (m == 0) {
    if (l == 0) evcnt[e] = 0;
    return;
  }
  if (m > EVW_MAX_MOVING) {
    if (l == 0) heavy[atomicAdd((unsigned long long *)&scal[SC_HEAVY], 1ull)] = e;
    return;
  }
  // the first chunks of the part table (parts ascending; pins | pins_in << 16),
  // loaded while the positions sort
  int32_t tp[EVN_PT_REG];
  uint32_t tc[EVN_PT_REG];
#pragma unroll
  for (int u = 0; u < EVN_PT_REG; ++u) {
    const int j = 64 * u + l;
    tp[u] = j < plen ? pt[b + j] : -1;
    tc[u] = j < plen ? ptc[b + j] : 0u;
  }
  wave_lds_sync();
  // moving pins in position order (positions are distinct)
  {
    auto sort_q = [&](auto kpl) {
      constexpr int KPL = decltype(kpl)::value;
      uint32_t k[KPL];
#pragma unroll
      for (int j = 0; j < KPL; ++j) {
        const int i = l * KPL + j;
        k[j] = i < m ? qs[i] : ~0u;
      }
      wave_bitonic_sort<KPL>(k);
      wave_lds_sync();
#pragma unroll
      for (int j = 0; j < KPL; ++j) {
        const int i = l * KPL + j;
        if (i < m) qs[i] = k[j];
      }
    };
    if (m <= 64) sort_q(std::integral_constant<int, 1>{});
    else if (m <= 128) sort_q(std::integral_constant<int, 2>{});
    else sort_q(std::integral_constant<int, 4>{});
  }
  wave_lds_sync();
  for (int r = l; r < m; r += 64) {
    const int slot = (int)(qs[r] & 255u);
    evk[2 * slot] |= (uint32_t)r << 2;
    evk[2 * slot + 1] |= (uint32_t)r << 2;
  }
  wave_lds_sync();
  const int nev = 2 * m;
  // table entry (p, c): the first sorted event of part p, if any, starts
  // from c instead of 0
  auto add_table = [&]() {
    auto one = [&](int32_t p, uint32_t cnt) {
      int lo = 0, hi = nev;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int32_t)(evk[mid] >> 10) < p) lo = mid + 1;
        else hi = mid;
      }
      if (lo < nev && (int32_t)(evk[lo] >> 10) == p) pre[lo] -= (int32_t)cnt;
    };
#pragma unroll
    for (int u = 0; u < EVN_PT_REG; ++u)
      if (tp[u] >= 0) one(tp[u], tc[u]);
    for (int j = 64 * EVN_PT_REG + l; j < plen; j += 64) one(pt[b + j], ptc[b + j]);
  };
  if (nev <= 64) ev_wave_sort_scan<1>(nev, 10, evk, pre, add_table);
  else if (nev <= 128) ev_wave_sort_scan<2>(nev, 10, evk, pre, add_table);
  else if (nev <= 256) ev_wave_sort_scan<4>(nev, 10, evk, pre, add_table);
  else ev_wave_sort_scan<8>(nev, 10, evk, pre, add_table);
  wave_lds_sync();
  uint32_t evbits = 0;  // bit t: event l + 64 t changes an inbound count
  int nout = 0;
  for (int t = 0; t * 64 < nev; ++t) {
    const int i = l + 64 * t;
    if (i >= nev) continue;
    const uint32_t k = evk[i];
    const int2 before = unpack_delta(pre[i]);  // pins / pins_in of the part before this move
    const bool dst_role = (k & 2u) != 0;
    const int slot = (int)(qs[(k >> 2) & 255u] & 255u);
    int2 *cp = &contrib[b + li[slot]];
    if (dst_role) cp->y = (before.x == 0) ? -we : 0;
    else cp->x = (before.x == 1) ? we : 0;
    if (k & 1u) {
      const int bin = before.y;
      if ((!dst_role && bin == 1) || (dst_role && bin == 0)) {
        evbits |= 1u << t;
        ++nout;
      }
    }
  }
  const int off = wave_exclusive_scan(nout);
  if (l == 63) evcnt[e] = off + nout;
  const int vshift = qbits + 2;
  int64_t o = 2 * (int64_t)b + off;
  for (int t = 0; evbits; ++t, evbits >>= 1) {
    if (!(evbits & 1u)) continue;
    const uint32_t k = evk[l + 64 * t];
    const uint64_t q = qs[(k >> 2) & 255u] >> 8;
    evpad[o++] = (KP)(((uint64_t)(k >> 10) << vshift) | (q << 2) | ((k >> 1) & 1u));
  }
}

// One workgroup per queued hedge (more than EVW_MAX_MOVING moving pins; at
// most kSegCap pins).  Same events as k_ev_wave with a 12-bit slot field:
// part << (qbits + 14) | position << 14 | slot << 2 | role << 1 | dst.
template <class KP>
__global__ __launch_bounds__(EVB_NT) void k_ev_block(
    const int32_t *__restrict__ hoff, const uint32_t *__restrict__ hpin, const int32_t *__restrict__ hw,
    const int32_t *__restrict__ rho, const int32_t *__restrict__ dest, const int32_t *__restrict__ pos,
    const int32_t *__restrict__ pt, const uint32_t *__restrict__ ptc, const int32_t *__restrict__ lam, int qbits,
    int2 *__restrict__ contrib, KP *__restrict__ evpad, int64_t *__restrict__ evcnt,
    const int64_t *__restrict__ scal, const int32_t *__restrict__ heavy) {
  __shared__ uint64_t key[2 * kSegCap];
  __shared__ int32_t dl[2 * kSegCap];
  __shared__ int32_t sp[kSegCap];
  __shared__ uint32_t sc[kSegCap];
  __shared__ int16_t li[kSegCap];
  __shared__ int32_t tmp[EVB_NT / 64 + 1];
  __shared__ int32_t s_wtot[EVB_NT / 64];
  __shared__ int32_t s_cnt;
  const int tid = threadIdx.x, l = lane_id();
  const int hshift = qbits + 14;
  const uint64_t qmask = (1ull << qbits) - 1ull;
  const int vshift = qbits + 2;
  const int64_t nh = scal[SC_HEAVY];
  for (int64_t h = blockIdx.x; h < nh; h += gridDim.x) {
    const int e = heavy[h];
    const int b = hoff[e], len = hoff[e + 1] - b;
    if (len > kSegCap) continue;  // k_ev_huge's
    if (tid == 0) s_cnt = 0;
    __syncthreads();
    for (int i = tid; i < len; i += EVB_NT) {
      const uint32_t x = hpin[b + i];
      const int v = (int)(x & kIdMask);
      const int q = pos[v];
      if (q > 0) {
        const int slot = atomicAdd(&s_cnt, 1);
        li[slot] = (int16_t)i;
        const uint64_t tail = ((uint64_t)q << 14) | ((uint64_t)slot << 2) | (uint64_t)(x >> 31);
        key[2 * slot] = ((uint64_t)(uint32_t)rho[v] << hshift) | tail;
        key[2 * slot + 1] = ((uint64_t)(uint32_t)dest[v] << hshift) | tail | 2ull;
      }
    }
    __syncthreads();
    const int nev = 2 * s_cnt;
    const int np = next_pow2(nev);
    for (int i = nev + tid; i < np; i += EVB_NT) key[i] = ~0ull;
    __syncthreads();
    block_bitonic_sort<uint64_t, EVB_NT>(key, np);
    for (int i = tid; i < nev; i += EVB_NT) {
      const uint64_t k = key[i];
      const int sgn = (k & 2ull) ? 1 : -1;
      dl[i] = sgn + ((k & 1ull) ? sgn * 65536 : 0);
    }
    __syncthreads();
    block_exclusive_scan<int32_t, EVB_NT>(dl, nev, tmp);
    const int32_t we = hw[e];
    const int plen = lam[e];
    for (int i = tid; i < plen; i += EVB_NT) {
      sp[i] = pt[b + i];
      sc[i] = ptc[b + i];
    }
    __syncthreads();
    uint32_t evbits = 0;  // bit t: event tid + EVB_NT t changes an inbound count (nev <= 32 EVB_NT)
    int nout = 0;
    for (int t = 0, i = tid; i < nev; ++t, i += EVB_NT) {
      const uint64_t k = key[i];
      const uint64_t part = k >> hshift;
      int lo = 0, hi = i;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((key[mid] >> hshift) < part) lo = mid + 1;
        else hi = mid;
      }
      const int2 before = unpack_delta(dl[i] - dl[lo]);
      const int2 c0 = pt_lookup_lds(sp, sc, plen, (int)part);
      const bool dst_role = (k & 2ull) != 0;
      int2 *cp = &contrib[b + li[(int)((k >> 2) & 4095ull)]];
      if (dst_role) cp->y = (c0.x + before.x == 0) ? -we : 0;
      else cp->x = (c0.x + before.x == 1) ? we : 0;
      if (k & 1ull) {
        const int bin = c0.y + before.y;
        if ((!dst_role && bin == 1) || (dst_role && bin == 0)) {
          evbits |= 1u << t;
          ++nout;
        }
      }
    }
    // this hedge's events go to evpad[2b ..), wave by wave
    const int off = wave_exclusive_scan(nout);
    if (l == 63) s_wtot[tid >> 6] = off + nout;
    __syncthreads();
    int wbase = 0, btot = 0;
    for (int q = 0; q < EVB_NT / 64; ++q) {
      if (q < (tid >> 6)) wbase += s_wtot[q];
      btot += s_wtot[q];
    }
    if (tid == 0) evcnt[e] = btot;
    int64_t o = 2 * (int64_t)b + wbase + off;
    for (int t = 0; evbits; ++t, evbits >>= 1) {
      if (!(evbits & 1u)) continue;
      const uint64_t k = key[tid + EVB_NT * t];
      const uint64_t q = (k >> 14) & qmask;
      evpad[o++] = (KP)(((k >> hshift) << vshift) | (q << 2) | ((k >> 1) & 1ull));
    }
    __syncthreads();
  }
}

// Queued hedges of more than kSegCap pins (at most kHugeCap): the events of
// k_ev_block built in global scratch (keys at four times the pin offset in
// gkey, their deltas at twice it in gdl).  The key carries the pin's
// position within the hedge instead of a slot, 16 bits wide:
// part << (qbits + 18) | position << 18 | pin << 2 | role << 1 | dst; keys
// are distinct (a node has one pin per hedge), so no slot is needed, and
// the hedge's inbound events take their places by an LDS counter (their
// order within the hedge's region does not matter: they are sorted later).
template <class KP>
__global__ __launch_bounds__(EVB_NT) void k_ev_huge(
    const int32_t *__restrict__ hoff, const uint32_t *__restrict__ hpin, const int32_t *__restrict__ hw,
    const int32_t *__restrict__ rho, const int32_t *__restrict__ dest, const int32_t *__restrict__ pos,
    const int32_t *__restrict__ pt, const uint32_t *__restrict__ ptc, const int32_t *__restrict__ lam, int qbits,
    int2 *__restrict__ contrib, KP *__restrict__ evpad, int64_t *__restrict__ evcnt,
    const int64_t *__restrict__ scal, const int32_t *__restrict__ heavy, uint64_t *__restrict__ gkey,
    int32_t *__restrict__ gdl) {
  __shared__ int32_t tmp[EVB_NT / 64 + 1];
  __shared__ int32_t s_cnt, s_out;
  const int tid = threadIdx.x;
  const int hshift = qbits + 18;
  const uint64_t qmask = (1ull << qbits) - 1ull;
  const int vshift = qbits + 2;
  const int64_t nh = scal[SC_HEAVY];
  for (int64_t h = blockIdx.x; h < nh; h += gridDim.x) {
    const int e = heavy[h];
    const int b = hoff[e], len = hoff[e + 1] - b;
    if (len <= kSegCap) continue;  // k_ev_block's
    uint64_t *key = gkey + 4 * (int64_t)b;
    int32_t *dl = gdl + 2 * (int64_t)b;
    if (tid == 0) {
      s_cnt = 0;
      s_out = 0;
    }
    __syncthreads();
    for (int i = tid; i < len; i += EVB_NT) {
      const uint32_t x = hpin[b + i];
      const int v = (int)(x & kIdMask);
      const int q = pos[v];
      if (q > 0) {
        const int slot = atomicAdd(&s_cnt, 1);
        const uint64_t tail = ((uint64_t)q << 18) | ((uint64_t)i << 2) | (uint64_t)(x >> 31);
        key[2 * slot] = ((uint64_t)(uint32_t)rho[v] << hshift) | tail;
        key[2 * slot + 1] = ((uint64_t)(uint32_t)dest[v] << hshift) | tail | 2ull;
      }
    }
    __syncthreads();
    const int nev = 2 * s_cnt;
    const int np = next_pow2(nev);
    for (int i = nev + tid; i < np; i += EVB_NT) key[i] = ~0ull;
    __syncthreads();
    block_bitonic_sort<uint64_t, EVB_NT>(key, np);
    for (int i = tid; i < nev; i += EVB_NT) {
      const uint64_t k = key[i];
      const int sgn = (k & 2ull) ? 1 : -1;
      dl[i] = sgn + ((k & 1ull) ? sgn * 65536 : 0);
    }
    __syncthreads();
    block_exclusive_scan<int32_t, EVB_NT>(dl, nev, tmp);
    const int32_t we = hw[e];
    const int plen = lam[e];
    for (int i = tid; i < nev; i += EVB_NT) {
      const uint64_t k = key[i];
      const uint64_t part = k >> hshift;
      int lo = 0, hi = i;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((key[mid] >> hshift) < part) lo = mid + 1;
        else hi = mid;
      }
      const int2 before = unpack_delta(dl[i] - dl[lo]);
      const int2 c0 = pt_lookup(pt, ptc, b, plen, (int)part);
      const bool dst_role = (k & 2ull) != 0;
      int2 *cp = &contrib[b + (int)((k >> 2) & 0xffffull)];
      if (dst_role) cp->y = (c0.x + before.x == 0) ? -we : 0;
      else cp->x = (c0.x + before.x == 1) ? we : 0;
      if (k & 1ull) {
        const int bin = c0.y + before.y;
        if ((!dst_role && bin == 1) || (dst_role && bin == 0)) {
          const int o = atomicAdd(&s_out, 1);
          const uint64_t q = (k >> 18) & qmask;
          evpad[2 * (int64_t)b + o] = (KP)(((k >> hshift) << vshift) | (q << 2) | ((k >> 1) & 1ull));
        }
      }
    }
    __syncthreads();
    if (tid == 0) evcnt[e] = s_out;
    __syncthreads();
  }
}

// Packs the inbound-count events of every hedge (evpad[2 hoff[e] ..), evcnt
// already scanned into offsets evoff) into ev[0 .. evoff[E]).  One wave per
// hedge.
template <class K>
__global__ __launch_bounds__(256) void k_ev_compact(const int32_t *__restrict__ hoff, int32_t E,
                                                    const int64_t *__restrict__ evoff,
                                                    const K *__restrict__ evpad, K *__restrict__ ev) {
  const int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (e >= E) return;
  const int64_t o = evoff[e], c = evoff[e + 1] - o;
  if (c == 0) return;
  const int64_t src = 2 * (int64_t)hoff[e];
  for (int64_t i = lane_id(); i < c; i += 64) ev[o + i] = evpad[src + i];
}

// g'(i) for move i = 1..S: the sum, over the incidences k of the moving node,
// of both terms stored at its pin perm[k].  One wave per move.
__global__ __launch_bounds__(256) void k_move_gain(const int32_t *__restrict__ seq, int64_t S,
                                                   const int32_t *__restrict__ ioff, const uint32_t *__restrict__ perm,
                                                   const int2 *__restrict__ contrib, int32_t *__restrict__ gp) {
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (i >= S) return;
  const int v = seq[i];
  const int a = ioff[v], z = ioff[v + 1];
  int32_t g = 0;
  for (int k = a + lane_id(); k < z; k += 64) {
    const int2 c = contrib[perm[k]];
    g += c.x + c.y;
  }
  g = wave_sum(g);
  if (lane_id() == 0) gp[i + 1] = g;
}

// size events (p_s, i, size) and (p_d, i, size) of every move i
template <class K>
__global__ void k_size_events(const int32_t *__restrict__ seq, int64_t S, const int32_t *__restrict__ rho,
                              const int32_t *__restrict__ dest, int vshift, K *__restrict__ ev, int64_t base) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  const int v = seq[i];
  const uint64_t tail = ((uint64_t)(i + 1) << 2) | 2ull;
  ev[base + 2 * i] = (K)(((uint64_t)(uint32_t)rho[v] << vshift) | tail);
  ev[base + 2 * i + 1] = (K)(((uint64_t)(uint32_t)dest[v] << vshift) | tail);
}

// After the sort, one pass decides every validity transition.  Deltas per
// sorted event: a size event (type 2) adds -size(v) to the part v leaves and
// +size(v) to the part it joins; an inbound event adds -1 (type 0) or +1
// (type 1).  The part's size and inbound count after event i are its initial
// values plus the prefix of the deltas within its part (a scan segmented at
// part changes).  For a (part, position) group, invalid_after - invalid_before
// is added to vdelta at the position: +1 where the part becomes invalid, -1
// where it becomes valid again (invalid = size > Omega or inbound > Delta).
// Two kernels over tiles of EVS_TILE events: per-tile aggregates of the
// segmented sum, then per tile its carry (a look-back over the aggregates of
// the tiles before it, as far as the nearest one where a part starts), its own
// scan and the group decisions.  Order within a group does not matter: only
// whole groups are compared.
constexpr int EVS_NT = 256;
constexpr int EVS_IPT = 8;
constexpr int EVS_TILE = EVS_NT * EVS_IPT;
static_assert(EVS_TILE == kEventTile, "tile arrays are sized by kEventTile");

template <class K>
__device__ __forceinline__ void ev_delta(uint64_t k, int vshift, uint64_t qmask, const int32_t *__restrict__ seq,
                                         const int32_t *__restrict__ rho, const int32_t *__restrict__ size,
                                         int64_t &ds, int32_t &di) {
  const int type = (int)(k & 3ull);
  ds = 0;
  di = 0;
  if (type == 2) {
    const int v = seq[((k >> 2) & qmask) - 1];
    ds = (uint64_t)(uint32_t)rho[v] == (k >> vshift) ? -(int64_t)size[v] : (int64_t)size[v];
  } else {
    di = type == 1 ? 1 : -1;
  }
}

// A segmented-sum element: f = a segment starts in it, (e, i) = the sums
// after its last start (of all of it when f = 0).
struct SegSum {
  int64_t e;
  int32_t i;
  int32_t f;
};
__device__ __forceinline__ SegSum seg_combine(const SegSum &a, const SegSum &b) {
  return b.f ? b : SegSum{a.e + b.e, a.i + b.i, a.f};
}
__device__ __forceinline__ SegSum seg_shfl_up(const SegSum &x, int o) {
  return SegSum{__shfl_up(x.e, o, 64), __shfl_up(x.i, o, 64), __shfl_up(x.f, o, 64)};
}
// Inclusive segmented scan over a wave.
__device__ __forceinline__ SegSum seg_wave_scan(SegSum x) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const SegSum y = seg_shfl_up(x, o);
    if (l >= o) x = seg_combine(y, x);
  }
  return x;
}
// Exclusive segmented scan over the block (thread order); returns the
// combination of all elements before this thread's.
template <int NT>
__device__ __forceinline__ SegSum seg_block_exclusive(SegSum x, SegSum *wtot) {
  const int w = threadIdx.x >> 6, l = lane_id();
  const SegSum inc = seg_wave_scan(x);
  if (l == 63) wtot[w] = inc;
  __syncthreads();
  SegSum pre{0, 0, 0};
  for (int q = 0; q < w; ++q) pre = seg_combine(pre, wtot[q]);
  SegSum ex = seg_shfl_up(inc, 1);
  if (l == 0) ex = SegSum{0, 0, 0};
  __syncthreads();
  return seg_combine(pre, ex);
}

template <class K>
__global__ __launch_bounds__(EVS_NT) void k_evs_tiles(const K *__restrict__ ev, int64_t nev, int vshift,
                                                      uint64_t qmask, const int32_t *__restrict__ seq,
                                                      const int32_t *__restrict__ rho,
                                                      const int32_t *__restrict__ size, int64_t *__restrict__ agg_e,
                                                      int32_t *__restrict__ agg_i, int32_t *__restrict__ agg_f) {
  __shared__ K kk[EVS_TILE + 1];  // kk[0]: the key before the tile
  __shared__ SegSum wtot[EVS_NT / 64];
  const int64_t t0 = (int64_t)blockIdx.x * EVS_TILE;
  const int tid = threadIdx.x;
  const int cnt = (int)min((int64_t)EVS_TILE, nev - t0);
  for (int j = tid; j < cnt; j += EVS_NT) kk[j + 1] = ev[t0 + j];
  if (tid == 0) kk[0] = t0 > 0 ? ev[t0 - 1] : K(0);
  __syncthreads();
  // contiguous items per thread, so that a thread's fold is in event order
  SegSum x{0, 0, 0};
#pragma unroll
  for (int j = 0; j < EVS_IPT; ++j) {
    const int lj = tid * EVS_IPT + j;
    if (lj >= cnt) break;
    const uint64_t k = (uint64_t)kk[lj + 1];
    const bool start = (t0 + lj == 0) || (k >> vshift) != ((uint64_t)kk[lj] >> vshift);
    int64_t ds;
    int32_t di;
    ev_delta<K>(k, vshift, qmask, seq, rho, size, ds, di);
    x = seg_combine(x, SegSum{ds, di, start ? 1 : 0});
  }
  const SegSum ex = seg_block_exclusive<EVS_NT>(x, wtot);
  if (tid == EVS_NT - 1) {
    const SegSum t = seg_combine(ex, x);
    agg_e[blockIdx.x] = t.e;
    agg_i[blockIdx.x] = t.i;
    agg_f[blockIdx.x] = t.f;
  }
}

template <class K>
__global__ __launch_bounds__(EVS_NT, sizeof(K) == 4 ? 8 : 1) void k_evs_trans(const K *__restrict__ ev, int64_t nev, int vshift,
                                                      uint64_t qmask, const int32_t *__restrict__ seq,
                                                      const int32_t *__restrict__ rho,
                                                      const int32_t *__restrict__ size,
                                                      const int64_t *__restrict__ agg_e,
                                                      const int32_t *__restrict__ agg_i,
                                                      const int32_t *__restrict__ agg_f,
                                                      const int32_t *__restrict__ psize,
                                                      const int32_t *__restrict__ pinb, int32_t omega, int32_t delta,
                                                      int32_t *__restrict__ vdelta) {
  __shared__ K kk[EVS_TILE];            // the tile's keys; key >> 2 identifies a (part, position) group
  __shared__ int8_t before[EVS_TILE];  // invalid before the group, at its first event
  __shared__ SegSum wtot[EVS_NT / 64];
  __shared__ int64_t s_ce;
  __shared__ int32_t s_ci;
  const int64_t t0 = (int64_t)blockIdx.x * EVS_TILE;
  const int tid = threadIdx.x;
  const int cnt = (int)min((int64_t)EVS_TILE, nev - t0);
  for (int j = tid; j < cnt; j += EVS_NT) kk[j] = ev[t0 + j];
  if (tid < 64) {
    // carry: the aggregates of the tiles before this one, back to the nearest
    // tile where a part starts (tile 0 always has one), 64 tiles per step
    const int l = lane_id();
    int64_t ce = 0;
    int32_t ci = 0;
    for (int64_t hi = blockIdx.x; hi > 0; hi -= 64) {
      const int64_t tt = hi - 1 - l;  // lane 0: the nearest tile
      const bool in = tt >= 0;
      const uint64_t fm = __ballot(in && agg_f[tt] != 0);
      const int stop = fm ? __ffsll((unsigned long long)fm) - 1 : 63;
      const bool take = in && l <= stop;
      ce += wave_sum<int64_t>(take ? agg_e[tt] : 0);
      ci += wave_sum<int32_t>(take ? agg_i[tt] : 0);
      if (fm) break;
    }
    if (l == 0) {
      s_ce = ce;
      s_ci = ci;
    }
  }
  __syncthreads();
  const int pshift = vshift - 2;
  // neighbours of the tile
  const uint64_t g_prev = t0 > 0 ? ((uint64_t)ev[t0 - 1] >> 2) : ~0ull;
  const uint64_t g_next = t0 + cnt < nev ? ((uint64_t)ev[t0 + cnt] >> 2) : ~0ull;
  int64_t dsv[EVS_IPT];
  int32_t div_[EVS_IPT];
  SegSum x{0, 0, 0};
  const int j0 = tid * EVS_IPT;
#pragma unroll
  for (int j = 0; j < EVS_IPT; ++j) {
    const int lj = j0 + j;
    dsv[j] = 0;
    div_[j] = 0;
    if (lj < cnt) {
      const uint64_t k = (uint64_t)kk[lj];
      const uint64_t gp = lj > 0 ? (uint64_t)kk[lj - 1] >> 2 : g_prev;
      const bool start = (t0 + lj == 0) || ((k >> 2) >> pshift) != (gp >> pshift);
      ev_delta<K>(k, vshift, qmask, seq, rho, size, dsv[j], div_[j]);
      x = seg_combine(x, SegSum{dsv[j], div_[j], start ? 1 : 0});
    }
  }
  SegSum run = seg_combine(SegSum{s_ce, s_ci, 0}, seg_block_exclusive<EVS_NT>(x, wtot));
  // inclusive part sums per item: the before-state at every group's first
  // event (to LDS) and the after-state at its last (bit j of after_bits)
  uint32_t after_bits = 0;
#pragma unroll
  for (int j = 0; j < EVS_IPT; ++j) {
    const int lj = j0 + j;
    if (lj < cnt) {
      const uint64_t g = (uint64_t)kk[lj] >> 2;
      const uint64_t gp = lj > 0 ? (uint64_t)kk[lj - 1] >> 2 : g_prev;
      const uint64_t gn = lj + 1 < cnt ? (uint64_t)kk[lj + 1] >> 2 : g_next;
      const bool pstart = (t0 + lj == 0) || (g >> pshift) != (gp >> pshift);
      run = seg_combine(run, SegSum{dsv[j], div_[j], pstart ? 1 : 0});
      const int p = (int)(g >> pshift);
      if (t0 + lj == 0 || g != gp) {
        const int64_t se = pstart ? 0 : run.e - dsv[j];
        const int64_t si = pstart ? 0 : (int64_t)run.i - div_[j];
        before[lj] = ((int64_t)psize[p] + se > omega || (int64_t)pinb[p] + si > delta) ? 1 : 0;
      }
      if (g != gn && ((int64_t)psize[p] + run.e > omega || (int64_t)pinb[p] + run.i > delta)) after_bits |= 1u << j;
    }
  }
  __syncthreads();
  const uint64_t g_first = (uint64_t)kk[0] >> 2, g_last = (uint64_t)kk[cnt - 1] >> 2;
#pragma unroll
  for (int j = 0; j < EVS_IPT; ++j) {
    const int lj = j0 + j;
    if (lj >= cnt) continue;
    const uint64_t g = (uint64_t)kk[lj] >> 2;
    const uint64_t gp = lj > 0 ? (uint64_t)kk[lj - 1] >> 2 : g_prev;
    const uint64_t gn = lj + 1 < cnt ? (uint64_t)kk[lj + 1] >> 2 : g_next;
    const bool first = (t0 + lj == 0) || g != gp;
    const bool last = g != gn;
    const int q = (int)(g & qmask);
    int d = 0;
    if (last) {
      const int after = (int)((after_bits >> j) & 1u);
      if (g == g_first && g == g_prev) {
        d = after;  // the group began in an earlier tile, which takes its before-state
      } else {
        int lo = 0, hi = lj;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (((uint64_t)kk[mid] >> 2) < g) lo = mid + 1;
          else hi = mid;
        }
        d = after - before[lo];
      }
    } else if (first && g == g_last && g == g_next) {
      d = -before[lj];  // the group ends in a later tile
    }
    if (d) atomicAdd(&vdelta[q], d);
  }
}

template <class K>
static void events_after_sort(const LevelView &L, const K *keys, int64_t nev, int vshift, uint64_t qmask,
                              const int32_t *rho, int32_t n_parts, int32_t omega, int32_t delta, RoundBufs &B,
                              hipStream_t s) {
  (void)n_parts;
  const int ntiles = (int)div_up(nev, EVS_TILE);
  if ((int64_t)ntiles > B.cap_tiles) throw Error(-7, "event tile buffer overflow");
  int64_t *agg_e = B.tile_e;
  int32_t *agg_i = B.tile_i, *agg_f = B.tile_i + ntiles;
  k_evs_tiles<K><<<ntiles, EVS_NT, 0, s>>>(keys, nev, vshift, qmask, B.seq, rho, L.size, agg_e, agg_i, agg_f);
  HGP_LAUNCH_CHECK();
  k_evs_trans<K><<<ntiles, EVS_NT, 0, s>>>(keys, nev, vshift, qmask, B.seq, rho, L.size, agg_e, agg_i, agg_f,
                                           B.psize, B.pinb, omega, delta, B.vdelta);
  HGP_LAUNCH_CHECK();
}

__global__ void k_init_invalid(const int32_t *__restrict__ psize, const int32_t *__restrict__ pinb, int32_t P,
                               int32_t omega, int32_t delta, int64_t *__restrict__ scal) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int bad = (p < P && (psize[p] > omega || pinb[p] > delta)) ? 1 : 0;
  bad = wave_sum(bad);
  if (lane_id() == 0 && bad) atomicAdd((unsigned long long *)&scal[SC_INVALID0], (unsigned long long)bad);
}

// Single workgroup: G(i) = prefix of g', viol(i) = viol(0) + prefix of the
// violation deltas, and i* = argmax over viol(i) = 0 of (G(i), i).
constexpr int FIN_NT = 1024;
__global__ __launch_bounds__(FIN_NT) void k_finish(const int32_t *__restrict__ gp, const int32_t *__restrict__ vdelta,
                                                   int64_t S, int64_t *__restrict__ G, int32_t *__restrict__ viol,
                                                   int64_t *__restrict__ scal, const int32_t *__restrict__ err) {
  __shared__ int64_t wsum[FIN_NT / 64];
  __shared__ int32_t wvs[FIN_NT / 64];
  __shared__ int64_t s_carry_g;
  __shared__ int32_t s_carry_v;
  __shared__ int64_t bestg[FIN_NT / 64];
  __shared__ int64_t besti[FIN_NT / 64];
  const int tid = threadIdx.x, w = tid >> 6, l = lane_id();
  if (tid == 0) {
    s_carry_g = 0;
    s_carry_v = (int32_t)scal[SC_INVALID0];
  }
  __syncthreads();
  int64_t my_g = 0, my_i = -1;
  for (int64_t c = 0; c <= S; c += FIN_NT) {
    const int64_t i = c + tid;
    const bool act = i <= S;
    const int64_t x = (act && i > 0) ? (int64_t)gp[i] : 0;
    const int32_t y = (act && i > 0) ? vdelta[i] : 0;
    const int64_t ix = wave_inclusive_scan(x);
    const int32_t iy = wave_inclusive_scan(y);
    if (l == 63) {
      wsum[w] = ix;
      wvs[w] = iy;
    }
    __syncthreads();
    int64_t og = s_carry_g;
    int32_t ov = s_carry_v;
    for (int q = 0; q < w; ++q) {
      og += wsum[q];
      ov += wvs[q];
    }
    const int64_t g = og + ix;
    const int32_t v = ov + iy;
    if (act) {
      G[i] = g;
      viol[i] = v;
      if (v == 0 && (my_i < 0 || g >= my_g)) {
        my_g = g;
        my_i = i;
      }
    }
    __syncthreads();
    if (tid == FIN_NT - 1) {
      int64_t tg = 0;
      int32_t tv = 0;
      for (int q = 0; q < FIN_NT / 64; ++q) {
        tg += wsum[q];
        tv += wvs[q];
      }
      s_carry_g += tg;
      s_carry_v += tv;
    }
    __syncthreads();
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t og = __shfl_xor(my_g, o, 64);
    const int64_t oi = __shfl_xor(my_i, o, 64);
    if (oi >= 0 && (my_i < 0 || og > my_g || (og == my_g && oi > my_i))) {
      my_g = og;
      my_i = oi;
    }
  }
  if (l == 0) {
    bestg[w] = my_g;
    besti[w] = my_i;
  }
  __syncthreads();
  if (tid == 0) {
    for (int q = 1; q < FIN_NT / 64; ++q)
      if (besti[q] >= 0 && (my_i < 0 || bestg[q] > my_g || (bestg[q] == my_g && besti[q] > my_i))) {
        my_g = bestg[q];
        my_i = besti[q];
      }
    scal[SC_ISTAR] = my_i;
    scal[SC_GSTAR] = my_i >= 0 ? my_g : 0;
    scal[SC_ERR] = *err;
  }
}


void evaluate_sequence(const LevelView &L, const int32_t *rho, int32_t n_parts, int32_t omega, int32_t delta,
                       int64_t S, RoundBufs &B, int32_t *err, DevBuf &scan_tmp, DevBuf &sort_tmp, hipStream_t s,
                       int64_t *istar, int64_t *gstar, int32_t *err_bits) {
  const int qbits = bits_for(S) > 0 ? bits_for(S) : 1;
  const int pbits = bits_for(n_parts > 1 ? n_parts - 1 : 1);
  const int vshift = qbits + 2;
  if (pbits + qbits + (L.big.huge_k ? 18 : 14) > 64) throw Error(-6, "sequence too long for the 64-bit event keys");
  // keys of at most 32 bits are packed and sorted as 32-bit words (half the
  // traffic): keys (as uint32) then holds them, keys2 is the sort's other half
  const int kbits = vshift + pbits;
  const bool narrow = kbits <= 32;
  uint32_t *k32 = reinterpret_cast<uint32_t *>(B.keys);
  fill_i32(B.vdelta, S + 1, 0, s);  // the round's scalars were reset by launch_round_reset
  if (S > 0) {
    KScope ks(kClsEvents, s);
    if (L.E > 0) {
      // inbound-count events per hedge into keys2 (one region of 2|e| per
      // hedge, 32-bit words when the packed keys fit), then packed into
      // keys[0 .. nin)
      auto emit = [&](auto *evpad, auto *ev) {
        using KP = std::remove_pointer_t<decltype(evpad)>;
        if (pbits <= EVN_PBITS && qbits <= EVN_QBITS)
          k_ev_wave32<KP><<<div_up(L.E, EVW_NT / 64), EVW_NT, 0, s>>>(L.hoff, L.hpin, L.E, L.hw, rho, B.dest,
                                                                      B.pos, B.pt, B.ptc, B.lam, qbits, B.contrib,
                                                                      evpad, B.evoff, B.scal, B.heavy);
        else
          k_ev_wave<KP><<<div_up(L.E, EVW_NT / 64), EVW_NT, 0, s>>>(L.hoff, L.hpin, L.E, L.hw, rho, B.dest, B.pos,
                                                                    B.pt, B.ptc, B.lam, qbits, B.contrib, evpad,
                                                                    B.evoff, B.scal, B.heavy);
        HGP_LAUNCH_CHECK();
        k_ev_block<KP><<<EVB_GRID, EVB_NT, 0, s>>>(L.hoff, L.hpin, L.hw, rho, B.dest, B.pos, B.pt, B.ptc, B.lam,
                                                   qbits, B.contrib, evpad, B.evoff, B.scal, B.heavy);
        HGP_LAUNCH_CHECK();
        if (L.big.huge_k) {
          k_ev_huge<KP><<<EVB_GRID, EVB_NT, 0, s>>>(L.hoff, L.hpin, L.hw, rho, B.dest, B.pos, B.pt, B.ptc, B.lam,
                                                    qbits, B.contrib, evpad, B.evoff, B.scal, B.heavy,
                                                    L.big.huge_k, L.big.huge_i);
          HGP_LAUNCH_CHECK();
        }
        scan_i64(B.evoff, B.evoff, (int64_t)L.E + 1, nullptr, scan_tmp, s);
        k_ev_compact<KP><<<div_up((int64_t)L.E, 4), 256, 0, s>>>(L.hoff, L.E, B.evoff, evpad, ev);
        HGP_LAUNCH_CHECK();
      };
      if (narrow) emit(reinterpret_cast<uint32_t *>(B.keys2), k32);
      else emit(B.keys2, B.keys);
    }
    k_move_gain<<<div_up(S, 4), 256, 0, s>>>(B.seq, S, L.ioff, L.perm, B.contrib, B.gp);
    HGP_LAUNCH_CHECK();
  }
  HGP_HIP(hipMemcpyAsync(B.hbox, B.evoff + L.E, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HGP_HIP(hipStreamSynchronize(s));
  const int64_t nin = B.hbox[0];
  const int64_t nev = nin + 2 * S;
  if (nev > B.cap_events) throw Error(-7, "event buffer overflow");
  add_units(kClsEvents, 16 * nev);  // algorithmic bytes: an 8-byte event key written and read once
  if (S > 0) {
    if (narrow)
      k_size_events<uint32_t><<<div_up(S, 256), 256, 0, s>>>(B.seq, S, rho, B.dest, vshift, k32, nin);
    else
      k_size_events<uint64_t><<<div_up(S, 256), 256, 0, s>>>(B.seq, S, rho, B.dest, vshift, B.keys, nin);
    HGP_LAUNCH_CHECK();
  }
  k_init_invalid<<<div_up(n_parts > 0 ? n_parts : 1, 256), 256, 0, s>>>(B.psize, B.pinb, n_parts, omega, delta,
                                                                         B.scal);
  HGP_LAUNCH_CHECK();
  if (narrow) {
    // the two type bits need no order: only whole (part, position) groups
    // are read after the sort
    sort_keys32(k32, reinterpret_cast<uint32_t *>(B.keys2), nev, kbits, sort_tmp, s, 2);
  } else {
    sort_keys(B.keys, B.keys2, nev, kbits, sort_tmp, s);
  }
  {
    KScope ks(kClsEvents, s);
    const uint64_t qmask = (1ull << qbits) - 1ull;
    if (nev > 0) {
      if (narrow)
        events_after_sort<uint32_t>(L, k32, nev, vshift, qmask, rho, n_parts, omega, delta, B, s);
      else
        events_after_sort<uint64_t>(L, B.keys, nev, vshift, qmask, rho, n_parts, omega, delta, B, s);
    }
    k_finish<<<1, FIN_NT, 0, s>>>(B.gp, B.vdelta, S, B.G, B.viol, B.scal, err);
    HGP_LAUNCH_CHECK();
  }
  // the result and the error bits (copied beside it by k_finish) in one copy
  HGP_HIP(hipMemcpyAsync(B.hbox, B.scal + SC_ISTAR, (SC_ERR - SC_ISTAR + 1) * sizeof(int64_t),
                         hipMemcpyDeviceToHost, s));
  HGP_HIP(hipStreamSynchronize(s));
  *istar = B.hbox[0];
  *gstar = B.hbox[SC_GSTAR - SC_ISTAR];
  *err_bits = (int32_t)B.hbox[SC_ERR - SC_ISTAR];
}

}  // namespace hgp
