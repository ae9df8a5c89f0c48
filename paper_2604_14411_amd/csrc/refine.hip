// Refinement kernels (Sec. IV): part tables, in-isolation proposals (Eq. 3),
// the move sequence, exact in-sequence gains, event-based constraint
// validity per prefix, the best valid prefix, projection and Eq. 1.
#include "coarsen.hpp"

namespace hgp {

constexpr int PT_NT = 256;
constexpr int PROP_NT = 256;
constexpr int PROP_LDS_BYTES = 64 * 1024;

enum { SC_S = 0, SC_EVENTS = 1, SC_ISTAR = 2, SC_GSTAR = 3, SC_INVALID0 = 4, SC_HEAVY = 5 };

__device__ __forceinline__ int lower_bound_u32(const uint32_t *a, int n, uint32_t x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Look up (pins, pins_in) of part p in hedge e's sorted part table.
__device__ __forceinline__ int2 pt_lookup(const int2 *__restrict__ pt, const int32_t *__restrict__ ptin, int b,
                                          int len, int p) {
  int lo = 0, hi = len;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (pt[b + mid].x < p) lo = mid + 1;
    else hi = mid;
  }
  if (lo < len && pt[b + lo].x == p) return make_int2(pt[b + lo].y, ptin[b + lo]);
  return make_int2(0, 0);
}

// ---------------------------------------------------------------------------
// part table: pins(p,e), pins_in(p,e) (Sec. IV-B, counting pins per partition)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(PT_NT) void k_part_table(const int32_t *__restrict__ hoff,
                                                      const uint32_t *__restrict__ hpin,
                                                      const int32_t *__restrict__ rho, int2 *__restrict__ pt,
                                                      int32_t *__restrict__ ptin, int32_t *__restrict__ lam,
                                                      int32_t *__restrict__ pinb, int32_t *err,
                                                      const int32_t *__restrict__ list) {
  __shared__ uint32_t key[kSegCap];
  __shared__ int32_t first[kSegCap];
  __shared__ int32_t tmp[PT_NT / 64 + 1];
  const int e = list[blockIdx.x];
  const int b = hoff[e];
  const int len = hoff[e + 1] - b;
  if (len <= 0 || len > kSegCap) {
    if (threadIdx.x == 0) {
      lam[e] = 0;
      if (len > kSegCap) atomicOr(err, kErrInternal);
    }
    return;
  }
  const int np = next_pow2(len);
  for (int i = threadIdx.x; i < np; i += PT_NT) {
    uint32_t k = 0xffffffffu;
    if (i < len) {
      const uint32_t x = hpin[b + i];
      k = ((uint32_t)rho[x & kIdMask] << 1) | (x >> 31);
    }
    key[i] = k;
  }
  __syncthreads();
  block_bitonic_sort<uint32_t, PT_NT>(key, np);
  for (int i = threadIdx.x; i < len; i += PT_NT) first[i] = (i == 0 || (key[i - 1] >> 1) != (key[i] >> 1)) ? 1 : 0;
  __syncthreads();
  const int runs = block_exclusive_scan<int32_t, PT_NT>(first, len, tmp);
  for (int i = threadIdx.x; i < len; i += PT_NT) {
    if (i == 0 || (key[i - 1] >> 1) != (key[i] >> 1)) {
      const uint32_t part = key[i] >> 1;
      const int end = lower_bound_u32(key, len, (part + 1) << 1);
      const int dst0 = lower_bound_u32(key, len, (part << 1) | 1u);
      const int r = first[i];
      pt[b + r] = make_int2((int)part, end - i);
      ptin[b + r] = end - dst0;
      if (end > dst0) atomicAdd(&pinb[part], 1);
    }
  }
  if (threadIdx.x == 0) lam[e] = runs;
}

__global__ void k_part_size(const int32_t *__restrict__ rho, const int32_t *__restrict__ size, int32_t N,
                            int32_t *__restrict__ psize) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < N) atomicAdd(&psize[rho[n]], size[n]);
}

void launch_part_table(const LevelView &L, const int32_t *rho, int32_t n_parts, RoundBufs &B, int32_t *err,
                       hipStream_t s) {
  fill_i32(B.pinb, n_parts, 0, s);
  fill_i32(B.psize, n_parts, 0, s);
  KScope ks(2, s);
  add_units(2, 0);
  if (L.E > 0) {
    launch_part_table_wave(L.hoff, L.hpin, L.E, rho, B.pt, B.ptin, B.lam, B.pinb, s);
    if (L.big.n > 0) {
      k_part_table<<<L.big.n, PT_NT, 0, s>>>(L.hoff, L.hpin, rho, B.pt, B.ptin, B.lam, B.pinb, err, L.big.list);
      HGP_LAUNCH_CHECK();
    }
  }
  if (L.n > 0 && L.size) {
    k_part_size<<<div_up(L.n, 256), 256, 0, s>>>(rho, L.size, L.n, B.psize);
    HGP_LAUNCH_CHECK();
  }
}

// ---------------------------------------------------------------------------
// proposals (Eq. 3)
// ---------------------------------------------------------------------------
// One workgroup per node n in part p_s (node list[t], or t when list is
// null; grid-stride over *count nodes).  saving(n) is summed first by one
// lookup of p_s per hedge; if it is zero no move can have positive gain
// (loss >= 0) and the node is done.  Otherwise every part table entry of
// every hedge of I(n) adds w(e) to conn[p] in LDS; then
//   gain(n,p) = saving - loss(n,p) = saving - total(n) + conn[p]
// and the best part by (gain, id) among those with size(p)+size(n) <= Omega
// is kept if gain > 0.
template <int NT>
__global__ __launch_bounds__(NT) void k_propose(const int32_t *__restrict__ list, const int64_t *__restrict__ count,
                                                int32_t N, const int32_t *__restrict__ ioff,
                                                const uint32_t *__restrict__ inc, const int32_t *__restrict__ hoff,
                                                const int2 *__restrict__ pt, const int32_t *__restrict__ ptin,
                                                const int32_t *__restrict__ lam, const int32_t *__restrict__ hw,
                                                const int32_t *__restrict__ rho, const int32_t *__restrict__ size,
                                                const int32_t *__restrict__ psize, const int32_t *__restrict__ total,
                                                int32_t n_parts, int32_t omega, int32_t words,
                                                int32_t *__restrict__ dest, int32_t *__restrict__ gain,
                                                unsigned long long *__restrict__ units) {
  extern __shared__ uint32_t conn[];
  __shared__ int64_t red[NT / 64];
  __shared__ int32_t redp[NT / 64];
  __shared__ int64_t s_saving;
  __shared__ int32_t tbl[NT / 64 * 192];
  const int tid = threadIdx.x, w = tid >> 6, l = lane_id();
  const int64_t cnt_nodes = list ? *count : (int64_t)N;
  int64_t streamed = 0;
  for (int64_t t = blockIdx.x; t < cnt_nodes; t += gridDim.x) {
    const int n = list ? list[t] : (int)t;
    const int ps = rho[n];
    const int i0 = ioff[n], i1 = ioff[n + 1];
    // saving(n)
    int64_t sav = 0;
    for (int i = i0 + tid; i < i1; i += NT) {
      const int e = (int)(inc[i] & kIdMask);
      const int2 c = pt_lookup(pt, ptin, hoff[e], lam[e], ps);
      if (c.x == 1) sav += hw[e];
    }
    sav = wave_sum(sav);
    if (l == 0) red[w] = sav;
    __syncthreads();
    if (tid == 0) {
      int64_t tt = 0;
      for (int q = 0; q < NT / 64; ++q) tt += red[q];
      s_saving = tt;
    }
    __syncthreads();
    const int64_t saving = s_saving;
    int bp = -1;
    int64_t bg = 0;
    if (saving > 0) {
      const int64_t tot = total[n];
      const int64_t sn = size[n];
      for (int lo = 0; lo < n_parts; lo += words) {
        const int span = min(words, n_parts - lo);
        for (int i = tid; i < span; i += NT) conn[i] = 0u;
        __syncthreads();
        streamed += stream_segments<NT / 64, 4, false, int32_t>(
            i0, i1, inc, hoff, lam, hw, tbl, [&](int j) { return pt[j].x; },
            [&](int32_t p, uint32_t info) {
              const uint32_t rel = (uint32_t)(p - lo);
              if (rel < (uint32_t)span) atomicAdd(&conn[rel], info & kIdMask);
            });
        __syncthreads();
        for (int i = tid; i < span; i += NT) {
          const uint32_t c = conn[i];
          if (!c) continue;
          const int p = lo + i;
          if (p == ps) continue;
          const int64_t g = saving - tot + (int64_t)c;
          if (g > 0 && (g > bg || (g == bg && p > bp)) && (int64_t)psize[p] + sn <= omega) {
            bg = g;
            bp = p;
          }
        }
        __syncthreads();
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const int64_t og = __shfl_xor(bg, o, 64);
      const int op = __shfl_xor(bp, o, 64);
      if (op >= 0 && (bp < 0 || og > bg || (og == bg && op > bp))) {
        bg = og;
        bp = op;
      }
    }
    if (l == 0) {
      red[w] = bg;
      redp[w] = bp;
    }
    __syncthreads();
    if (tid == 0) {
      for (int q = 1; q < NT / 64; ++q) {
        const int op = redp[q];
        const int64_t og = red[q];
        if (op >= 0 && (bp < 0 || og > bg || (og == bg && op > bp))) {
          bg = og;
          bp = op;
        }
      }
      dest[n] = bp;
      gain[n] = bp >= 0 ? (int32_t)bg : 0;
    }
    __syncthreads();
  }
  add_wave_units(units, streamed);
}

constexpr int PROP_GRID = 8192;

void launch_propose(const LevelView &L, const int32_t *total, const int32_t *rho, int32_t n_parts, int32_t omega,
                    RoundBufs &B, hipStream_t s, const int32_t *list, const int64_t *count) {
  if (L.n <= 0) return;
  const int max_words = PROP_LDS_BYTES / 4;
  const int words = n_parts < max_words ? (n_parts > 0 ? n_parts : 1) : max_words;
  KScope ks(1, s);
  const int grid = list ? (L.n < PROP_GRID ? L.n : PROP_GRID) : L.n;
  k_propose<PROP_NT><<<grid, PROP_NT, (size_t)words * 4, s>>>(list, count, L.n, L.ioff, L.inc, L.hoff, B.pt, B.ptin,
                                                             B.lam, L.hw, rho, L.size, B.psize, total, n_parts, omega,
                                                             words, B.dest, B.gain, units_ptr(1));
  HGP_LAUNCH_CHECK();
}

// Proposals carried over from the next coarser level: a node whose cluster
// was not split there keeps that cluster's proposal (same parts, sizes and
// per-hedge part sets, hence the same Eq. 3 values); split nodes are queued.
__global__ void k_prop_gather(int32_t n, const int32_t *__restrict__ match, const int32_t *__restrict__ gamma,
                              const int32_t *__restrict__ cdest, const int32_t *__restrict__ cgain,
                              int32_t *__restrict__ dest, int32_t *__restrict__ gain, int32_t *__restrict__ list,
                              int64_t *__restrict__ cnt) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (match[v] == v) {
    const int c = gamma[v];
    dest[v] = cdest[c];
    gain[v] = cgain[c];
  } else {
    list[atomicAdd((unsigned long long *)cnt, 1ull)] = (int32_t)v;
  }
}

void launch_prop_gather(int32_t n, const int32_t *match, const int32_t *gamma, const int32_t *cdest,
                        const int32_t *cgain, RoundBufs &B, int32_t *list, int64_t *cnt, hipStream_t s) {
  fill_i64(cnt, 1, 0, s);
  if (n <= 0) return;
  k_prop_gather<<<div_up(n, 256), 256, 0, s>>>(n, match, gamma, cdest, cgain, B.dest, B.gain, list, cnt);
  HGP_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// sequence: moves sorted by (gain, id) descending (Sec. IV-A)
// ---------------------------------------------------------------------------
__global__ void k_move_flags(const int32_t *__restrict__ dest, int32_t N, int32_t *__restrict__ flag,
                             int32_t *__restrict__ pos) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < N) {
    flag[n] = dest[n] >= 0 ? 1 : 0;
    pos[n] = 0;
  }
}

__global__ void k_move_keys(const int32_t *__restrict__ dest, const int32_t *__restrict__ gain,
                            const int32_t *__restrict__ off, int32_t N, int idbits, uint64_t *__restrict__ keys) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < N && dest[n] >= 0)
    keys[off[n]] = ((uint64_t)(uint32_t)(0x7fffffff - gain[n]) << idbits) | (uint64_t)(uint32_t)(N - 1 - n);
}

__global__ void k_seq_from_keys(const uint64_t *__restrict__ keys, int64_t S, int32_t N, int idbits,
                                int32_t *__restrict__ seq, int32_t *__restrict__ pos) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < S) {
    const int n = N - 1 - (int)(keys[i] & ((1ull << idbits) - 1ull));
    seq[i] = n;
    pos[n] = (int32_t)(i + 1);
  }
}

constexpr int SMALL_SORT_NT = 1024;
constexpr int SMALL_SORT_CAP = 8192;

__global__ __launch_bounds__(SMALL_SORT_NT) void k_small_sort(uint64_t *keys, int n) {
  __shared__ uint64_t s[SMALL_SORT_CAP];
  const int np = next_pow2(n);
  for (int i = threadIdx.x; i < np; i += SMALL_SORT_NT) s[i] = i < n ? keys[i] : ~0ull;
  __syncthreads();
  block_bitonic_sort<uint64_t, SMALL_SORT_NT>(s, np);
  for (int i = threadIdx.x; i < n; i += SMALL_SORT_NT) keys[i] = s[i];
}

static void sort_keys(uint64_t *keys, uint64_t *alt, int64_t n, int bits, DevBuf &sort_tmp, hipStream_t s) {
  if (n <= 1) return;
  KScope ks(6, s);
  add_units(6, n);
  if (n <= SMALL_SORT_CAP) {
    k_small_sort<<<1, SMALL_SORT_NT, 0, s>>>(keys, (int)n);
    HGP_LAUNCH_CHECK();
  } else {
    radix_sort_u64(keys, alt, nullptr, nullptr, n, bits, sort_tmp, s);
  }
}

static int bits_for(int64_t x) {
  int b = 0;
  while (b < 63 && (int64_t(1) << b) <= x) ++b;
  return b;
}

int64_t build_sequence(const LevelView &L, RoundBufs &B, DevBuf &scan_tmp, DevBuf &sort_tmp, hipStream_t s) {
  const int32_t N = L.n;
  if (N <= 0) return 0;
  k_move_flags<<<div_up(N, 256), 256, 0, s>>>(B.dest, N, B.flag, B.pos);
  HGP_LAUNCH_CHECK();
  scan_i32(B.flag, B.flag, N, reinterpret_cast<int32_t *>(B.scal + SC_S), scan_tmp, s);
  int32_t S32 = 0;
  HGP_HIP(hipMemcpyAsync(&S32, B.scal + SC_S, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HGP_HIP(hipStreamSynchronize(s));
  const int64_t S = S32;
  if (S == 0) return 0;
  const int idbits = bits_for(N - 1) > 0 ? bits_for(N - 1) : 1;
  k_move_keys<<<div_up(N, 256), 256, 0, s>>>(B.dest, B.gain, B.flag, N, idbits, B.keys);
  HGP_LAUNCH_CHECK();
  sort_keys(B.keys, B.keys2, S, 31 + idbits, sort_tmp, s);
  k_seq_from_keys<<<div_up(S, 256), 256, 0, s>>>(B.keys, S, N, idbits, B.seq, B.pos);
  HGP_LAUNCH_CHECK();
  return S;
}

// ---------------------------------------------------------------------------
// in-sequence gains and inbound transitions, one workgroup per hedge
// ---------------------------------------------------------------------------
// For the moving pins of hedge e, every move i of node v (p_s -> p_d)
// yields a source event on (p_s, i) and a destination event on (p_d, i).
// Sorted by (part, position), an exclusive prefix within each part gives
// pins_{i-1}(p, e) = pins_0(p, e) + (earlier arrivals - earlier departures).
// The exact change of Eq. 1 caused by move i on hedge e is
//   +w(e) if pins_{i-1}(p_s, e) = 1   (p_s leaves the hedge)
//   -w(e) if pins_{i-1}(p_d, e) = 0   (p_d joins the hedge)
// summed into g'(i).  Destination pins do the same on pins_in(p, e) and emit
// an inbound-count event (p, i, -1) on a 1 -> 0 transition of p_s and
// (p, i, +1) on a 0 -> 1 transition of p_d.
//
// Event key layout: part << 32 | position << 2 | role << 1 | is_dst
// (role 0 = source, 1 = destination).  Validity events use
// part << 32 | position << 2 | type (type 0: inbound -1, 1: inbound +1,
// 2: size change).
// Part table of the hedge staged in LDS (parts ascending; counts packed as
// pins | pins_in << 16, both <= 4096).
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

template <int CAPEV, int PTCAP>
__device__ void seq_events_hedge(int e, int moving, const int32_t *__restrict__ hoff,
                                 const uint32_t *__restrict__ hpin, const int32_t *__restrict__ hw,
                                 const int32_t *__restrict__ rho, const int32_t *__restrict__ dest,
                                 const int32_t *__restrict__ pos, const int2 *__restrict__ pt,
                                 const int32_t *__restrict__ ptin, const int32_t *__restrict__ lam, int pshift,
                                 int32_t *__restrict__ gp, uint64_t *__restrict__ ev, int32_t *__restrict__ pcnt,
                                 int64_t *__restrict__ scal, uint64_t *key, int32_t *dl, int32_t *tmp,
                                 int32_t *s_cnt, int64_t *s_base, int32_t *sp, uint32_t *sc) {
  const int b = hoff[e];
  const int len = hoff[e + 1] - b;
  if (threadIdx.x == 0) *s_cnt = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < len; i += PT_NT) {
    const uint32_t x = hpin[b + i];
    const int v = (int)(x & kIdMask);
    const int q = pos[v];
    if (q > 0) {
      const int slot = atomicAdd(s_cnt, 2);
      const uint64_t d = x >> 31;
      key[slot] = ((uint64_t)(uint32_t)rho[v] << 32) | ((uint64_t)q << 2) | d;
      key[slot + 1] = ((uint64_t)(uint32_t)dest[v] << 32) | ((uint64_t)q << 2) | 2ull | d;
    }
  }
  const int nev = 2 * moving;
  const int np = next_pow2(nev);
  __syncthreads();
  for (int i = nev + threadIdx.x; i < np; i += PT_NT) key[i] = ~0ull;
  __syncthreads();
  block_bitonic_sort<uint64_t, PT_NT>(key, np);
  // deltas: low 16 bits pins, high 16 bits pins_in (both signed, |.| <= 4096)
  for (int i = threadIdx.x; i < nev; i += PT_NT) {
    const uint64_t k = key[i];
    const int sgn = (k & 2ull) ? 1 : -1;
    dl[i] = sgn + ((k & 1ull) ? sgn * 65536 : 0);
  }
  __syncthreads();
  block_exclusive_scan<int32_t, PT_NT>(dl, nev, tmp);
  if (threadIdx.x == 0) *s_cnt = 0;
  __syncthreads();
  const int32_t we = hw[e];
  const int plen = lam[e];
  const bool staged = plen <= PTCAP;
  if (staged) {
    for (int i = threadIdx.x; i < plen; i += PT_NT) {
      const int2 x = pt[b + i];
      sp[i] = x.x;
      sc[i] = (uint32_t)x.y | ((uint32_t)ptin[b + i] << 16);
    }
  }
  __syncthreads();
  // pass 1: gains, and count inbound events; pass 2: write inbound events
  int my_events = 0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int i = threadIdx.x; i < nev; i += PT_NT) {
      const uint64_t k = key[i];
      if (pass == 1 && !(k & 1ull)) continue;
      const uint32_t part = (uint32_t)(k >> 32);
      const int q = (int)((k >> 2) & 0x3fffffffull);
      const bool is_dst_role = (k & 2ull) != 0;
      int lo = 0, hi = i;  // first event of this part
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((uint32_t)(key[mid] >> 32) < part) lo = mid + 1;
        else hi = mid;
      }
      const int32_t pre = dl[i] - dl[lo];
      const int32_t pre_pins = (int32_t)(int16_t)(pre & 0xffff);
      const int32_t pre_in = (pre - pre_pins) >> 16;
      const int2 c0 = staged ? pt_lookup_lds(sp, sc, plen, (int)part) : pt_lookup(pt, ptin, b, plen, (int)part);
      if (pass == 0) {
        const int before = c0.x + pre_pins;
        if (!is_dst_role && before == 1) atomicAdd(&gp[q], we);
        if (is_dst_role && before == 0) atomicAdd(&gp[q], -we);
      }
      if (k & 1ull) {
        const int bin = c0.y + pre_in;
        int type = -1;
        if (!is_dst_role && bin == 1) type = 0;
        if (is_dst_role && bin == 0) type = 1;
        if (type >= 0) {
          if (pass == 0) {
            ++my_events;
          } else {
            const int64_t slot = *s_base + atomicAdd(s_cnt, 1);
            ev[slot] = ((uint64_t)part << pshift) | ((uint64_t)q << 2) | (uint64_t)type;
            atomicAdd(&pcnt[part], 1);
          }
        }
      }
    }
    if (pass == 0) {
      my_events = wave_sum(my_events);
      if (lane_id() == 0 && my_events) atomicAdd(s_cnt, my_events);
      __syncthreads();
      if (threadIdx.x == 0) {
        const int c = *s_cnt;
        *s_base = c ? (int64_t)atomicAdd((unsigned long long *)&scal[SC_EVENTS], (unsigned long long)c) : 0;
        *s_cnt = 0;
      }
      __syncthreads();
    }
  }
  __syncthreads();
}

__device__ __forceinline__ int count_moving(const uint32_t *__restrict__ hpin, const int32_t *__restrict__ pos,
                                            int b, int len, int32_t *s_cnt) {
  if (threadIdx.x == 0) *s_cnt = 0;
  __syncthreads();
  int mine = 0;
  for (int i = threadIdx.x; i < len; i += PT_NT) mine += pos[hpin[b + i] & kIdMask] > 0 ? 1 : 0;
  mine = wave_sum(mine);
  if (lane_id() == 0 && mine) atomicAdd(s_cnt, mine);
  __syncthreads();
  const int m = *s_cnt;
  __syncthreads();
  return m;
}

constexpr int EV_LIGHT = 512;  // moving pins per hedge handled by the small-LDS kernel

// One workgroup per hedge; hedges with more than EV_LIGHT moving pins are
// queued for k_seq_events_heavy.
__global__ __launch_bounds__(PT_NT) void k_seq_events_light(
    const int32_t *__restrict__ hoff, const uint32_t *__restrict__ hpin, const int32_t *__restrict__ hw,
    const int32_t *__restrict__ rho, const int32_t *__restrict__ dest, const int32_t *__restrict__ pos,
    const int2 *__restrict__ pt, const int32_t *__restrict__ ptin, const int32_t *__restrict__ lam, int pshift,
    int32_t *__restrict__ gp, uint64_t *__restrict__ ev, int32_t *__restrict__ pcnt, int64_t *__restrict__ scal,
    int32_t *__restrict__ heavy) {
  __shared__ uint64_t key[2 * EV_LIGHT];
  __shared__ int32_t dl[2 * EV_LIGHT];
  __shared__ int32_t sp[1024];
  __shared__ uint32_t sc[1024];
  __shared__ int32_t tmp[PT_NT / 64 + 1];
  __shared__ int32_t s_cnt;
  __shared__ int64_t s_base;
  const int e = blockIdx.x;
  const int moving = count_moving(hpin, pos, hoff[e], hoff[e + 1] - hoff[e], &s_cnt);
  if (moving == 0) return;
  if (moving > EV_LIGHT) {
    if (threadIdx.x == 0) heavy[atomicAdd((unsigned long long *)&scal[SC_HEAVY], 1ull)] = e;
    return;
  }
  seq_events_hedge<2 * EV_LIGHT, 1024>(e, moving, hoff, hpin, hw, rho, dest, pos, pt, ptin, lam, pshift, gp, ev,
                                       pcnt, scal, key, dl, tmp, &s_cnt, &s_base, sp, sc);
}

constexpr int EV_HEAVY_GRID = 512;

__global__ __launch_bounds__(PT_NT) void k_seq_events_heavy(
    const int32_t *__restrict__ hoff, const uint32_t *__restrict__ hpin, const int32_t *__restrict__ hw,
    const int32_t *__restrict__ rho, const int32_t *__restrict__ dest, const int32_t *__restrict__ pos,
    const int2 *__restrict__ pt, const int32_t *__restrict__ ptin, const int32_t *__restrict__ lam, int pshift,
    int32_t *__restrict__ gp, uint64_t *__restrict__ ev, int32_t *__restrict__ pcnt, int64_t *__restrict__ scal,
    const int32_t *__restrict__ heavy) {
  __shared__ uint64_t key[2 * kSegCap];
  __shared__ int32_t dl[2 * kSegCap];
  __shared__ int32_t sp[kSegCap];
  __shared__ uint32_t sc[kSegCap];
  __shared__ int32_t tmp[PT_NT / 64 + 1];
  __shared__ int32_t s_cnt;
  __shared__ int64_t s_base;
  const int64_t nh = scal[SC_HEAVY];
  for (int64_t t = blockIdx.x; t < nh; t += gridDim.x) {
    const int e = heavy[t];
    const int moving = count_moving(hpin, pos, hoff[e], hoff[e + 1] - hoff[e], &s_cnt);
    seq_events_hedge<2 * kSegCap, kSegCap>(e, moving, hoff, hpin, hw, rho, dest, pos, pt, ptin, lam, pshift, gp, ev,
                                           pcnt, scal, key, dl, tmp, &s_cnt, &s_base, sp, sc);
  }
}

// size events: (p_s, i, size) and (p_d, i, size) for every move i
__global__ void k_size_events(const int32_t *__restrict__ seq, int64_t S, const int32_t *__restrict__ rho,
                              const int32_t *__restrict__ dest, int pshift, uint64_t *__restrict__ ev, int64_t base,
                              int32_t *__restrict__ pcnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  const int v = seq[i];
  const uint64_t q = (uint64_t)(i + 1);
  const uint32_t ps = (uint32_t)rho[v], pd = (uint32_t)dest[v];
  ev[base + 2 * i] = ((uint64_t)ps << pshift) | (q << 2) | 2ull;
  ev[base + 2 * i + 1] = ((uint64_t)pd << pshift) | (q << 2) | 2ull;
  atomicAdd(&pcnt[ps], 1);
  atomicAdd(&pcnt[pd], 1);
}

__global__ void k_init_invalid(const int32_t *__restrict__ psize, const int32_t *__restrict__ pinb, int32_t P,
                               int32_t omega, int32_t delta, int64_t *__restrict__ scal) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int bad = (p < P && (psize[p] > omega || pinb[p] > delta)) ? 1 : 0;
  bad = wave_sum(bad);
  if (lane_id() == 0 && bad) atomicAdd((unsigned long long *)&scal[SC_INVALID0], (unsigned long long)bad);
}

// One wave per part: walk the part's events in position order, keep the
// running size and inbound count, and at the last event of every position
// compare validity with the previous position's; a valid -> invalid change
// adds +1 to viol at that position, invalid -> valid adds -1.
__global__ void k_part_validity(const uint64_t *__restrict__ ev, const int32_t *__restrict__ poff, int32_t P,
                                const int32_t *__restrict__ psize, const int32_t *__restrict__ pinb,
                                const int32_t *__restrict__ seq, const int32_t *__restrict__ rho,
                                const int32_t *__restrict__ size, int32_t omega, int32_t delta, uint64_t qmask,
                                int32_t *__restrict__ vdelta) {
  const int p = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (p >= P) return;
  const int l = lane_id();
  const int b = poff[p], en = poff[p + 1];
  if (b == en) return;
  int64_t run_size = psize[p];
  int64_t run_inb = pinb[p];
  bool prev_valid = run_size <= omega && run_inb <= delta;
  const uint64_t lt = (l == 0) ? 0ull : ((~0ull) >> (64 - l));
  for (int c = b; c < en; c += 64) {
    const int i = c + l;
    const bool act = i < en;
    int64_t ds = 0, di = 0;
    int q = -1;
    if (act) {
      const uint64_t k = ev[i];
      q = (int)((k >> 2) & qmask);
      const int type = (int)(k & 3ull);
      if (type == 0) di = -1;
      else if (type == 1) di = 1;
      else {
        const int v = seq[q - 1];
        ds = rho[v] == p ? -(int64_t)size[v] : (int64_t)size[v];
      }
    }
    const int64_t cs = wave_inclusive_scan(ds) + run_size;
    const int64_t ci = wave_inclusive_scan(di) + run_inb;
    int qn = __shfl_down(q, 1, 64);
    if (l == 63) qn = (i + 1 < en) ? (int)((ev[i + 1] >> 2) & qmask) : -1;
    const bool last = act && (i + 1 >= en || qn != q);
    const bool valid = cs <= omega && ci <= delta;
    const uint64_t lastmask = __ballot(last);
    const uint64_t validmask = __ballot(last && valid);
    if (last) {
      const uint64_t below = lastmask & lt;
      const bool pv = below ? ((validmask >> (63 - __clzll(below))) & 1ull) != 0 : prev_valid;
      if (pv != valid) atomicAdd(&vdelta[q], valid ? -1 : 1);
    }
    if (lastmask) prev_valid = ((validmask >> (63 - __clzll(lastmask))) & 1ull) != 0;
    run_size = __shfl(cs, 63, 64);
    run_inb = __shfl(ci, 63, 64);
  }
}

// Single workgroup: G(i) = prefix of g', viol(i) = viol(0) + prefix of the
// violation deltas, and i* = argmax over viol(i) = 0 of (G(i), i).
constexpr int FIN_NT = 1024;
__global__ __launch_bounds__(FIN_NT) void k_finish(const int32_t *__restrict__ gp, const int32_t *__restrict__ vdelta,
                                                   int64_t S, int64_t *__restrict__ G, int32_t *__restrict__ viol,
                                                   int64_t *__restrict__ scal) {
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
  }
}

void evaluate_sequence(const LevelView &L, const int32_t *rho, int32_t n_parts, int32_t omega, int32_t delta,
                       int64_t S, RoundBufs &B, int32_t *err, DevBuf &scan_tmp, DevBuf &sort_tmp, hipStream_t s,
                       int64_t *istar, int64_t *gstar) {
  fill_i32(B.gp, S + 1, 0, s);
  fill_i32(B.vdelta, S + 1, 0, s);
  fill_i32(B.pcnt, (int64_t)n_parts + 1, 0, s);
  fill_i64(B.scal + SC_EVENTS, 1, 0, s);
  fill_i64(B.scal + SC_INVALID0, 1, 0, s);
  const int posbits = bits_for(S);
  const int pshift = posbits + 2;
  fill_i64(B.scal + SC_HEAVY, 1, 0, s);
  if (S > 0 && L.E > 0) {
    KScope ks(3, s);
    k_seq_events_light<<<L.E, PT_NT, 0, s>>>(L.hoff, L.hpin, L.hw, rho, B.dest, B.pos, B.pt, B.ptin, B.lam, pshift,
                                            B.gp, B.keys, B.pcnt, B.scal, B.heavy);
    HGP_LAUNCH_CHECK();
    k_seq_events_heavy<<<EV_HEAVY_GRID, PT_NT, 0, s>>>(L.hoff, L.hpin, L.hw, rho, B.dest, B.pos, B.pt, B.ptin,
                                                       B.lam, pshift, B.gp, B.keys, B.pcnt, B.scal, B.heavy);
    HGP_LAUNCH_CHECK();
  }
  int64_t nin = 0;
  HGP_HIP(hipMemcpyAsync(&nin, B.scal + SC_EVENTS, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HGP_HIP(hipStreamSynchronize(s));
  const int64_t nev = nin + 2 * S;
  if (nev > B.cap_events) throw Error(-7, "event buffer overflow");
  if (S > 0) {
    k_size_events<<<div_up(S, 256), 256, 0, s>>>(B.seq, S, rho, B.dest, pshift, B.keys, nin, B.pcnt);
    HGP_LAUNCH_CHECK();
  }
  k_init_invalid<<<div_up(n_parts > 0 ? n_parts : 1, 256), 256, 0, s>>>(B.psize, B.pinb, n_parts, omega, delta,
                                                                         B.scal);
  HGP_LAUNCH_CHECK();
  int pbits = bits_for(n_parts > 0 ? n_parts - 1 : 0);
  if (pbits < 1) pbits = 1;
  sort_keys(B.keys, B.keys2, nev, pshift + pbits, sort_tmp, s);
  scan_i32(B.pcnt, B.pcnt, (int64_t)n_parts + 1, nullptr, scan_tmp, s);
  if (n_parts > 0 && nev > 0) {
    k_part_validity<<<div_up((int64_t)n_parts * 64, 256), 256, 0, s>>>(B.keys, B.pcnt, n_parts, B.psize, B.pinb,
                                                                        B.seq, rho, L.size, omega, delta,
                                                                        (1ull << posbits) - 1ull, B.vdelta);
    HGP_LAUNCH_CHECK();
  }
  k_finish<<<1, FIN_NT, 0, s>>>(B.gp, B.vdelta, S, B.G, B.viol, B.scal);
  HGP_LAUNCH_CHECK();
  int64_t res[2];
  HGP_HIP(hipMemcpyAsync(res, B.scal + SC_ISTAR, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HGP_HIP(hipStreamSynchronize(s));
  *istar = res[0];
  *gstar = res[1];
}

__global__ void k_apply(int32_t *__restrict__ rho, const int32_t *__restrict__ seq, const int32_t *__restrict__ dest,
                        int64_t istar) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < istar) {
    const int v = seq[i];
    rho[v] = dest[v];
  }
}

void launch_apply(int32_t *rho, RoundBufs &B, int64_t istar, hipStream_t s) {
  if (istar <= 0) return;
  k_apply<<<div_up(istar, 256), 256, 0, s>>>(rho, B.seq, B.dest, istar);
  HGP_LAUNCH_CHECK();
}

__global__ void k_project(const int32_t *__restrict__ gamma, const int32_t *__restrict__ rc, int32_t n,
                          int32_t *__restrict__ rf) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) rf[v] = rc[gamma[v]];
}

void launch_project(const int32_t *gamma, const int32_t *rho_coarse, int32_t n, int32_t *rho_fine, hipStream_t s) {
  if (n <= 0) return;
  k_project<<<div_up(n, 256), 256, 0, s>>>(gamma, rho_coarse, n, rho_fine);
  HGP_LAUNCH_CHECK();
}

__global__ void k_conn(const int32_t *__restrict__ lam, const int32_t *__restrict__ hw, int32_t E,
                       int64_t *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t c = 0;
  if (e < E && lam[e] > 1) c = (int64_t)hw[e] * (lam[e] - 1);
  c = wave_sum(c);
  if (lane_id() == 0 && c) atomicAdd((unsigned long long *)out, (unsigned long long)c);
}

void launch_connectivity(const LevelView &L, const RoundBufs &B, int64_t *conn_dev, hipStream_t s) {
  fill_i64(conn_dev, 1, 0, s);
  if (L.E <= 0) return;
  k_conn<<<div_up(L.E, 256), 256, 0, s>>>(B.lam, L.hw, L.E, conn_dev);
  HGP_LAUNCH_CHECK();
}

__global__ void k_mark_used(const int32_t *__restrict__ rho, int32_t n, int32_t *__restrict__ used) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) used[rho[v]] = 1;
}

__global__ void k_rename(const int32_t *__restrict__ rho, int32_t n, const int32_t *__restrict__ ren,
                         int32_t *__restrict__ out) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) out[v] = ren[rho[v]];
}

void launch_compact_parts(const int32_t *rho, int32_t n, int32_t n_parts, int32_t *used, int32_t *part_out,
                          int32_t *np_dev, DevBuf &scan_tmp, hipStream_t s) {
  fill_i32(used, n_parts, 0, s);
  if (n > 0) {
    k_mark_used<<<div_up(n, 256), 256, 0, s>>>(rho, n, used);
    HGP_LAUNCH_CHECK();
  }
  scan_i32(used, used, n_parts, np_dev, scan_tmp, s);
  if (n > 0) {
    k_rename<<<div_up(n, 256), 256, 0, s>>>(rho, n, used, part_out);
    HGP_LAUNCH_CHECK();
  }
}

__global__ void k_cluster_size_sum(const int32_t *__restrict__ gamma, const int32_t *__restrict__ size, int32_t n,
                                   int32_t *__restrict__ out) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) atomicAdd(&out[gamma[v]], size[v]);
}

void launch_cluster_size_sum(const int32_t *gamma, const int32_t *size, int32_t n, int32_t *out, hipStream_t s) {
  if (n <= 0) return;
  k_cluster_size_sum<<<div_up(n, 256), 256, 0, s>>>(gamma, size, n, out);
  HGP_LAUNCH_CHECK();
}

__global__ void k_widen(const int32_t *__restrict__ dest, const int32_t *__restrict__ gain, int32_t n,
                        int32_t *__restrict__ d2, int64_t *__restrict__ g2) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) {
    d2[v] = dest[v];
    g2[v] = gain[v];
  }
}

void launch_widen(const int32_t *dest, const int32_t *gain, int32_t n, int32_t *d2, int64_t *g2, hipStream_t s) {
  if (n <= 0) return;
  k_widen<<<div_up(n, 256), 256, 0, s>>>(dest, gain, n, d2, g2);
  HGP_LAUNCH_CHECK();
}

}  // namespace hgp
