// Per-hedge kernels: hedges of at most kThreadSegMax pins are handled by one
// thread each (keys sorted by a register network), longer ones by one wave
// each (keys sorted in registers by wave_bitonic_sort, no workgroup
// barriers).  Hedges with more than kWaveSegMax pins are left to the
// workgroup-per-hedge kernels, which run over the list of such hedges.
#include <algorithm>

#include "coarsen.hpp"

namespace hgp {

__device__ __forceinline__ int lb_u32(const uint32_t *a, int n, uint32_t x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Coarse pins of one hedge (Sec. III-B): keys (map(v) << 1 | dst) sorted;
// the last key of every id run survives, its low bit being the OR of the
// run's destination flags.  Survivors go to out[b ..], their count to cnt[e].
template <int KPL>
__device__ __forceinline__ void contract_wave(int e, int b, int len, const uint32_t *__restrict__ hpin,
                                              const int32_t *__restrict__ map, uint32_t *__restrict__ out,
                                              int32_t *__restrict__ cnt) {
  const int l = lane_id();
  uint32_t k[KPL];
#pragma unroll
  for (int j = 0; j < KPL; ++j) {
    const int i = l * KPL + j;
    uint32_t key = 0xffffffffu;
    if (i < len) {
      const uint32_t x = hpin[b + i];
      key = ((uint32_t)map[x & kIdMask] << 1) | (x >> 31);
    }
    k[j] = key;
  }
  wave_bitonic_sort<KPL>(k);
  const uint32_t next_lane_first = __shfl_down(k[0], 1, 64);
  bool kept[KPL];
  int c = 0;
#pragma unroll
  for (int j = 0; j < KPL; ++j) {
    const int i = l * KPL + j;
    const uint32_t nx = (j + 1 < KPL) ? k[j + 1] : next_lane_first;
    kept[j] = i < len && (i + 1 == len || (nx >> 1) != (k[j] >> 1));
    c += kept[j] ? 1 : 0;
  }
  int pos = wave_exclusive_scan(c);
  const int total = __shfl(pos + c, 63, 64);
#pragma unroll
  for (int j = 0; j < KPL; ++j)
    if (kept[j]) out[b + pos++] = (k[j] >> 1) | ((k[j] & 1u) << 31);
  if (l == 0) cnt[e] = total;
}

// Part table of one hedge (Sec. IV-B): keys (rho(v) << 1 | dst) sorted; each
// run of one part gives (part, pins(p,e)) and pins_in(p,e), written at the
// hedge's pin offset; lam[e] = number of runs.  solo[b + i] = 1 when pin i is
// the only pin of its part in the hedge (pins(rho(v), e) = 1: the hedge is
// in saving(v) of Eq. 3).  s: 64*KPL words of LDS.
template <int KPL>
__device__ __forceinline__ void part_table_wave(int e, int b, int len, const uint32_t *__restrict__ hpin,
                                                const int32_t *__restrict__ rho, int32_t *__restrict__ pt,
                                                uint32_t *__restrict__ ptc, int32_t *__restrict__ lam,
                                                uint8_t *__restrict__ solo, int32_t *__restrict__ pinb,
                                                uint32_t *s) {
  const int l = lane_id();
  uint32_t k[KPL];
#pragma unroll
  for (int j = 0; j < KPL; ++j) {
    const int i = l * KPL + j;
    uint32_t key = 0xffffffffu;
    if (i < len) {
      const uint32_t x = hpin[b + i];
      key = ((uint32_t)rho[x & kIdMask] << 1) | (x >> 31);
    }
    k[j] = key;
  }
  uint32_t ku[KPL];  // keys in pin order
#pragma unroll
  for (int j = 0; j < KPL; ++j) ku[j] = k[j];
  wave_bitonic_sort<KPL>(k);
#pragma unroll
  for (int j = 0; j < KPL; ++j) s[l * KPL + j] = k[j];
  wave_lds_sync();
#pragma unroll
  for (int j = 0; j < KPL; ++j) {
    const int i = l * KPL + j;
    if (i < len) {
      const uint32_t part = ku[j] >> 1;
      solo[b + i] = (lb_u32(s, len, (part + 1) << 1) - lb_u32(s, len, part << 1)) == 1 ? 1 : 0;
    }
  }
  const uint32_t prev_lane_last = __shfl_up(k[KPL - 1], 1, 64);
  bool first[KPL];
  int c = 0;
#pragma unroll
  for (int j = 0; j < KPL; ++j) {
    const int i = l * KPL + j;
    const uint32_t pv = (j > 0) ? k[j - 1] : prev_lane_last;
    first[j] = i < len && (i == 0 || (pv >> 1) != (k[j] >> 1));
    c += first[j] ? 1 : 0;
  }
  int r = wave_exclusive_scan(c);
  const int runs = __shfl(r + c, 63, 64);
#pragma unroll
  for (int j = 0; j < KPL; ++j) {
    if (first[j]) {
      const int i = l * KPL + j;
      const uint32_t part = k[j] >> 1;
      const int end = lb_u32(s, len, (part + 1) << 1);
      const int dst0 = lb_u32(s, len, (part << 1) | 1u);
      pt[b + r] = (int)part;
      ptc[b + r] = (uint32_t)(end - i) | ((uint32_t)(end - dst0) << 16);
      if (end > dst0) atomicAdd(&pinb[part], 1);
      ++r;
    }
  }
  if (l == 0) lam[e] = runs;
  wave_lds_sync();
}

// Grid-stride over hedges, one wave each.  inb(p) counts go to `cnt`: the
// workgroup's LDS histogram (dynamic LDS, n_parts words) when it covers every
// part (flushed to row blockIdx.x of `partial`, summed per part by
// k_pinb_reduce), else the global pinb array.  MAXKPL bounds the hedge length
// handled here (64 * MAXKPL); a variant with MAXKPL = 8 is used when no hedge
// is longer than 512 pins, for its lower register and LDS use.
constexpr int PTW_LDS_PARTS = 8192;

template <int MAXKPL>
__global__ __launch_bounds__(256) void k_part_table_wave(const int32_t *__restrict__ hoff,
                                                         const uint32_t *__restrict__ hpin, int32_t E,
                                                         const int32_t *__restrict__ list,
                                                         const int32_t *__restrict__ list_n,
                                                         const int32_t *__restrict__ rho, int32_t *__restrict__ pt,
                                                         uint32_t *__restrict__ ptc, int32_t *__restrict__ lam,
                                                         uint8_t *__restrict__ solo, int32_t *__restrict__ pinb,
                                                         int32_t n_parts,
                                                         int32_t *__restrict__ partial) {
  __shared__ uint32_t sbuf[4][64 * MAXKPL];
  extern __shared__ int32_t hist[];
  const bool local = partial != nullptr;
  const int count = list ? *list_n : E;
  // workgroups past the list (the grid is sized for every hedge; a coarse
  // level lists few) neither clear nor flush a histogram row: k_pinb_reduce
  // reads the rows of the first ceil(count / 4) workgroups only
  if ((int64_t)blockIdx.x * 4 >= count) return;
  if (local) {
    for (int i = threadIdx.x; i < n_parts; i += 256) hist[i] = 0;
    __syncthreads();
  }
  int32_t *cnt = local ? hist : pinb;
  const int w = threadIdx.x >> 6;
  uint32_t *s = sbuf[w];
  for (int t = (int)(blockIdx.x * 4 + w); t < count; t += (int)(gridDim.x * 4)) {
    const int e = list ? list[t] : t;
    const int b = hoff[e], len = hoff[e + 1] - b;
    if (len > 64 * MAXKPL || len <= kThreadSegMax) continue;
    if (len <= 64) part_table_wave<1>(e, b, len, hpin, rho, pt, ptc, lam, solo, cnt, s);
    else if (len <= 128) part_table_wave<2>(e, b, len, hpin, rho, pt, ptc, lam, solo, cnt, s);
    else if (len <= 256) part_table_wave<4>(e, b, len, hpin, rho, pt, ptc, lam, solo, cnt, s);
    else if (MAXKPL == 8 || len <= 512) part_table_wave<8>(e, b, len, hpin, rho, pt, ptc, lam, solo, cnt, s);
    else part_table_wave<MAXKPL>(e, b, len, hpin, rho, pt, ptc, lam, solo, cnt, s);
  }
  if (local) {
    __syncthreads();
    int32_t *row = partial + (int64_t)blockIdx.x * n_parts;
    for (int i = threadIdx.x; i < n_parts; i += 256) row[i] = hist[i];
  }
}
static_assert(kWaveSegMax == 1024, "k_part_table_wave<16> covers the wave-path hedge lengths");

// pinb[p] = sum over the rows of partial written by the wave kernel: those of
// its first ceil(count / 4) workgroups (count = *list_n, or E without a
// list), at most `rows`.  A workgroup covers 64 parts (one per lane); its
// PR_W waves sum interleaved rows, 8 loads in flight each.
constexpr int PR_W = 16;

__global__ __launch_bounds__(64 * PR_W) void k_pinb_reduce(const int32_t *__restrict__ partial, int grid_rows,
                                                           const int32_t *__restrict__ list_n, int32_t E,
                                                           int32_t n_parts, int32_t *__restrict__ pinb) {
  __shared__ int32_t red[PR_W][64];
  const int count = list_n ? *list_n : E;
  const int rows = (int)min((int64_t)grid_rows, ((int64_t)count + 3) / 4);
  const int l = lane_id(), w = (int)(threadIdx.x >> 6);
  const int p = (int)(blockIdx.x * 64) + l;
  int32_t t = 0;
  if (p < n_parts) {
    int r = w;
    for (; r + 7 * PR_W < rows; r += 8 * PR_W) {
      int32_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = partial[(int64_t)(r + u * PR_W) * n_parts + p];
#pragma unroll
      for (int u = 0; u < 8; ++u) t += v[u];
    }
    for (; r < rows; r += PR_W) t += partial[(int64_t)r * n_parts + p];
  }
  red[w][l] = t;
  __syncthreads();
  if (w == 0 && p < n_parts) {
    int32_t sum = 0;
    for (int q = 0; q < PR_W; ++q) sum += red[q][l];
    pinb[p] = sum;
  }
}

template <int MAXKPL>
static void launch_ptw(int grid, size_t lds, const int32_t *hoff, const uint32_t *hpin, int32_t E,
                       const int32_t *list, const int32_t *list_n, const int32_t *rho, int32_t *pt, uint32_t *ptc,
                       int32_t *lam, uint8_t *solo, int32_t *pinb, int32_t n_parts, int32_t *partial, hipStream_t s) {
  k_part_table_wave<MAXKPL><<<grid, 256, lds, s>>>(hoff, hpin, E, list, list_n, rho, pt, ptc, lam, solo, pinb,
                                                   n_parts, partial);
  HGP_LAUNCH_CHECK();
}

void launch_part_table_wave(const int32_t *hoff, const uint32_t *hpin, int32_t E, const int32_t *list,
                            const int32_t *list_n, const int32_t *rho, int32_t *pt, uint32_t *ptc, int32_t *lam,
                            uint8_t *solo, int32_t *pinb, int32_t n_parts, int32_t max_len, DevBuf &partial,
                            hipStream_t s) {
  const bool small = max_len <= 512;
  const bool local = n_parts > 0 && n_parts <= PTW_LDS_PARTS;
  const size_t lds = local ? (size_t)n_parts * sizeof(int32_t) : 0;
  // resident workgroups per CU (registers: 5 or 3; LDS: 160 KB), 256 CUs
  const size_t lds_wg = lds + (small ? 8u : 16u) * 1024u;
  const int per_cu = std::max(1, std::min(small ? 5 : 3, (int)((160u * 1024u) / lds_wg)));
  const int grid = E > 0 ? std::min(256 * per_cu, div_up(E, 4)) : 0;
  if (!local) fill_i32(pinb, n_parts, 0, s);
  if (grid <= 0) {
    if (local) fill_i32(pinb, n_parts, 0, s);
    return;
  }
  int32_t *rows = nullptr;
  if (local) {
    partial.reserve((size_t)grid * n_parts * sizeof(int32_t));
    rows = partial.as<int32_t>();
  }
  if (small)
    launch_ptw<8>(grid, lds, hoff, hpin, E, list, list_n, rho, pt, ptc, lam, solo, pinb, n_parts, rows, s);
  else
    launch_ptw<16>(grid, lds, hoff, hpin, E, list, list_n, rho, pt, ptc, lam, solo, pinb, n_parts, rows, s);
  if (local) {
    k_pinb_reduce<<<div_up(n_parts, 64), 64 * PR_W, 0, s>>>(rows, grid, list ? list_n : nullptr, E, n_parts,
                                                           pinb);
    HGP_LAUNCH_CHECK();
  }
}

// ---------------------------------------------------------------------------
// part tables of short hedges: one thread per hedge
// ---------------------------------------------------------------------------
// Coarse levels leave most hedges with a few pins, and a wave per hedge then
// spends its time on the latency of one hedge's loads at a time.  Here each
// thread owns a hedge of at most kThreadSegMax pins: it loads the pins and
// their parts (all loads of a thread issued together), sorts the 64-bit keys
// (rho(v) << 1 | dst) << 32 | position in registers with a bitonic network of
// T keys (T chosen per wave from its longest hedge), and walks the sorted runs
// once, writing the same part table, solo flags and inb(p) counts as the wave
// kernel.
template <int T, class K>
__device__ __forceinline__ void reg_bitonic_sort(K (&k)[T]) {
#pragma unroll
  for (int size = 2; size <= T; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
      for (int i = 0; i < T; ++i) {
        const int j = i ^ stride;
        if (j > i) {
          const bool asc = (i & size) == 0;
          const K a = k[i], b = k[j];
          const bool sw = (a > b) == asc;
          k[i] = sw ? b : a;
          k[j] = sw ? a : b;
        }
      }
    }
  }
}

template <int T>
__device__ __forceinline__ void part_table_thread(int e, int b, int len, const uint32_t *__restrict__ hpin,
                                                  const int32_t *__restrict__ rho, int32_t *__restrict__ pt,
                                                  uint32_t *__restrict__ ptc, int32_t *__restrict__ lam,
                                                  uint8_t *__restrict__ solo, int32_t *cnt) {
  uint32_t x[T];
#pragma unroll
  for (int j = 0; j < T; ++j) x[j] = j < len ? hpin[b + j] : 0u;
  uint64_t k[T];
#pragma unroll
  for (int j = 0; j < T; ++j) {
    k[j] = ~0ull;
    if (j < len) {
      const uint32_t hi = ((uint32_t)rho[x[j] & kIdMask] << 1) | (x[j] >> 31);
      k[j] = ((uint64_t)hi << 32) | (uint64_t)j;
    }
  }
  reg_bitonic_sort<T, uint64_t>(k);
  int r = 0, start = 0, din = 0;
#pragma unroll
  for (int j = 0; j < T; ++j) {
    if (j < len) {
      const uint32_t hi = (uint32_t)(k[j] >> 32);
      din += (int)(hi & 1u);
      const bool last = (j + 1 == len) || (j + 1 < T && (uint32_t)(k[j + 1] >> 33) != (hi >> 1));
      solo[b + (int)(uint32_t)k[j]] = (last && j == start) ? 1 : 0;
      if (last) {
        const int32_t part = (int32_t)(hi >> 1);
        pt[b + r] = part;
        ptc[b + r] = (uint32_t)(j + 1 - start) | ((uint32_t)din << 16);
        if (din) atomicAdd(&cnt[part], 1);
        ++r;
        start = j + 1;
        din = 0;
      }
    }
  }
  lam[e] = r;
}

// Grid-stride over hedges; those longer than kThreadSegMax are left to the
// wave and workgroup kernels.  inb(p) counts are summed in an LDS histogram
// per workgroup when n_parts <= PTW_LDS_PARTS and added to pinb (which holds
// the other kernels' counts) by one atomic per non-zero bin.
__global__ __launch_bounds__(256) void k_part_table_thread(const int32_t *__restrict__ hoff,
                                                           const uint32_t *__restrict__ hpin, int32_t E,
                                                           const int32_t *__restrict__ rho, int32_t *__restrict__ pt,
                                                           uint32_t *__restrict__ ptc, int32_t *__restrict__ lam,
                                                           uint8_t *__restrict__ solo, int32_t *__restrict__ pinb,
                                                           int32_t n_parts) {
  extern __shared__ int32_t hist[];
  const bool local = n_parts > 0 && n_parts <= PTW_LDS_PARTS;
  if (local) {
    for (int i = threadIdx.x; i < n_parts; i += 256) hist[i] = 0;
    __syncthreads();
  }
  int32_t *cnt = local ? hist : pinb;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t e0 = (int64_t)blockIdx.x * 256; e0 < E; e0 += stride) {
    const int e = (int)(e0 + threadIdx.x);
    int b = 0, len = kThreadSegMax + 1;
    if (e < E) {
      b = hoff[e];
      len = hoff[e + 1] - b;
    }
    const bool mine = len <= kThreadSegMax;
    // wave-uniform network width: the longest of the wave's short hedges
    int wl = mine ? len : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wl = max(wl, __shfl_xor(wl, o, 64));
    if (mine) {
      if (len == 0) lam[e] = 0;
      else if (wl <= 4) part_table_thread<4>(e, b, len, hpin, rho, pt, ptc, lam, solo, cnt);
      else if (wl <= 8) part_table_thread<8>(e, b, len, hpin, rho, pt, ptc, lam, solo, cnt);
      else part_table_thread<16>(e, b, len, hpin, rho, pt, ptc, lam, solo, cnt);
    }
  }
  if (local) {
    __syncthreads();
    for (int i = threadIdx.x; i < n_parts; i += 256)
      if (hist[i]) atomicAdd(&pinb[i], hist[i]);
  }
}
static_assert(kThreadSegMax == 16, "k_part_table_thread's networks cover kThreadSegMax keys");

void launch_part_table_thread(const int32_t *hoff, const uint32_t *hpin, int32_t E, const int32_t *rho, int32_t *pt,
                              uint32_t *ptc, int32_t *lam, uint8_t *solo, int32_t *pinb, int32_t n_parts,
                              hipStream_t s) {
  if (E <= 0) return;
  const bool local = n_parts > 0 && n_parts <= PTW_LDS_PARTS;
  const int grid = std::min(div_up(E, 256), 2048);
  k_part_table_thread<<<grid, 256, local ? (size_t)n_parts * sizeof(int32_t) : 0, s>>>(hoff, hpin, E, rho, pt, ptc,
                                                                                        lam, solo, pinb, n_parts);
  HGP_LAUNCH_CHECK();
}

// list[0 .. *count) = hedges with lo < |e| <= hi (any order).
__global__ __launch_bounds__(256) void k_mid_hedges(const int32_t *__restrict__ hoff, int32_t E, int32_t lo,
                                                    int32_t hi, int32_t *__restrict__ list,
                                                    int32_t *__restrict__ count) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool mid = false;
  if (e < E) {
    const int len = hoff[e + 1] - hoff[e];
    mid = len > lo && len <= hi;
  }
  const uint64_t m = __ballot(mid);
  int base = 0;
  if (lane_id() == 0 && m) base = atomicAdd(count, __popcll(m));
  base = __shfl(base, 0, 64);
  if (mid) list[base + __popcll(m & ((1ull << lane_id()) - 1ull))] = (int32_t)e;
}

void launch_mid_hedges(const int32_t *hoff, int32_t E, int32_t *list, int32_t *count, hipStream_t s, int32_t lo,
                       int32_t hi) {
  fill_i32(count, 1, 0, s);
  if (E <= 0) return;
  k_mid_hedges<<<div_up(E, 256), 256, 0, s>>>(hoff, E, lo, hi, list, count);
  HGP_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// contraction of short hedges: one thread per hedge
// ---------------------------------------------------------------------------
// As contract_wave for a hedge of at most kThreadSegMax pins held by one
// thread: keys (map(v) << 1 | dst) sorted in registers, the last key of every
// id run kept (its low bit is the OR of the run's destination flags).
template <int T>
__device__ __forceinline__ void contract_thread(int e, int b, int len, const uint32_t *__restrict__ hpin,
                                                const int32_t *__restrict__ map, uint32_t *__restrict__ out,
                                                int32_t *__restrict__ cnt) {
  uint32_t x[T];
#pragma unroll
  for (int j = 0; j < T; ++j) x[j] = j < len ? hpin[b + j] : 0u;
  uint32_t k[T];
#pragma unroll
  for (int j = 0; j < T; ++j) k[j] = j < len ? (((uint32_t)map[x[j] & kIdMask] << 1) | (x[j] >> 31)) : 0xffffffffu;
  reg_bitonic_sort<T, uint32_t>(k);
  int c = 0;
#pragma unroll
  for (int j = 0; j < T; ++j) {
    if (j < len) {
      const bool kept = (j + 1 == len) || (j + 1 < T && (k[j + 1] >> 1) != (k[j] >> 1));
      if (kept) out[b + c++] = (k[j] >> 1) | ((k[j] & 1u) << 31);
    }
  }
  cnt[e] = c;
}

__global__ __launch_bounds__(256) void k_contract_thread(const int32_t *__restrict__ hoff,
                                                         const uint32_t *__restrict__ hpin, int32_t E,
                                                         const int32_t *__restrict__ map, uint32_t *__restrict__ out,
                                                         int32_t *__restrict__ cnt) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t e0 = (int64_t)blockIdx.x * 256; e0 < E; e0 += stride) {
    const int e = (int)(e0 + threadIdx.x);
    int b = 0, len = kThreadSegMax + 1;
    if (e < E) {
      b = hoff[e];
      len = hoff[e + 1] - b;
    }
    const bool mine = len <= kThreadSegMax;
    int wl = mine ? len : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wl = max(wl, __shfl_xor(wl, o, 64));
    if (mine) {
      if (len == 0) cnt[e] = 0;
      else if (wl <= 4) contract_thread<4>(e, b, len, hpin, map, out, cnt);
      else if (wl <= 8) contract_thread<8>(e, b, len, hpin, map, out, cnt);
      else contract_thread<16>(e, b, len, hpin, map, out, cnt);
    }
  }
}

// Contraction of the hedges of list[0 .. *count) (lengths above
// kThreadSegMax; those above kWaveSegMax are left to the workgroup kernel),
// one wave each, grid-stride over the list.
__global__ __launch_bounds__(256) void k_contract_wave_list(const int32_t *__restrict__ hoff,
                                                            const uint32_t *__restrict__ hpin,
                                                            const int32_t *__restrict__ list,
                                                            const int32_t *__restrict__ count,
                                                            const int32_t *__restrict__ map,
                                                            uint32_t *__restrict__ out, int32_t *__restrict__ cnt) {
  const int n = *count;
  for (int t = (int)(blockIdx.x * 4 + (threadIdx.x >> 6)); t < n; t += (int)(gridDim.x * 4)) {
    const int e = list[t];
    const int b = hoff[e], len = hoff[e + 1] - b;
    if (len > kWaveSegMax) continue;
    if (len <= 64) contract_wave<1>(e, b, len, hpin, map, out, cnt);
    else if (len <= 128) contract_wave<2>(e, b, len, hpin, map, out, cnt);
    else if (len <= 256) contract_wave<4>(e, b, len, hpin, map, out, cnt);
    else if (len <= 512) contract_wave<8>(e, b, len, hpin, map, out, cnt);
    else contract_wave<16>(e, b, len, hpin, map, out, cnt);
  }
}

// Packing of the coarse pins: a thread copies a hedge whose old length is at
// most kThreadSegMax; a wave copies each hedge of the list (the longer ones).
__global__ __launch_bounds__(256) void k_pack_thread(const int32_t *__restrict__ old_off,
                                                     const int32_t *__restrict__ new_off, int32_t E,
                                                     const uint32_t *__restrict__ src, uint32_t *__restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int a = old_off[e];
  if (old_off[e + 1] - a > kThreadSegMax) return;
  const int b = new_off[e], len = new_off[e + 1] - b;
  uint32_t v[kThreadSegMax];
#pragma unroll
  for (int j = 0; j < kThreadSegMax; ++j) v[j] = j < len ? src[a + j] : 0u;
#pragma unroll
  for (int j = 0; j < kThreadSegMax; ++j)
    if (j < len) dst[b + j] = v[j];
}

__global__ __launch_bounds__(256) void k_pack_wave_list(const int32_t *__restrict__ old_off,
                                                        const int32_t *__restrict__ new_off,
                                                        const int32_t *__restrict__ list,
                                                        const int32_t *__restrict__ count,
                                                        const uint32_t *__restrict__ src, uint32_t *__restrict__ dst) {
  const int n = *count;
  for (int t = (int)(blockIdx.x * 4 + (threadIdx.x >> 6)); t < n; t += (int)(gridDim.x * 4)) {
    const int e = list[t];
    const int a = old_off[e], b = new_off[e], len = new_off[e + 1] - b;
    for (int j = lane_id(); j < len; j += 64) dst[b + j] = src[a + j];
  }
}

void launch_contract_split(const int32_t *hoff, const uint32_t *hpin, int32_t E, const int32_t *map, uint32_t *out,
                           int32_t *cnt, int32_t *list_buf, hipStream_t s) {
  if (E <= 0) return;
  launch_mid_hedges(hoff, E, list_buf + 1, list_buf, s, kThreadSegMax, 0x7fffffff);
  k_contract_thread<<<std::min(div_up(E, 256), 2048), 256, 0, s>>>(hoff, hpin, E, map, out, cnt);
  HGP_LAUNCH_CHECK();
  k_contract_wave_list<<<std::min(div_up(E, 4), 2048), 256, 0, s>>>(hoff, hpin, list_buf + 1, list_buf, map, out,
                                                                    cnt);
  HGP_LAUNCH_CHECK();
}

void launch_pack_split(const int32_t *old_off, const int32_t *new_off, int32_t E, const uint32_t *src, uint32_t *dst,
                       const int32_t *list_buf, hipStream_t s) {
  if (E <= 0) return;
  k_pack_thread<<<div_up(E, 256), 256, 0, s>>>(old_off, new_off, E, src, dst);
  HGP_LAUNCH_CHECK();
  k_pack_wave_list<<<std::min(div_up(E, 4), 2048), 256, 0, s>>>(old_off, new_off, list_buf + 1, list_buf, src, dst);
  HGP_LAUNCH_CHECK();
}

// Hedges longer than kWaveSegMax pins (fixed by level 0: coarse hedges only shrink).
__global__ __launch_bounds__(256) void k_big_hedges(const int32_t *__restrict__ hoff, int32_t E,
                                                    int32_t *__restrict__ list, int32_t *__restrict__ count) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int len = 0;
  if (e < E) {
    len = hoff[e + 1] - hoff[e];
    if (len > kWaveSegMax) list[atomicAdd(count, 1)] = (int32_t)e;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) len = max(len, __shfl_xor(len, o, 64));
  if (lane_id() == 0 && len > 0) atomicMax(count + 1, len);
}

void launch_big_hedges(const int32_t *hoff, int32_t E, int32_t *list, int32_t *count, hipStream_t s) {
  fill_i32(count, 2, 0, s);
  if (E <= 0) return;
  k_big_hedges<<<div_up(E, 256), 256, 0, s>>>(hoff, E, list, count);
  HGP_LAUNCH_CHECK();
}

}  // namespace hgp
