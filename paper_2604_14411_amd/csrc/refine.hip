// Refinement kernels (Sec. IV): part tables, in-isolation proposals (Eq. 3),
// the move sequence, exact in-sequence gains, event-based constraint
// validity per prefix, the best valid prefix, projection and Eq. 1.
#include "coarsen.hpp"

#include <algorithm>

namespace hgp {

constexpr int PT_NT = 256;
constexpr int PROP_NT = 256;
constexpr int PROP_LDS_BYTES = 64 * 1024;


__device__ __forceinline__ int lower_bound_u32(const uint32_t *a, int n, uint32_t x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// part table: pins(p,e), pins_in(p,e) (Sec. IV-B, counting pins per partition)
// ---------------------------------------------------------------------------
// Part table of one hedge of at most kSegCap pins by a workgroup (LDS sort).
__device__ __forceinline__ void part_table_block(int e, const int32_t *__restrict__ hoff,
                                                 const uint32_t *__restrict__ hpin, const int32_t *__restrict__ rho,
                                                 int32_t *__restrict__ pt, uint32_t *__restrict__ ptc,
                                                 int32_t *__restrict__ lam, uint8_t *__restrict__ solo,
                                                 int32_t *__restrict__ pinb, int32_t *err, uint32_t *key,
                                                 int32_t *first, int32_t *tmp) {
  const int b = hoff[e];
  const int len = hoff[e + 1] - b;
  if (len <= 0 || len > kHugeCap) {
    if (threadIdx.x == 0) {
      lam[e] = 0;
      if (len > kHugeCap) atomicOr(err, kErrInternal);
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
      pt[b + r] = (int)part;
      ptc[b + r] = (uint32_t)(end - i) | ((uint32_t)(end - dst0) << 16);
      if (end > dst0) atomicAdd(&pinb[part], 1);
    }
  }
  if (threadIdx.x == 0) lam[e] = runs;
  // solo flags in pin order (the only pin of its part in the hedge)
  for (int i = threadIdx.x; i < len; i += PT_NT) {
    const uint32_t part = (uint32_t)rho[hpin[b + i] & kIdMask];
    solo[b + i] = (lower_bound_u32(key, len, (part + 1) << 1) - lower_bound_u32(key, len, part << 1)) == 1 ? 1 : 0;
  }
}

// Workgroup per hedge, grid-stride over list[0 .. count).
__global__ __launch_bounds__(PT_NT) void k_part_table(const int32_t *__restrict__ hoff,
                                                      const uint32_t *__restrict__ hpin,
                                                      const int32_t *__restrict__ rho, int32_t *__restrict__ pt,
                                                      uint32_t *__restrict__ ptc, int32_t *__restrict__ lam,
                                                      uint8_t *__restrict__ solo, int32_t *__restrict__ pinb,
                                                      int32_t *err, const int32_t *__restrict__ list,
                                                      const int32_t *__restrict__ list_n, int32_t n_fixed,
                                                      uint64_t *__restrict__ huge_k, int32_t *__restrict__ huge_i) {
  __shared__ uint32_t key[kSegCap];
  __shared__ int32_t first[kSegCap];
  __shared__ int32_t tmp[PT_NT / 64 + 1];
  // grid-stride over list[0 .. count): count from the device when list_n is set
  const int count = list_n ? *list_n : n_fixed;
  for (int t = blockIdx.x; t < count; t += gridDim.x) {
    const int e = list[t];
    const int b = hoff[e], len = hoff[e + 1] - b;
    if (len <= kSegCap || !huge_k)
      part_table_block(e, hoff, hpin, rho, pt, ptc, lam, solo, pinb, err, key, first, tmp);
    else  // keys at twice the pin offset, run flags at the pin offset of the global scratch
      part_table_block(e, hoff, hpin, rho, pt, ptc, lam, solo, pinb, err,
                       reinterpret_cast<uint32_t *>(huge_i) + 2 * (int64_t)b,
                       reinterpret_cast<int32_t *>(huge_k) + b, tmp);
    __syncthreads();
  }
}

__global__ void k_part_size(const int32_t *__restrict__ rho, const int32_t *__restrict__ size, int32_t N,
                            int32_t *__restrict__ psize) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < N) atomicAdd(&psize[rho[n]], size[n]);
}

// As k_part_size for n_parts <= PS_LDS_PARTS: each workgroup sums its nodes in
// an LDS histogram first and flushes its non-zero bins, so a part gets one
// global atomic per workgroup (at coarse levels a part can hold thousands of
// nodes, whose per-node atomics serialise on one address; with many more
// parts, clearing and scanning every workgroup's histogram would cost more
// than it saves).
constexpr int PS_LDS_PARTS = 8192;
constexpr int PS_GRID = 512;
__global__ __launch_bounds__(256) void k_part_size_lds(const int32_t *__restrict__ rho,
                                                       const int32_t *__restrict__ size, int32_t N, int32_t n_parts,
                                                       int32_t *__restrict__ psize) {
  extern __shared__ int32_t h[];
  for (int p = threadIdx.x; p < n_parts; p += 256) h[p] = 0;
  __syncthreads();
  for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < N; n += (int64_t)gridDim.x * 256)
    atomicAdd(&h[rho[n]], size[n]);
  __syncthreads();
  for (int p = threadIdx.x; p < n_parts; p += 256)
    if (h[p]) atomicAdd(&psize[p], h[p]);
}

void launch_part_table(const LevelView &L, const int32_t *rho, int32_t n_parts, RoundBufs &B, int32_t *err,
                       hipStream_t s) {
  fill_i32(B.psize, n_parts, 0, s);
  KScope ks(2, s);
  add_units(2, 0);
  if (!B.partial) throw Error(-7, "part-table scratch missing");
  // pinb is written by the wave kernel's reduction (or zeroed by it), then
  // the workgroup and thread kernels add their hedges' counts
  launch_part_table_wave(L.hoff, L.hpin, L.E, L.mid.list, L.mid.count, rho, B.pt, B.ptc, B.lam, B.solo, B.pinb,
                         n_parts, L.big.max_len, *B.partial, s);
  if (L.E > 0) {
    const int grid = std::min(std::min(L.big.n, L.big.bound), 2048);
    if (grid > 0) {
      // the level's own long hedges when listed (fewer than level 0's at coarse levels)
      if (L.mid.big_list)
        k_part_table<<<grid, PT_NT, 0, s>>>(L.hoff, L.hpin, rho, B.pt, B.ptc, B.lam, B.solo, B.pinb, err,
                                            L.mid.big_list, L.mid.big_count, 0, L.big.huge_k, L.big.huge_i);
      else
        k_part_table<<<grid, PT_NT, 0, s>>>(L.hoff, L.hpin, rho, B.pt, B.ptc, B.lam, B.solo, B.pinb, err,
                                            L.big.list, nullptr, L.big.n, L.big.huge_k, L.big.huge_i);
      HGP_LAUNCH_CHECK();
    }
    launch_part_table_thread(L.hoff, L.hpin, L.E, rho, B.pt, B.ptc, B.lam, B.solo, B.pinb, n_parts, s);
  }
  if (L.n > 0 && L.size) {
    if (n_parts > 0 && n_parts <= PS_LDS_PARTS) {
      const int grid = (int)std::min<int64_t>(div_up(L.n, 1024), PS_GRID);
      k_part_size_lds<<<grid, 256, (size_t)n_parts * 4, s>>>(rho, L.size, L.n, n_parts, B.psize);
    } else {
      k_part_size<<<div_up(L.n, 256), 256, 0, s>>>(rho, L.size, L.n, B.psize);
    }
    HGP_LAUNCH_CHECK();
  }
}

// ---------------------------------------------------------------------------
// proposals (Eq. 3)
// ---------------------------------------------------------------------------
// One workgroup per node n in part p_s (node list[t], or t when list is
// null; grid-stride over *count nodes).  saving(n) is summed first from the
// solo flags of n's pins (pins(p_s, e) = 1); if it is zero no move can have positive gain
// (loss >= 0) and the node is done.  Otherwise every part table entry of
// every hedge of I(n) adds w(e) to conn[p] in LDS; then
//   gain(n,p) = saving - loss(n,p) = saving - total(n) + conn[p]
// and the best part by (gain, id) among those with size(p)+size(n) <= Omega
// is kept if gain > 0.  With DEFER, nodes of more than kPropHeavyDeg
// incidences are only queued (hlist, *hcnt): the second launch gives each of
// them a workgroup of many more waves, since a few such nodes (large clusters
// at coarse levels) would otherwise decide the whole launch's duration (128
// measured best against 256 and 512 on the random and layered networks).
constexpr int kPropHeavyDeg = PROP_NT / 2;
template <int NT, int U, bool DEFER>
__global__ __launch_bounds__(NT) void k_propose(const int32_t *__restrict__ list, const int64_t *__restrict__ count,
                                                int32_t N, const int32_t *__restrict__ ioff,
                                                const uint32_t *__restrict__ inc, const uint32_t *__restrict__ perm,
                                                const int32_t *__restrict__ hoff, const int32_t *__restrict__ pt,
                                                const uint8_t *__restrict__ solo,
                                                const int32_t *__restrict__ lam, const int32_t *__restrict__ hw,
                                                const int32_t *__restrict__ rho, const int32_t *__restrict__ size,
                                                const int32_t *__restrict__ psize, const int32_t *__restrict__ total,
                                                int32_t n_parts, int32_t omega, int32_t words,
                                                int32_t *__restrict__ dest, int32_t *__restrict__ gain,
                                                int32_t *__restrict__ hlist, unsigned long long *__restrict__ hcnt,
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
    if (DEFER && i1 - i0 > kPropHeavyDeg) {
      if (tid == 0) hlist[atomicAdd(hcnt, 1ull)] = n;
      continue;
    }
    // saving(n): hedges where n is the only pin of p_s; eight incidences
    // per thread in flight (a coarse cluster has tens of thousands)
    int64_t sav = 0;
    for (int i = i0 + tid; i < i1; i += 8 * NT) {
      uint32_t pp[8], x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int j = i + u * NT;
        pp[u] = j < i1 ? perm[j] : 0u;
        x[u] = j < i1 ? inc[j] : 0u;
      }
      uint8_t so[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) so[u] = i + u * NT < i1 ? solo[pp[u]] : (uint8_t)0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (so[u]) sav += hw[x[u] & kIdMask];
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
        streamed += stream_segments<NT / 64, U, false, int32_t>(
            i0, i1, inc, hoff, lam, hw, tbl, [&](int j) { return pt[j]; },
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
constexpr int PROP_HEAVY_NT = 1024;
constexpr int PROP_HEAVY_GRID = 512;  // two 1024-thread workgroups per CU

void launch_propose(const LevelView &L, const int32_t *total, const int32_t *rho, int32_t n_parts, int32_t omega,
                    RoundBufs &B, hipStream_t s, const int32_t *list, const int64_t *count) {
  if (L.n <= 0) return;
  const int max_words = PROP_LDS_BYTES / 4;
  const int words = n_parts < max_words ? (n_parts > 0 ? n_parts : 1) : max_words;
  KScope ks(1, s);
  const int grid = list ? (L.n < PROP_GRID ? L.n : PROP_GRID) : L.n;
  // heavy nodes queue into flag (free until the sequence is built)
  int64_t *hcnt = B.scal + SC_PHEAVY;  // zeroed by launch_round_reset
  k_propose<PROP_NT, 4, true><<<grid, PROP_NT, (size_t)words * 4, s>>>(
      list, count, L.n, L.ioff, L.inc, L.perm, L.hoff, B.pt, B.solo, B.lam, L.hw, rho, L.size, B.psize, total, n_parts,
      omega, words, B.dest, B.gain, B.flag, reinterpret_cast<unsigned long long *>(hcnt), units_ptr(1));
  HGP_LAUNCH_CHECK();
  const int hgrid = L.n < PROP_HEAVY_GRID ? L.n : PROP_HEAVY_GRID;
  k_propose<PROP_HEAVY_NT, 8, false><<<hgrid, PROP_HEAVY_NT, (size_t)words * 4, s>>>(
      B.flag, hcnt, L.n, L.ioff, L.inc, L.perm, L.hoff, B.pt, B.solo, B.lam, L.hw, rho, L.size, B.psize, total,
      n_parts, omega, words, B.dest, B.gain, nullptr, nullptr, units_ptr(1));
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

// The round's device scalars in one launch: heavy-node and heavy-hedge
// counters, the largest gain, the initially invalid parts, g'(0), the end of
// the event-count scan and (when given) the count of nodes to propose.
__global__ void k_round_reset(int64_t *__restrict__ scal, int32_t *__restrict__ gp, int64_t *__restrict__ evoff_end,
                              int64_t *__restrict__ cnt) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    scal[SC_INVALID0] = 0;
    scal[SC_HEAVY] = 0;
    scal[SC_PHEAVY] = 0;
    scal[SC_GMAX] = 0;
    gp[0] = 0;
    *evoff_end = 0;
    if (cnt) *cnt = 0;
  }
}

void launch_round_reset(RoundBufs &B, int32_t E, int64_t *cnt, hipStream_t s) {
  k_round_reset<<<1, 64, 0, s>>>(B.scal, B.gp, B.evoff + E, cnt);
  HGP_LAUNCH_CHECK();
}

void launch_prop_gather(int32_t n, const int32_t *match, const int32_t *gamma, const int32_t *cdest,
                        const int32_t *cgain, RoundBufs &B, int32_t *list, int64_t *cnt, hipStream_t s) {
  if (n <= 0) return;
  k_prop_gather<<<div_up(n, 256), 256, 0, s>>>(n, match, gamma, cdest, cgain, B.dest, B.gain, list, cnt);
  HGP_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// sequence: moves sorted by (gain, id) descending (Sec. IV-A)
// ---------------------------------------------------------------------------
// Move flags, and the largest proposed gain into *gmax (zeroed by the caller).
__global__ void k_move_flags(const int32_t *__restrict__ dest, const int32_t *__restrict__ gain, int32_t N,
                             int32_t *__restrict__ flag, int32_t *__restrict__ pos,
                             unsigned long long *__restrict__ gmax) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t g = 0;
  if (n < N) {
    const bool mv = dest[n] >= 0;
    flag[n] = mv ? 1 : 0;
    pos[n] = 0;
    if (mv) g = gain[n];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) g = max(g, __shfl_xor(g, o, 64));
  if (lane_id() == 0 && g > 0) atomicMax(gmax, (unsigned long long)g);
}

// Sequence order (Sec. IV-B): gain descending, then node id descending; the
// key is (gmax - gain) << idbits | (N - 1 - n), ascending.
template <class K>
__global__ void k_move_keys(const int32_t *__restrict__ dest, const int32_t *__restrict__ gain,
                            const int32_t *__restrict__ off, int32_t N, int idbits, int32_t gmax,
                            K *__restrict__ keys) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < N && dest[n] >= 0)
    keys[off[n]] = (K)(((uint64_t)(uint32_t)(gmax - gain[n]) << idbits) | (uint64_t)(uint32_t)(N - 1 - n));
}

template <class K>
__global__ void k_seq_from_keys(const K *__restrict__ keys, int64_t S, int32_t N, int idbits,
                                int32_t *__restrict__ seq, int32_t *__restrict__ pos) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < S) {
    const int n = N - 1 - (int)((uint64_t)keys[i] & ((1ull << idbits) - 1ull));
    seq[i] = n;
    pos[n] = (int32_t)(i + 1);
  }
}

constexpr int SMALL_SORT_NT = 1024;
constexpr int SMALL_SORT_CAP = 8192;

template <class K>
__global__ __launch_bounds__(SMALL_SORT_NT) void k_small_sort(K *keys, int n) {
  __shared__ K s[SMALL_SORT_CAP];
  const int np = next_pow2(n);
  for (int i = threadIdx.x; i < np; i += SMALL_SORT_NT) s[i] = i < n ? keys[i] : ~K(0);
  __syncthreads();
  block_bitonic_sort<K, SMALL_SORT_NT>(s, np);
  for (int i = threadIdx.x; i < n; i += SMALL_SORT_NT) keys[i] = s[i];
}

void sort_keys(uint64_t *keys, uint64_t *alt, int64_t n, int bits, DevBuf &sort_tmp, hipStream_t s) {
  if (n <= 1) return;
  KScope ks(6, s);
  add_units(6, n);
  if (n <= SMALL_SORT_CAP) {
    k_small_sort<uint64_t><<<1, SMALL_SORT_NT, 0, s>>>(keys, (int)n);
    HGP_LAUNCH_CHECK();
  } else {
    radix_sort_u64(keys, alt, nullptr, nullptr, n, bits, sort_tmp, s);
  }
}

void sort_keys32(uint32_t *keys, uint32_t *alt, int64_t n, int bits, DevBuf &sort_tmp, hipStream_t s, int lo) {
  if (n <= 1) return;
  KScope ks(6, s);
  add_units(6, n);
  if (n <= SMALL_SORT_CAP) {
    k_small_sort<uint32_t><<<1, SMALL_SORT_NT, 0, s>>>(keys, (int)n);
    HGP_LAUNCH_CHECK();
  } else {
    radix_sort_u32(keys, alt, nullptr, nullptr, n, bits, sort_tmp, s, lo);
  }
}

int bits_for(int64_t x) {
  int b = 0;
  while (b < 63 && (int64_t(1) << b) <= x) ++b;
  return b;
}

int64_t build_sequence(const LevelView &L, RoundBufs &B, DevBuf &scan_tmp, DevBuf &sort_tmp, hipStream_t s) {
  const int32_t N = L.n;
  if (N <= 0) return 0;
  k_move_flags<<<div_up(N, 256), 256, 0, s>>>(B.dest, B.gain, N, B.flag, B.pos,
                                              reinterpret_cast<unsigned long long *>(B.scal + SC_GMAX));
  HGP_LAUNCH_CHECK();
  scan_i32(B.flag, B.flag, N, reinterpret_cast<int32_t *>(B.scal + SC_S), scan_tmp, s);
  // |S| and the largest gain in one copy (scal[SC_S .. SC_GMAX])
  HGP_HIP(hipMemcpyAsync(B.hbox, B.scal + SC_S, (SC_GMAX - SC_S + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HGP_HIP(hipStreamSynchronize(s));
  const int64_t S = *reinterpret_cast<const int32_t *>(B.hbox + SC_S);
  const int64_t gmax = B.hbox[SC_GMAX];
  if (S == 0) return 0;
  const int idbits = bits_for(N - 1) > 0 ? bits_for(N - 1) : 1;
  const int gbits = bits_for(gmax);
  const int bits = gbits + idbits;
  if (bits <= 32) {
    uint32_t *k32 = reinterpret_cast<uint32_t *>(B.keys);
    k_move_keys<uint32_t><<<div_up(N, 256), 256, 0, s>>>(B.dest, B.gain, B.flag, N, idbits, (int32_t)gmax, k32);
    HGP_LAUNCH_CHECK();
    sort_keys32(k32, reinterpret_cast<uint32_t *>(B.keys2), S, bits, sort_tmp, s, 0);
    k_seq_from_keys<uint32_t><<<div_up(S, 256), 256, 0, s>>>(k32, S, N, idbits, B.seq, B.pos);
  } else {
    k_move_keys<uint64_t><<<div_up(N, 256), 256, 0, s>>>(B.dest, B.gain, B.flag, N, idbits, (int32_t)gmax, B.keys);
    HGP_LAUNCH_CHECK();
    sort_keys(B.keys, B.keys2, S, bits, sort_tmp, s);
    k_seq_from_keys<uint64_t><<<div_up(S, 256), 256, 0, s>>>(B.keys, S, N, idbits, B.seq, B.pos);
  }
  HGP_LAUNCH_CHECK();
  return S;
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
