// Incremental coarsening for the late levels (Sec. III-A selection, exact).
//
// When a level merges only a few pairs, the candidate sets of most nodes are
// unchanged: for nodes n, m that both stay unmerged, hist(n,m), c(n,m), their
// sizes and |in| do not change, hence neither does the validity of m for n.
// Each node therefore keeps the exact top-TK valid candidates of its last
// full rating (key = hist << 32 | id) and kappa, the hist of the best valid
// candidate left off the list (0 if none was left off).  Invariant: every
// valid candidate not in the list has hist <= kappa.  Only hist is kept in
// the bound because ids are renumbered at every level and the renumbering
// does not preserve order against clusters that merged.
//
// At the next level:
//  - every new cluster c' gets a full rating; its histogram row gives
//    hist(n', c') for every node n' (Eq. 2 is symmetric) and is offered to
//    the unmerged nodes;
//  - an unmerged node drops listed candidates that merged, renames the rest
//    through gamma (order-preserving on unmerged nodes), inserts offers with
//    hist > kappa, and if the list overflows TK the evicted hist raises kappa;
//  - the head is the best valid candidate when its hist exceeds kappa;
//    otherwise (empty list with kappa > 0, or a tie with hidden candidates)
//    the node gets a full rating again.
#include <algorithm>

#include "coarsen.hpp"
#include "tail.hpp"

namespace hgp {

__device__ __forceinline__ uint64_t cand_key(uint64_t h, uint32_t m) { return (h << 32) | (uint64_t)m; }

// Full rating with top-(TK+1) extraction of the nodes in list[0 .. *count)
// (or of every node when list is null).  The whole id range [0, N) must fit
// the LDS window (2N words).  Valid histogram entries of the nodes with a
// row slot are written to rows[slot * N + m].
template <int NT>
__global__ __launch_bounds__(NT) void k_rate_topk(int32_t N, const int32_t *__restrict__ list,
                                                  const int64_t *__restrict__ count, const int32_t *__restrict__ ioff,
                                                  const uint32_t *__restrict__ inc, const int32_t *__restrict__ hoff,
                                                  const uint32_t *__restrict__ hpin, const int32_t *__restrict__ hw,
                                                  const int32_t *__restrict__ size, const int32_t *__restrict__ indeg,
                                                  const int32_t *__restrict__ total, int32_t omega, int32_t delta,
                                                  const int32_t *__restrict__ row_slot, int32_t *__restrict__ rows,
                                                  int32_t *__restrict__ pair, int64_t *__restrict__ score,
                                                  uint64_t *__restrict__ tk_key, int32_t *__restrict__ tk_cnt,
                                                  uint64_t *__restrict__ tk_kappa, int32_t words,
                                                  const uint32_t *__restrict__ pre, int32_t *err,
                                                  unsigned long long *__restrict__ units) {
  extern __shared__ uint32_t lds[];
  __shared__ int32_t tbl[NT / 64 * 192];
  __shared__ uint64_t red[NT / 64];
  __shared__ uint64_t found[kTopK + 1];
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
    const uint64_t hmask = (hb >= 32) ? 0xffffffffull : ((1ull << hb) - 1ull);
    const int zw = packed ? N : 2 * N;
    if (zw > words) {  // the window was sized for packed counters only
      if (tid == 0) atomicOr(err, kErrInternal);
      continue;
    }
    if (pre) {
      // histogram row summed by k_tail_hist
      for (int i = tid; i < zw; i += NT) lds[i] = pre[t * (int64_t)words + i];
      __syncthreads();
    } else {
      for (int i = tid; i < zw; i += NT) lds[i] = 0u;
      __syncthreads();
    }
    if (!pre && sn < omega) {
      streamed += with_mode(packed ? 1 : 2, [&](auto mode) {
        constexpr int MODE = decltype(mode)::value;
        return stream_segments<NT / 64, 4, true, uint32_t>(
            ioff[n], ioff[n + 1], inc, hoff, nullptr, hw, tbl, [&](int j) { return hpin[j]; },
            [&](uint32_t y, uint32_t info) {
              const int m = (int)(y & kIdMask);
              if (m != n) {
                const uint32_t we = info & kIdMask;
                const uint32_t both = (info & y) >> 31;
                if constexpr (MODE == 1)
                  atomicAdd(&lds[m], we + (both << hb));
                else
                  atomicAdd((unsigned long long *)&lds64[m],
                            (unsigned long long)we | ((unsigned long long)both << 32));
              }
            });
      });
    }
    __syncthreads();
    // validity pass fused with the top-(TK+1) selection by key (hist, id):
    // each thread keeps the largest TK+1 keys of its own counters, in
    // registers, descending
    const int slot = row_slot ? row_slot[n] : -1;
    uint64_t top[kTopK + 1];
#pragma unroll
    for (int z = 0; z <= kTopK; ++z) top[z] = 0ull;
    for (int i = tid; i < N; i += NT) {
      uint64_t h = 0, c = 0;
      if (packed) {
        const uint32_t v = lds[i];
        h = v & hmask;
        c = (hb >= 32) ? 0 : (v >> hb);
      } else {
        const uint64_t v = lds64[i];
        h = v & 0xffffffffull;
        c = v >> 32;
      }
      bool ok = false;
      if (h) {
        const int64_t un = (int64_t)din + indeg[i] - (int64_t)c;
        ok = sn + size[i] <= omega && un <= delta;
      }
      if (slot >= 0) rows[(int64_t)slot * N + i] = ok ? (int32_t)h : 0;
      if (ok) {
        uint64_t x = cand_key(h, (uint32_t)i);
        if (x > top[kTopK]) {
#pragma unroll
          for (int z = 0; z <= kTopK; ++z) {
            if (x > top[z]) {
              const uint64_t t = top[z];
              top[z] = x;
              x = t;
            }
          }
        }
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
#pragma unroll
        for (int z = 0; z < kTopK; ++z) top[z] = top[z + 1];
        top[kTopK] = 0ull;
      }
    }
    if (tid == 0) {
      const int keep = nf < kTopK ? nf : kTopK;
      for (int q = 0; q < kTopK; ++q) tk_key[(int64_t)n * kTopK + q] = q < keep ? found[q] : 0ull;
      tk_cnt[n] = keep;
      tk_kappa[n] = nf > kTopK ? (found[kTopK] >> 32) : 0ull;
      pair[n] = keep ? (int32_t)(found[0] & 0xffffffffull) : -1;
      score[n] = keep ? (int64_t)(found[0] >> 32) : 0;
    }
    __syncthreads();
  }
  add_wave_units(units, streamed);
}

// Carry the lists of unmerged level-l nodes to level l+1 and offer the new
// clusters (one thread per level-l node).  Nodes whose list empties with
// kappa > 0 are queued in rerate[] (count in *rerate_cnt).
__global__ void k_rate_update(int32_t n_fine, const int32_t *__restrict__ match, const int32_t *__restrict__ gamma,
                              const uint64_t *__restrict__ old_key, const int32_t *__restrict__ old_cnt,
                              const uint64_t *__restrict__ old_kappa, int32_t n_new, const int32_t *__restrict__ newc,
                              const int32_t *__restrict__ rows, int32_t n_coarse, uint64_t *__restrict__ tk_key,
                              int32_t *__restrict__ tk_cnt, uint64_t *__restrict__ tk_kappa,
                              int32_t *__restrict__ pair, int64_t *__restrict__ score, int32_t *__restrict__ rerate,
                              int64_t *__restrict__ rerate_cnt) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= n_fine || match[n] != n) return;
  const int nc = gamma[n];
  uint64_t a[kTopK];
#pragma unroll
  for (int q = 0; q < kTopK; ++q) a[q] = 0ull;
  uint64_t kap = old_kappa[n];  // hist bound of candidates left off the list
  const int c0 = old_cnt[n];
  // surviving old candidates, renamed (already in descending key order)
  int k = 0;
  for (int q = 0; q < c0; ++q) {
    const uint64_t key = old_key[n * kTopK + q];
    const int m = (int)(key & 0xffffffffull);
    if (match[m] != m) continue;
    const uint64_t nk = (key & 0xffffffff00000000ull) | (uint64_t)(uint32_t)gamma[m];
#pragma unroll
    for (int z = 0; z < kTopK; ++z)
      if (z == k) a[z] = nk;
    ++k;
  }
  // offers from the new clusters (hist > kappa only)
  for (int j = 0; j < n_new; ++j) {
    const int32_t h = rows[(int64_t)j * n_coarse + nc];
    if (h <= 0 || (uint64_t)h <= kap) continue;
    uint64_t x = cand_key((uint64_t)h, (uint32_t)newc[j]);
#pragma unroll
    for (int z = 0; z < kTopK; ++z) {
      if (x > a[z]) {
        const uint64_t t = a[z];
        a[z] = x;
        x = t;
      }
    }
    if ((x >> 32) > kap) kap = x >> 32;  // evicted (0 if the list had room)
  }
  int cnt = 0;
#pragma unroll
  for (int z = 0; z < kTopK; ++z) {
    tk_key[(int64_t)nc * kTopK + z] = a[z];
    cnt += a[z] ? 1 : 0;
  }
  tk_cnt[nc] = cnt;
  tk_kappa[nc] = kap;
  // the head is certain only above every hidden candidate's hist
  const bool certain = cnt > 0 && (a[0] >> 32) > kap;
  if (!certain && (cnt > 0 || kap != 0)) {
    rerate[atomicAdd((unsigned long long *)rerate_cnt, 1ull)] = nc;
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
// `slices` parts streamed by different workgroups (a late level rates only a
// few large clusters: one workgroup per row would leave the device idle).
// Workgroup b handles slice b % slices of row b / slices and adds its LDS
// counters to acc[row * words ..] (same packing as k_rate_topk).
template <int NT>
__global__ __launch_bounds__(NT) void k_tail_hist(int32_t N, const int32_t *__restrict__ list, int32_t rows_n,
                                                  int32_t slices, const int32_t *__restrict__ ioff,
                                                  const uint32_t *__restrict__ inc, const int32_t *__restrict__ hoff,
                                                  const uint32_t *__restrict__ hpin, const int32_t *__restrict__ hw,
                                                  const int32_t *__restrict__ size, const int32_t *__restrict__ indeg,
                                                  const int32_t *__restrict__ total, int32_t omega, int32_t words,
                                                  uint32_t *__restrict__ acc, int32_t *err,
                                                  unsigned long long *__restrict__ units) {
  extern __shared__ uint32_t lds[];
  __shared__ int32_t tbl[NT / 64 * 192];
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
  const int zw = packed ? N : 2 * N;
  if (zw > words) {
    if (tid == 0) atomicOr(err, kErrInternal);
    return;
  }
  const int i0 = ioff[n], i1 = ioff[n + 1];
  const int chunk = (i1 - i0 + slices - 1) / slices;
  const int a = i0 + sl * chunk, z = min(i1, a + chunk);
  if (a >= z) return;
  uint64_t *lds64 = reinterpret_cast<uint64_t *>(lds);
  for (int i = tid; i < zw; i += NT) lds[i] = 0u;
  __syncthreads();
  const int64_t streamed = with_mode(packed ? 1 : 2, [&](auto mode) {
    constexpr int MODE = decltype(mode)::value;
    return stream_segments<NT / 64, 4, true, uint32_t>(
        a, z, inc, hoff, nullptr, hw, tbl, [&](int j) { return hpin[j]; },
        [&](uint32_t y, uint32_t info) {
          const int m = (int)(y & kIdMask);
          if (m != n) {
            const uint32_t we = info & kIdMask;
            const uint32_t both = (info & y) >> 31;
            if constexpr (MODE == 1)
              atomicAdd(&lds[m], we + (both << hb));
            else
              atomicAdd((unsigned long long *)&lds64[m], (unsigned long long)we | ((unsigned long long)both << 32));
          }
        });
  });
  __syncthreads();
  uint32_t *row = acc + (int64_t)r * words;
  if (packed) {
    for (int i = tid; i < N; i += NT) {
      const uint32_t v = lds[i];
      if (v) atomicAdd(&row[i], v);
    }
  } else {
    unsigned long long *row64 = reinterpret_cast<unsigned long long *>(row);
    for (int i = tid; i < N; i += NT) {
      const unsigned long long v = lds64[i];
      if (v) atomicAdd(&row64[i], v);
    }
  }
  add_wave_units(units, streamed);
}

constexpr int TOPK_NT = 256;
constexpr int TOPK_GRID = 2048;

void launch_rate_topk(const LevelView &L, const int32_t *total, int32_t omega, int32_t delta, const int32_t *list,
                      const int64_t *count, int64_t grid_nodes, const int32_t *row_slot, int32_t *rows, int32_t *pair,
                      int64_t *score, TopK &tk, int words_per_id, int32_t *err, hipStream_t s) {
  if (L.n <= 0 || grid_nodes <= 0) return;
  const int64_t words = (int64_t)words_per_id * L.n;
  if (words > kTopKMaxWords) throw Error(-7, "top-K window exceeds LDS");
  KScope ks(8, s);
  const size_t bytes = (size_t)words * 4;
  // thread-safe one-time opt-in to the large dynamic LDS size
  static const bool attr_set = [] {
    HGP_HIP(hipFuncSetAttribute((const void *)k_rate_topk<TOPK_NT>, hipFuncAttributeMaxDynamicSharedMemorySize, kTopKMaxWords * 4));
    return true;
  }();
  (void)attr_set;
  const int grid = (int)(grid_nodes < TOPK_GRID ? grid_nodes : TOPK_GRID);
  k_rate_topk<TOPK_NT><<<grid, TOPK_NT, bytes, s>>>(L.n, list, count, L.ioff, L.inc, L.hoff, L.hpin, L.hw, L.size,
                                                    L.indeg, total, omega, delta, row_slot, rows, pair, score, tk.key,
                                                    tk.cnt, tk.kappa, (int32_t)words, nullptr, err, units_ptr(8));
  HGP_LAUNCH_CHECK();
}

void launch_rate_topk_rows(const LevelView &L, const int32_t *total, int32_t omega, int32_t delta,
                           const int32_t *list, const int64_t *count, int32_t n_rows, const int32_t *row_slot,
                           int32_t *rows, int32_t *pair, int64_t *score, TopK &tk, int words_per_id, DevBuf &acc,
                           int32_t *err, hipStream_t s) {
  if (L.n <= 0 || n_rows <= 0) return;
  const int64_t words = (int64_t)words_per_id * L.n;
  if (words > kTopKMaxWords) throw Error(-7, "top-K window exceeds LDS");
  KScope ks(8, s);
  const size_t bytes = (size_t)words * 4;
  static const bool attr_set = [] {
    HGP_HIP(hipFuncSetAttribute((const void *)k_rate_topk<TOPK_NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                kTopKMaxWords * 4));
    HGP_HIP(hipFuncSetAttribute((const void *)k_tail_hist<TOPK_NT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                kTopKMaxWords * 4));
    return true;
  }();
  (void)attr_set;
  // about 2048 workgroups over the rows, at most 256 slices per row
  const int slices = (int)std::max<int64_t>(1, std::min<int64_t>(256, (2048 + n_rows - 1) / n_rows));
  acc.reserve((size_t)n_rows * words * 4);
  uint32_t *a = acc.as<uint32_t>();
  fill_i32(reinterpret_cast<int32_t *>(a), (int64_t)n_rows * words, 0, s);
  k_tail_hist<TOPK_NT><<<n_rows * slices, TOPK_NT, bytes, s>>>(L.n, list, n_rows, slices, L.ioff, L.inc, L.hoff,
                                                               L.hpin, L.hw, L.size, L.indeg, total, omega,
                                                               (int32_t)words, a, err, units_ptr(8));
  HGP_LAUNCH_CHECK();
  const int grid = n_rows < TOPK_GRID ? n_rows : TOPK_GRID;
  k_rate_topk<TOPK_NT><<<grid, TOPK_NT, bytes, s>>>(L.n, list, count, L.ioff, L.inc, L.hoff, L.hpin, L.hw, L.size,
                                                    L.indeg, total, omega, delta, row_slot, rows, pair, score, tk.key,
                                                    tk.cnt, tk.kappa, (int32_t)words, a, err, units_ptr(8));
  HGP_LAUNCH_CHECK();
}

void launch_rate_update(int32_t n_fine, const int32_t *match, const int32_t *gamma, const TopK &old_tk,
                        int32_t n_new, const int32_t *newc, const int32_t *rows, int32_t n_coarse, TopK &tk,
                        int32_t *pair, int64_t *score, int32_t *rerate, int64_t *rerate_cnt, hipStream_t s) {
  if (n_fine <= 0) return;
  KScope ks(8, s);
  k_rate_update<<<div_up(n_fine, 256), 256, 0, s>>>(n_fine, match, gamma, old_tk.key, old_tk.cnt, old_tk.kappa, n_new,
                                                    newc, rows, n_coarse, tk.key, tk.cnt, tk.kappa, pair, score,
                                                    rerate, rerate_cnt);
  HGP_LAUNCH_CHECK();
}

__global__ void k_max_counter_bits(const int32_t *__restrict__ total, const int32_t *__restrict__ indeg, int32_t n,
                                   int32_t *out) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int b = 0;
  if (v < n) {
    const uint32_t t = (uint32_t)total[v], d = (uint32_t)indeg[v];
    b = (t ? 32 - __clz(t) : 0) + (d ? 32 - __clz(d) : 0);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) b = max(b, __shfl_xor(b, o, 64));
  if (lane_id() == 0 && b) atomicMax(out, b);
}

void launch_max_counter_bits(const int32_t *total, const int32_t *indeg, int32_t n, int32_t *out, hipStream_t s) {
  fill_i32(out, 1, 0, s);
  if (n <= 0) return;
  k_max_counter_bits<<<div_up(n, 256), 256, 0, s>>>(total, indeg, n, out);
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

}  // namespace hgp
