// Internal declarations shared by the libhgp translation units (gfx950, wave64).
#pragma once
#include <type_traits>

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace hgp {

constexpr uint32_t kDst = 0x80000000u;  // destination flag carried in bit 31 of pins / incidences
constexpr uint32_t kIdMask = 0x7fffffffu;

// Largest hedge handled by the LDS-resident per-hedge kernels (pins).
constexpr int kSegCap = 4096;
// Largest hedge supported at all: longer than kSegCap, the per-hedge
// workgroup kernels sort in global scratch; pin positions within a hedge
// then still fit 15 bits and pin counts the 16-bit fields of the part tables.
constexpr int kHugeCap = 32767;

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void hip_fail(hipError_t e, const char *what, const char *file, int line);

#define HGP_HIP(call)                                              \
  do {                                                             \
    hipError_t _e = (call);                                        \
    if (_e != hipSuccess) ::hgp::hip_fail(_e, #call, __FILE__, __LINE__); \
  } while (0)

#define HGP_LAUNCH_CHECK() HGP_HIP(hipGetLastError())

inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Counts of DevBuf device allocations and frees (diagnostics).
extern std::atomic<int64_t> g_dev_allocs, g_dev_frees;

// Pinned host words for small device-to-host reads.  A copy into pageable
// memory is staged and blocks the host copy by copy; into pinned memory it is
// a plain asynchronous copy, so the reads of one step share a single stream
// synchronisation.
struct HostBox {
  static constexpr int kWords = 64;
  int64_t *p = nullptr;
  int64_t *get();  // allocated on first use
  void release();
};

// Grow-only device buffer owned by a context.
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  void reserve(size_t need);
  void release();
  template <class T>
  T *as() const {
    return static_cast<T *>(ptr);
  }
};

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

template <class T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T t = __shfl_up(v, o, 64);
    if (l >= o) v += t;
  }
  return v;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Slots of the LDS hash set of inbound_common for a node with `din` inbound
// hedges: the power of two at least twice din (at least 64).
__host__ __device__ inline int inbound_slots(uint32_t din) {
  int s = 64;
  while ((uint32_t)s < 2u * din) s <<= 1;
  return s;
}

// c(n, m) = |in(n) ∩ in(m)| (hedges holding both nodes as destinations) for
// the candidates m = key[r] & 0xffffffff, r < cnt, into c[r]: n's inbound
// hedges go into an open-addressing hash set of `slots` LDS words (a power
// of two, at least twice their number: probes always end), then one wave per
// candidate looks up the candidate's inbound hedges.  Block-wide; the caller
// synchronises before the table's words are reused.
template <int NT>
__device__ void inbound_common(int n, const int32_t *__restrict__ ioff, const uint32_t *__restrict__ inc,
                               uint32_t *table, int slots, const uint64_t *key, int32_t *c, int cnt) {
  const int tid = threadIdx.x, w = tid >> 6, l = lane_id();
  const uint32_t mask = (uint32_t)slots - 1u, empty = 0xffffffffu;
  for (int i = tid; i < slots; i += NT) table[i] = empty;
  __syncthreads();
  for (int i = ioff[n] + tid; i < ioff[n + 1]; i += NT) {
    const uint32_t v = inc[i];
    if (!(v >> 31)) continue;  // n is a source of this hedge
    const uint32_t e = v & kIdMask;
    for (uint32_t h = (e * 2654435761u) & mask;; h = (h + 1u) & mask) {
      const uint32_t old = atomicCAS(&table[h], empty, e);
      if (old == empty || old == e) break;
    }
  }
  __syncthreads();
  constexpr int B = 8;  // incidences loaded per lane before they are looked up
  for (int r = w; r < cnt; r += NT / 64) {
    const int m = (int)(key[r] & 0xffffffffull);
    const int j1 = ioff[m + 1];
    int k = 0;
    for (int j0 = ioff[m]; j0 < j1; j0 += 64 * B) {
      uint32_t v[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int j = j0 + u * 64 + l;
        v[u] = j < j1 ? inc[j] : 0u;  // 0: not a destination, skipped
      }
#pragma unroll
      for (int u = 0; u < B; ++u) {
        if (!(v[u] >> 31)) continue;
        const uint32_t e = v[u] & kIdMask;
        for (uint32_t h = (e * 2654435761u) & mask;; h = (h + 1u) & mask) {
          const uint32_t t = table[h];
          if (t == e) {
            ++k;
            break;
          }
          if (t == empty) break;
        }
      }
    }
    k = wave_sum(k);
    if (l == 0) c[r] = k;
  }
}

// Block-wide exclusive scan of a[0..n) in place (any address space).  Each
// thread scans a contiguous chunk; chunk totals are scanned by wave shuffles.
// `tmp` must hold NT/64 + 1 elements of shared memory.  Returns the total.
template <class T, int NT>
__device__ T block_exclusive_scan(T *a, int n, T *tmp) {
  const int tid = threadIdx.x;
  const int chunk = (n + NT - 1) / NT;
  const int b = tid * chunk;
  const int e = min(n, b + chunk);
  T s = 0;
  for (int i = b; i < e; ++i) s += a[i];
  T inc = wave_inclusive_scan(s);
  const int w = tid >> 6;
  if (lane_id() == 63) tmp[w] = inc;
  __syncthreads();
  if (tid == 0) {
    T run = 0;
    for (int i = 0; i < NT / 64; ++i) {
      T x = tmp[i];
      tmp[i] = run;
      run += x;
    }
    tmp[NT / 64] = run;
  }
  __syncthreads();
  T run = tmp[w] + inc - s;
  for (int i = b; i < e; ++i) {
    T x = a[i];
    a[i] = run;
    run += x;
  }
  T total = tmp[NT / 64];
  __syncthreads();
  return total;
}

// Block-wide bitonic sort (ascending) of s[0..n), n a power of two.
template <class K, int NT>
__device__ void block_bitonic_sort(K *s, int n) {
  for (int k = 2; k <= n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < (n >> 1); i += NT) {
        const int lo = ((i & ~(j - 1)) << 1) | (i & (j - 1));
        const int hi = lo + j;
        const bool asc = (lo & k) == 0;
        K a = s[lo], c = s[hi];
        if ((a > c) == asc) {
          s[lo] = c;
          s[hi] = a;
        }
      }
      __syncthreads();
    }
  }
}

// Make this wave's LDS writes visible to its other lanes (LDS operations of
// one wave execute in order; this keeps the compiler from reordering them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Streams, for the incidences i in [i0, i1) of one node (inc[i] = hedge |
// dst << 31), every entry j of each hedge's segment [soff[e], soff[e] + len)
// with len = soff[e+1] - soff[e] (LEN_FROM_END) or slen[e].  Each wave takes
// 64 incidences at a time, loads their segment bounds and weights in one
// round, then walks the concatenation of the 64 segments with every lane
// busy and U loads in flight per lane: load(j) fetches entry j, apply(v, info)
// consumes it with info = w(e) | (dst << 31).  tbl: 192 ints of LDS per wave.
// Returns the number of entries this wave streamed (uniform across the wave).
// With clip non-null (the segments' ascending pin ids, bit 31 masked off),
// each segment is first narrowed by binary search to the entries whose id
// lies in [clip_lo, clip_hi): a rating over several LDS windows then streams
// each pin once instead of once per window.
// ROLE 1 streams only the incidences with the destination bit (the hedges
// whose destination the node is), ROLE 2 only the others, ROLE 0 all.
// With PASS_OK, apply(v, info, ok) is called for every lane of every round,
// ok false for the lanes past the end (their v and info repeat the last
// entry), so that a caller can fold the mask into its update instead of
// branching around it.
// Loads in flight per lane in the ratings' pin streams: each round of U
// loads waits out one cache latency before its LDS updates, so the pin rate
// of a latency-bound stream grows with U.
constexpr int kRateU = 16;

template <int NW, int U, bool LEN_FROM_END, class V, bool PASS_OK = false, int ROLE = 0, class Load, class Apply>
__device__ __forceinline__ int64_t stream_segments(int i0, int i1, const uint32_t *__restrict__ inc,
                                                   const int32_t *__restrict__ soff, const int32_t *__restrict__ slen,
                                                   const int32_t *__restrict__ hw, int32_t *tbl, Load load,
                                                   Apply apply, const uint32_t *__restrict__ clip = nullptr,
                                                   int clip_lo = 0, int clip_hi = 0) {
  const int w = threadIdx.x >> 6, l = lane_id();
  int64_t streamed = 0;
  int32_t *t_end = tbl + w * 192;
  int32_t *t_shift = t_end + 64;
  uint32_t *t_info = reinterpret_cast<uint32_t *>(t_end + 128);
  for (int base = i0 + w * 64; base < i1; base += NW * 64) {
    const int idx = base + l;
    int b = 0, len = 0;
    uint32_t info = 0;
    uint32_t x = 0;
    bool take = idx < i1;
    if (take) {
      x = inc[idx];
      if constexpr (ROLE == 1) take = (x & kDst) != 0u;
      if constexpr (ROLE == 2) take = (x & kDst) == 0u;
    }
    if (take) {
      const int e = (int)(x & kIdMask);
      b = soff[e];
      len = LEN_FROM_END ? soff[e + 1] - b : slen[e];
      info = (uint32_t)hw[e] | (x & kDst);
      if (clip) {
        int a = b, z = b + len;
        while (a < z) {
          const int mid = (a + z) >> 1;
          if ((int)(clip[mid] & kIdMask) < clip_lo) a = mid + 1;
          else z = mid;
        }
        int c = a;
        z = b + len;
        while (c < z) {
          const int mid = (c + z) >> 1;
          if ((int)(clip[mid] & kIdMask) < clip_hi) c = mid + 1;
          else z = mid;
        }
        b = a;
        len = c - a;
      }
    }
    const int incl = wave_inclusive_scan(len);
    const int total = __shfl(incl, 63, 64);
    t_end[l] = incl;
    t_shift[l] = b - (incl - len);
    t_info[l] = info;
    wave_lds_sync();
    // per-lane cursor over the 64 segments, its bounds cached in registers
    int k = 0;
    int k_end = t_end[0];
    int k_shift = t_shift[0];
    uint32_t k_info = t_info[0];
    streamed += total;
    // lanes past the end re-read the last entry (always in bounds), so the
    // loads need no branch; only apply is masked
    for (int v0 = 0; v0 < total; v0 += 64 * U) {
      int jj[U];
      uint32_t ii[U];
      bool ok[U];
      V vv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int v = v0 + u * 64 + l;
        ok[u] = v < total;
        const int vc = ok[u] ? v : total - 1;
        while (k_end <= vc) {
          ++k;
          k_end = t_end[k];
          k_shift = t_shift[k];
          k_info = t_info[k];
        }
        jj[u] = vc + k_shift;
        ii[u] = k_info;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) vv[u] = load(jj[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if constexpr (PASS_OK)
          apply(vv[u], ii[u], ok[u]);
        else if (ok[u])
          apply(vv[u], ii[u]);
      }
    }
    wave_lds_sync();
  }
  return streamed;
}

// Calls f(std::integral_constant<int, mode>) for mode 0, 1 or 2, so that a
// streaming loop is compiled once per counter layout instead of branching on
// it for every entry.
template <class F>
__device__ __forceinline__ int64_t with_mode(int mode, F f) {
  if (mode == 0) return f(std::integral_constant<int, 0>{});
  if (mode == 1) return f(std::integral_constant<int, 1>{});
  return f(std::integral_constant<int, 2>{});
}

// Workgroups are dealt to the device's 8 XCDs round-robin by workgroup index.
// xcd_node maps workgroup b of a grid of xcd_grid(N) to a node so that XCD x
// handles the contiguous ids [x*per, (x+1)*per): nodes with nearby ids share
// hedges in layered networks, and their pin re-reads then hit the same L2.
// Returns -1 for the padding workgroups.
constexpr int kXcds = 8;
__host__ __device__ inline int xcd_grid(int N) { return ((N + kXcds - 1) / kXcds) * kXcds; }
__device__ __forceinline__ int xcd_node(int b, int N) {
  const int per = (N + kXcds - 1) / kXcds;
  const int n = (b % kXcds) * per + b / kXcds;
  return n < N ? n : -1;
}

// Smallest and largest pin id over the hedges of incidences [i0, i1) (pins are
// ascending per hedge: first and last pin).  Block-wide; red: NT/64 int2 of LDS.
// Empty range: (INT_MAX, -1).
template <int NT>
__device__ int2 neighbour_range(int i0, int i1, const uint32_t *__restrict__ inc, const int32_t *__restrict__ hoff,
                                const uint32_t *__restrict__ hpin, int2 *red) {
  int lo = 0x7fffffff, hi = -1;
  // four incidences per thread in flight through the three dependent loads
  // (a coarse cluster has tens of thousands of incidences)
  for (int i = i0 + (int)threadIdx.x; i < i1; i += 4 * NT) {
    int e[4], b[4], en[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) e[u] = i + u * NT < i1 ? (int)(inc[i + u * NT] & kIdMask) : -1;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      b[u] = e[u] >= 0 ? hoff[e[u]] : 0;
      en[u] = e[u] >= 0 ? hoff[e[u] + 1] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (en[u] > b[u]) {
        lo = min(lo, (int)(hpin[b[u]] & kIdMask));
        hi = max(hi, (int)(hpin[en[u] - 1] & kIdMask));
      }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o, 64));
    hi = max(hi, __shfl_xor(hi, o, 64));
  }
  if (lane_id() == 0) red[threadIdx.x >> 6] = make_int2(lo, hi);
  __syncthreads();
  int2 r = red[0];
#pragma unroll
  for (int q = 1; q < NT / 64; ++q) {
    r.x = min(r.x, red[q].x);
    r.y = max(r.y, red[q].y);
  }
  __syncthreads();
  return r;
}

// Adds a per-wave count to a device counter (one atomic per wave).
__device__ __forceinline__ void add_wave_units(unsigned long long *units, int64_t v) {
  if (units && lane_id() == 0 && v) atomicAdd(units, (unsigned long long)v);
}

// Bitonic sort (ascending) of 64*KPL keys held by one wave in registers; key
// i = lane * KPL + j sits in k[j] of that lane.  Compare-exchange partners
// closer than KPL are in the same lane, the others one xor-shuffle away.
template <int KPL, class K>
__device__ __forceinline__ void wave_bitonic_sort(K (&k)[KPL]) {
  const int l = lane_id();
#pragma unroll
  for (int size = 2; size <= 64 * KPL; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride >= KPL) {
        const int lx = stride / KPL;
        const bool lower = (l & lx) == 0;
#pragma unroll
        for (int j = 0; j < KPL; ++j) {
          const bool asc = ((l * KPL + j) & size) == 0;
          const K other = __shfl_xor(k[j], lx, 64);
          k[j] = (lower == asc) ? (k[j] < other ? k[j] : other) : (k[j] < other ? other : k[j]);
        }
      } else {
#pragma unroll
        for (int j = 0; j < KPL; ++j) {
          const int p = j ^ stride;
          if (p > j) {
            const bool asc = ((l * KPL + j) & size) == 0;
            const K a = k[j], b = k[p];
            if ((a > b) == asc) {
              k[j] = b;
              k[p] = a;
            }
          }
        }
      }
    }
  }
}

template <class T>
__device__ __forceinline__ T wave_exclusive_scan(T v) {
  return wave_inclusive_scan(v) - v;
}

__host__ __device__ inline int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// ---------------------------------------------------------------------------
// Optional per-kernel-class timing with HIP events (enabled per call).
// ---------------------------------------------------------------------------
constexpr int kNKClass = 10;
struct KTimer {
  bool on = false;
  uint32_t mask = ~0u;  // classes timed while on; kernels count their own units only for these
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  hipEvent_t pending = nullptr;
  int64_t units[kNKClass] = {};
  unsigned long long *units_dev = nullptr;  // device counters, one per class
  hipEvent_t take();
  void begin(hipStream_t s);
  void end(int cls, hipStream_t s);
  void reset();
  void resolve(double *ms, int64_t *cnt);
  void destroy();
};
extern thread_local KTimer *g_ktimer;

struct KScope {
  int cls;
  hipStream_t s;
  bool on;
  KScope(int c, hipStream_t st) : cls(c), s(st), on(g_ktimer && g_ktimer->on && ((g_ktimer->mask >> c) & 1u)) {
    if (on) g_ktimer->begin(s);
  }
  ~KScope() {
    if (on) g_ktimer->end(cls, s);
  }
};
inline void add_units(int cls, int64_t u) {
  if (g_ktimer && g_ktimer->on) g_ktimer->units[cls] += u;
}
// Device counter for kernels that count their own algorithmic units (per
// wave, atomics on one address: only for the classes being timed).
inline unsigned long long *units_ptr(int cls) {
  return (g_ktimer && g_ktimer->on && g_ktimer->units_dev && ((g_ktimer->mask >> cls) & 1u))
             ? g_ktimer->units_dev + cls
             : nullptr;
}

// ---------------------------------------------------------------------------
// Host-side primitives (prims.hip)
// ---------------------------------------------------------------------------

// Exclusive scan of n int32 (or int64) values; out may alias in.  If total is
// non-null the grand total is written there (device).
void scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *total, DevBuf &tmp, hipStream_t s);
void scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total, DevBuf &tmp, hipStream_t s);

// Stable LSD radix sort of n uint64 keys over bits [0, bits); keys are in
// `keys` on entry and exit (ping-pong through `alt`).  Optional uint32 values
// travel with the keys (vals / valt).
void radix_sort_u64(uint64_t *keys, uint64_t *alt, uint32_t *vals, uint32_t *valt, int64_t n, int bits,
                    DevBuf &tmp, hipStream_t s);

// (32-bit keys: bits [lo, bits) only; keys equal on them keep their order.)
void radix_sort_u32(uint32_t *keys, uint32_t *alt, uint32_t *vals, uint32_t *valt, int64_t n, int bits,
                    DevBuf &tmp, hipStream_t s, int lo = 0);
// Sorts 32-bit keys (bits [0, bits)) with 64-bit values, stable; the sorted
// values are written as their high halves to out_hi and low halves to out_lo
// (the keys end sorted in keys; vals and valt are overwritten).
void radix_sort_u32_split(uint32_t *keys, uint32_t *alt, uint64_t *vals, uint64_t *valt, int64_t n, int bits,
                          uint32_t *out_hi, uint32_t *out_lo, DevBuf &tmp, hipStream_t s);

// Fill / iota helpers.
void fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
void fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s);
void iota_i32(int32_t *p, int64_t n, hipStream_t s);

}  // namespace hgp
