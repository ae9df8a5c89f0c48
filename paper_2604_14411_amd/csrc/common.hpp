// Internal declarations shared by the libhgp translation units (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace hgp {

constexpr uint32_t kDst = 0x80000000u;  // destination flag carried in bit 31 of pins / incidences
constexpr uint32_t kIdMask = 0x7fffffffu;

// Largest hedge handled by the LDS-resident per-hedge kernels (pins).
constexpr int kSegCap = 4096;

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

__host__ __device__ inline int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// ---------------------------------------------------------------------------
// Optional per-kernel-class timing with HIP events (enabled per call).
// ---------------------------------------------------------------------------
constexpr int kNKClass = 8;
struct KTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  hipEvent_t pending = nullptr;
  int64_t units[kNKClass] = {};
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
  KScope(int c, hipStream_t st) : cls(c), s(st), on(g_ktimer && g_ktimer->on) {
    if (on) g_ktimer->begin(s);
  }
  ~KScope() {
    if (on) g_ktimer->end(cls, s);
  }
};
inline void add_units(int cls, int64_t u) {
  if (g_ktimer && g_ktimer->on) g_ktimer->units[cls] += u;
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

// Fill / iota helpers.
void fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
void fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s);
void iota_i32(int32_t *p, int64_t n, hipStream_t s);

}  // namespace hgp
