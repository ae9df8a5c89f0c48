// Device-wide primitives: exclusive scans, stable LSD radix sort, fills.
#include "common.hpp"

#include <atomic>

#include <cstdio>

namespace hgp {

void hip_fail(hipError_t e, const char *what, const char *file, int line) {
  char buf[512];
  snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  if (e == hipErrorOutOfMemory) throw Error(-4, buf);
  throw Error(-5, buf);
}

thread_local KTimer *g_ktimer = nullptr;

hipEvent_t KTimer::take() {
  if (used == pool.size()) {
    hipEvent_t e;
    HGP_HIP(hipEventCreate(&e));
    pool.push_back(e);
  }
  return pool[used++];
}

void KTimer::begin(hipStream_t s) {
  pending = take();
  HGP_HIP(hipEventRecord(pending, s));
}

void KTimer::end(int cls, hipStream_t s) {
  hipEvent_t b = take();
  HGP_HIP(hipEventRecord(b, s));
  recs.push_back({cls, pending, b});
}

void KTimer::reset() {
  used = 0;
  recs.clear();
  for (auto &u : units) u = 0;
}

void KTimer::resolve(double *ms, int64_t *cnt) {
  for (const Rec &r : recs) {
    float t = 0.f;
    HGP_HIP(hipEventSynchronize(r.b));
    HGP_HIP(hipEventElapsedTime(&t, r.a, r.b));
    ms[r.cls] += t;
    cnt[r.cls] += 1;
  }
}

void KTimer::destroy() {
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  pool.clear();
  used = 0;
  recs.clear();
}

// Device allocations and frees made through DevBuf (diagnostics: printed per
// partition with HGP_LOG=1).
std::atomic<int64_t> g_dev_allocs{0}, g_dev_frees{0};

void DevBuf::reserve(size_t need) {
  if (need <= bytes) return;
  const size_t old = bytes;
  release();
  g_dev_allocs.fetch_add(1, std::memory_order_relaxed);
  // grow by at least a quarter: fewer reallocations (each hipFree
  // synchronises the device)
  size_t b = need < 256 ? 256 : need;
  if (old && b < old + old / 4) b = old + old / 4;
  b = (b + 255) & ~size_t(255);
  hipError_t e = hipMalloc(&ptr, b);
  if (e != hipSuccess) {
    ptr = nullptr;
    bytes = 0;
    (void)hipGetLastError();
    throw Error(-4, "device allocation of " + std::to_string(b) + " bytes failed");
  }
  bytes = b;
}

int64_t *HostBox::get() {
  if (!p) {
    void *q = nullptr;
    HGP_HIP(hipHostMalloc(&q, kWords * sizeof(int64_t), hipHostMallocDefault));
    p = static_cast<int64_t *>(q);
  }
  return p;
}

void HostBox::release() {
  if (p) (void)hipHostFree(p);
  p = nullptr;
}

void DevBuf::release() {
  if (ptr) {
    (void)hipFree(ptr);
    g_dev_frees.fetch_add(1, std::memory_order_relaxed);
  }
  ptr = nullptr;
  bytes = 0;
}

// ---------------------------------------------------------------------------
// fills
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_fill(T *p, int64_t n, T v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_iota(int32_t *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// scans
// ---------------------------------------------------------------------------
constexpr int SC_NT = 256;
constexpr int SC_TILE = 4096;

template <class T>
__global__ __launch_bounds__(SC_NT) void k_tile_sum(const T *__restrict__ in, int64_t n, T *__restrict__ bsum) {
  __shared__ T red[SC_NT / 64];
  const int64_t base = (int64_t)blockIdx.x * SC_TILE;
  T s = 0;
  for (int i = threadIdx.x; i < SC_TILE; i += SC_NT) {
    const int64_t j = base + i;
    if (j < n) s += in[j];
  }
  s = wave_sum(s);
  if (lane_id() == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    T t = 0;
    for (int w = 0; w < SC_NT / 64; ++w) t += red[w];
    bsum[blockIdx.x] = t;
  }
}

template <class T>
__global__ __launch_bounds__(SC_NT) void k_tile_scan(const T *in, T *out, int64_t n, const T *__restrict__ boff,
                                                     T *total) {
  __shared__ T tile[SC_TILE];
  __shared__ T tmp[SC_NT / 64 + 1];
  const int64_t base = (int64_t)blockIdx.x * SC_TILE;
  for (int i = threadIdx.x; i < SC_TILE; i += SC_NT) {
    const int64_t j = base + i;
    tile[i] = j < n ? in[j] : T(0);
  }
  __syncthreads();
  T tot = block_exclusive_scan<T, SC_NT>(tile, SC_TILE, tmp);
  const T off = boff ? boff[blockIdx.x] : T(0);
  for (int i = threadIdx.x; i < SC_TILE; i += SC_NT) {
    const int64_t j = base + i;
    if (j < n) out[j] = tile[i] + off;
  }
  if (total && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *total = off + tot;
}

// Exclusive scan of up to SC_ONE_MAX elements by one workgroup (one launch
// where the tiled scan takes three): in is copied to out, then scanned in
// place, each thread owning a contiguous chunk.
constexpr int SC_ONE_NT = 1024;
constexpr int64_t SC_ONE_MAX = 16384;

template <class T>
__global__ __launch_bounds__(SC_ONE_NT) void k_scan_one(const T *in, T *out, int n, T *total) {
  __shared__ T tmp[SC_ONE_NT / 64 + 1];
  if (in != out)
    for (int i = threadIdx.x; i < n; i += SC_ONE_NT) out[i] = in[i];
  __syncthreads();
  const T tot = block_exclusive_scan<T, SC_ONE_NT>(out, n, tmp);
  if (total && threadIdx.x == 0) *total = tot;
}

template <class T>
static void scan_impl(const T *in, T *out, int64_t n, T *total, T *tmp, hipStream_t s) {
  if (n <= 0) {
    if (total) {
      k_fill<T><<<1, 1, 0, s>>>(total, 1, T(0));
      HGP_LAUNCH_CHECK();
    }
    return;
  }
  const int64_t nb = (n + SC_TILE - 1) / SC_TILE;
  if (nb > 1 && n <= SC_ONE_MAX) {
    k_scan_one<T><<<1, SC_ONE_NT, 0, s>>>(in, out, (int)n, total);
    HGP_LAUNCH_CHECK();
    return;
  }
  if (nb == 1) {
    k_tile_scan<T><<<1, SC_NT, 0, s>>>(in, out, n, nullptr, total);
    HGP_LAUNCH_CHECK();
    return;
  }
  T *bsum = tmp;
  k_tile_sum<T><<<(unsigned)nb, SC_NT, 0, s>>>(in, n, bsum);
  HGP_LAUNCH_CHECK();
  scan_impl<T>(bsum, bsum, nb, nullptr, tmp + ((nb + 63) & ~int64_t(63)), s);
  k_tile_scan<T><<<(unsigned)nb, SC_NT, 0, s>>>(in, out, n, bsum, total);
  HGP_LAUNCH_CHECK();
}

static size_t scan_tmp_elems(int64_t n) {
  size_t t = 0;
  while (n > SC_TILE) {
    n = (n + SC_TILE - 1) / SC_TILE;
    t += (size_t)((n + 63) & ~int64_t(63));
  }
  return t + 64;
}

void scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *total, DevBuf &tmp, hipStream_t s) {
  tmp.reserve(scan_tmp_elems(n) * sizeof(int32_t));
  scan_impl<int32_t>(in, out, n, total, tmp.as<int32_t>(), s);
}

void scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total, DevBuf &tmp, hipStream_t s) {
  tmp.reserve(scan_tmp_elems(n) * sizeof(int64_t));
  scan_impl<int64_t>(in, out, n, total, tmp.as<int64_t>(), s);
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, DB-bit digits (8 in use), 4096-key tiles
// ---------------------------------------------------------------------------
constexpr int RS_NT = 256;
constexpr int RS_ROUNDS = 16;
constexpr int RS_TILE = RS_NT * RS_ROUNDS;

// Rank of a key within its digit among the valid lanes of the wave (match
// mask from DB ballots); returns the rank, *cnt = size of the digit group.
template <int DB>
__device__ __forceinline__ int rs_wave_rank(bool valid, uint32_t d, uint64_t lt, int *cnt) {
  uint64_t match = __ballot(valid);
#pragma unroll
  for (int b = 0; b < DB; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bb = __ballot(valid && bit);
    match &= bit ? bb : ~bb;
  }
  *cnt = __popcll(match);
  return __popcll(match & lt);
}

// Wave w of a tile owns its keys w * RS_WKEYS + r * 64 + lane (r < RS_ROUNDS):
// the waves' key ranges are contiguous and in tile order, so a wave ranks
// its keys alone (tile order within the wave: round, then lane) and the
// waves' digit counts are combined once.
constexpr int RS_WKEYS = RS_ROUNDS * 64;

// Digit counts of one 4096-key tile: LDS atomics on per-wave counters.  All of
// the tile's loads are issued first.
// hist is digit-major: hist[d * ntiles + tile].
template <class K, int DB>
__global__ __launch_bounds__(RS_NT) void k_rs_hist(const K *__restrict__ keys, int64_t n, int shift,
                                                   int32_t *__restrict__ hist, int ntiles) {
  constexpr int RADIX = 1 << DB;
  __shared__ int32_t cw[RS_NT / 64][RADIX];
  const int tid = threadIdx.x, w = tid >> 6, l = lane_id();
  for (int i = tid; i < RS_NT / 64 * RADIX; i += RS_NT) (&cw[0][0])[i] = 0;
  const int64_t base = (int64_t)blockIdx.x * RS_TILE + w * RS_WKEYS + l;
  K kr[RS_ROUNDS];
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t j = base + r * 64;
    kr[r] = j < n ? keys[j] : K(0);
  }
  __syncthreads();
  // LDS atomics on the wave's own counters (lanes of one digit serialise in
  // the LDS unit, but no ranks are needed here)
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const bool valid = base + r * 64 < n;
    const uint32_t d = (uint32_t)(kr[r] >> shift) & (uint32_t)(RADIX - 1);
    if (valid) atomicAdd(&cw[w][d], 1);
  }
  __syncthreads();
  for (int d = tid; d < RADIX; d += RS_NT) {
    int32_t c = 0;
#pragma unroll
    for (int q = 0; q < RS_NT / 64; ++q) c += cw[q][d];
    hist[(int64_t)d * ntiles + blockIdx.x] = c;
  }
}

// Per digit d (one workgroup each): exclusive scan over the tiles of
// hist[d * ntiles ..], in place, and the digit's total in dtot[d].
__global__ __launch_bounds__(RS_NT) void k_rs_dscan(int32_t *__restrict__ hist, int ntiles,
                                                    int32_t *__restrict__ dtot) {
  __shared__ int32_t stmp[RS_NT / 64 + 1];
  const int32_t t = block_exclusive_scan<int32_t, RS_NT>(hist + (int64_t)blockIdx.x * ntiles, ntiles, stmp);
  if (threadIdx.x == 0) dtot[blockIdx.x] = t;
}

// gbase[d] = start of digit d in the output (exclusive scan of dtot, in LDS)
// + start of this tile within digit d.
template <int RADIX>
__device__ __forceinline__ void rs_tile_bases(const int32_t *__restrict__ offs, const int32_t *__restrict__ dtot,
                                              int ntiles, int32_t *gbase, int32_t *stmp) {
  for (int d = threadIdx.x; d < RADIX; d += RS_NT) gbase[d] = dtot[d];
  __syncthreads();
  block_exclusive_scan<int32_t, RS_NT>(gbase, RADIX, stmp);
  for (int d = threadIdx.x; d < RADIX; d += RS_NT) gbase[d] += offs[(int64_t)d * ntiles + blockIdx.x];
  __syncthreads();
}

template <class VT, bool SPLIT>
__device__ __forceinline__ void rs_put_val(VT v, int64_t pos, VT *__restrict__ ovals, uint32_t *__restrict__ ohi,
                                           uint32_t *__restrict__ olo) {
  if constexpr (SPLIT) {
    ohi[pos] = (uint32_t)((uint64_t)v >> 32);
    olo[pos] = (uint32_t)v;
  } else {
    ovals[pos] = v;
  }
}

// Stable scatter of one 4096-key tile.  Each wave loads its contiguous key
// range into registers and ranks every key within its digit among the
// wave's earlier keys (ballot match masks and a running per-wave count in
// LDS, no workgroup barrier); one barrier later the waves' counts give each
// digit's offset per wave.  With LDS staging (32-bit keys) the tile is placed
// in LDS in digit order and written out so that each digit's run goes to
// consecutive addresses; 64-bit keys go straight to their slots.
// offs: scanned (digit, tile) offsets within each digit; dtot: digit totals.
// VT: the value word; with SPLIT (64-bit values) the values are written as
// their high and low halves to ohi / olo instead of to ovals.
template <class K, bool V, bool STAGE, int DB, class VT = uint32_t, bool SPLIT = false>
__global__ __launch_bounds__(RS_NT) void k_rs_scatter(const K *__restrict__ keys, const VT *__restrict__ vals,
                                                      int64_t n, int shift, const int32_t *__restrict__ offs,
                                                      const int32_t *__restrict__ dtot, int ntiles,
                                                      K *__restrict__ okeys, VT *__restrict__ ovals,
                                                      uint32_t *__restrict__ ohi, uint32_t *__restrict__ olo) {
  constexpr int RADIX = 1 << DB;
  __shared__ int32_t gbase[RADIX];
  __shared__ int32_t lstart[RADIX];
  __shared__ int32_t cw[RS_NT / 64][RADIX];
  __shared__ int32_t stmp[RS_NT / 64 + 1];
  __shared__ K lkeys[STAGE ? RS_TILE : 1];
  __shared__ VT lvals[(STAGE && V) ? RS_TILE : 1];
  const int tid = threadIdx.x, w = tid >> 6, l = lane_id();
  const int64_t tbase = (int64_t)blockIdx.x * RS_TILE;
  const int64_t base = tbase + w * RS_WKEYS + l;
  K kr[RS_ROUNDS];
  VT vr[V ? RS_ROUNDS : 1];
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const int64_t j = base + r * 64;
    kr[r] = j < n ? keys[j] : K(0);
    if (V) vr[r] = j < n ? vals[j] : VT(0);
  }
  for (int i = tid; i < RS_NT / 64 * RADIX; i += RS_NT) (&cw[0][0])[i] = 0;
  rs_tile_bases<RADIX>(offs, dtot, ntiles, gbase, stmp);  // its barriers also order the zeroing above
  // ranks within the wave (running per-wave digit counts)
  const uint64_t lt = (l == 0) ? 0ull : ((~0ull) >> (64 - l));
  int16_t rk[RS_ROUNDS];
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const bool valid = base + r * 64 < n;
    const uint32_t d = (uint32_t)(kr[r] >> shift) & (uint32_t)(RADIX - 1);
    int cnt;
    const int rank = rs_wave_rank<DB>(valid, d, lt, &cnt);
    rk[r] = (int16_t)(cw[w][d] + rank);
    wave_lds_sync();
    if (valid && rank == cnt - 1) cw[w][d] += cnt;
    wave_lds_sync();
  }
  __syncthreads();
  // per digit: counts of the earlier waves, and the digit's start in the tile
  for (int d = tid; d < RADIX; d += RS_NT) {
    int32_t run = 0;
#pragma unroll
    for (int q = 0; q < RS_NT / 64; ++q) {
      const int32_t c = cw[q][d];
      cw[q][d] = run;
      run += c;
    }
    lstart[d] = run;
  }
  __syncthreads();
  block_exclusive_scan<int32_t, RS_NT>(lstart, RADIX, stmp);
#pragma unroll
  for (int r = 0; r < RS_ROUNDS; ++r) {
    if (base + r * 64 >= n) continue;
    const uint32_t d = (uint32_t)(kr[r] >> shift) & (uint32_t)(RADIX - 1);
    const int within = cw[w][d] + rk[r];  // position among the tile's keys of digit d
    if (STAGE) {
      const int lp = lstart[d] + within;
      lkeys[lp] = kr[r];
      if (V) lvals[lp] = vr[r];
    } else {
      const int64_t pos = (int64_t)gbase[d] + within;
      okeys[pos] = kr[r];
      if (V) rs_put_val<VT, SPLIT>(vr[r], pos, ovals, ohi, olo);
    }
  }
  if (STAGE) {
    __syncthreads();
    const int tn = (int)min((int64_t)RS_TILE, n - tbase);
    for (int i = tid; i < tn; i += RS_NT) {
      const K key = lkeys[i];
      const uint32_t d = (uint32_t)(key >> shift) & (uint32_t)(RADIX - 1);
      const int64_t pos = (int64_t)gbase[d] + (i - lstart[d]);
      okeys[pos] = key;
      if (V) rs_put_val<VT, SPLIT>(lvals[i], pos, ovals, ohi, olo);
    }
  }
}

template <class K, int DB>
static void radix_pass(const K *src, const uint32_t *vs, int64_t n, int shift, int ntiles, int32_t *hist,
                       int32_t *dtot, K *dst, uint32_t *vd, hipStream_t s) {
  k_rs_hist<K, DB><<<ntiles, RS_NT, 0, s>>>(src, n, shift, hist, ntiles);
  HGP_LAUNCH_CHECK();
  k_rs_dscan<<<1 << DB, RS_NT, 0, s>>>(hist, ntiles, dtot);
  HGP_LAUNCH_CHECK();
  // 32-bit keys are staged in LDS for coalesced runs; 64-bit keys go direct
  constexpr bool kStage = sizeof(K) == 4;
  if (vs)
    k_rs_scatter<K, true, kStage, DB><<<ntiles, RS_NT, 0, s>>>(src, vs, n, shift, hist, dtot, ntiles, dst, vd,
                                                               nullptr, nullptr);
  else
    k_rs_scatter<K, false, kStage, DB><<<ntiles, RS_NT, 0, s>>>(src, vs, n, shift, hist, dtot, ntiles, dst, vd,
                                                                nullptr, nullptr);
  HGP_LAUNCH_CHECK();
}

// Sorts by bits [lo, bits) with 8-bit digits.  (10-bit digits, 3 passes
// instead of 4 for 25-30 bits, measured slower on rand64k: 1,024 digit runs
// per 4,096-key tile leave the scatter's writes poorly coalesced.)
template <class K>
static void radix_sort_impl(K *keys, K *alt, uint32_t *vals, uint32_t *valt, int64_t n, int lo, int bits,
                            DevBuf &tmp, hipStream_t s) {
  if (n <= 1 || bits <= lo) return;
  constexpr int db = 8;
  const int ntiles = (int)((n + RS_TILE - 1) / RS_TILE);
  const int64_t hn = (int64_t)(1 << db) * ntiles;
  const size_t hist_bytes = ((size_t)hn * sizeof(int32_t) + 255) & ~size_t(255);
  tmp.reserve(hist_bytes + 1024 * sizeof(int32_t));
  int32_t *hist = tmp.as<int32_t>();
  int32_t *dtot = reinterpret_cast<int32_t *>(static_cast<char *>(tmp.ptr) + hist_bytes);
  K *src = keys, *dst = alt;
  uint32_t *vs = vals, *vd = valt;
  int passes = 0;
  for (int shift = lo; shift < bits; shift += db, ++passes) {
    radix_pass<K, db>(src, vs, n, shift, ntiles, hist, dtot, dst, vd, s);
    std::swap(src, dst);
    std::swap(vs, vd);
  }
  if (passes & 1) {
    HGP_HIP(hipMemcpyAsync(keys, src, (size_t)n * sizeof(K), hipMemcpyDeviceToDevice, s));
    if (vals) HGP_HIP(hipMemcpyAsync(vals, vs, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  }
}

void radix_sort_u64(uint64_t *keys, uint64_t *alt, uint32_t *vals, uint32_t *valt, int64_t n, int bits,
                    DevBuf &tmp, hipStream_t s) {
  radix_sort_impl<uint64_t>(keys, alt, vals, valt, n, 0, bits, tmp, s);
}

void radix_sort_u32(uint32_t *keys, uint32_t *alt, uint32_t *vals, uint32_t *valt, int64_t n, int bits,
                    DevBuf &tmp, hipStream_t s, int lo) {
  radix_sort_impl<uint32_t>(keys, alt, vals, valt, n, lo, bits > 32 ? 32 : bits, tmp, s);
}

__global__ void k_split_u64(const uint64_t *__restrict__ v, int64_t n, uint32_t *__restrict__ hi,
                            uint32_t *__restrict__ lo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    hi[i] = (uint32_t)(v[i] >> 32);
    lo[i] = (uint32_t)v[i];
  }
}

void radix_sort_u32_split(uint32_t *keys, uint32_t *alt, uint64_t *vals, uint64_t *valt, int64_t n, int bits,
                          uint32_t *out_hi, uint32_t *out_lo, DevBuf &tmp, hipStream_t s) {
  if (n <= 0) return;
  constexpr int db = 8;
  bits = bits > 32 ? 32 : bits;
  if (n == 1 || bits <= 0) {
    k_split_u64<<<div_up(n, 256), 256, 0, s>>>(vals, n, out_hi, out_lo);
    HGP_LAUNCH_CHECK();
    return;
  }
  const int ntiles = (int)((n + RS_TILE - 1) / RS_TILE);
  const int64_t hn = (int64_t)(1 << db) * ntiles;
  const size_t hist_bytes = ((size_t)hn * sizeof(int32_t) + 255) & ~size_t(255);
  tmp.reserve(hist_bytes + 1024 * sizeof(int32_t));
  int32_t *hist = tmp.as<int32_t>();
  int32_t *dtot = reinterpret_cast<int32_t *>(static_cast<char *>(tmp.ptr) + hist_bytes);
  uint32_t *src = keys, *dst = alt;
  uint64_t *vs = vals, *vd = valt;
  int passes = 0;
  for (int shift = 0; shift < bits; shift += db, ++passes) {
    const bool last = shift + db >= bits;
    k_rs_hist<uint32_t, db><<<ntiles, RS_NT, 0, s>>>(src, n, shift, hist, ntiles);
    HGP_LAUNCH_CHECK();
    k_rs_dscan<<<1 << db, RS_NT, 0, s>>>(hist, ntiles, dtot);
    HGP_LAUNCH_CHECK();
    if (last)
      k_rs_scatter<uint32_t, true, true, db, uint64_t, true><<<ntiles, RS_NT, 0, s>>>(
          src, vs, n, shift, hist, dtot, ntiles, dst, nullptr, out_hi, out_lo);
    else
      k_rs_scatter<uint32_t, true, true, db, uint64_t, false><<<ntiles, RS_NT, 0, s>>>(
          src, vs, n, shift, hist, dtot, ntiles, dst, vd, nullptr, nullptr);
    HGP_LAUNCH_CHECK();
    std::swap(src, dst);
    std::swap(vs, vd);
  }
  if (passes & 1) HGP_HIP(hipMemcpyAsync(keys, src, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
}

void fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return;
  k_fill<int32_t><<<div_up(n, 256), 256, 0, s>>>(p, n, v);
  HGP_LAUNCH_CHECK();
}

void fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s) {
  if (n <= 0) return;
  k_fill<int64_t><<<div_up(n, 256), 256, 0, s>>>(p, n, v);
  HGP_LAUNCH_CHECK();
}

void iota_i32(int32_t *p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_iota<<<div_up(n, 256), 256, 0, s>>>(p, n);
  HGP_LAUNCH_CHECK();
}

}  // namespace hgp
