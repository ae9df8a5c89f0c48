// Micro-benchmark behind the peak that the LDS-atomic-bound kernels (the
// ratings' and proposals' part and neighbour histograms) are priced against:
// the rate of 32-bit LDS atomic adds without a return value that the whole
// device sustains.  Built as its own library (libhgp_probe.so); the
// partitioner does not use it.
//
//   int hgp_probe_lds_atomics(int random, int grid, int iters, uint32_t *out,
//                             void *stream, float *ms)
//
// Launches `grid` workgroups of 1024 threads on `stream` (a hipStream_t; null
// is the default stream).  Each workgroup clears 8192 LDS counters, each
// thread adds 8 times per iteration, `iters` iterations (the value added in
// iteration i is i + 1), and the counters are written to out[grid * 8192]
// (device memory, owned by the caller).  random = 0: lane t of a workgroup
// adds to words t, t + 1024, ..., t + 7168 (no bank conflicts; each counter
// ends at iters (iters + 1) / 2 modulo 2^32); random = 1: to 8 pseudo-random
// words per lane, shifted by 97 words every iteration (the conflict degree
// of random addresses; the workgroup's counters sum to 8192 iters (iters + 1)
// / 2 modulo 2^32).  *ms receives the launch's duration from HIP events
// recorded on `stream` around it.  Returns 0, or -1 for arguments outside
// grid >= 1, iters >= 1, out and ms non-null, or the HIP error code.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kNT = 1024;
constexpr int kU = 8;
constexpr int kWords = kU * kNT;

template <bool RANDOM>
__global__ __launch_bounds__(kNT) void k_lds_atomics(int iters, uint32_t *__restrict__ out) {
  __shared__ uint32_t cnt[kWords];
  const int tid = threadIdx.x;
  for (int i = tid; i < kWords; i += kNT) cnt[i] = 0u;
  __syncthreads();
  uint32_t base[kU];
  uint32_t h = (uint32_t)tid * 2654435761u ^ ((uint32_t)blockIdx.x * 40503u + 0x9E3779B9u);
#pragma unroll
  for (int u = 0; u < kU; ++u) {
    // xorshift32 per lane for the random bases
    h ^= h << 13;
    h ^= h >> 17;
    h ^= h << 5;
    base[u] = RANDOM ? h : (uint32_t)(u * kNT + tid);
  }
  uint32_t shift = 0;
  for (int it = 0; it < iters; ++it) {
    const uint32_t v = (uint32_t)it + 1u;
#pragma unroll
    for (int u = 0; u < kU; ++u) atomicAdd(&cnt[(base[u] + shift) & (kWords - 1)], v);
    if (RANDOM) shift += 97u;
  }
  __syncthreads();
  uint32_t *o = out + (int64_t)blockIdx.x * kWords;
  for (int i = tid; i < kWords; i += kNT) o[i] = cnt[i];
}

}  // namespace

extern "C" int hgp_probe_lds_atomics(int random, int grid, int iters, uint32_t *out, void *stream, float *ms) {
  if (grid < 1 || iters < 1 || !out || !ms) return -1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t err = hipEventCreate(&e0);
  if (err == hipSuccess) err = hipEventCreate(&e1);
  if (err == hipSuccess) err = hipEventRecord(e0, s);
  if (err == hipSuccess) {
    if (random)
      k_lds_atomics<true><<<grid, kNT, 0, s>>>(iters, out);
    else
      k_lds_atomics<false><<<grid, kNT, 0, s>>>(iters, out);
    err = hipGetLastError();
  }
  if (err == hipSuccess) err = hipEventRecord(e1, s);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  if (err == hipSuccess) err = hipEventElapsedTime(ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return err == hipSuccess ? 0 : (int)err;
}
