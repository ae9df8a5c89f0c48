// Training of the learned proposal's network (FP32 master weights) and its
// quantisation to the integer network of hgp_mlp.
//
// Model (float): x = code / 8 (code = the 8-bit feature code, ~ log2(1+f)),
//   h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), z = h2 . w3 + b3,
//   loss = mean over rows of softplus(z) - y z  (binary cross-entropy on
//   logits; y = 1 if the pair ended in one part of the plain run).
// k_mlp_grad: one wave per group of rows, lane j owning hidden unit j in both
// layers: forward, backward and the per-wave gradient sums (column j of W1
// and W2 in registers).  k_mlp_reduce_adam sums the per-wave partials in a
// fixed order (deterministic) and applies Adam or returns the gradient.
#include <cmath>
#include <cstring>
#include <vector>

#include "learned.hpp"

namespace hgp {

constexpr int TR_NT = 256;
constexpr int kW1 = 0, kB1 = kW1 + kMlpF * kMlpH, kW2 = kB1 + kMlpH, kB2 = kW2 + kMlpH * kMlpH, kW3 = kB2 + kMlpH,
              kB3 = kW3 + kMlpH, kNPar = kB3 + 1;
static_assert(kNPar * sizeof(float) == sizeof(hgp_mlp_f32), "parameter layout of hgp_mlp_f32");
constexpr int kPartStride = kNPar + 1;  // per-wave partial: gradient, then the loss sum
constexpr int W2_LD = 65;

__global__ __launch_bounds__(TR_NT) void k_mlp_grad(const float *__restrict__ prm, const int32_t *__restrict__ xq,
                                                    const float *__restrict__ y, const int64_t *__restrict__ idx,
                                                    int64_t row0, int64_t nrows, float inv_batch,
                                                    float *__restrict__ partial) {
  __shared__ float W2s[kMlpH * W2_LD];
  __shared__ float h1s[TR_NT / 64][kMlpH];
  __shared__ float d2s[TR_NT / 64][kMlpH];
  for (int t = threadIdx.x; t < kMlpH * kMlpH; t += TR_NT) W2s[(t / kMlpH) * W2_LD + (t % kMlpH)] = prm[kW2 + t];
  __syncthreads();
  const int w = threadIdx.x >> 6, j = lane_id();
  const int64_t gw = (int64_t)blockIdx.x * (TR_NT / 64) + w;
  const int64_t GW = (int64_t)gridDim.x * (TR_NT / 64);
  float w1c[kMlpF];
#pragma unroll
  for (int f = 0; f < kMlpF; ++f) w1c[f] = prm[kW1 + f * kMlpH + j];
  const float b1j = prm[kB1 + j], b2j = prm[kB2 + j], w3j = prm[kW3 + j], b3 = prm[kB3];
  float g_w1[kMlpF], g_w2[kMlpH];
#pragma unroll
  for (int f = 0; f < kMlpF; ++f) g_w1[f] = 0.f;
#pragma unroll
  for (int i = 0; i < kMlpH; ++i) g_w2[i] = 0.f;
  float g_b1 = 0.f, g_b2 = 0.f, g_w3 = 0.f, g_b3 = 0.f;
  double loss = 0.0;
  for (int64_t r = gw; r < nrows; r += GW) {
    const int64_t rr = idx ? idx[row0 + r] : row0 + r;
    float x[kMlpF];
#pragma unroll
    for (int f = 0; f < kMlpF; ++f) x[f] = (float)xq[rr * kMlpF + f] * 0.125f;
    float pre1 = b1j;
#pragma unroll
    for (int f = 0; f < kMlpF; ++f) pre1 = fmaf(x[f], w1c[f], pre1);
    h1s[w][j] = fmaxf(pre1, 0.f);
    wave_lds_sync();
    float pre2 = b2j;
#pragma unroll 16
    for (int i = 0; i < kMlpH; ++i) pre2 = fmaf(h1s[w][i], W2s[i * W2_LD + j], pre2);
    const float h2 = fmaxf(pre2, 0.f);
    const float z = wave_sum(h2 * w3j) + b3;
    const float yv = y[rr];
    // softplus(z) - y z, written to stay finite for large |z|
    loss += (double)(fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))) - yv * z);
    const float p = 1.f / (1.f + expf(-z));
    const float dz = (p - yv) * inv_batch;
    g_w3 = fmaf(dz, h2, g_w3);
    g_b3 += dz;
    const float d2 = pre2 > 0.f ? dz * w3j : 0.f;
    g_b2 += d2;
    d2s[w][j] = d2;
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < kMlpH; ++i) g_w2[i] = fmaf(h1s[w][i], d2, g_w2[i]);
    float dh1 = 0.f;
#pragma unroll 16
    for (int k = 0; k < kMlpH; ++k) dh1 = fmaf(d2s[w][k], W2s[j * W2_LD + k], dh1);
    const float d1 = pre1 > 0.f ? dh1 : 0.f;
    g_b1 += d1;
#pragma unroll
    for (int f = 0; f < kMlpF; ++f) g_w1[f] = fmaf(x[f], d1, g_w1[f]);
    wave_lds_sync();
  }
  float *out = partial + gw * kPartStride;
#pragma unroll
  for (int f = 0; f < kMlpF; ++f) out[kW1 + f * kMlpH + j] = g_w1[f];
  out[kB1 + j] = g_b1;
#pragma unroll
  for (int i = 0; i < kMlpH; ++i) out[kW2 + i * kMlpH + j] = g_w2[i];
  out[kB2 + j] = g_b2;
  out[kW3 + j] = g_w3;
  if (j == 0) {
    out[kB3] = g_b3;
    out[kNPar] = (float)loss;
  }
}

// Sums the partials of `waves` waves per parameter (fixed order).  mode 0:
// gradient to grad[], loss sum to *loss; mode 1: Adam step t (1-based) on
// prm with moments m, v; the loss sum is added to *loss.
__global__ void k_mlp_reduce_adam(const float *__restrict__ partial, int waves, int mode, float *__restrict__ prm,
                                  float *__restrict__ m, float *__restrict__ v, float lr, float beta1, float beta2,
                                  float eps, int step, float *__restrict__ grad, double *__restrict__ loss) {
  const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (p > kNPar) return;
  double g = 0.0;
  for (int w = 0; w < waves; ++w) g += (double)partial[(int64_t)w * kPartStride + p];
  if (p == kNPar) {
    *loss += g;
    return;
  }
  if (mode == 0) {
    grad[p] = (float)g;
    return;
  }
  const float gf = (float)g;
  const float mn = beta1 * m[p] + (1.f - beta1) * gf;
  const float vn = beta2 * v[p] + (1.f - beta2) * gf * gf;
  m[p] = mn;
  v[p] = vn;
  const float mh = mn / (1.f - powf(beta1, (float)step));
  const float vh = vn / (1.f - powf(beta2, (float)step));
  prm[p] -= lr * mh / (sqrtf(vh) + eps);
}

static int grad_waves(int64_t rows) {
  const int64_t w = (rows + 15) / 16;
  return (int)std::max<int64_t>(4, std::min<int64_t>((w + 3) / 4 * 4, 1024));
}

void mlp_grad(const hgp_mlp_f32 *w, const int32_t *xq, const float *y, int64_t n, DevBuf &prm, DevBuf &part,
              DevBuf &grad, DevBuf &lossb, hgp_mlp_f32 *g_out, double *loss_out, hipStream_t s) {
  prm.reserve(sizeof(hgp_mlp_f32));
  HGP_HIP(hipMemcpyAsync(prm.ptr, w, sizeof(hgp_mlp_f32), hipMemcpyHostToDevice, s));
  const int waves = grad_waves(n);
  part.reserve((size_t)waves * kPartStride * sizeof(float));
  grad.reserve(sizeof(hgp_mlp_f32));
  lossb.reserve(sizeof(double));
  fill_i64(lossb.as<int64_t>(), 1, 0, s);  // +0.0
  k_mlp_grad<<<waves / 4, TR_NT, 0, s>>>(prm.as<float>(), xq, y, nullptr, 0, n, 1.0f / (float)n, part.as<float>());
  HGP_LAUNCH_CHECK();
  k_mlp_reduce_adam<<<div_up(kNPar + 1, 256), 256, 0, s>>>(part.as<float>(), waves, 0, nullptr, nullptr, nullptr, 0,
                                                           0, 0, 0, 0, grad.as<float>(), lossb.as<double>());
  HGP_LAUNCH_CHECK();
  double ls = 0;
  HGP_HIP(hipMemcpyAsync(g_out, grad.ptr, sizeof(hgp_mlp_f32), hipMemcpyDeviceToHost, s));
  HGP_HIP(hipMemcpyAsync(&ls, lossb.ptr, sizeof ls, hipMemcpyDeviceToHost, s));
  HGP_HIP(hipStreamSynchronize(s));
  *loss_out = ls / (double)n;
}

// SplitMix64 (Steele, Lea, Flood 2014): the seeded generator of shuffles and
// initial weights.
static uint64_t splitmix64(uint64_t &st) {
  uint64_t z = (st += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double unit_double(uint64_t &st) { return (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0); }

void mlp_init(hgp_mlp_f32 *w, uint64_t seed) {
  std::memset(w, 0, sizeof *w);
  uint64_t st = seed ^ 0x6a09e667f3bcc909ull;
  const double a1 = std::sqrt(6.0 / kMlpNFeat), a2 = std::sqrt(6.0 / kMlpH);
  for (int f = 0; f < kMlpNFeat; ++f)
    for (int j = 0; j < kMlpH; ++j) w->w1[f * kMlpH + j] = (float)((2 * unit_double(st) - 1) * a1);
  for (int i = 0; i < kMlpH * kMlpH; ++i) w->w2[i] = (float)((2 * unit_double(st) - 1) * a2);
  for (int j = 0; j < kMlpH; ++j) w->w3[j] = (float)((2 * unit_double(st) - 1) * a2);
  for (int j = 0; j < kMlpH; ++j) {
    w->b1[j] = 0.01f;
    w->b2[j] = 0.01f;
  }
}

void train_state_init(hgp_train_state *st, const hgp_mlp_f32 *w, uint64_t seed) {
  std::memset(st, 0, sizeof *st);
  st->w = *w;
  st->rng = seed ^ 0xbb67ae8584caa73bull;
}

// `epochs` epochs of minibatch Adam from state st (host), which is updated:
// weights and moments live on the device during the run, the shuffle order of
// each epoch is drawn on the host from st->rng (Fisher-Yates), and the Adam
// step count carries over, so a run split at an epoch boundary is
// bit-identical to an uninterrupted one.
void mlp_train(hgp_train_state *st, const int32_t *xq, const float *y, int64_t n, const hgp_train_opts &o,
               int32_t epochs, DevBuf &prm, DevBuf &mom, DevBuf &part, DevBuf &perm, DevBuf &lossb,
               float *loss_epochs, hipStream_t s) {
  if (n <= 0 || epochs <= 0) return;
  prm.reserve(sizeof(hgp_mlp_f32));
  mom.reserve(2 * sizeof(hgp_mlp_f32));
  HGP_HIP(hipMemcpyAsync(prm.ptr, &st->w, sizeof(hgp_mlp_f32), hipMemcpyHostToDevice, s));
  float *m = mom.as<float>(), *v = mom.as<float>() + kNPar;
  HGP_HIP(hipMemcpyAsync(m, &st->m, sizeof(hgp_mlp_f32), hipMemcpyHostToDevice, s));
  HGP_HIP(hipMemcpyAsync(v, &st->v, sizeof(hgp_mlp_f32), hipMemcpyHostToDevice, s));
  const int64_t batch = std::min<int64_t>(o.batch, n);
  const int waves = grad_waves(batch);
  part.reserve((size_t)waves * kPartStride * sizeof(float));
  perm.reserve((size_t)n * sizeof(int64_t));
  lossb.reserve(sizeof(double));
  std::vector<int64_t> order((size_t)n);
  uint64_t rng = st->rng;
  int64_t step = st->step;
  for (int ep = 0; ep < epochs; ++ep) {
    for (int64_t i = 0; i < n; ++i) order[(size_t)i] = i;
    for (int64_t i = n - 1; i > 0; --i) std::swap(order[(size_t)i], order[(size_t)(splitmix64(rng) % (uint64_t)(i + 1))]);
    HGP_HIP(hipMemcpyAsync(perm.ptr, order.data(), (size_t)n * sizeof(int64_t), hipMemcpyHostToDevice, s));
    fill_i64(lossb.as<int64_t>(), 1, 0, s);
    for (int64_t b0 = 0; b0 < n; b0 += batch) {
      const int64_t rows = std::min<int64_t>(batch, n - b0);
      const int wv = grad_waves(rows);
      k_mlp_grad<<<wv / 4, TR_NT, 0, s>>>(prm.as<float>(), xq, y, perm.as<int64_t>(), b0, rows, 1.0f / (float)rows,
                                          part.as<float>());
      HGP_LAUNCH_CHECK();
      ++step;
      k_mlp_reduce_adam<<<div_up(kNPar + 1, 256), 256, 0, s>>>(part.as<float>(), wv, 1, prm.as<float>(), m, v, o.lr,
                                                               o.beta1, o.beta2, o.eps, (int)step, nullptr,
                                                               lossb.as<double>());
      HGP_LAUNCH_CHECK();
    }
    double ls = 0;
    HGP_HIP(hipMemcpyAsync(&ls, lossb.ptr, sizeof ls, hipMemcpyDeviceToHost, s));
    HGP_HIP(hipStreamSynchronize(s));
    if (loss_epochs) loss_epochs[ep] = (float)(ls / (double)n);
  }
  HGP_HIP(hipMemcpyAsync(&st->w, prm.ptr, sizeof(hgp_mlp_f32), hipMemcpyDeviceToHost, s));
  HGP_HIP(hipMemcpyAsync(&st->m, m, sizeof(hgp_mlp_f32), hipMemcpyDeviceToHost, s));
  HGP_HIP(hipMemcpyAsync(&st->v, v, sizeof(hgp_mlp_f32), hipMemcpyDeviceToHost, s));
  HGP_HIP(hipStreamSynchronize(s));
  st->rng = rng;
  st->step = step;
  st->epoch += epochs;
}

// ---------------------------------------------------------------------------
// quantisation
// ---------------------------------------------------------------------------
static int pow2_exp_for(double maxabs, double target) {
  // largest e with maxabs * 2^e <= target
  if (!(maxabs > 0)) return 0;
  return (int)std::floor(std::log2(target / maxabs));
}

static int32_t qround(double v, int64_t lim) {
  const double r = std::nearbyint(v);
  return (int32_t)std::max<double>(-(double)lim, std::min<double>((double)lim, r));
}

void mlp_quantize(const hgp_mlp_f32 *w, const int32_t *xq, int64_t n, int32_t k, hgp_mlp *q, int32_t *score_shift) {
  std::memset(q, 0, sizeof *q);
  q->k = k;
  double m1 = 0, m2 = 0, m3 = 0;
  for (int i = 0; i < kMlpF * kMlpH; ++i) m1 = std::max(m1, (double)std::fabs(w->w1[i]));
  for (int i = 0; i < kMlpH * kMlpH; ++i) m2 = std::max(m2, (double)std::fabs(w->w2[i]));
  for (int i = 0; i < kMlpH; ++i) m3 = std::max(m3, (double)std::fabs(w->w3[i]));
  const int s1 = std::min(pow2_exp_for(m1, 255.0), 24), s2 = std::min(pow2_exp_for(m2, 255.0), 24),
            s3 = std::min(pow2_exp_for(m3, 255.0), 24);
  // activation ranges of the float model on the calibration rows
  double a1max = 0, a2max = 0;
  std::vector<double> h1(kMlpH);
  for (int64_t r = 0; r < n; ++r) {
    for (int j = 0; j < kMlpH; ++j) {
      double a = w->b1[j];
      for (int f = 0; f < kMlpF; ++f) a += (double)xq[r * kMlpF + f] * 0.125 * w->w1[f * kMlpH + j];
      h1[j] = std::max(a, 0.0);
      a1max = std::max(a1max, h1[j]);
    }
    for (int j = 0; j < kMlpH; ++j) {
      double a = w->b2[j];
      for (int i = 0; i < kMlpH; ++i) a += h1[i] * w->w2[i * kMlpH + j];
      a2max = std::max(a2max, a);
    }
  }
  // a1 = h1 2^t1 with r1 = s1 + 3 - t1; a2 = h2 2^t2 with r2 = t1 + s2 - t2
  int t1 = pow2_exp_for(a1max, 255.0);
  int r1 = s1 + 3 - t1;
  r1 = std::max(0, std::min(30, r1));
  t1 = s1 + 3 - r1;
  int t2 = pow2_exp_for(a2max, 255.0);
  int r2 = t1 + s2 - t2;
  r2 = std::max(0, std::min(30, r2));
  t2 = t1 + s2 - r2;
  const int64_t blim = int64_t(1) << 22;
  for (int i = 0; i < kMlpF * kMlpH; ++i) q->w1[i] = qround(std::ldexp((double)w->w1[i], s1), 255);
  for (int i = 0; i < kMlpH * kMlpH; ++i) q->w2[i] = qround(std::ldexp((double)w->w2[i], s2), 255);
  for (int i = 0; i < kMlpH; ++i) {
    q->w3[i] = qround(std::ldexp((double)w->w3[i], s3), 255);
    q->b1[i] = qround(std::ldexp((double)w->b1[i], s1 + 3), blim);
    q->b2[i] = qround(std::ldexp((double)w->b2[i], t1 + s2), blim);
  }
  q->b3 = qround(std::ldexp((double)w->b3, t2 + s3), blim);
  q->r1 = r1;
  q->r2 = r2;
  if (score_shift) *score_shift = t2 + s3;
}

}  // namespace hgp
