/*
 * Seeded synthetic spiking-network hypergraphs.
 *
 * This module only draws inputs; it holds none of the partitioner's
 * arithmetic.  Both the GPU library's tests/benchmarks and the CPU oracle
 * consume the exact bytes produced here.
 *
 * Every node v owns one hyperedge e_v whose single source pin is v and whose
 * destination pins are the neurons v projects to (the incidence model of
 * Sec. II-A: src(e), dst(e), in(n), out(n)).  Two families stand in for the
 * spiking networks of Tab. I:
 *   - random SNN: |T_v| = min(Poisson(mu)+1, n-1) targets drawn uniformly
 *     without replacement from N \ {v};
 *   - layered conv-like SNN: L layers of C x H x W neurons, neuron (l,c,y,x)
 *     targets every channel of layer l+1 inside the k x k window centred at
 *     (y,x) (clipped at the borders); the last layer owns singleton edges.
 *
 * Output CSR (int32): hedge_off[E+1], pins[P] (source pin first, then the
 * destinations in ascending id order), n_src[E] (= 1), hedge_w[E].
 *
 * RNG: xoshiro256** seeded through SplitMix64 (Blackman & Vigna); bounded
 * integers by Lemire's multiply-shift rejection method; Poisson by sequential
 * search inversion; sampling without replacement by Floyd's algorithm;
 * geometric on {1,2,...} by inversion.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t n_nodes;
  int32_t n_hedges;
  int64_t n_pins;
  int32_t *hedge_off; /* [n_hedges + 1] */
  int32_t *pins;      /* [n_pins] */
  int32_t *n_src;     /* [n_hedges] */
  int32_t *hedge_w;   /* [n_hedges] */
  int32_t *node_w;    /* [n_nodes] */
} synth_graph;

typedef struct {
  uint64_t s[4];
} rng_t;

static uint64_t splitmix64(uint64_t *x) {
  uint64_t z = (*x += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

static void rng_seed(rng_t *r, uint64_t seed) {
  uint64_t x = seed;
  for (int i = 0; i < 4; ++i) r->s[i] = splitmix64(&x);
}

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t rng_next(rng_t *r) {
  uint64_t *s = r->s;
  uint64_t result = rotl(s[1] * 5, 7) * 9;
  uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = rotl(s[3], 45);
  return result;
}

/* uniform integer in [0, bound), bound >= 1 (Lemire 2019) */
static uint32_t rng_below(rng_t *r, uint32_t bound) {
  uint32_t x = (uint32_t)(rng_next(r) >> 32);
  uint64_t m = (uint64_t)x * bound;
  uint32_t l = (uint32_t)m;
  if (l < bound) {
    uint32_t t = (uint32_t)(-bound) % bound;
    while (l < t) {
      x = (uint32_t)(rng_next(r) >> 32);
      m = (uint64_t)x * bound;
      l = (uint32_t)m;
    }
  }
  return (uint32_t)(m >> 32);
}

/* uniform double in [0, 1) */
static double rng_u01(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* uniform double in (0, 1) */
static double rng_u01_open(rng_t *r) { return ((double)(rng_next(r) >> 11) + 0.5) * 0x1.0p-53; }

static int32_t rng_poisson(rng_t *r, double mu) {
  double u = rng_u01(r);
  double p = exp(-mu);
  double f = p;
  int32_t k = 0;
  int32_t cap = (int32_t)(10.0 * mu) + 100;
  while (u > f && k < cap) {
    ++k;
    p *= mu / (double)k;
    f += p;
  }
  return k;
}

static int32_t rng_geometric(rng_t *r, double p) {
  double u = rng_u01_open(r);
  double k = ceil(log(u) / log1p(-p));
  if (!(k >= 1.0)) k = 1.0;
  if (k > 2147483647.0) k = 2147483647.0;
  return (int32_t)k;
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* growable int32 buffer */
typedef struct {
  int32_t *d;
  int64_t n, cap;
} vec32;

static int vec_reserve(vec32 *v, int64_t need) {
  if (need <= v->cap) return 0;
  int64_t c = v->cap ? v->cap : 1024;
  while (c < need) c *= 2;
  int32_t *p = (int32_t *)realloc(v->d, (size_t)c * sizeof(int32_t));
  if (!p) return -1;
  v->d = p;
  v->cap = c;
  return 0;
}

void synth_free(synth_graph *g) {
  if (!g) return;
  free(g->hedge_off);
  free(g->pins);
  free(g->n_src);
  free(g->hedge_w);
  free(g->node_w);
  free(g);
}

static synth_graph *alloc_graph(int32_t n) {
  synth_graph *g = (synth_graph *)calloc(1, sizeof(synth_graph));
  if (!g) return NULL;
  g->n_nodes = n;
  g->n_hedges = n;
  g->hedge_off = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
  g->n_src = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n > 0 ? (size_t)n : 1));
  g->hedge_w = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n > 0 ? (size_t)n : 1));
  g->node_w = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n > 0 ? (size_t)n : 1));
  if (!g->hedge_off || !g->n_src || !g->hedge_w || !g->node_w) {
    synth_free(g);
    return NULL;
  }
  for (int32_t i = 0; i < n; ++i) g->node_w[i] = 1;
  return g;
}

/*
 * Floyd's sampling of t distinct values from [0, m) into out[0..t), using an
 * open-addressing set of capacity cap (power of two > 2t) held in tab.
 */
static void floyd_sample(rng_t *r, uint32_t m, int32_t t, int32_t *out, int32_t *tab, uint32_t cap) {
  for (uint32_t i = 0; i < cap; ++i) tab[i] = -1;
  int32_t cnt = 0;
  for (uint32_t j = m - (uint32_t)t; j < m; ++j) {
    uint32_t x = rng_below(r, j + 1);
    /* insert x, or j if x is present */
    uint32_t h = (x * 2654435761u) & (cap - 1);
    int present = 0;
    while (tab[h] != -1) {
      if ((uint32_t)tab[h] == x) {
        present = 1;
        break;
      }
      h = (h + 1) & (cap - 1);
    }
    uint32_t y = present ? j : x;
    if (present) {
      h = (y * 2654435761u) & (cap - 1);
      while (tab[h] != -1) h = (h + 1) & (cap - 1);
    }
    tab[h] = (int32_t)y;
    out[cnt++] = (int32_t)y;
  }
}

/*
 * Random SNN: n nodes, targets per node min(Poisson(mu)+1, n-1), hedge weights
 * uniform in [wmin, wmax].  Draw order per node v: Poisson count, Floyd
 * sample, weight.
 */
synth_graph *synth_random_snn(int32_t n, double mu, uint64_t seed, int32_t wmin, int32_t wmax) {
  if (n < 0 || wmin < 1 || wmax < wmin) return NULL;
  synth_graph *g = alloc_graph(n);
  if (!g) return NULL;
  rng_t r;
  rng_seed(&r, seed);
  vec32 pins = {0, 0, 0};
  int32_t cap_t = 16;
  int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * 16);
  int32_t *tab = (int32_t *)malloc(sizeof(int32_t) * 64);
  uint32_t tabcap = 64;
  if (!tmp || !tab) goto fail;
  g->hedge_off[0] = 0;
  for (int32_t v = 0; v < n; ++v) {
    int32_t t = rng_poisson(&r, mu) + 1;
    if (t > n - 1) t = n - 1;
    if (t > cap_t) {
      while (cap_t < t) cap_t *= 2;
      int32_t *p = (int32_t *)realloc(tmp, sizeof(int32_t) * (size_t)cap_t);
      if (!p) goto fail;
      tmp = p;
    }
    while (tabcap < 2u * (uint32_t)t + 2u) tabcap *= 2;
    {
      int32_t *p = (int32_t *)realloc(tab, sizeof(int32_t) * tabcap);
      if (!p) goto fail;
      tab = p;
    }
    if (t > 0) floyd_sample(&r, (uint32_t)(n - 1), t, tmp, tab, tabcap);
    for (int32_t i = 0; i < t; ++i)
      if (tmp[i] >= v) tmp[i] += 1; /* skip v itself */
    qsort(tmp, (size_t)t, sizeof(int32_t), cmp_i32);
    if (vec_reserve(&pins, pins.n + t + 1)) goto fail;
    pins.d[pins.n++] = v;
    for (int32_t i = 0; i < t; ++i) pins.d[pins.n++] = tmp[i];
    if (pins.n > 2147483647LL) goto fail;
    g->hedge_off[v + 1] = (int32_t)pins.n;
    g->n_src[v] = 1;
    g->hedge_w[v] = wmin + (int32_t)rng_below(&r, (uint32_t)(wmax - wmin + 1));
  }
  free(tmp);
  free(tab);
  g->pins = pins.d ? pins.d : (int32_t *)malloc(sizeof(int32_t));
  g->n_pins = pins.n;
  return g;
fail:
  free(tmp);
  free(tab);
  free(pins.d);
  synth_free(g);
  return NULL;
}

/*
 * Layered conv-like SNN: `layers` layers of C x H x W neurons; node id
 * l*CHW + c*HW + y*W + x.  Neuron (l < layers-1, c, y, x) targets all
 * channels of layer l+1 in the k x k window centred at (y, x), clipped.
 * Hedge weights ~ Geometric(p_geo) on {1, 2, ...}, drawn in node order.
 */
synth_graph *synth_layered_conv(int32_t layers, int32_t C, int32_t H, int32_t W, int32_t k, double p_geo,
                                uint64_t seed) {
  if (layers < 1 || C < 1 || H < 1 || W < 1 || k < 1 || (k % 2) == 0) return NULL;
  if (!(p_geo > 0.0 && p_geo <= 1.0)) return NULL;
  int64_t chw = (int64_t)C * H * W;
  int64_t n64 = chw * layers;
  if (n64 > 2147483647LL) return NULL;
  int32_t n = (int32_t)n64;
  int32_t hw = H * W, rad = k / 2;
  /* count pins first */
  int64_t total = 0;
  for (int32_t l = 0; l < layers; ++l)
    for (int32_t y = 0; y < H; ++y)
      for (int32_t x = 0; x < W; ++x) {
        int64_t per = 1;
        if (l + 1 < layers) {
          int32_t y0 = y - rad < 0 ? 0 : y - rad, y1 = y + rad >= H ? H - 1 : y + rad;
          int32_t x0 = x - rad < 0 ? 0 : x - rad, x1 = x + rad >= W ? W - 1 : x + rad;
          per += (int64_t)C * (y1 - y0 + 1) * (x1 - x0 + 1);
        }
        total += per * C;
      }
  if (total > 2147483647LL) return NULL;
  synth_graph *g = alloc_graph(n);
  if (!g) return NULL;
  g->pins = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
  if (!g->pins) {
    synth_free(g);
    return NULL;
  }
  rng_t r;
  rng_seed(&r, seed);
  int64_t pos = 0;
  g->hedge_off[0] = 0;
  for (int32_t v = 0; v < n; ++v) {
    int32_t l = (int32_t)(v / chw);
    int32_t rem = (int32_t)(v % chw);
    int32_t y = (rem % hw) / W, x = rem % W;
    g->pins[pos++] = v;
    if (l + 1 < layers) {
      int32_t y0 = y - rad < 0 ? 0 : y - rad, y1 = y + rad >= H ? H - 1 : y + rad;
      int32_t x0 = x - rad < 0 ? 0 : x - rad, x1 = x + rad >= W ? W - 1 : x + rad;
      int64_t base = (int64_t)(l + 1) * chw;
      for (int32_t c2 = 0; c2 < C; ++c2)
        for (int32_t yy = y0; yy <= y1; ++yy)
          for (int32_t xx = x0; xx <= x1; ++xx) g->pins[pos++] = (int32_t)(base + (int64_t)c2 * hw + yy * W + xx);
    }
    g->hedge_off[v + 1] = (int32_t)pos;
    g->n_src[v] = 1;
    g->hedge_w[v] = rng_geometric(&r, p_geo);
  }
  g->n_pins = pos;
  return g;
}

/*
 * One member of a family of random SNNs: the node count is round(2^U) with U
 * uniform in [log2_lo, log2_hi], the target mean mu uniform in [mu_lo, mu_hi];
 * both are drawn first from the seed's stream, then the graph is drawn from a
 * stream seeded with seed ^ 0x5bd1e995.
 */
synth_graph *synth_random_snn_family(uint64_t seed, double log2_lo, double log2_hi, double mu_lo, double mu_hi,
                                     int32_t wmin, int32_t wmax, int32_t *n_out, double *mu_out) {
  rng_t r;
  rng_seed(&r, seed);
  double u = log2_lo + (log2_hi - log2_lo) * rng_u01(&r);
  double mu = mu_lo + (mu_hi - mu_lo) * rng_u01(&r);
  int32_t n = (int32_t)llround(pow(2.0, u));
  if (n_out) *n_out = n;
  if (mu_out) *mu_out = mu;
  return synth_random_snn(n, mu, seed ^ 0x5bd1e995ULL, wmin, wmax);
}
