// Runs the CPU oracle and the seeded input generator under AddressSanitizer
// and UndefinedBehaviorSanitizer (built by tests/test_sanitize_cpu.py): plain,
// learned, exact-matching and constraint-role partitions with traces,
// malformed inputs, connectivity and the network on random rows.  Exit
// status 0 when every call returned its expected code; a sanitizer report
// aborts the process.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../oracle/hgpo.h"

extern "C" {
typedef struct {
  int32_t n_nodes;
  int32_t n_hedges;
  int64_t n_pins;
  int32_t *hedge_off;
  int32_t *pins;
  int32_t *n_src;
  int32_t *hedge_w;
  int32_t *node_w;
} synth_graph;
synth_graph *synth_random_snn(int32_t n, double mu, uint64_t seed, int32_t wmin, int32_t wmax);
synth_graph *synth_layered_conv(int32_t layers, int32_t C, int32_t H, int32_t W, int32_t k, double p_geo,
                                uint64_t seed);
void synth_free(synth_graph *g);
}

static int failures = 0;

static void expect(int got, int want, const char *what) {
  if (got != want) {
    std::fprintf(stderr, "%s: rc %d, expected %d\n", what, got, want);
    ++failures;
  }
}

static hgpo_hypergraph view(const synth_graph *g) {
  hgpo_hypergraph h;
  h.n_nodes = g->n_nodes;
  h.n_hedges = g->n_hedges;
  h.hedge_off = g->hedge_off;
  h.pins = g->pins;
  h.n_src = g->n_src;
  h.hedge_w = g->hedge_w;
  h.node_w = g->node_w;
  return h;
}

static void random_mlp(hgpo_mlp *m, uint64_t seed) {
  uint64_t x = seed * 0x9E3779B97F4A7C15ull + 1;
  auto next = [&](int lo, int hi) {
    x ^= x << 13;
    x ^= x >> 7;
    x ^= x << 17;
    return lo + (int)(x % (uint64_t)(hi - lo + 1));
  };
  m->k = 8;
  m->r1 = 7;
  m->r2 = 9;
  m->b3 = next(-4096, 4096);
  for (int i = 0; i < HGPO_MLP_F * HGPO_MLP_H; ++i) m->w1[i] = (i / HGPO_MLP_H) < 10 ? next(-255, 255) : 0;
  for (int i = 0; i < HGPO_MLP_H * HGPO_MLP_H; ++i) m->w2[i] = next(-255, 255);
  for (int i = 0; i < HGPO_MLP_H; ++i) {
    m->b1[i] = next(-4096, 4096);
    m->b2[i] = next(-4096, 4096);
    m->w3[i] = next(-255, 255);
  }
}

static void run_graph(const synth_graph *sg, int32_t omega, int32_t delta, uint64_t seed) {
  const hgpo_hypergraph g = view(sg);
  std::vector<int32_t> part((size_t)g.n_nodes + 1);
  hgpo_result res;
  for (int role = 0; role < 3; ++role) {
    hgpo_trace *t = hgpo_trace_new();
    expect(hgpo_partition_role(&g, omega, delta, 0, 8, role, part.data(), &res, t), HGPO_OK, "partition_role");
    for (int l = 0; l < hgpo_trace_levels(t); ++l) {
      const void *d = nullptr;
      int32_t eb = 0;
      (void)hgpo_trace_get(t, HGPO_LV_PAIR, l, &d, &eb);
      (void)hgpo_trace_get(t, HGPO_LV_FEAT, l, &d, &eb);
    }
    hgpo_trace_free(t);
    int64_t conn = 0;
    expect(hgpo_connectivity(&g, part.data(), &conn), HGPO_OK, "connectivity");
    if (conn != res.connectivity) {
      std::fprintf(stderr, "connectivity %lld != %lld\n", (long long)conn, (long long)res.connectivity);
      ++failures;
    }
  }
  expect(hgpo_partition_ex(&g, omega, delta, 0, 8, HGPO_INBOUND, HGPO_MATCH_EXACT, part.data(), &res, nullptr),
         HGPO_OK, "exact matching");
  hgpo_mlp m;
  random_mlp(&m, seed);
  hgpo_trace *t = hgpo_trace_new();
  expect(hgpo_partition_learned(&g, omega, delta, 0, 8, &m, part.data(), &res, t), HGPO_OK, "learned");
  hgpo_trace_free(t);
}

int main() {
  synth_graph *a = synth_random_snn(600, 12.0, 5, 1, 16);
  run_graph(a, 32, 150, 1);
  synth_free(a);
  synth_graph *b = synth_random_snn(400, 10.0, 6, 1, 60000);
  run_graph(b, 24, 120, 2);
  synth_free(b);
  synth_graph *c = synth_layered_conv(4, 4, 6, 6, 3, 0.1, 7);
  run_graph(c, 64, 2000, 3);
  synth_free(c);
  // malformed inputs
  const int32_t off_bad[3] = {0, 3, 2}, pins[4] = {0, 1, 2, 3}, dup[3] = {1, 1, 0}, off2[3] = {0, 2, 3};
  hgpo_hypergraph g{4, 2, off_bad, pins, nullptr, nullptr, nullptr};
  std::vector<int32_t> part(8);
  hgpo_result res;
  expect(hgpo_partition(&g, 4, 4, 0, 8, part.data(), &res, nullptr), HGPO_EBADCSR, "offsets");
  g.hedge_off = off2;
  g.pins = dup;
  expect(hgpo_partition(&g, 4, 4, 0, 8, part.data(), &res, nullptr), HGPO_EBADCSR, "duplicate");
  expect(hgpo_partition(nullptr, 4, 4, 0, 8, part.data(), &res, nullptr), HGPO_EINVAL, "null");
  // the network on random rows, and feature codes
  hgpo_mlp m;
  random_mlp(&m, 9);
  std::vector<int32_t> xq(16 * 257);
  for (size_t i = 0; i < xq.size(); ++i) xq[i] = (int32_t)((i * 37) % 256);
  std::vector<int64_t> sc(257);
  expect(hgpo_mlp_score(&m, xq.data(), 257, sc.data()), HGPO_OK, "mlp_score");
  for (int64_t f = 0; f < 100000; f += 97) (void)hgpo_qlog(f);
  std::printf("oracle under sanitizers: %d failures\n", failures);
  return failures ? 1 : 0;
}
