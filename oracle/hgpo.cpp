/*
 * hgpo -- CPU oracle (TEST INFRASTRUCTURE ONLY; see hgpo.h).
 *
 * A sequential restatement of the multilevel scheme of Sec. II-B:
 * coarsening by constrained candidate pairs and pseudo-forest matching
 * (Sec. III-A), contraction (Sec. III-B, coarse hypergraph construction),
 * and FM-style refinement by sorted move sequences with in-sequence gains and
 * per-prefix constraint validity (Sec. IV-A, IV-B).  Each function names the
 * passage it follows.  Parallel machinery of the paper (warp histograms,
 * atomic pseudo-forest walks, event sort/scan pipelines) is replaced by the
 * plain definitions those pipelines compute.
 *
 * Readings where the paper is silent or ambiguous (all ties toward the larger
 * id; exact four-term in-sequence gain; inbound = destination pins; ...) are
 * listed in the project's design notes and restated at each use below.
 */
#include "hgpo.h"

#include <algorithm>
#include <array>
#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <utility>
#include <stdexcept>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

struct hgpo_trace {
  struct Rec {
    std::vector<int32_t> i32;
    std::vector<int64_t> i64;
    int32_t bytes = 4;
  };
  std::map<std::pair<int32_t, int32_t>, Rec> recs;
  int32_t levels = 0;
  int32_t rounds = 0;

  void put32(int32_t kind, int32_t idx, const std::vector<int32_t> &v) {
    Rec &r = recs[{kind, idx}];
    r.i32 = v;
    r.bytes = 4;
  }
  void put64(int32_t kind, int32_t idx, const std::vector<int64_t> &v) {
    Rec &r = recs[{kind, idx}];
    r.i64 = v;
    r.bytes = 8;
  }
};

namespace {

constexpr int64_t kInt32Max = 2147483647LL;

/* One level G_l of the hierarchy.  Hedge ids and weights never change across
 * levels; pins are (cluster id, destination flag), ascending by id. */
struct Level {
  int32_t n = 0;
  std::vector<int64_t> hoff;  /* [E+1] */
  std::vector<int32_t> hpin;  /* pin node ids */
  std::vector<uint8_t> hdst;  /* 1 iff the pin is a destination of the hedge */
  std::vector<int64_t> size;  /* node weight (cluster size), Sec. III-B */
  std::vector<int64_t> ioff;  /* incidence I(n) = in(n) u out(n), Sec. II-A */
  std::vector<int32_t> ihe;   /* hedge ids, ascending within each node */
  std::vector<uint8_t> idst;  /* 1 iff n in dst(e), i.e. e in in(n) */
  std::vector<int32_t> indeg; /* |in(n)| */
  std::vector<int32_t> gamma; /* map to the next level (empty: none) */
};

/* I(n), in(n) from the hedge lists (Sec. II-A definitions). */
void build_incidence(Level &L, int32_t E) {
  L.ioff.assign((size_t)L.n + 1, 0);
  L.indeg.assign((size_t)L.n, 0);
  for (int32_t e = 0; e < E; ++e)
    for (int64_t j = L.hoff[e]; j < L.hoff[e + 1]; ++j) {
      L.ioff[(size_t)L.hpin[j] + 1]++;
      if (L.hdst[j]) L.indeg[L.hpin[j]]++;
    }
  for (int32_t v = 0; v < L.n; ++v) L.ioff[v + 1] += L.ioff[v];
  L.ihe.assign((size_t)L.ioff[L.n], 0);
  L.idst.assign((size_t)L.ioff[L.n], 0);
  std::vector<int64_t> fill(L.ioff.begin(), L.ioff.end() - 1);
  for (int32_t e = 0; e < E; ++e)
    for (int64_t j = L.hoff[e]; j < L.hoff[e + 1]; ++j) {
      int32_t v = L.hpin[j];
      L.ihe[fill[v]] = e;
      L.idst[fill[v]] = L.hdst[j];
      fill[v]++;
    }
}

/* Memory only: the incidence of a level is not needed while other levels run. */
void drop_incidence(Level &L) {
  std::vector<int64_t>().swap(L.ioff);
  std::vector<int32_t>().swap(L.ihe);
  std::vector<uint8_t>().swap(L.idst);
}

/* Eq. 1: sum over hedges of w(e) * (number of distinct parts among its pins
 * minus one).  A hedge with no pins contributes nothing. */
int64_t connectivity_of(const Level &L, int32_t E, const std::vector<int32_t> &w, const std::vector<int32_t> &rho) {
  int64_t conn = 0;
  std::vector<int32_t> parts;
  for (int32_t e = 0; e < E; ++e) {
    parts.clear();
    for (int64_t j = L.hoff[e]; j < L.hoff[e + 1]; ++j) parts.push_back(rho[L.hpin[j]]);
    std::sort(parts.begin(), parts.end());
    int64_t lambda = std::unique(parts.begin(), parts.end()) - parts.begin();
    if (lambda > 0) conn += (int64_t)w[e] * (lambda - 1);
  }
  return conn;
}

/*
 * Candidate selection, Sec. III-A with Eq. 2.  For every node n and every
 * other pin m of a hedge in I(n):
 *   hist(n,m) = sum of w(e) over e in I(n) containing m             (Eq. 2)
 *   c(n,m)    = #{e in in(n) : m in dst(e)} = |in(n) n in(m)|
 * m is valid iff size(n)+size(m) <= Omega and |in(n) u in(m)| <= Delta, where
 * |in(n) u in(m)| = |in(n)| + |in(m)| - c(n,m) (inclusion-exclusion, exact).
 * pair(n) = the valid m maximising (hist, id): the global best valid
 * candidate, larger id on ties; -1 if no valid m.  n is not its own
 * neighbour.  score(n) = hist(n, pair(n)).
 */
void rate_select(const Level &L, const std::vector<int32_t> &w, int64_t omega, int64_t delta,
                 std::vector<int32_t> &pair, std::vector<int64_t> &score) {
  const int32_t N = L.n;
  pair.assign((size_t)N, -1);
  score.assign((size_t)N, 0);
#pragma omp parallel
  {
    std::vector<int64_t> hist((size_t)N, 0);
    std::vector<int64_t> common((size_t)N, 0);
    std::vector<uint8_t> seen((size_t)N, 0);
    std::vector<int32_t> touched;
#pragma omp for schedule(dynamic, 64)
    for (int32_t n = 0; n < N; ++n) {
      touched.clear();
      for (int64_t i = L.ioff[n]; i < L.ioff[n + 1]; ++i) {
        const int32_t e = L.ihe[i];
        const bool n_dst = L.idst[i] != 0;
        for (int64_t j = L.hoff[e]; j < L.hoff[e + 1]; ++j) {
          const int32_t m = L.hpin[j];
          if (m == n) continue;
          if (!seen[m]) {
            seen[m] = 1;
            touched.push_back(m);
          }
          hist[m] += w[e];
          if (n_dst && L.hdst[j]) common[m] += 1;
        }
      }
      int32_t best = -1;
      int64_t best_h = 0;
      for (int32_t m : touched) {
        const bool ok_size = L.size[n] + L.size[m] <= omega;
        const bool ok_inb = (int64_t)L.indeg[n] + L.indeg[m] - common[m] <= delta;
        if (ok_size && ok_inb && (best < 0 || hist[m] > best_h || (hist[m] == best_h && m > best))) {
          best = m;
          best_h = hist[m];
        }
        hist[m] = 0;
        common[m] = 0;
        seen[m] = 0;
      }
      pair[n] = best;
      score[n] = best < 0 ? 0 : best_h;
    }
  }
}

/*
 * Matching over the pairing pseudo-forest, Sec. III-A and the parallel walk of
 * Sec. III-B, written as the recursion the two traversals evaluate:
 *   best(p) = the m with pair(m) = p maximising (score(m), id), if any
 *   up(n)   = true  if n lies on a 2-cycle (pair(pair(n)) = n),
 *             false if n proposes nothing (such nodes are roots),
 *             [best(pair(n)) = n] and not up(pair(n))   otherwise
 *   match(n) = pair(n) if up(n); best(n) if best(n) exists and up(best(n));
 *              n otherwise.
 * Walking a pair chain ends at a 2-cycle or at a node without candidate,
 * because score is non-decreasing along pair edges and cycles have length 2.
 */
void match_pairs(const std::vector<int32_t> &pair, const std::vector<int64_t> &score, std::vector<int32_t> &match) {
  const int32_t N = (int32_t)pair.size();
  std::vector<int32_t> best((size_t)N, -1);
  for (int32_t m = 0; m < N; ++m) {
    const int32_t p = pair[m];
    if (p < 0) continue;
    const int32_t b = best[p];
    if (b < 0 || score[m] > score[b] || (score[m] == score[b] && m > b)) best[p] = m;
  }
  /* up: -1 unknown, 0 false, 1 true */
  std::vector<int8_t> up((size_t)N, -1);
  std::vector<int32_t> path;
  for (int32_t s = 0; s < N; ++s) {
    if (up[s] >= 0) continue;
    path.clear();
    int32_t v = s;
    int8_t val = -1;
    while (true) {
      if (up[v] >= 0) {
        val = up[v];
        break;
      }
      const int32_t p = pair[v];
      if (p < 0) {
        up[v] = 0;
        val = 0;
        break;
      }
      if (pair[p] == v) {
        up[v] = 1;
        up[p] = 1;
        val = 1;
        break;
      }
      path.push_back(v);
      v = p;
    }
    /* unwind: val is up(parent) for the last node of the path */
    for (size_t i = path.size(); i-- > 0;) {
      const int32_t x = path[i];
      const int8_t ux = (best[pair[x]] == x && val == 0) ? 1 : 0;
      up[x] = ux;
      val = ux;
    }
  }
  match.assign((size_t)N, 0);
  for (int32_t n = 0; n < N; ++n) {
    if (up[n] == 1)
      match[n] = pair[n];
    else if (best[n] >= 0 && up[best[n]] == 1)
      match[n] = best[n];
    else
      match[n] = n;
  }
}

/*
 * Exact matching on the pairing pseudo-forest: the dynamic-programming
 * formulation the paper names as future work (Sec. VI), replacing the
 * two-traversal heuristic of Sec. III-A.  Each component is a tree hanging
 * from a 2-cycle, or from a node without candidate; its edges are the pairing
 * edges {n, pair(n)} of weight score(n).  The textbook tree recursion gives a
 * maximum-weight matching:
 *   children(v) = {c : pair(c) = v}, without v's 2-cycle partner
 *   g(v) = sum of f(c) over the children      (v left free for its parent)
 *   d(v) = max over the children of g(c) + score(c) - f(c), argmax c*(v)
 *          by (value, id), larger id on ties; no children: no d(v)
 *   f(v) = g(v) + max(0, d(v))                (best matching of v's subtree)
 *   v is matched to c*(v) unless matched upward, when d(v) >= 0
 * A 2-cycle {a, b} is matched iff g(a) + g(b) + score(a) >= f(a) + f(b).
 * Ties favour matching (d(v) = 0 still takes c*(v)), which fixes one
 * matching among those of maximum weight.  Whether a node is matched to its
 * parent follows the recursion of match_pairs with best = c* and the 2-cycle
 * decision.
 */
void match_exact(const std::vector<int32_t> &pair, const std::vector<int64_t> &score, std::vector<int32_t> &match) {
  const int32_t N = (int32_t)pair.size();
  auto root = [&](int32_t v) { return pair[v] < 0 || pair[pair[v]] == v; };
  /* children lists, and the nodes in an order where children come first
   * (reverse of a breadth-first order from the roots) */
  std::vector<std::vector<int32_t>> kids((size_t)N);
  for (int32_t c = 0; c < N; ++c)
    if (!root(c)) kids[(size_t)pair[c]].push_back(c);
  std::vector<int32_t> order;
  for (int32_t v = 0; v < N; ++v)
    if (root(v)) order.push_back(v);
  for (size_t i = 0; i < order.size(); ++i)
    for (int32_t c : kids[(size_t)order[i]]) order.push_back(c);
  if ((int32_t)order.size() != N) throw std::logic_error("pairing graph has a cycle longer than two");
  std::vector<int64_t> g((size_t)N, 0), f((size_t)N, 0);
  std::vector<int32_t> cstar((size_t)N, -1);
  for (size_t i = order.size(); i-- > 0;) {
    const int32_t v = order[i];
    int64_t gv = 0, best = 0;
    int32_t bc = -1;
    for (int32_t c : kids[(size_t)v]) {
      gv += f[c];
      const int64_t val = g[c] + score[c] - f[c];
      if (bc < 0 || val > best || (val == best && c > bc)) {
        best = val;
        bc = c;
      }
    }
    g[v] = gv;
    f[v] = gv + (bc >= 0 && best > 0 ? best : 0);
    if (bc >= 0 && best >= 0) cstar[v] = bc;
  }
  /* up(v): matched to pair(v) */
  std::vector<int8_t> up((size_t)N, 0);
  for (int32_t v : order) {
    const int32_t p = pair[v];
    if (p < 0) {
      up[v] = 0;
    } else if (pair[p] == v) {
      const int32_t a = std::min(v, p), b = std::max(v, p);
      up[v] = (g[a] + g[b] + score[a] >= f[a] + f[b]) ? 1 : 0;
    } else {
      up[v] = (cstar[p] == v && up[p] == 0) ? 1 : 0; /* the parent comes earlier in `order` */
    }
  }
  match.assign((size_t)N, 0);
  for (int32_t n = 0; n < N; ++n) {
    if (up[n] == 1)
      match[n] = pair[n];
    else if (cstar[n] >= 0 && up[cstar[n]] == 1)
      match[n] = cstar[n];
    else
      match[n] = n;
  }
}

/*
 * Learned merge proposal (an extension outside the paper's method; the
 * definitions are stated in hgpo.h).  Everything is integer arithmetic.
 */

/* 8 * floor(log2(f+1)) + the three bits below the leading one of f+1, capped
 * at 255. */
int32_t qlog_code(int64_t f) {
  const uint64_t v = (uint64_t)f + 1u;
  int e = 63;
  while (!((v >> e) & 1u)) --e;
  const uint64_t t = e >= 3 ? (v >> (e - 3)) & 7u : (v << (3 - e)) & 7u;
  const int64_t code = 8 * (int64_t)e + (int64_t)t;
  return (int32_t)std::min<int64_t>(code, 255);
}

/* x / 2^r rounded to nearest, ties to even. */
int64_t rshift_rne(int64_t x, int32_t r) {
  if (r == 0) return x;
  const int64_t q = x >> r; /* floor */
  const int64_t rem = x - q * ((int64_t)1 << r);
  const int64_t half = (int64_t)1 << (r - 1);
  return (rem > half || (rem == half && (q & 1))) ? q + 1 : q;
}

int64_t clamp255(int64_t v) { return v < 0 ? 0 : (v > 255 ? 255 : v); }

/* The fixed-point network: two hidden layers of 64 ReLU units (requantised
 * to 0..255 by a rounded right shift) and a linear output. */
int64_t mlp_forward(const hgpo_mlp &q, const int32_t *x) {
  int64_t a1[HGPO_MLP_H], a2[HGPO_MLP_H];
  for (int j = 0; j < HGPO_MLP_H; ++j) {
    int64_t acc = q.b1[j];
    for (int f = 0; f < HGPO_MLP_F; ++f) acc += (int64_t)x[f] * q.w1[f * HGPO_MLP_H + j];
    a1[j] = clamp255(rshift_rne(acc, q.r1));
  }
  for (int k = 0; k < HGPO_MLP_H; ++k) {
    int64_t acc = q.b2[k];
    for (int j = 0; j < HGPO_MLP_H; ++j) acc += a1[j] * q.w2[j * HGPO_MLP_H + k];
    a2[k] = clamp255(rshift_rne(acc, q.r2));
  }
  int64_t s = q.b3;
  for (int k = 0; k < HGPO_MLP_H; ++k) s += a2[k] * q.w3[k];
  return s;
}

bool mlp_ok(const hgpo_mlp *q) {
  if (!q || q->k < 1 || q->r1 < 0 || q->r1 > 30 || q->r2 < 0 || q->r2 > 30) return false;
  const int64_t bmax = (int64_t)1 << 22;
  auto wok = [](int32_t v) { return v >= -255 && v <= 255; };
  auto bok = [bmax](int32_t v) { return (int64_t)v >= -bmax && (int64_t)v <= bmax; };
  for (int i = 0; i < HGPO_MLP_F * HGPO_MLP_H; ++i)
    if (!wok(q->w1[i])) return false;
  for (int i = 0; i < HGPO_MLP_H * HGPO_MLP_H; ++i)
    if (!wok(q->w2[i])) return false;
  for (int i = 0; i < HGPO_MLP_H; ++i)
    if (!wok(q->w3[i]) || !bok(q->b1[i]) || !bok(q->b2[i])) return false;
  return bok(q->b3);
}

/* A valid candidate m of n with hist(n,m) and c(n,m). */
struct Cand {
  int32_t m;
  int64_t h;
  int64_t c;
};

/* Codes of the features of the unordered pair {n, m} (see hgpo.h). */
void pair_codes(const Level &L, int32_t level, int64_t omega, int64_t delta, int32_t n, const Cand &cd, int32_t *x) {
  const int32_t a = std::min(n, cd.m), b = std::max(n, cd.m);
  const int64_t uni = (int64_t)L.indeg[a] + L.indeg[b] - cd.c;
  const int64_t f[HGPO_MLP_NFEAT] = {cd.h,
                                     cd.c,
                                     L.size[a],
                                     L.size[b],
                                     uni,
                                     L.ioff[a + 1] - L.ioff[a],
                                     L.ioff[b + 1] - L.ioff[b],
                                     level,
                                     omega - L.size[a] - L.size[b],
                                     delta - uni};
  for (int i = 0; i < HGPO_MLP_F; ++i) x[i] = i < HGPO_MLP_NFEAT ? qlog_code(f[i]) : 0;
}

/* The K best valid candidates of every node by (hist, id), descending, with
 * the same hist / c / validity as rate_select (Eq. 2, Sec. III-A). */
void rate_topk(const Level &L, const std::vector<int32_t> &w, int64_t omega, int64_t delta, int32_t K,
               std::vector<std::vector<Cand>> &top) {
  const int32_t N = L.n;
  top.assign((size_t)N, {});
#pragma omp parallel
  {
    std::vector<int64_t> hist((size_t)N, 0);
    std::vector<int64_t> common((size_t)N, 0);
    std::vector<uint8_t> seen((size_t)N, 0);
    std::vector<int32_t> touched;
    std::vector<Cand> valid;
#pragma omp for schedule(dynamic, 64)
    for (int32_t n = 0; n < N; ++n) {
      touched.clear();
      for (int64_t i = L.ioff[n]; i < L.ioff[n + 1]; ++i) {
        const int32_t e = L.ihe[i];
        const bool n_dst = L.idst[i] != 0;
        for (int64_t j = L.hoff[e]; j < L.hoff[e + 1]; ++j) {
          const int32_t m = L.hpin[j];
          if (m == n) continue;
          if (!seen[m]) {
            seen[m] = 1;
            touched.push_back(m);
          }
          hist[m] += w[e];
          if (n_dst && L.hdst[j]) common[m] += 1;
        }
      }
      valid.clear();
      for (int32_t m : touched) {
        if (L.size[n] + L.size[m] <= omega && (int64_t)L.indeg[n] + L.indeg[m] - common[m] <= delta)
          valid.push_back({m, hist[m], common[m]});
        hist[m] = 0;
        common[m] = 0;
        seen[m] = 0;
      }
      std::sort(valid.begin(), valid.end(),
                [](const Cand &x, const Cand &y) { return x.h != y.h ? x.h > y.h : x.m > y.m; });
      if ((int32_t)valid.size() > K) valid.resize((size_t)K);
      top[n] = valid;
    }
  }
}

/* C(n) = topK(n) u {m : n in topK(m)}, ascending by id. */
void symmetric_candidates(const std::vector<std::vector<Cand>> &top, std::vector<std::vector<Cand>> &cand) {
  const int32_t N = (int32_t)top.size();
  cand.assign((size_t)N, {});
  for (int32_t n = 0; n < N; ++n)
    for (const Cand &x : top[n]) {
      cand[n].push_back(x);
      cand[x.m].push_back({n, x.h, x.c});
    }
  for (auto &v : cand) {
    std::sort(v.begin(), v.end(), [](const Cand &x, const Cand &y) { return x.m < y.m; });
    v.erase(std::unique(v.begin(), v.end(), [](const Cand &x, const Cand &y) { return x.m == y.m; }), v.end());
  }
}

/* Plain runs with a tracer also record the symmetric 8-best candidate sets
 * and their input codes (the rows a learned network is trained on). */
void record_candidates(const Level &L, int32_t level, const std::vector<int32_t> &w, int64_t omega, int64_t delta,
                       hgpo_trace *trace) {
  std::vector<std::vector<Cand>> top, cand;
  rate_topk(L, w, omega, delta, 8, top);
  symmetric_candidates(top, cand);
  std::vector<int64_t> coff((size_t)L.n + 1, 0);
  std::vector<int32_t> cid, feat;
  int32_t x[HGPO_MLP_F];
  for (int32_t n = 0; n < L.n; ++n) {
    for (const Cand &cd : cand[n]) {
      cid.push_back(cd.m);
      pair_codes(L, level, omega, delta, n, cd, x);
      feat.insert(feat.end(), x, x + HGPO_MLP_F);
    }
    coff[(size_t)n + 1] = (int64_t)cid.size();
  }
  trace->put64(HGPO_LV_COFF, level, coff);
  trace->put32(HGPO_LV_CAND, level, cid);
  trace->put32(HGPO_LV_FEAT, level, feat);
}

/* One coarsening level with the learned proposal: top-K rating, symmetric
 * candidate sets, network scores, pair(n) = argmax (score, id) over C(n),
 * the matching of Sec. III-A on those pairs, and the plain fallback. */
void learned_level(const Level &L, int32_t level, const std::vector<int32_t> &w, int64_t omega, int64_t delta,
                   const hgpo_mlp &q, std::vector<int32_t> &pair, std::vector<int64_t> &score,
                   std::vector<int32_t> &match, int32_t &n_fallback, hgpo_trace *trace) {
  const int32_t N = L.n;
  std::vector<std::vector<Cand>> top, cand;
  rate_topk(L, w, omega, delta, q.k, top);
  std::vector<int32_t> ppair((size_t)N, -1), pmatch;
  std::vector<int64_t> pscore((size_t)N, 0);
  for (int32_t n = 0; n < N; ++n)
    if (!top[n].empty()) {
      ppair[n] = top[n][0].m;
      pscore[n] = top[n][0].h;
    }
  symmetric_candidates(top, cand);
  std::vector<std::vector<int64_t>> cs((size_t)N);
  pair.assign((size_t)N, -1);
  score.assign((size_t)N, 0);
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t n = 0; n < N; ++n) {
    int32_t x[HGPO_MLP_F];
    cs[n].resize(cand[n].size());
    for (size_t i = 0; i < cand[n].size(); ++i) {
      pair_codes(L, level, omega, delta, n, cand[n][i], x);
      const int64_t s = mlp_forward(q, x);
      cs[n][i] = s;
      if (pair[n] < 0 || s > score[n] || (s == score[n] && cand[n][i].m > pair[n])) {
        pair[n] = cand[n][i].m;
        score[n] = s;
      }
    }
  }
  match_pairs(pair, score, match);
  match_pairs(ppair, pscore, pmatch);
  int64_t ml = 0, mp = 0;
  for (int32_t n = 0; n < N; ++n) {
    ml += match[n] > n;
    mp += pmatch[n] > n;
  }
  const bool fb = 2 * ml < mp;
  if (fb) {
    match.swap(pmatch);
    ++n_fallback;
  }
  if (trace) {
    std::vector<int64_t> coff((size_t)N + 1, 0), csc;
    std::vector<int32_t> cid, feat;
    int32_t x[HGPO_MLP_F];
    for (int32_t n = 0; n < N; ++n) {
      for (size_t i = 0; i < cand[n].size(); ++i) {
        cid.push_back(cand[n][i].m);
        csc.push_back(cs[n][i]);
        pair_codes(L, level, omega, delta, n, cand[n][i], x);
        feat.insert(feat.end(), x, x + HGPO_MLP_F);
      }
      coff[(size_t)n + 1] = (int64_t)cid.size();
    }
    trace->put64(HGPO_LV_COFF, level, coff);
    trace->put32(HGPO_LV_CAND, level, cid);
    trace->put64(HGPO_LV_CSCORE, level, csc);
    trace->put32(HGPO_LV_FEAT, level, feat);
    trace->put32(HGPO_LV_PPAIR, level, ppair);
    trace->put32(HGPO_LV_FALLBACK, level, std::vector<int32_t>{fb ? 1 : 0});
  }
}

/*
 * Coarse hypergraph, Sec. III-B: N' = {{n, match(n)}}, gamma(n) = the rank of
 * the cluster's smaller member among all such representatives (ascending).
 * Every hedge keeps its id and weight; its pins become the set of clusters of
 * its pins, a cluster being a destination iff one of its members is.
 * Coarse node weight = sum of member weights.
 */
void cluster_map(const std::vector<int32_t> &match, std::vector<int32_t> &gamma, int32_t &n_next) {
  const int32_t N = (int32_t)match.size();
  gamma.assign((size_t)N, 0);
  int32_t next = 0;
  for (int32_t n = 0; n < N; ++n)
    if (match[n] >= n) gamma[n] = next++;
  for (int32_t n = 0; n < N; ++n)
    if (match[n] < n) gamma[n] = gamma[match[n]];
  n_next = next;
}

void contract(const Level &L, int32_t E, const std::vector<int32_t> &gamma, int32_t n_next, Level &C) {
  C.n = n_next;
  C.size.assign((size_t)n_next, 0);
  for (int32_t v = 0; v < L.n; ++v) C.size[gamma[v]] += L.size[v];
  C.hoff.assign((size_t)E + 1, 0);
  C.hpin.clear();
  C.hdst.clear();
  std::vector<std::pair<int32_t, uint8_t>> buf;
  for (int32_t e = 0; e < E; ++e) {
    buf.clear();
    for (int64_t j = L.hoff[e]; j < L.hoff[e + 1]; ++j) buf.push_back({gamma[L.hpin[j]], L.hdst[j]});
    std::sort(buf.begin(), buf.end());
    for (size_t i = 0; i < buf.size(); ++i) {
      if (!C.hpin.empty() && (int64_t)C.hpin.size() > C.hoff[e] && C.hpin.back() == buf[i].first) {
        C.hdst.back() = (uint8_t)(C.hdst.back() | buf[i].second);
      } else {
        C.hpin.push_back(buf[i].first);
        C.hdst.push_back(buf[i].second);
      }
    }
    C.hoff[e + 1] = (int64_t)C.hpin.size();
  }
  build_incidence(C, E);
}

/* Per-hedge part table entry: pins(p,e) and pins_in(p,e) of Sec. IV-B. */
struct PT {
  int32_t part;
  int32_t pins;
  int32_t pins_in;
};

using PartTables = std::vector<std::vector<PT>>;

/* pins(p,e) = |{n in e : rho(n) = p}|, pins_in(p,e) = |{n in dst(e) : rho(n) = p}|
 * (Sec. IV-B, counting pins per partition), ascending by part. */
void part_tables(const Level &L, int32_t E, const std::vector<int32_t> &rho, PartTables &pt) {
  pt.assign((size_t)E, {});
  std::vector<std::pair<int32_t, uint8_t>> buf;
  for (int32_t e = 0; e < E; ++e) {
    buf.clear();
    for (int64_t j = L.hoff[e]; j < L.hoff[e + 1]; ++j) buf.push_back({rho[L.hpin[j]], L.hdst[j]});
    std::sort(buf.begin(), buf.end());
    for (auto &b : buf) {
      if (pt[e].empty() || pt[e].back().part != b.first) pt[e].push_back({b.first, 0, 0});
      pt[e].back().pins += 1;
      pt[e].back().pins_in += b.second;
    }
  }
}

PT *pt_find(std::vector<PT> &t, int32_t p) {
  auto it = std::lower_bound(t.begin(), t.end(), p, [](const PT &a, int32_t q) { return a.part < q; });
  if (it != t.end() && it->part == p) return &*it;
  return nullptr;
}

int32_t pt_pins(const std::vector<PT> &t, int32_t p) {
  auto it = std::lower_bound(t.begin(), t.end(), p, [](const PT &a, int32_t q) { return a.part < q; });
  return (it != t.end() && it->part == p) ? it->pins : 0;
}

PT &pt_get(std::vector<PT> &t, int32_t p) {
  auto it = std::lower_bound(t.begin(), t.end(), p, [](const PT &a, int32_t q) { return a.part < q; });
  if (it != t.end() && it->part == p) return *it;
  return *t.insert(it, PT{p, 0, 0});
}

/*
 * Move proposal, Eq. 3 and Sec. IV-B "moves proposal": with p_s = rho(n),
 *   saving(n)  = sum of w(e), e in I(n), pins(p_s,e) = 1
 *   loss(n,p)  = sum of w(e), e in I(n), pins(p,e)  = 0
 *   gain(n,p)  = saving(n) - loss(n,p)
 * over parts p != p_s with size(p) + size(n) <= Omega (parts that cannot take
 * n are excluded a priori).  The proposal is the p maximising (gain, part
 * id), kept only if gain > 0.  loss(n,p) is evaluated as
 *   sum_{e in I(n)} w(e) - sum_{e in I(n), pins(p,e) > 0} w(e),
 * the same sum split over the indicator; a part touching no hedge of n has
 * loss = sum_{e in I(n)} w(e) >= saving(n), so it can never carry a gain > 0
 * and only parts present in some hedge of I(n) are enumerated.
 */
void propose(const Level &L, const std::vector<int32_t> &w, const PartTables &pt, const std::vector<int32_t> &rho,
             const std::vector<int64_t> &psize, int64_t omega, int32_t n_parts, std::vector<int32_t> &dest,
             std::vector<int64_t> &gain) {
  const int32_t N = L.n;
  dest.assign((size_t)N, -1);
  gain.assign((size_t)N, 0);
#pragma omp parallel
  {
    std::vector<int64_t> conn((size_t)n_parts, 0);
    std::vector<uint8_t> seen((size_t)n_parts, 0);
    std::vector<int32_t> touched;
#pragma omp for schedule(dynamic, 64)
    for (int32_t n = 0; n < N; ++n) {
      const int32_t ps = rho[n];
      int64_t total = 0, saving = 0;
      touched.clear();
      for (int64_t i = L.ioff[n]; i < L.ioff[n + 1]; ++i) {
        const int32_t e = L.ihe[i];
        total += w[e];
        if (pt_pins(pt[e], ps) == 1) saving += w[e];
        for (const PT &x : pt[e]) {
          if (x.pins <= 0) continue;
          if (!seen[x.part]) {
            seen[x.part] = 1;
            touched.push_back(x.part);
          }
          conn[x.part] += w[e];
        }
      }
      int32_t bp = -1;
      int64_t bg = 0;
      for (int32_t p : touched) {
        if (p != ps && psize[p] + L.size[n] <= omega) {
          const int64_t loss = total - conn[p];
          const int64_t g = saving - loss;
          if (bp < 0 || g > bg || (g == bg && p > bp)) {
            bp = p;
            bg = g;
          }
        }
        conn[p] = 0;
        seen[p] = 0;
      }
      if (bp >= 0 && bg > 0) {
        dest[n] = bp;
        gain[n] = bg;
      }
    }
  }
}

struct RoundOut {
  bool applied = false;
};

/*
 * One refinement round, Sec. IV-A/IV-B:
 *  (a) part tables, part sizes and distinct inbound counts
 *      inb(p) = #{e : pins_in(p,e) > 0}                      (Sec. IV-B)
 *  (b) in-isolation proposals (Eq. 3)
 *  (c) sequence S sorted by (gain, id) descending
 *  (d) state_i = state_{i-1} with move i applied; the in-sequence gain is
 *      g'(i) = Conn(state_{i-1}) - Conn(state_i), exactly.  Only hedges of
 *      I(n) change, each by w(e) * ([pins(p_s,e) = 1] - [pins(p_d,e) = 0])
 *      in state_{i-1}; G(i) = sum_{j <= i} g'(j)
 *  (e) viol(i) = number of parts with size > Omega or inb > Delta in state_i
 *  (f) i* = argmax over i in [0, |S|] with viol(i) = 0 of (G(i), i); the
 *      prefix is applied iff G(i*) > 0.
 */
RoundOut refine_round(const Level &L, int32_t E, const std::vector<int32_t> &w, std::vector<int32_t> &rho,
                      int32_t n_parts, int64_t omega, int64_t delta, hgpo_trace *trace, int32_t level) {
  RoundOut out;
  PartTables pt;
  part_tables(L, E, rho, pt);
  std::vector<int64_t> psize((size_t)n_parts, 0);
  for (int32_t n = 0; n < L.n; ++n) psize[rho[n]] += L.size[n];
  std::vector<int32_t> pinb((size_t)n_parts, 0);
  for (int32_t e = 0; e < E; ++e)
    for (const PT &x : pt[e])
      if (x.pins_in > 0) pinb[x.part]++;

  std::vector<int32_t> dest;
  std::vector<int64_t> gain;
  propose(L, w, pt, rho, psize, omega, n_parts, dest, gain);

  std::vector<int32_t> seq;
  for (int32_t n = 0; n < L.n; ++n)
    if (dest[n] >= 0) seq.push_back(n);
  std::sort(seq.begin(), seq.end(), [&](int32_t a, int32_t b) {
    if (gain[a] != gain[b]) return gain[a] > gain[b];
    return a > b;
  });
  const int64_t S = (int64_t)seq.size();

  /* sequential replay of the sequence on live copies */
  std::vector<int32_t> state = rho;
  PartTables live = pt;
  std::vector<int64_t> lsize = psize;
  std::vector<int32_t> linb = pinb;
  auto part_invalid = [&](int32_t p) { return lsize[p] > omega || (int64_t)linb[p] > delta; };
  int32_t invalid = 0;
  for (int32_t p = 0; p < n_parts; ++p) invalid += part_invalid(p) ? 1 : 0;
  std::vector<int64_t> gp((size_t)S + 1, 0), G((size_t)S + 1, 0);
  std::vector<int32_t> viol((size_t)S + 1, 0);
  viol[0] = invalid;
  for (int64_t i = 1; i <= S; ++i) {
    const int32_t n = seq[(size_t)i - 1];
    const int32_t ps = state[n], pd = dest[n];
    const int32_t before = (part_invalid(ps) ? 1 : 0) + (part_invalid(pd) ? 1 : 0);
    int64_t g = 0;
    for (int64_t k = L.ioff[n]; k < L.ioff[n + 1]; ++k) {
      const int32_t e = L.ihe[k];
      const bool n_dst = L.idst[k] != 0;
      PT &s = pt_get(live[e], ps);
      if (s.pins == 1) g += w[e];
      PT &d0 = pt_get(live[e], pd);
      if (d0.pins == 0) g -= w[e];
      /* re-look-up: the insertion above may have moved the source entry */
      PT &s2 = *pt_find(live[e], ps);
      s2.pins -= 1;
      if (n_dst) {
        s2.pins_in -= 1;
        if (s2.pins_in == 0) linb[ps] -= 1;
      }
      PT &d = *pt_find(live[e], pd);
      d.pins += 1;
      if (n_dst) {
        d.pins_in += 1;
        if (d.pins_in == 1) linb[pd] += 1;
      }
    }
    lsize[ps] -= L.size[n];
    lsize[pd] += L.size[n];
    state[n] = pd;
    const int32_t after = (part_invalid(ps) ? 1 : 0) + (part_invalid(pd) ? 1 : 0);
    invalid += after - before;
    gp[(size_t)i] = g;
    G[(size_t)i] = G[(size_t)i - 1] + g;
    viol[(size_t)i] = invalid;
  }
  int64_t istar = -1;
  for (int64_t i = 0; i <= S; ++i)
    if (viol[(size_t)i] == 0 && (istar < 0 || G[(size_t)i] >= G[(size_t)istar])) istar = i;
  const int64_t Gstar = istar >= 0 ? G[(size_t)istar] : 0;

  if (trace) {
    const int32_t r = trace->rounds;
    trace->put32(HGPO_RD_RHO, r, rho);
    trace->put32(HGPO_RD_PDEST, r, dest);
    trace->put64(HGPO_RD_PGAIN, r, gain);
    trace->put32(HGPO_RD_SEQ, r, seq);
    trace->put64(HGPO_RD_GP, r, gp);
    trace->put64(HGPO_RD_G, r, G);
    trace->put32(HGPO_RD_VIOL, r, viol);
    std::vector<int64_t> ptoff((size_t)E + 1, 0);
    std::vector<int32_t> ptv;
    for (int32_t e = 0; e < E; ++e) {
      for (const PT &x : pt[e]) {
        ptv.push_back(x.part);
        ptv.push_back(x.pins);
        ptv.push_back(x.pins_in);
      }
      ptoff[(size_t)e + 1] = ptoff[(size_t)e] + (int64_t)pt[e].size();
    }
    trace->put64(HGPO_RD_PTOFF, r, ptoff);
    trace->put32(HGPO_RD_PT, r, ptv);
    trace->put64(HGPO_RD_PSIZE, r, psize);
    trace->put32(HGPO_RD_PINB, r, pinb);
    trace->put64(HGPO_RD_INFO, r, {level, S, istar, Gstar, (int64_t)(istar >= 0 && Gstar > 0), n_parts});
    trace->rounds++;
  }
  if (istar >= 0 && Gstar > 0) {
    for (int64_t i = 0; i < istar; ++i) rho[seq[(size_t)i]] = dest[seq[(size_t)i]];
    out.applied = true;
  }
  return out;
}

int validate(const hgpo_hypergraph *g, int32_t omega, int32_t delta, int32_t k, int32_t max_rounds) {
  if (!g || g->n_nodes < 0 || g->n_hedges < 0 || omega < 1 || delta < 0 || k < 0 || max_rounds < 0)
    return HGPO_EINVAL;
  if (!g->hedge_off) return HGPO_EINVAL;
  const int32_t N = g->n_nodes, E = g->n_hedges;
  if (g->hedge_off[0] != 0) return HGPO_EBADCSR;
  for (int32_t e = 0; e < E; ++e)
    if (g->hedge_off[e + 1] < g->hedge_off[e]) return HGPO_EBADCSR;
  const int64_t P = g->hedge_off[E];
  if (P > 0 && !g->pins) return HGPO_EINVAL;
  for (int64_t j = 0; j < P; ++j)
    if (g->pins[j] < 0 || g->pins[j] >= N) return HGPO_EBADCSR;
  if (g->n_src)
    for (int32_t e = 0; e < E; ++e)
      if (g->n_src[e] < 0 || g->n_src[e] > g->hedge_off[e + 1] - g->hedge_off[e]) return HGPO_EBADCSR;
  int64_t wsum = 0, nsum = 0;
  for (int32_t e = 0; e < E; ++e) {
    const int64_t x = g->hedge_w ? g->hedge_w[e] : 1;
    if (x < 1) return HGPO_EINVAL;
    wsum += x;
  }
  for (int32_t v = 0; v < N; ++v) {
    const int64_t x = g->node_w ? g->node_w[v] : 1;
    if (x < 1) return HGPO_EINVAL;
    nsum += x;
  }
  /* input domain shared with the GPU library: totals fit in int32 */
  if (wsum > kInt32Max || nsum > kInt32Max) return HGPO_EUNSUPPORTED;
  std::vector<int32_t> tmp;
  for (int32_t e = 0; e < E; ++e) {
    tmp.assign(g->pins + g->hedge_off[e], g->pins + g->hedge_off[e + 1]);
    std::sort(tmp.begin(), tmp.end());
    if (std::adjacent_find(tmp.begin(), tmp.end()) != tmp.end()) return HGPO_EBADCSR;
  }
  return HGPO_OK;
}

}  // namespace

extern "C" {

hgpo_trace *hgpo_trace_new(void) { return new (std::nothrow) hgpo_trace(); }
void hgpo_trace_free(hgpo_trace *t) { delete t; }
int32_t hgpo_trace_levels(const hgpo_trace *t) { return t ? t->levels : 0; }
int32_t hgpo_trace_rounds(const hgpo_trace *t) { return t ? t->rounds : 0; }

int64_t hgpo_trace_get(const hgpo_trace *t, int32_t kind, int32_t index, const void **data, int32_t *elem_bytes) {
  if (!t) return -1;
  auto it = t->recs.find({kind, index});
  if (it == t->recs.end()) return -1;
  const hgpo_trace::Rec &r = it->second;
  if (elem_bytes) *elem_bytes = r.bytes;
  if (r.bytes == 4) {
    if (data) *data = r.i32.data();
    return (int64_t)r.i32.size();
  }
  if (data) *data = r.i64.data();
  return (int64_t)r.i64.size();
}

int hgpo_connectivity(const hgpo_hypergraph *g, const int32_t *part, int64_t *out) {
  if (!g || !part || !out || !g->hedge_off || g->n_nodes < 0 || g->n_hedges < 0) return HGPO_EINVAL;
  int64_t conn = 0;
  std::vector<int32_t> parts;
  for (int32_t e = 0; e < g->n_hedges; ++e) {
    parts.clear();
    for (int32_t j = g->hedge_off[e]; j < g->hedge_off[e + 1]; ++j) parts.push_back(part[g->pins[j]]);
    std::sort(parts.begin(), parts.end());
    const int64_t lambda = std::unique(parts.begin(), parts.end()) - parts.begin();
    if (lambda > 0) conn += (int64_t)(g->hedge_w ? g->hedge_w[e] : 1) * (lambda - 1);
  }
  *out = conn;
  return HGPO_OK;
}

/*
 * The multilevel scheme of Sec. II-B.  Coarsening repeats rating, matching
 * and contraction (Sec. III) until, after a matching, the number of clusters
 * is at most T = ceil(sum of node weights / Omega) (or T = k when k > 0), or
 * no pair can be formed; the clusters of the last matching (or the nodes
 * themselves if nothing matched) are the initial parts, and no coarse
 * hypergraph is built for them.  Refinement (Sec. IV) then runs at every
 * level from the coarsest down, projecting the partition through the cluster
 * maps; each level runs rounds until one applies no move, at most
 * max_rounds.  Output part ids are renumbered 0..n_parts-1 by ascending
 * initial-part id, skipping emptied parts.
 */
static int partition_impl(const hgpo_hypergraph *g, int32_t omega, int32_t delta, int32_t k, int32_t max_rounds,
                          const hgpo_mlp *mlp, int32_t role, int32_t *part_out, hgpo_result *res, hgpo_trace *trace,
                          int32_t matching = HGPO_MATCH_TRAVERSAL) {
  int rc = validate(g, omega, delta, k, max_rounds);
  if (rc != HGPO_OK) return rc;
  if (!part_out && g->n_nodes > 0) return HGPO_EINVAL;
  try {
    const int32_t N = g->n_nodes, E = g->n_hedges;
    std::vector<int32_t> w((size_t)E);
    for (int32_t e = 0; e < E; ++e) w[e] = g->hedge_w ? g->hedge_w[e] : 1;

    std::vector<Level> levels(1);
    Level &L0 = levels[0];
    L0.n = N;
    L0.size.assign((size_t)N, 1);
    int64_t wsum = 0;
    for (int32_t v = 0; v < N; ++v) {
      L0.size[v] = g->node_w ? g->node_w[v] : 1;
      wsum += L0.size[v];
    }
    L0.hoff.assign((size_t)E + 1, 0);
    std::vector<std::pair<int32_t, uint8_t>> buf;
    for (int32_t e = 0; e < E; ++e) {
      const int32_t b = g->hedge_off[e], en = g->hedge_off[e + 1];
      const int32_t ns = g->n_src ? g->n_src[e] : 1;
      buf.clear();
      /* the pins whose hedges count toward Delta: destinations (inbound,
       * Sec. II-A), sources (outbound) or all pins (incident) */
      for (int32_t j = b; j < en; ++j) {
        const bool dst = (j - b) >= ns;
        const bool counted = role == HGPO_INBOUND ? dst : (role == HGPO_OUTBOUND ? !dst : true);
        buf.push_back({g->pins[j], (uint8_t)(counted ? 1 : 0)});
      }
      std::sort(buf.begin(), buf.end());
      for (auto &x : buf) {
        L0.hpin.push_back(x.first);
        L0.hdst.push_back(x.second);
      }
      L0.hoff[(size_t)e + 1] = (int64_t)L0.hpin.size();
    }
    build_incidence(L0, E);
    for (int32_t v = 0; v < N; ++v)
      if (L0.size[v] > omega || L0.indeg[v] > delta) return HGPO_EINFEASIBLE;

    const int64_t T = k > 0 ? (int64_t)k : (wsum + omega - 1) / omega;

    /* coarsening */
    int32_t n_fallback = 0;
    std::vector<int32_t> rho;
    int32_t n_parts = 0;
    int32_t l = 0;
    while (true) {
      Level &L = levels[(size_t)l];
      std::vector<int32_t> pair, match;
      std::vector<int64_t> score;
      if (!mlp) {
        rate_select(L, w, omega, delta, pair, score);
        if (matching == HGPO_MATCH_EXACT)
          match_exact(pair, score, match);
        else
          match_pairs(pair, score, match);
        if (trace) record_candidates(L, l, w, omega, delta, trace);
      } else {
        learned_level(L, l, w, omega, delta, *mlp, pair, score, match, n_fallback, trace);
      }
      int32_t M = 0;
      for (int32_t n = 0; n < L.n; ++n)
        if (match[n] > n) ++M;
      if (trace) {
        std::vector<int32_t> hp(L.hpin.size());
        for (size_t j = 0; j < hp.size(); ++j) hp[j] = L.hpin[j] | (L.hdst[j] ? (int32_t)0x80000000u : 0);
        trace->put64(HGPO_LV_HOFF, l, L.hoff);
        trace->put32(HGPO_LV_HPIN, l, hp);
        trace->put64(HGPO_LV_SIZE, l, L.size);
        trace->put32(HGPO_LV_PAIR, l, pair);
        trace->put64(HGPO_LV_SCORE, l, score);
        trace->put32(HGPO_LV_MATCH, l, match);
      }
      if (M == 0) {
        rho.resize((size_t)L.n);
        for (int32_t n = 0; n < L.n; ++n) rho[n] = n;
        n_parts = L.n;
        break;
      }
      int32_t n_next = 0;
      cluster_map(match, L.gamma, n_next);
      if (trace) trace->put32(HGPO_LV_GAMMA, l, L.gamma);
      if ((int64_t)n_next <= T) {
        rho = L.gamma;
        n_parts = n_next;
        break;
      }
      levels.emplace_back();
      contract(levels[(size_t)l], E, levels[(size_t)l].gamma, n_next, levels[(size_t)l + 1]);
      drop_incidence(levels[(size_t)l]);  /* rebuilt when refinement returns to this level */
      ++l;
    }
    const int32_t Lmax = l;
    if (trace) trace->levels = Lmax + 1;

    /* refinement, coarsest level first */
    int32_t rounds = 0;
    for (int32_t lv = Lmax; lv >= 0; --lv) {
      Level &L = levels[(size_t)lv];
      if (L.ioff.empty()) build_incidence(L, E);
      if (lv < Lmax) {
        std::vector<int32_t> finer((size_t)L.n);
        for (int32_t v = 0; v < L.n; ++v) finer[v] = rho[L.gamma[v]];
        rho.swap(finer);
      }
      if (trace) trace->put32(HGPO_LV_RHO0, lv, rho);
      for (int32_t r = 0; r < max_rounds; ++r) {
        ++rounds;
        RoundOut ro = refine_round(L, E, w, rho, n_parts, omega, delta, trace, lv);
        if (!ro.applied) break;
      }
      if (trace) trace->put32(HGPO_LV_RHO1, lv, rho);
      if (lv > 0) {
        drop_incidence(L);
        std::vector<int32_t>().swap(L.hpin);
        std::vector<uint8_t>().swap(L.hdst);
      }
    }

    /* output: renumber non-empty parts ascending */
    std::vector<int32_t> rename((size_t)n_parts, -1);
    for (int32_t v = 0; v < N; ++v) rename[rho[v]] = 0;
    int32_t np = 0;
    for (int32_t p = 0; p < n_parts; ++p)
      if (rename[p] == 0) rename[p] = np++;
    for (int32_t v = 0; v < N; ++v) part_out[v] = rename[rho[v]];
    if (res) {
      std::vector<int32_t> fin(part_out, part_out + N);
      res->connectivity = connectivity_of(levels[0], E, w, fin);
      res->n_parts = np;
      res->n_levels = Lmax + 1;
      res->n_rounds = rounds;
      res->n_fallback = n_fallback;
    }
  } catch (const std::bad_alloc &) {
    return HGPO_ENOMEM;
  }
  return HGPO_OK;
}

int hgpo_partition(const hgpo_hypergraph *g, int32_t omega, int32_t delta, int32_t k, int32_t max_rounds,
                   int32_t *part_out, hgpo_result *res, hgpo_trace *trace) {
  return partition_impl(g, omega, delta, k, max_rounds, nullptr, HGPO_INBOUND, part_out, res, trace);
}

int hgpo_partition_role(const hgpo_hypergraph *g, int32_t omega, int32_t delta, int32_t k, int32_t max_rounds,
                        int32_t role, int32_t *part_out, hgpo_result *res, hgpo_trace *trace) {
  if (role != HGPO_INBOUND && role != HGPO_OUTBOUND && role != HGPO_INCIDENT) return HGPO_EINVAL;
  return partition_impl(g, omega, delta, k, max_rounds, nullptr, role, part_out, res, trace);
}

int hgpo_partition_ex(const hgpo_hypergraph *g, int32_t omega, int32_t delta, int32_t k, int32_t max_rounds,
                      int32_t role, int32_t matching, int32_t *part_out, hgpo_result *res, hgpo_trace *trace) {
  if (role != HGPO_INBOUND && role != HGPO_OUTBOUND && role != HGPO_INCIDENT) return HGPO_EINVAL;
  if (matching != HGPO_MATCH_TRAVERSAL && matching != HGPO_MATCH_EXACT) return HGPO_EINVAL;
  return partition_impl(g, omega, delta, k, max_rounds, nullptr, role, part_out, res, trace, matching);
}

int hgpo_match(int32_t n, const int32_t *pair, const int64_t *score, int32_t matching, int32_t *match_out) {
  if (n < 0 || (n > 0 && (!pair || !score || !match_out))) return HGPO_EINVAL;
  if (matching != HGPO_MATCH_TRAVERSAL && matching != HGPO_MATCH_EXACT) return HGPO_EINVAL;
  for (int32_t v = 0; v < n; ++v)
    if (pair[v] < -1 || pair[v] >= n || pair[v] == v) return HGPO_EINVAL;
  try {
    std::vector<int32_t> p(pair, pair + n), m;
    std::vector<int64_t> sc(score, score + n);
    if (matching == HGPO_MATCH_EXACT)
      match_exact(p, sc, m);
    else
      match_pairs(p, sc, m);
    std::copy(m.begin(), m.end(), match_out);
  } catch (const std::logic_error &) {
    return HGPO_EINVAL;
  }
  return HGPO_OK;
}

int hgpo_partition_learned(const hgpo_hypergraph *g, int32_t omega, int32_t delta, int32_t k, int32_t max_rounds,
                           const hgpo_mlp *mlp, int32_t *part_out, hgpo_result *res, hgpo_trace *trace) {
  if (!mlp_ok(mlp)) return HGPO_EINVAL;
  return partition_impl(g, omega, delta, k, max_rounds, mlp, HGPO_INBOUND, part_out, res, trace);
}

int hgpo_mlp_score(const hgpo_mlp *mlp, const int32_t *xq, int64_t n, int64_t *score) {
  if (!mlp_ok(mlp) || n < 0 || (n > 0 && (!xq || !score))) return HGPO_EINVAL;
  for (int64_t i = 0; i < n * HGPO_MLP_F; ++i)
    if (xq[i] < 0 || xq[i] > 255) return HGPO_EINVAL;
  for (int64_t i = 0; i < n; ++i) score[i] = mlp_forward(*mlp, xq + i * HGPO_MLP_F);
  return HGPO_OK;
}

int32_t hgpo_qlog(int64_t f) { return f < 0 ? -1 : qlog_code(f); }

}  // extern "C"
