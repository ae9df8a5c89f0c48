/*
 * hgpo -- CPU oracle for incidence-constrained multilevel hypergraph
 * partitioning (Ronzani & Silvano, "Incidence Constraints in Hypergraph
 * Partitioning on GPU").
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, sequential restatement of
 * the method used to check the GPU library; it shares no code with it and the
 * product never calls it.
 *
 * Inputs use the int32 CSR layout: hedge_off[E+1], pins[P] with the n_src[e]
 * source pins of each hedge first, hedge_w[E] >= 1, node_w[N] >= 1.
 * All arithmetic is integer (int64 accumulators); ties go to the larger id.
 */
#ifndef HGPO_H
#define HGPO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HGPO_OK = 0,
  HGPO_EINVAL = -1,
  HGPO_EBADCSR = -2,
  HGPO_EINFEASIBLE = -3,
  HGPO_ENOMEM = -4,
  HGPO_EUNSUPPORTED = -6
};

typedef struct {
  int32_t n_nodes;
  int32_t n_hedges;
  const int32_t *hedge_off; /* [n_hedges+1] */
  const int32_t *pins;      /* [hedge_off[n_hedges]] */
  const int32_t *n_src;     /* [n_hedges] or NULL (=> 1) */
  const int32_t *hedge_w;   /* [n_hedges] or NULL (=> 1) */
  const int32_t *node_w;    /* [n_nodes] or NULL (=> 1) */
} hgpo_hypergraph;

typedef struct {
  int64_t connectivity; /* Eq. 1 on the input hypergraph */
  int32_t n_parts;
  int32_t n_levels; /* levels built: 1 + number of contractions */
  int32_t n_rounds; /* refinement rounds run, summed over levels */
  int32_t n_fallback; /* learned proposal: levels that took the plain matching */
} hgpo_result;

/*
 * Learned merge proposal (an extension outside the paper's method).  At each
 * coarsening level the rating of Eq. 2 yields, per node, its K best valid
 * candidates by (hist, id).  The candidate sets are made symmetric
 * (C(n) = topK(n) u {m : n in topK(m)}), every pair is scored by a small
 * fixed-point network on exact integer features of the unordered pair, and
 * pair(n) = the m in C(n) maximising (score, id).  Scores are symmetric and
 * candidate sets are symmetric, so the pairing graph keeps the "cycles of
 * length two only" property the matching relies on.
 *
 * Features of the unordered pair {a < b} (all exact integers, Sec. II-A/III-A
 * quantities): hist(a,b), c(a,b), size(a), size(b), |in(a) u in(b)|, |I(a)|,
 * |I(b)|, the level, Omega - size(a) - size(b), Delta - |in(a) u in(b)|,
 * then six zeros.  Each feature f enters the network as the 8-bit code
 * qlog(f) = min(255, 8 e + t) with e = floor(log2(f+1)) and t the three bits
 * of f+1 below its leading one (a piecewise-linear log2 with 3 fraction bits).
 *
 * Network (integers throughout, round-half-even right shifts):
 *   a1 = clamp(rshift(W1^T x + b1, r1), 0, 255)      64 units
 *   a2 = clamp(rshift(W2^T a1 + b2, r2), 0, 255)     64 units
 *   score = w3 . a2 + b3
 * with |W1|, |W2|, |w3| <= 255 and |b| <= 2^22, so every partial sum stays
 * below 2^24 in magnitude.
 *
 * Fallback: the plain pair (the first of the K candidates) gives a second
 * matching at every level; when the learned matching merges fewer than half
 * as many pairs, the plain matching is used for that level.
 */
enum { HGPO_MLP_F = 16, HGPO_MLP_H = 64, HGPO_MLP_NFEAT = 10 };
typedef struct {
  int32_t k;                          /* candidates per node (>= 1)         */
  int32_t r1, r2;                     /* requantisation shifts (0 .. 30)    */
  int32_t b3;
  int32_t w1[HGPO_MLP_F * HGPO_MLP_H];  /* [f][j] */
  int32_t b1[HGPO_MLP_H];
  int32_t w2[HGPO_MLP_H * HGPO_MLP_H];  /* [j][k] */
  int32_t b2[HGPO_MLP_H];
  int32_t w3[HGPO_MLP_H];
} hgpo_mlp;

typedef struct hgpo_trace hgpo_trace;

/* Trace record kinds.  Level records take the level index; round records
 * take the global round index (0 .. n_rounds-1). */
enum {
  HGPO_LV_HOFF = 0,   /* int64 [E+1]  canonical hedge offsets at the level   */
  HGPO_LV_HPIN = 1,   /* int32 [P_l]  pin id | (dst << 31), ascending id      */
  HGPO_LV_SIZE = 2,   /* int32 [N_l]  node weights                            */
  HGPO_LV_PAIR = 3,   /* int32 [N_l]  candidate, -1 = none                    */
  HGPO_LV_SCORE = 4,  /* int64 [N_l]  hist(n, pair(n)), 0 if none             */
  HGPO_LV_MATCH = 5,  /* int32 [N_l]                                          */
  HGPO_LV_GAMMA = 6,  /* int32 [N_l]  cluster map (empty if no match)         */
  HGPO_LV_RHO0 = 7,   /* int32 [N_l]  partition entering refinement           */
  HGPO_LV_RHO1 = 8,   /* int32 [N_l]  partition after refinement              */
  HGPO_LV_COFF = 9,   /* int64 [N_l+1] learned: candidate offsets              */
  HGPO_LV_CAND = 10,  /* int32 [C]    learned: candidate ids, ascending per node */
  HGPO_LV_CSCORE = 11, /* int64 [C]   learned: network score of each candidate */
  HGPO_LV_FEAT = 12,  /* int32 [C*16] learned: input codes qlog(f) per candidate */
  HGPO_LV_PPAIR = 13, /* int32 [N_l]  learned: plain pair (first candidate)    */
  HGPO_LV_FALLBACK = 14, /* int32 [1] learned: 1 if the plain matching was used */
  HGPO_RD_INFO = 20,  /* int64 [6]: level, |S|, i*, G(i*), applied, n_parts   */
  HGPO_RD_RHO = 21,   /* int32 [N_l]  partition at round start                */
  HGPO_RD_PDEST = 22, /* int32 [N_l]  proposed destination, -1 = none         */
  HGPO_RD_PGAIN = 23, /* int64 [N_l]  in-isolation gain of the proposal       */
  HGPO_RD_SEQ = 24,   /* int32 [|S|]  nodes in sequence order                 */
  HGPO_RD_GP = 25,    /* int64 [|S|+1] in-sequence gain g'(i), g'(0) = 0      */
  HGPO_RD_G = 26,     /* int64 [|S|+1] prefix G(i)                            */
  HGPO_RD_VIOL = 27,  /* int32 [|S|+1] violated parts after prefix i          */
  HGPO_RD_PTOFF = 28, /* int64 [E+1]  part-table offsets at round start       */
  HGPO_RD_PT = 29,    /* int32 [3*sum lambda] (part, pins, pins_in) ascending */
  HGPO_RD_PSIZE = 30, /* int64 [n_parts] part sizes at round start            */
  HGPO_RD_PINB = 31   /* int32 [n_parts] distinct inbound hedges per part     */
};

int hgpo_partition(const hgpo_hypergraph *g, int32_t omega, int32_t delta, int32_t k, int32_t max_rounds,
                   int32_t *part_out, hgpo_result *res, hgpo_trace *trace);

/* Roles of the pins whose hedges count toward Delta: inbound (destination
 * pins, the paper's constraint), outbound (source pins), incident (all). */
enum { HGPO_INBOUND = 0, HGPO_OUTBOUND = 1, HGPO_INCIDENT = 2 };

/* As hgpo_partition with the Delta bound counting the hedges of `role`. */
int hgpo_partition_role(const hgpo_hypergraph *g, int32_t omega, int32_t delta, int32_t k, int32_t max_rounds,
                        int32_t role, int32_t *part_out, hgpo_result *res, hgpo_trace *trace);

/* Matching rules over the pairing pseudo-forest: the two traversals of
 * Sec. III-A (the paper's), or the exact maximum-weight matching by the tree
 * recursion of the dynamic-programming formulation of Sec. VI. */
enum { HGPO_MATCH_TRAVERSAL = 0, HGPO_MATCH_EXACT = 1 };

/* As hgpo_partition_role with the given matching rule (plain method). */
int hgpo_partition_ex(const hgpo_hypergraph *g, int32_t omega, int32_t delta, int32_t k, int32_t max_rounds,
                      int32_t role, int32_t matching, int32_t *part_out, hgpo_result *res, hgpo_trace *trace);

/* One matching of n nodes from pair[n] (-1: none; no self pairs, cycles of
 * length two only) and score[n]: match_out[n] (n itself if unmatched). */
int hgpo_match(int32_t n, const int32_t *pair, const int64_t *score, int32_t matching, int32_t *match_out);

/* As hgpo_partition with the learned merge proposal (mlp non-NULL). */
int hgpo_partition_learned(const hgpo_hypergraph *g, int32_t omega, int32_t delta, int32_t k, int32_t max_rounds,
                           const hgpo_mlp *mlp, int32_t *part_out, hgpo_result *res, hgpo_trace *trace);

/* The network on n input rows xq[n*16] (codes 0..255): score[n]. */
int hgpo_mlp_score(const hgpo_mlp *mlp, const int32_t *xq, int64_t n, int64_t *score);

/* The 8-bit feature code qlog(f) of f >= 0. */
int32_t hgpo_qlog(int64_t f);

/* Eq. 1 for an arbitrary partition vector (part ids >= 0). */
int hgpo_connectivity(const hgpo_hypergraph *g, const int32_t *part, int64_t *out);

hgpo_trace *hgpo_trace_new(void);
void hgpo_trace_free(hgpo_trace *t);
int32_t hgpo_trace_levels(const hgpo_trace *t);
int32_t hgpo_trace_rounds(const hgpo_trace *t);
/* Returns the element count of record (kind, index) and sets *data to its
 * storage (owned by the trace), or -1 if absent.  *elem_bytes is 4 or 8. */
int64_t hgpo_trace_get(const hgpo_trace *t, int32_t kind, int32_t index, const void **data, int32_t *elem_bytes);

#ifdef __cplusplus
}
#endif
#endif
