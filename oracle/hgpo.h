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
  int32_t pad;
} hgpo_result;

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
