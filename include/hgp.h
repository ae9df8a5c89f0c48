/*
 * libhgp -- incidence-constrained multilevel hypergraph partitioning on
 * MI355X (gfx950), after Ronzani & Silvano, "Incidence Constraints in
 * Hypergraph Partitioning on GPU".
 *
 * Problem (Sec. II-A): a directed weighted hypergraph G(N, E, w) is split
 * into disjoint non-empty parts so that every part p holds at most Omega
 * node weight and at most Delta distinct inbound hyperedges
 * (|U_{n in p} in(n)| <= Delta, in(n) = {e : n in dst(e)}), minimising the
 * connectivity of Eq. 1, Conn = sum_e w(e) * (lambda(e) - 1), lambda(e) being
 * the number of distinct parts among the pins of e.  The number of parts is
 * not fixed: it emerges from multilevel coarsening (Sec. II-B, III) followed
 * by refinement (Sec. IV).
 *
 * All arithmetic is integer and every tie is broken by id, so a given input
 * yields the same bits whatever the stream, launch shape or run.
 *
 * Conventions
 *  - Return value: 0 on success, a negative HGP_E* code on failure.  On
 *    failure no output buffer is written and hgp_last_error() holds a
 *    message for the calling thread.  No C++ exception crosses the ABI.
 *  - The caller owns every buffer it passes; inputs are only read.  The
 *    context owns its device scratch until hgp_ctx_destroy().
 *  - "device pointer" means memory on the context's device (hipMalloc or a
 *    torch tensor's data_ptr()); "stream" is a hipStream_t (NULL = the null
 *    stream).  Device-side calls are ordered on the given stream; calls that
 *    return scalars to the host synchronise that stream.
 *  - One context must not be used by two threads at once.
 */
#ifndef HGP_H
#define HGP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define HGP_OK 0
#define HGP_EINVAL (-1)        /* NULL pointer, negative count, Omega < 1, Delta < 0, weight < 1 */
#define HGP_EBADCSR (-2)       /* offsets not monotone, pin out of range, duplicate pin, n_src > |e| */
#define HGP_EINFEASIBLE (-3)   /* a node with w(n) > Omega or |in(n)| > Delta: no valid partition */
#define HGP_ENOMEM (-4)        /* device allocation failed */
#define HGP_EDEVICE (-5)       /* HIP runtime error (text in hgp_last_error) */
#define HGP_EUNSUPPORTED (-6)  /* outside the supported domain (see hgp_partition) */
#define HGP_EINTERNAL (-7)     /* an internal consistency check failed */

/*
 * Input hypergraph in int32 CSR form (Sec. II-C: offsets + segmented data).
 * Hedge e has pins pins[hedge_off[e] .. hedge_off[e+1]); the first n_src[e]
 * of them are its sources src(e), the rest its destinations dst(e).  A node
 * appears at most once per hedge.  NULL n_src means one source per hedge,
 * NULL hedge_w / node_w mean unit weights.  Either all pointers are host
 * pointers (hgp_partition) or all are device pointers (the _device calls).
 */
typedef struct {
  int32_t n_nodes;          /* |N| >= 0 */
  int32_t n_hedges;         /* |E| >= 0 */
  const int32_t *hedge_off; /* [n_hedges + 1], hedge_off[0] = 0, non-decreasing */
  const int32_t *pins;      /* [hedge_off[n_hedges]], values in [0, n_nodes) */
  const int32_t *n_src;     /* [n_hedges], 0 <= n_src[e] <= |e|, or NULL */
  const int32_t *hedge_w;   /* [n_hedges], >= 1, or NULL */
  const int32_t *node_w;    /* [n_nodes], >= 1, or NULL */
} hgp_hypergraph;

#define HGP_PLAIN 0

/* hgp_options.flags */
#define HGP_FLAG_TIME_KERNELS 1   /* time kernel classes with HIP events on the call's stream */
#define HGP_FLAG_NO_INCREMENTAL 2 /* rate every level and propose every round from scratch (same result) */

/* kernel classes reported in hgp_result.ms_kernel / n_kernel / units_kernel */
#define HGP_K_RATE 0       /* candidate rating + selection; unit: pin-pair visit (sum |e|^2 per level) */
#define HGP_K_PROPOSE 1    /* move proposal; unit: part-table entry visit (sum over e of |e| * lambda(e)) */
#define HGP_K_PARTTABLE 2  /* per-hedge part tables; unit: pin */
#define HGP_K_SEQEVENTS 3  /* in-sequence gains and inbound transitions; unit: pin */
#define HGP_K_CONTRACT 4   /* coarse hedge construction; unit: pin */
#define HGP_K_INCIDENCE 5  /* incidence transpose; unit: pin */
#define HGP_K_SORT 6       /* move / event sorts; unit: key */
#define HGP_K_MATCH 7      /* pseudo-forest matching; unit: node */
#define HGP_K_RATE_TAIL 8  /* late-level rating with top-K lists; unit: pin-pair visit */
#define HGP_NKERNEL 9

typedef struct {
  int32_t k;                 /* 0: coarsen to ceil(sum w / Omega) clusters (Sec. II-B); k > 0: to k */
  int32_t max_refine_rounds; /* refinement rounds per level (default 8); a level stops early
                                once a round applies no move */
  uint64_t seed;             /* not used by the plain method (its result is seed-independent) */
  int32_t proposal;          /* HGP_PLAIN */
  int32_t flags;             /* HGP_FLAG_* bits, 0 by default */
} hgp_options;

typedef struct {
  int64_t connectivity; /* Eq. 1 of the returned partition on the input hypergraph */
  int32_t n_parts;      /* parts are numbered 0 .. n_parts-1 */
  int32_t n_levels;     /* hypergraph levels built (1 + contractions) */
  int32_t n_rounds;     /* refinement rounds run, all levels */
  int32_t pad;
  double ms_coarsen;    /* host wall-clock of the coarsening phase */
  double ms_refine;     /* host wall-clock of the refinement phase */
  /* with HGP_FLAG_TIME_KERNELS: summed kernel time, launches and algorithmic
     units per kernel class (HGP_K_*); zero otherwise */
  double ms_kernel[HGP_NKERNEL];
  int64_t n_kernel[HGP_NKERNEL];
  int64_t units_kernel[HGP_NKERNEL];
} hgp_result;

typedef struct hgp_ctx hgp_ctx;

/* Create a context on HIP device `device`.  *ctx receives the handle. */
int hgp_ctx_create(hgp_ctx **ctx, int device);
/* Free a context and all its device scratch.  NULL is ignored. */
void hgp_ctx_destroy(hgp_ctx *ctx);

/* Fill *opt with the defaults: k = 0, max_refine_rounds = 8, seed = 0, plain. */
void hgp_options_default(hgp_options *opt);

/*
 * Partition a hypergraph given in host memory (Sec. II-B multilevel scheme).
 * part_out (host, [n_nodes], caller-owned) receives part ids; res (may be
 * NULL) the connectivity and statistics.  opt may be NULL (defaults).
 * Supported domain: total node weight and total hedge weight each at most
 * 2^31 - 1 (else HGP_EUNSUPPORTED).  The whole call is synchronous.
 */
int hgp_partition(hgp_ctx *ctx, const hgp_hypergraph *g, int32_t omega, int32_t delta, const hgp_options *opt,
                  int32_t *part_out, hgp_result *res);

/*
 * Same as hgp_partition with every array of *g and part_out (device,
 * [n_nodes]) in device memory; work is ordered on `stream`.  The call
 * returns when part_out has been written (the stream is synchronised).
 */
int hgp_partition_device(hgp_ctx *ctx, const hgp_hypergraph *g, int32_t omega, int32_t delta,
                         const hgp_options *opt, void *stream, int32_t *part_out, hgp_result *res);

/*
 * Eq. 1 for a partition vector part (device, [n_nodes], values in [0, n_nodes)) of the
 * device hypergraph *g.  *out (host) receives the connectivity.
 */
int hgp_connectivity_device(hgp_ctx *ctx, const hgp_hypergraph *g, const int32_t *part, void *stream,
                            int64_t *out);

const char *hgp_strerror(int code);
/* Message of the last failure on the calling thread ("" if none). */
const char *hgp_last_error(void);

/* ------------------------------------------------------------------------
 * Level API: the individual steps of the hot path on one hierarchy level,
 * for step-by-step checking.  A level is held in canonical form:
 *   hoff[E+1]    int32 offsets,
 *   hpin[P]      int32, pin id | (1 << 31) if the pin is a destination,
 *                ids strictly ascending within each hedge,
 *   size[n]      int32 node weights (cluster sizes),
 *   hedge_w[E]   int32 hedge weights (the same at every level).
 * All pointers are device pointers; calls are ordered on `stream` and
 * synchronise it before returning host scalars.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t n_nodes;
  int32_t n_hedges;
  const int32_t *hoff;
  const int32_t *hpin;
  const int32_t *size;
  const int32_t *hedge_w;
} hgp_level;

/*
 * Canonical level-0 form of an input hypergraph (Sec. II-C): every hedge's
 * pins sorted by id with the destination flag in bit 31.  hoff_out [E+1] and
 * hpin_out [P] are device buffers.  Validates the input like hgp_partition
 * (HGP_EBADCSR / HGP_EINVAL / HGP_EINFEASIBLE / HGP_EUNSUPPORTED).
 */
int hgp_level_canonical(hgp_ctx *ctx, const hgp_hypergraph *g, int32_t omega, int32_t delta, void *stream,
                        int32_t *hoff_out, int32_t *hpin_out);

/*
 * Candidate selection (Sec. III-A, Eq. 2): for every node n, pair_out[n] =
 * the valid neighbour m maximising (hist(n,m), m), -1 if none, where
 * hist(n,m) = sum of w(e) over hedges of I(n) containing m, and m is valid
 * iff size(n)+size(m) <= Omega and |in(n) u in(m)| <= Delta;
 * score_out[n] = hist(n, pair_out[n]) (0 if none).  [n] int32 / int64.
 */
int hgp_level_rate(hgp_ctx *ctx, const hgp_level *lv, int32_t omega, int32_t delta, void *stream,
                   int32_t *pair_out, int64_t *score_out);

/*
 * Pseudo-forest matching (Sec. III-A/B): match_out[n] (int32 [n]) is the
 * partner of n (n itself if unmatched): 2-cycles of pair match, and a node
 * matches its candidate iff it is the candidate's best proposer by (score,
 * id) and the candidate is not matched upward.  gamma_out[n] is the coarse
 * id (rank of the cluster's smaller member); *n_next (host) the number of
 * clusters.
 */
int hgp_level_match(hgp_ctx *ctx, int32_t n, const int32_t *pair, const int64_t *score, void *stream,
                    int32_t *match_out, int32_t *gamma_out, int32_t *n_next);

/*
 * Coarse hypergraph (Sec. III-B): hedge pins mapped through gamma and
 * deduplicated (a cluster is a destination iff a member is), node sizes
 * summed.  hoff_out [E+1], hpin_out [>= P of the input level], size_out
 * [n_next] are device buffers.
 */
int hgp_level_contract(hgp_ctx *ctx, const hgp_level *lv, const int32_t *gamma, int32_t n_next, void *stream,
                       int32_t *hoff_out, int32_t *hpin_out, int32_t *size_out);

/*
 * One refinement round (Sec. IV) on partition rho (device, [n], values in
 * [0, n_parts)).  Outputs (device buffers):
 *   pdest [n]  proposed part (Eq. 3 best, gain > 0) or -1;  pgain [n] int64
 *   seq   [n]  first |S| entries: moving nodes sorted by (gain, id) desc
 *   gsum  [n+1] int64 G(i) = sum of in-sequence gains of moves 1..i
 *   viol  [n+1] int32 parts violating Omega or Delta after move i
 *   rho_out [n] rho with the best valid prefix applied (if its gain > 0)
 * info (host, int64[4]): |S|, i*, G(i*), applied (0/1).
 */
int hgp_level_refine_round(hgp_ctx *ctx, const hgp_level *lv, const int32_t *rho, int32_t n_parts, int32_t omega,
                           int32_t delta, void *stream, int32_t *pdest, int64_t *pgain, int32_t *seq, int64_t *gsum,
                           int32_t *viol, int32_t *rho_out, int64_t *info);

#ifdef __cplusplus
}
#endif
#endif
