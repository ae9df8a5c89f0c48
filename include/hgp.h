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
#define HGP_EIO (-8)           /* a checkpoint file could not be opened, read or written */
#define HGP_EFORMAT (-9)       /* a checkpoint file is not in the format of hgp_mlp_save (or is corrupt) */

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
#define HGP_LEARNED 1 /* learned merge proposal (hgp_options.mlp) */

/* hgp_options.constraint: which distinct hedges a part's Delta bound counts.
 * The paper's constraint (Sec. II-A) counts inbound hedges (a destination pin
 * in the part); the variants count hedges with a source pin in the part, or
 * with any pin in it.  Every step runs unchanged on the selected pin role. */
#define HGP_INBOUND 0
#define HGP_OUTBOUND 1
#define HGP_INCIDENT 2

/* hgp_options.flags */
#define HGP_FLAG_TIME_KERNELS 1   /* time kernel classes with HIP events on the call's stream */
#define HGP_FLAG_NO_INCREMENTAL 2 /* rate every level and propose every round from scratch (same result) */
#define HGP_FLAG_EXACT_MATCHING 4 /* plain proposal: exact maximum-weight matching of the pairing
                                     pseudo-forest (hgp_level_match_ex, HGP_MATCH_EXACT) instead of
                                     the two traversals of Sec. III-A; changes the result */

/* kernel classes reported in hgp_result.ms_kernel / n_kernel / units_kernel */
#define HGP_K_RATE 0       /* candidate rating + selection; unit: pin-pair visit (sum |e|^2 per level) */
#define HGP_K_PROPOSE 1    /* move proposal; unit: part-table entry visit (sum over e of |e| * lambda(e)) */
#define HGP_K_PARTTABLE 2  /* per-hedge part tables; unit: pin */
#define HGP_K_SEQEVENTS 3  /* in-sequence gains and inbound transitions; unit: algorithmic byte (4 per pin, 16 per event) */
#define HGP_K_CONTRACT 4   /* coarse hedge construction; unit: pin */
#define HGP_K_INCIDENCE 5  /* incidence transpose; unit: pin */
#define HGP_K_SORT 6       /* move / event sorts; unit: key */
#define HGP_K_MATCH 7      /* pseudo-forest matching; unit: node */
#define HGP_K_RATE_TAIL 8  /* late-level rating with top-K lists; unit: pin-pair visit */
#define HGP_K_MLP 9        /* learned proposal: candidate sets, features, network; unit: scored pair */
#define HGP_NKERNEL 10

/*
 * Network of the learned merge proposal (an extension outside the paper's
 * method; HGP_LEARNED).  At each coarsening level the rating of Eq. 2 keeps,
 * per node n, its k best valid candidates by (hist, id) (k <= 8).  The sets
 * are made symmetric, C(n) = topk(n) u {m : n in topk(m)}, every unordered pair
 * {a < b} in them is scored, and pair(n) = the m in C(n) maximising
 * (score, id).  Symmetric sets and scores keep the pairing graph free of
 * cycles longer than two, which the matching of Sec. III-A relies on.
 *
 * Input codes of {a < b} (exact integers f, code = min(255, 8 e + t) with
 * e = floor(log2(f+1)) and t the three bits of f+1 below its leading one):
 *   hist(a,b), c(a,b) = |in(a) n in(b)|, size(a), size(b), |in(a) u in(b)|,
 *   |I(a)|, |I(b)|, level, Omega - size(a) - size(b), Delta - |in(a) u in(b)|,
 *   then six zero inputs.
 * Network, integers throughout (rshift rounds half to even):
 *   a1[j] = clamp(rshift(b1[j] + sum_f x[f] w1[f][j], r1), 0, 255)   j < 64
 *   a2[j] = clamp(rshift(b2[j] + sum_i a1[i] w2[i][j], r2), 0, 255)
 *   score = b3 + sum_j a2[j] w3[j]
 * with |w| <= 255, |b| <= 2^22, 0 <= r <= 30.  Every partial sum stays below
 * 2^24, so the library's BF16 MFMA evaluation with FP32 accumulation is exact.
 * Fallback: the plain pairs (each node's first candidate) are matched too;
 * a level whose learned matching merges fewer than half as many pairs uses
 * the plain matching (counted in hgp_result.n_fallback).
 */
#define HGP_MLP_F 16
#define HGP_MLP_H 64
typedef struct {
  int32_t k;  /* candidates per node, 1..8 */
  int32_t r1, r2;
  int32_t b3;
  int32_t w1[HGP_MLP_F * HGP_MLP_H]; /* [f][j] */
  int32_t b1[HGP_MLP_H];
  int32_t w2[HGP_MLP_H * HGP_MLP_H]; /* [i][j] */
  int32_t b2[HGP_MLP_H];
  int32_t w3[HGP_MLP_H];
} hgp_mlp;

typedef struct {
  int32_t k;                 /* 0: coarsen to ceil(sum w / Omega) clusters (Sec. II-B); k > 0: to k */
  int32_t max_refine_rounds; /* refinement rounds per level (default 8); a level stops early
                                once a round applies no move */
  uint64_t seed;             /* not used by the plain method (its result is seed-independent) */
  int32_t proposal;          /* HGP_PLAIN or HGP_LEARNED */
  int32_t flags;             /* HGP_FLAG_* bits, 0 by default */
  const hgp_mlp *mlp;        /* host memory; required with HGP_LEARNED, read during the call */
  int32_t constraint;        /* HGP_INBOUND (default), HGP_OUTBOUND or HGP_INCIDENT */
  int32_t time_classes;      /* with HGP_FLAG_TIME_KERNELS: bit c set times class c (HGP_K_*) with
                                HIP events and counts its units, 0 does so for every class; each timed
                                launch records two events on the stream and the counting kernels add
                                atomics, so timing fewer classes perturbs the run less */
} hgp_options;

typedef struct {
  int64_t connectivity; /* Eq. 1 of the returned partition on the input hypergraph */
  int32_t n_parts;      /* parts are numbered 0 .. n_parts-1 */
  int32_t n_levels;     /* hypergraph levels built (1 + contractions) */
  int32_t n_rounds;     /* refinement rounds run, all levels */
  int32_t n_fallback;   /* HGP_LEARNED: levels that used the plain matching */
  int32_t n_kept;       /* coarse levels refinement found kept in device memory (the others
                           were rebuilt from level 0; see hgp_set_level_cache) */
  double ms_coarsen;    /* host wall-clock of the coarsening phase */
  double ms_refine;     /* host wall-clock of the refinement phase */
  /* with HGP_FLAG_TIME_KERNELS: summed kernel time, launches and algorithmic
     units per kernel class (HGP_K_*) of the timed classes (time_classes);
     zero otherwise (units counted on the host may appear for every class) */
  double ms_kernel[HGP_NKERNEL];
  int64_t n_kernel[HGP_NKERNEL];
  int64_t units_kernel[HGP_NKERNEL];
} hgp_result;

typedef struct hgp_ctx hgp_ctx;

/* Create a context on HIP device `device`.  *ctx receives the handle. */
int hgp_ctx_create(hgp_ctx **ctx, int device);
/* Free a context and all its device scratch.  NULL is ignored. */
void hgp_ctx_destroy(hgp_ctx *ctx);

/*
 * Device memory the context may keep coarse levels in between coarsening and
 * refinement (Sec. II-B: refinement visits the levels coarsening built, from
 * the coarsest down).  Kept levels (the most recent ones that fit) are read
 * back directly; the others are rebuilt from level 0 by the composed cluster
 * map when refinement reaches them, so the partition does not depend on the
 * budget, only the time does.  bytes = 0 keeps no level; bytes < 0 restores
 * the default (HGP_LEVEL_CACHE_GB in the environment, else 48 GiB).  The
 * memory is one device allocation, made by the next partition that needs it
 * and reused by later ones; it is released here when the budget falls below
 * it, and by hgp_ctx_destroy.  *held (may be NULL) receives the bytes the
 * context holds for it after the call.  Applies to hgp_partition and
 * hgp_partition_device; batch workers share it (see
 * hgp_partition_batch_device).  HGP_EINVAL if ctx is NULL.
 */
int hgp_set_level_cache(hgp_ctx *ctx, int64_t bytes, int64_t *held);

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

/*
 * Eq. 1 for a partition vector in host memory: *g holds host arrays (as for
 * hgp_partition), part (host, [n_nodes]) values in [0, n_nodes).  The arrays
 * are copied to the context's device and the connectivity is computed there
 * by the same kernels as hgp_connectivity_device; *out (host) receives it.
 * Synchronous.  HGP_EBADCSR / HGP_EINVAL as for hgp_partition; a part id
 * outside [0, n_nodes) gives HGP_EBADCSR.
 */
int hgp_connectivity(hgp_ctx *ctx, const hgp_hypergraph *g, const int32_t *part, int64_t *out);

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
 * Matching rules.  HGP_MATCH_TRAVERSAL is hgp_level_match above (Sec. III-A).
 * HGP_MATCH_EXACT is the dynamic-programming formulation Sec. VI names as
 * future work: a maximum-weight matching of the pairing edges {n, pair(n)}
 * (weight score(n)) in each component, by the tree recursion
 *   children(v) = {c : pair(c) = v} without v's 2-cycle partner,
 *   g(v) = sum of f(c) over the children, d(v) = max over the children of
 *   g(c) + score(c) - f(c) (argmax c*(v) by value, then larger id),
 *   f(v) = g(v) + max(0, d(v)); v takes c*(v) when d(v) >= 0 and it is not
 *   matched upward; a 2-cycle {a, b} matches iff
 *   g(a) + g(b) + score(a) >= f(a) + f(b).
 * Scores of nodes with a candidate must lie in [0, 2^31) (HGP_EINVAL).
 * Outputs as hgp_level_match.
 */
#define HGP_MATCH_TRAVERSAL 0
#define HGP_MATCH_EXACT 1
int hgp_level_match_ex(hgp_ctx *ctx, int32_t n, const int32_t *pair, const int64_t *score, int32_t rule,
                       void *stream, int32_t *match_out, int32_t *gamma_out, int32_t *n_next);

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

/*
 * Learned proposal, one level (see hgp_mlp): the candidate sets, their input
 * codes and scores, and the learned and plain pairs of level `level` (the
 * level index enters the features).  mlp is host memory.  Device outputs,
 * capacities as given (cap >= 16 * n_nodes always suffices):
 *   coff [n+1]          offsets of each node's entries (ascending neighbour ids)
 *   cand [cap]          neighbour id of each entry
 *   xq   [cap * 16]     input codes of each entry (may be NULL)
 *   cscore [cap]        network score of each entry (int64)
 *   pair [n], score [n] learned pair (-1: none) and its score (0 if none)
 *   ppair [n]           plain pair: the first candidate by (hist, id)
 * *count (host) receives the number of entries; HGP_EINVAL if it exceeds cap.
 */
int hgp_level_learned(hgp_ctx *ctx, const hgp_level *lv, int32_t level, int32_t omega, int32_t delta,
                      const hgp_mlp *mlp, void *stream, int64_t cap, int64_t *coff, int32_t *cand, int32_t *xq,
                      int64_t *cscore, int32_t *pair, int64_t *score, int32_t *ppair, int64_t *count);

/*
 * The network of hgp_mlp on n rows of 16 input codes (device xq[n*16], each
 * code 0..255; not checked), scores to device score[n].  Stream-ordered.
 */
int hgp_mlp_score_device(hgp_ctx *ctx, const hgp_mlp *mlp, const int32_t *xq, int64_t n, int64_t *score,
                         void *stream);

/*
 * hgp_mlp_score_device for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments and results, but the staged copy of the network
 * and the intermediate int32 scores live in a fixed scratch array of the
 * library instead of context buffers, so the call makes no device allocation.
 * The array holds HGP_NOALLOC_MAX_ROWS rows (about 16 MiB); every device the
 * library runs on keeps its own copy until the process ends.  n above
 * HGP_NOALLOC_MAX_ROWS gives HGP_EUNSUPPORTED (nothing is launched).  All
 * calls on one device share that device's scratch: calls that overlap on a
 * device (other streams or threads) race, and the caller must order them.
 */
#define HGP_NOALLOC_MAX_ROWS (1 << 22)
int hgp_mlp_score_device_noalloc(hgp_ctx *ctx, const hgp_mlp *mlp, const int32_t *xq, int64_t n, int64_t *score,
                                 void *stream);

/* ---------------------------------------------------------------------------
 * Batches of independent hypergraphs
 * ------------------------------------------------------------------------- */

#define HGP_ORDER_LPT 1        /* largest pin count first */
#define HGP_ORDER_INPUT 2      /* the caller's order */
#define HGP_LATE_INCREMENTAL 1 /* incremental late-level rating and proposal carry */
#define HGP_LATE_FULL 2        /* every level and round from scratch */

/* Schedule of a batch; every knob leaves each graph's result unchanged.
 * Zero fields take the context's tuned value (hgp_batch_tune), else the
 * default (4 workers, LPT, 1024, incremental). */
typedef struct {
  int32_t workers;     /* concurrent streams, each with its own workspace: 1..16 */
  int32_t order;       /* HGP_ORDER_* */
  int32_t rate_tile;   /* workgroup size of the rating kernel: 256, 512 or 1024 */
  int32_t late_levels; /* HGP_LATE_* */
} hgp_batch_sched;

/*
 * Partitions n_graphs independent hypergraphs held in device memory
 * (graphs[i] as for hgp_partition_device, with its own omega[i], delta[i]).
 * part_out[i] (device, [graphs[i].n_nodes]) receives graph i's part ids,
 * identical to a single hgp_partition_device call on it.  res (host,
 * [n_graphs]) and t_start_ms / t_end_ms (host, [n_graphs]: ms from the batch
 * start to graph i's start and completion, read from the device's constant-
 * rate wall clock by stamps on the streams that run the graphs) may be NULL.
 * `stream` is synchronised before the batch starts; the call returns when
 * every graph is done.  The first failing graph's error is returned.  Each
 * worker keeps coarse levels in a ring of its own, sized once per batch for
 * the largest graph within an equal share of the context's level budget
 * (hgp_set_level_cache).
 */
int hgp_partition_batch_device(hgp_ctx *ctx, int32_t n_graphs, const hgp_hypergraph *graphs, const int32_t *omega,
                               const int32_t *delta, const hgp_options *opt, const hgp_batch_sched *sched,
                               void *stream, int32_t *const *part_out, hgp_result *res, double *t_start_ms,
                               double *t_end_ms);

/*
 * Autotuner: runs the batch under candidate schedules (coordinate search over
 * workers 1/2/4/8, then order, rating tile and late-level schedule), keeps the
 * fastest in the context for later batches and returns it in *best (and its
 * wall time in *best_ms); both may be NULL.  part_out receives valid results.
 */
int hgp_batch_tune(hgp_ctx *ctx, int32_t n_graphs, const hgp_hypergraph *graphs, const int32_t *omega,
                   const int32_t *delta, const hgp_options *opt, void *stream, int32_t *const *part_out,
                   hgp_batch_sched *best, double *best_ms);

/* ---------------------------------------------------------------------------
 * Training the learned proposal's network (hand-written GPU kernels)
 * ------------------------------------------------------------------------- */

/* Float model with the shape of hgp_mlp: inputs x[f] = code[f] / 8,
 * h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), z = h2 . w3 + b3. */
typedef struct {
  float w1[HGP_MLP_F * HGP_MLP_H]; /* [f][j] */
  float b1[HGP_MLP_H];
  float w2[HGP_MLP_H * HGP_MLP_H]; /* [i][j] */
  float b2[HGP_MLP_H];
  float w3[HGP_MLP_H];
  float b3;
} hgp_mlp_f32;

typedef struct {
  int32_t epochs;  /* passes over the rows */
  int32_t batch;   /* rows per Adam step */
  float lr, beta1, beta2, eps;
  uint64_t seed;   /* shuffle order */
} hgp_train_opts;

/* Seeded initial weights (uniform, scaled by fan-in; unused inputs 10..15 zero). */
void hgp_mlp_init(hgp_mlp_f32 *w, uint64_t seed);

/*
 * Mean binary cross-entropy on logits, (1/n) sum softplus(z) - y z, and its
 * gradient over n device rows: xq [n*16] codes, y [n] labels in {0, 1}.
 * w, grad and loss are host memory.  Synchronous.
 */
int hgp_mlp_grad(hgp_ctx *ctx, const hgp_mlp_f32 *w, const int32_t *xq, const float *y, int64_t n,
                 hgp_mlp_f32 *grad, double *loss, void *stream);

/*
 * Adam on minibatches of the rows in a seeded shuffled order; w (host) holds
 * the initial weights and receives the trained ones; loss_epochs (host,
 * [opt->epochs], may be NULL) the mean loss of each epoch.  Deterministic for
 * a given seed.  Synchronous.
 */
int hgp_mlp_train(hgp_ctx *ctx, hgp_mlp_f32 *w, const int32_t *xq, const float *y, int64_t n,
                  const hgp_train_opts *opt, float *loss_epochs, void *stream);

/*
 * Resumable training.  The state holds everything a run of
 * hgp_mlp_train_state carries from one epoch to the next: the FP32 master
 * weights, Adam's first and second moments, the number of Adam steps taken,
 * the number of epochs completed and the state of the shuffle generator.
 * Training e1 epochs, saving the state (hgp_mlp_save), loading it and
 * training e2 more gives bit-identical weights to e1 + e2 epochs in one run.
 */
typedef struct {
  hgp_mlp_f32 w;  /* master weights */
  hgp_mlp_f32 m;  /* Adam first moments (same layout as the weights) */
  hgp_mlp_f32 v;  /* Adam second moments */
  int64_t step;   /* Adam steps taken (bias corrections use step + 1 next) */
  int64_t epoch;  /* epochs completed */
  uint64_t rng;   /* shuffle generator state */
} hgp_train_state;

/* Fresh state: weights *w, zero moments, step = epoch = 0, the shuffle
 * generator seeded from opt->seed. */
void hgp_train_state_init(hgp_train_state *st, const hgp_mlp_f32 *w, const hgp_train_opts *opt);

/*
 * `epochs` more epochs of hgp_mlp_train from state *st (host memory, updated
 * in place); opt->epochs is ignored and opt->seed only matters through
 * hgp_train_state_init.  loss_epochs (host, [epochs], may be NULL) receives
 * the mean loss of each epoch.  hgp_mlp_train(w, ..., opt) equals
 * hgp_train_state_init followed by this call with opt->epochs.  Synchronous.
 */
int hgp_mlp_train_state(hgp_ctx *ctx, hgp_train_state *st, const int32_t *xq, const float *y, int64_t n,
                        const hgp_train_opts *opt, int32_t epochs, float *loss_epochs, void *stream);

/*
 * Checkpoint file of the learned proposal (host code, no device needed).
 * A versioned little-endian binary file:
 *   header (48 bytes): magic "HGPMLP\0\0", version 1, header size 48,
 *     inputs 16, hidden 64, parameter count 5249, section bits (1: training
 *     state, 2: integer network), score shift, reserved 0, payload bytes;
 *   payload: the training state when bit 1 is set (weights, first and second
 *     moments as 5249 floats each in hgp_mlp_f32 order, step, epoch, rng),
 *     then the integer network of hgp_mlp when bit 2 is set;
 *   trailer: CRC-32 (IEEE 802.3, reflected polynomial 0xEDB88320) of header
 *     and payload.
 * hgp_mlp_save writes the sections whose pointer is non-NULL (at least one);
 * the integer network is checked as for HGP_LEARNED (HGP_EINVAL).
 * hgp_mlp_load reads them back; st / q / score_shift may be NULL to skip a
 * section, and asking for a section the file lacks gives HGP_EFORMAT, as do
 * a wrong magic, version, shape, size or CRC.  File errors give HGP_EIO.
 */
int hgp_mlp_save(const char *path, const hgp_train_state *st, const hgp_mlp *q, int32_t score_shift);
int hgp_mlp_load(const char *path, hgp_train_state *st, hgp_mlp *q, int32_t *score_shift);

/*
 * Integer network from float weights: power-of-two scales per layer chosen
 * from the largest weight and from the largest activations on n host
 * calibration rows xq [n*16].  score ~ z * 2^score_shift.  k: candidates per
 * node (1..8).
 */
int hgp_mlp_quantize(const hgp_mlp_f32 *w, const int32_t *xq, int64_t n, int32_t k, hgp_mlp *out,
                     int32_t *score_shift);

/*
 * Merge traces of the plain method.  hgp_partition_traced runs the plain
 * partitioner (host arrays, like hgp_partition) and records, at every
 * coarsening level, each unordered candidate pair {n < m} of the symmetric
 * 8-best candidate sets (see hgp_mlp) with its 16 input codes; after the run
 * each pair is labelled 1 if the smallest level-0 members of n and of m end
 * in the same part, else 0.  The partition is the plain method's.
 */
typedef struct hgp_trace hgp_trace;
int hgp_trace_create(hgp_trace **t);
void hgp_trace_destroy(hgp_trace *t);
int hgp_partition_traced(hgp_ctx *ctx, const hgp_hypergraph *g, int32_t omega, int32_t delta,
                         const hgp_options *opt, hgp_trace *t, int32_t *part_out, hgp_result *res);
/* Rows recorded (-1 if t is NULL). */
int64_t hgp_trace_rows(const hgp_trace *t);
/* Copies the rows out (host arrays; any may be NULL): xq [rows*16], label
 * [rows], level [rows], node [rows] and cand [rows] (n < m). */
int hgp_trace_read(const hgp_trace *t, int32_t *xq, float *label, int32_t *level, int32_t *node, int32_t *cand);

#ifdef __cplusplus
}
#endif
#endif
