// Learned merge proposal: candidate sets, the fixed-point network on MFMA and
// the selection of pairs (learned.hip).
#pragma once

#include <algorithm>

#include "../../include/hgp.h"
#include "coarsen.hpp"

namespace hgp {

constexpr int kCandK = 8;      // candidates kept per node by the rating
constexpr int kMlpF = HGP_MLP_F;
constexpr int kMlpH = HGP_MLP_H;
constexpr int kMlpNFeat = 10;  // features in use; the other inputs are zero

// Device buffers of one learned level (capacities: N*8 for ck/cc, 16N for the
// directed and deduplicated pair lists).
struct CandBufs {
  uint64_t *ck = nullptr;    // [N*8] hist << 32 | m, descending per node
  int32_t *cc = nullptr;     // [N*8] c(n, m)
  int32_t *ccnt = nullptr;   // [N]
  int32_t *coff32 = nullptr; // [N] exclusive prefix of ccnt
  int32_t *tot32 = nullptr;  // [2] device totals
  uint64_t *key = nullptr, *key2 = nullptr;  // [16N] directed pairs n << idbits | m
  uint32_t *val = nullptr, *val2 = nullptr;  // [16N] slot in ck / cc
  int32_t *flag = nullptr;   // [16N]
  uint64_t *cnm = nullptr;   // [16N] deduplicated pairs
  uint32_t *csrc = nullptr;  // [16N]
  int32_t *cs = nullptr;     // [16N] network score
  int64_t *coff = nullptr;   // [N+1]
  int32_t *pair = nullptr;   // [N] learned pair
  int64_t *score = nullptr;  // [N] matching key score + 2^31
  int32_t *ppair = nullptr;  // [N] plain pair
  int64_t *pscore = nullptr; // [N] its hist
  unsigned long long *best = nullptr;  // [N] selection scratch: best packed (score, id) per node
  int64_t *hbox = nullptr;             // pinned host words for read-backs
  // with device counts (candidate_sets_dev): the number of entries C on the
  // device; the host then knows a bound only
  const int32_t *cdev = nullptr;
};

// Validates a network (HGP_EINVAL / HGP_EUNSUPPORTED) and copies it to buf.
void check_mlp(const hgp_mlp *q);
const int32_t *upload_mlp(DevBuf &buf, const hgp_mlp *q, hipStream_t s);

// Scores n rows of 16 codes (device) with the network params (device copy of hgp_mlp).
void launch_mlp_score_codes(const int32_t *xq, int64_t n, const int32_t *params, int32_t *out, hipStream_t s);

// One learned level: top-8 rating, symmetric sets, scores, learned and plain
// pairs.  Returns the number of candidate entries C (host sync).
int64_t learned_candidates(const LevelView &L, const int32_t *total, int32_t omega, int32_t delta, int level,
                           int keep, const int32_t *params, CandBufs &B, DevBuf &scan_tmp, DevBuf &sort_tmp,
                           hipStream_t s);
// Steps 1-2 only (rating, symmetric sets, offsets); returns C (host sync).
// keep: candidates per node (1..8).
int64_t build_candidates(const LevelView &L, const int32_t *total, int32_t omega, int32_t delta, int keep,
                         CandBufs &B, DevBuf &scan_tmp, DevBuf &sort_tmp, hipStream_t s);
// Symmetric candidate sets, deduplicated pairs and offsets from ck / cc / ccnt
// (the second half of build_candidates); returns the number of pairs.
int64_t candidate_sets(const LevelView &L, CandBufs &B, DevBuf &scan_tmp, DevBuf &sort_tmp, hipStream_t s);
// As candidate_sets without a host round trip: the arrays are built for the
// bound of 2 N keep mirrored entries (keep: the most candidates of a node),
// the exact counts stay on the device (B.cdev), and the bound is returned.
int64_t candidate_sets_dev(const LevelView &L, CandBufs &B, int keep, DevBuf &scan_tmp, DevBuf &sort_tmp,
                           hipStream_t s);
// Steps 3-4 on C entries built by build_candidates (C a bound when B.cdev is set).
void score_and_select(const LevelView &L, int32_t omega, int32_t delta, int level, const int32_t *params,
                      CandBufs &B, int64_t C, hipStream_t s);
// Input codes of the C entries of B ([C*16]).
void launch_cand_codes(const LevelView &L, int32_t omega, int32_t delta, int level, const CandBufs &B, int64_t C,
                       int32_t *xq, hipStream_t s);
void launch_widen_scores(const int32_t *in, int64_t n, int64_t *out, hipStream_t s);
void launch_unkey(const int32_t *pair, const int64_t *key, int32_t n, int64_t *out, hipStream_t s);
// Neighbour ids of the C entries (ascending per node).
void launch_cand_ids(const CandBufs &B, int64_t C, int32_t N, int32_t *ids, hipStream_t s);

// --- training.hip ---
void mlp_init(hgp_mlp_f32 *w, uint64_t seed);
// Mean loss and full-batch gradient on n device rows.
void mlp_grad(const hgp_mlp_f32 *w, const int32_t *xq, const float *y, int64_t n, DevBuf &prm, DevBuf &part,
              DevBuf &grad, DevBuf &lossb, hgp_mlp_f32 *g_out, double *loss_out, hipStream_t s);
// Adam on shuffled minibatches; w (host) in/out; loss_epochs[epochs] (host, optional).
// Fresh training state: weights w, zero moments, shuffle generator from seed.
void train_state_init(hgp_train_state *st, const hgp_mlp_f32 *w, uint64_t seed);
// `epochs` epochs of minibatch Adam continuing from state st (updated).
void mlp_train(hgp_train_state *st, const int32_t *xq, const float *y, int64_t n, const hgp_train_opts &o,
               int32_t epochs, DevBuf &prm, DevBuf &mom, DevBuf &part, DevBuf &perm, DevBuf &lossb,
               float *loss_epochs, hipStream_t s);
// Allocation-free scoring: the per-device scratch address (looked up once per
// device, with that device current) and the scoring on it.
void *noalloc_scratch_init(int device);
void mlp_score_noalloc(void *scratch_dev, const hgp_mlp *q, const int32_t *xq, int64_t n, int64_t *score,
                       hipStream_t s);
// Checkpoint files (checkpoint.hip); throw Error on failure.
void ckpt_save(const char *path, const hgp_train_state *st, const hgp_mlp *q, int32_t score_shift);
void ckpt_load(const char *path, hgp_train_state *st, hgp_mlp *q, int32_t *score_shift);
// Integer network from float weights and host calibration rows.
void mlp_quantize(const hgp_mlp_f32 *w, const int32_t *xq, int64_t n, int32_t k, hgp_mlp *q, int32_t *score_shift);

}  // namespace hgp
