// Incremental late-level rating (internal).
#pragma once

#include "coarsen.hpp"

namespace hgp {

constexpr int kTopK = 8;             // candidates kept per node
constexpr int kTopKMaxWords = 38912; // LDS window of the top-K rating (one or two 32-bit words per id)
constexpr int kTailRatio = 8;        // a matching with M * kTailRatio <= n starts the incremental regime
constexpr int64_t kRowBudget = int64_t(1) << 25;  // new-cluster rows: M * n_next int32 entries

struct TopK {
  uint64_t *key = nullptr;    // [n * kTopK] (hist << 32 | id), descending, 0 = empty
  int32_t *cnt = nullptr;     // [n]
  uint64_t *kappa = nullptr;  // [n] largest hist of a valid candidate left off the list, 0 if none
};

// words_per_id: 1 when every node's counters pack in 32 bits, else 2;
// requires words_per_id * n <= kTopKMaxWords.
void launch_rate_topk(const LevelView &L, const int32_t *total, int32_t omega, int32_t delta, const int32_t *list,
                      const int64_t *count, int64_t grid_nodes, const int32_t *row_slot, int32_t *rows, int32_t *pair,
                      int64_t *score, TopK &tk, int words_per_id, int32_t *err, hipStream_t s);
// As launch_rate_topk for the n_rows (host) nodes of list, with each row's
// pin stream split over many workgroups (acc: scratch of n_rows windows).
// *count must equal n_rows.
void launch_rate_topk_rows(const LevelView &L, const int32_t *total, int32_t omega, int32_t delta,
                           const int32_t *list, const int64_t *count, int32_t n_rows, const int32_t *row_slot,
                           int32_t *rows, int32_t *pair, int64_t *score, TopK &tk, int words_per_id, DevBuf &acc,
                           int32_t *err, hipStream_t s);
// Largest bits(total(n)) + bits(|in(n)|) over the level (device int32, reset inside).
void launch_max_counter_bits(const int32_t *total, const int32_t *indeg, int32_t n, int32_t *out, hipStream_t s);
void launch_rate_update(int32_t n_fine, const int32_t *match, const int32_t *gamma, const TopK &old_tk,
                        int32_t n_new, const int32_t *newc, const int32_t *rows, int32_t n_coarse, TopK &tk,
                        int32_t *pair, int64_t *score, int32_t *rerate, int64_t *rerate_cnt, hipStream_t s);
void launch_new_clusters(const int32_t *match, const int32_t *gamma, int32_t n_fine, int32_t n_coarse,
                         int32_t *flag_tmp, int32_t *newc, int32_t *row_slot, DevBuf &scan_tmp, hipStream_t s);

}  // namespace hgp
