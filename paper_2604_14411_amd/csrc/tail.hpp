// Incremental rating of levels that merge few pairs (internal).
#pragma once

#include "coarsen.hpp"

namespace hgp {

constexpr int kTopK = 16;            // candidates kept per node (the learned proposal needs up to 8 certain)
constexpr int kTailRatio = 8;        // a matching with M * kTailRatio <= n starts the incremental regime
constexpr int64_t kRowBudget = int64_t(1) << 32;  // new-cluster rows: M * n_next 64-bit entries (32 GB)

struct TopK {
  uint64_t *key = nullptr;    // [n * kTopK] (hist << 32 | id), descending, 0 = empty
  int32_t *c = nullptr;       // [n * kTopK] c(n, id) of each entry
  int32_t *cnt = nullptr;     // [n]
  uint64_t *kappa = nullptr;  // [n] bound of the keys of valid candidates left off the list, 0 if none
};

// Exact top-(TK+1) rating of list[0 .. *count) (every node when list is null);
// grid_nodes: a host bound of the node count (grid size).
void launch_rate_topk(const LevelView &L, const int32_t *total, int32_t omega, int32_t delta, const int32_t *list,
                      const int64_t *count, int64_t grid_nodes, int32_t *pair, int64_t *score, TopK &tk,
                      hipStream_t s);
// Work buffers of the grouped rating: keys, alt, vals, valt, pos, goff of
// `bound` (+1 for goff) entries, the device group count, and the scratch
// windows (group_scratch_words(n) words).
struct GroupBufs {
  uint32_t *keys = nullptr, *alt = nullptr, *vals = nullptr, *valt = nullptr;
  int32_t *pos = nullptr, *goff = nullptr, *groups = nullptr;
  uint32_t *scratch = nullptr;
  DevBuf *tmp = nullptr, *scan_tmp = nullptr;
};
int64_t group_scratch_words(int32_t n);
// The listed nodes (list null: every node; *count of them, count null:
// bound, a host bound of the count) sorted by a hash of their inbound hedge
// sets into G.vals and cut into groups of equal keys (at most kGroupCap
// nodes): G.goff, and their number in *G.groups.
void launch_group_order(const LevelView &L, const int32_t *list, const int64_t *count, int64_t bound,
                        const GroupBufs &G, hipStream_t s);
// As launch_rate_topk over the groups of launch_group_order: groups of equal
// inbound hedge sets share those hedges' histogram (results exactly equal).
// stat (device, may be null) receives the number of groups and of rated nodes.
void launch_rate_topk_grouped(const LevelView &L, const int32_t *total, int32_t omega, int32_t delta,
                              const int64_t *count, int64_t bound, int32_t *pair, int64_t *score, TopK &tk,
                              const GroupBufs &G, int32_t *stat, hipStream_t s);
// As launch_rate_topk for the n_rows (host) nodes of list, with each row's
// pin stream split over many workgroups.  Returns the rows (in acc): row
// row_slot[list[j]] = j holds hist | c << 32 of every valid pair, 0 elsewhere.
// *count must equal n_rows.
uint64_t *launch_rate_topk_rows(const LevelView &L, const int32_t *total, int32_t omega, int32_t delta,
                                const int32_t *list, const int64_t *count, int32_t n_rows, const int32_t *row_slot,
                                int32_t *pair, int64_t *score, TopK &tk, DevBuf &acc, hipStream_t s);
// Carries the lists to the next level; nodes whose first `need` entries are
// not certain go to rerate (need 1: the plain head; k: the learned proposal).
void launch_rate_update(int32_t n_fine, const int32_t *match, const int32_t *gamma, const TopK &old_tk,
                        int32_t n_new, const int32_t *newc, const uint64_t *rows, int32_t n_coarse,
                        const int32_t *csize, const int32_t *cindeg, int32_t omega, int32_t delta, int32_t need,
                        TopK &tk, int32_t *pair, int64_t *score, int32_t *rflag, int32_t *rerate,
                        int64_t *rerate_cnt, DevBuf &scan_tmp, hipStream_t s, int64_t *why = nullptr);
void launch_new_clusters(const int32_t *match, const int32_t *gamma, int32_t n_fine, int32_t n_coarse,
                         int32_t *flag_tmp, int32_t *newc, int32_t *row_slot, DevBuf &scan_tmp, hipStream_t s);
// ck / cc / ccnt of the learned proposal from exact lists (first min(cnt, keep) entries).
void launch_cand_from_lists(int32_t n, int32_t keep, const TopK &tk, uint64_t *ck, int32_t *cc, int32_t *ccnt,
                            hipStream_t s);

}  // namespace hgp
