// Host launchers of the coarsening and refinement kernels (internal).
#pragma once

#include "common.hpp"

namespace hgp {

// device error-flag bits
constexpr int32_t kErrCsr = 1;         // offsets not monotone / not starting at 0
constexpr int32_t kErrPin = 2;         // pin id out of range
constexpr int32_t kErrDup = 4;         // duplicate pin within a hedge
constexpr int32_t kErrNsrc = 8;        // n_src outside [0, |e|]
constexpr int32_t kErrWeight = 16;     // weight < 1
constexpr int32_t kErrInfeasible = 32; // node exceeding Omega or Delta on its own
constexpr int32_t kErrBigHedge = 64;   // hedge larger than kHugeCap pins
constexpr int32_t kErrInternal = 128;  // internal consistency check

// Hedges longer than kWaveSegMax pins, handled by workgroup-per-hedge kernels.
constexpr int kWaveSegMax = 1024;
// Hedges of at most kThreadSegMax pins get their part tables from one thread each.
constexpr int kThreadSegMax = 16;
// A level's hedges by length class, lists on the device with device counts:
// list[0 .. *count) with kThreadSegMax < |e| <= kWaveSegMax, and
// big_list[0 .. *big_count) with |e| > kWaveSegMax.  A null list means every
// hedge, filtered by length in the kernel (mid), or the level-0 superset
// BigHedges (big).
struct MidHedges {
  const int32_t *list = nullptr;
  const int32_t *count = nullptr;
  const int32_t *big_list = nullptr;
  const int32_t *big_count = nullptr;
};
struct BigHedges {
  const int32_t *list = nullptr;
  int32_t n = 0;
  int32_t max_len = 0x7fffffff;  // bound of the hedge lengths (coarse hedges only shrink)
  // bound of this level's count of hedges above kWaveSegMax (n at level 0,
  // the finer level's count below it: coarse hedges only shrink); sizes the
  // grids of the long-hedge kernels, which skip the level when it is 0
  int32_t bound = 0x7fffffff;
  // Global scratch of the workgroup kernels for hedges above kSegCap pins
  // (null when the input has none), oversized at each hedge's pin offset b:
  // huge_k[4b .. 4b + 4|e|) 64-bit words, huge_i[2b .. 2b + 2|e|) 32-bit words.
  uint64_t *huge_k = nullptr;
  int32_t *huge_i = nullptr;
};

// One hierarchy level resident on the device.
struct LevelView {
  int32_t n = 0;  // nodes
  int32_t E = 0;  // hedges
  const int32_t *hoff = nullptr;   // [E+1]
  const uint32_t *hpin = nullptr;  // [P] id | dst << 31, ascending ids per hedge
  const int32_t *ioff = nullptr;   // [n+1]
  const uint32_t *inc = nullptr;   // [P] hedge | dst << 31, ascending hedge ids within a node
  const uint32_t *perm = nullptr;  // [P] pin position of incidence k
  const int32_t *size = nullptr;   // [n]
  const int32_t *indeg = nullptr;  // [n]
  const int32_t *total = nullptr;  // [n] sum of w(e) over I(n)
  const int32_t *maxin = nullptr;  // [1] largest indeg of the level (set for the levels coarsening rates)
  const int32_t *hw = nullptr;     // [E]
  BigHedges big;                   // hedges longer than kWaveSegMax (a superset is fine)
  MidHedges mid;                   // this level's hedges for the wave part-table kernel
};

// --- coarsen.hip ---
void launch_check_offsets(const int32_t *off, int32_t E, int32_t *err, hipStream_t s);
void launch_check_weights(const int32_t *hw, int32_t E, const int32_t *nw, int32_t N, int32_t *err,
                          unsigned long long *sums, hipStream_t s);
// huge_keys: 2 P words of scratch when some hedge exceeds kSegCap pins, else null.
void launch_canon(const int32_t *off, const int32_t *pins, const int32_t *nsrc, int32_t E, int32_t N, int32_t role, int32_t *err,
                  uint32_t *hpin, uint32_t *huge_keys, hipStream_t s);
// Incidence I(n) (ascending hedge ids, destination flag in bit 31), the pin
// position perm[k] of every incidence k, |in(n)| and total(n) of a level;
// tkey/tkey2/tval/tval2 are P-element scratch.
void build_incidence(const int32_t *hoff, const uint32_t *hpin, int32_t E, int32_t N, int64_t P, const int32_t *hw,
                     int32_t *ioff, uint32_t *inc, uint32_t *perm, int32_t *indeg, int32_t *total, uint32_t *tkey,
                     uint32_t *tkey2, uint64_t *tval, uint64_t *tval2, DevBuf &sort_tmp, hipStream_t s);
void launch_feasible(const int32_t *size, const int32_t *indeg, int32_t N, int32_t omega, int32_t delta,
                     int32_t *err, hipStream_t s);
// maxin: one device int32 of scratch (max |in(n)| of the level)
// *out = max(0, a[0 .. n)).
void launch_max_i32(const int32_t *a, int32_t n, int32_t *out, hipStream_t s);
void launch_rate(const LevelView &L, const int32_t *total, int32_t omega, int32_t delta, int32_t *pair,
                 int64_t *score, int32_t *maxin, hipStream_t s, int tile = 512);
void launch_match(const int32_t *pair, const int64_t *score, int32_t N, unsigned long long *best, uint8_t *up,
                  int32_t *match, int32_t *gamma, int32_t *rep, int32_t *n_next_dev, int32_t *err,
                  DevBuf &scan_tmp, hipStream_t s);
// Scratch of the exact matching, N elements each.
struct MatchScratch {
  int32_t *nchild = nullptr;
  int32_t *arrived = nullptr;
  unsigned long long *gsum = nullptr;
  unsigned long long *dkey = nullptr;
  int64_t *f = nullptr;
  uint8_t *root = nullptr;
};
// Exact maximum-weight matching over the pairing pseudo-forest (tree
// recursion; outputs as launch_match).  A score outside [0, 2^31) of a node
// with a candidate sets kErrWeight.
void launch_match_exact(const int32_t *pair, const int64_t *score, int32_t N, const MatchScratch &m,
                        unsigned long long *best, uint8_t *up, int32_t *match, int32_t *gamma, int32_t *rep,
                        int32_t *n_next_dev, int32_t *err, DevBuf &scan_tmp, hipStream_t s);
void launch_cluster_size(const int32_t *match, const int32_t *gamma, const int32_t *size, int32_t N, int32_t *csize,
                         hipStream_t s);
// list_buf: 2 (E + 1) ints of scratch.
void launch_contract(const int32_t *hoff, const uint32_t *hpin, int32_t E, const int32_t *map, uint32_t *tmp_pins,
                     int32_t *cnt, int32_t *new_hoff, uint32_t *new_hpin, const BigHedges &big, DevBuf &scan_tmp,
                     int32_t *list_buf, int32_t *err, hipStream_t s);
// --- seg.hip ---
// Part tables of hedges with at most kWaveSegMax pins and inb(p) of their
// entries: pinb[0 .. n_parts) is written (not accumulated).  partial: scratch.
// max_len: an upper bound of the hedge lengths (selects the kernel variant).
// Hedges are list[0 .. *list_n) if list is non-null, else all E (those of at
// most kThreadSegMax pins are skipped: launch_part_table_thread covers them).
void launch_part_table_wave(const int32_t *hoff, const uint32_t *hpin, int32_t E, const int32_t *list,
                            const int32_t *list_n, const int32_t *rho, int32_t *pt, uint32_t *ptc, int32_t *lam,
                            uint8_t *solo, int32_t *pinb, int32_t n_parts, int32_t max_len, DevBuf &partial,
                            hipStream_t s);
// Part tables of the hedges of at most kThreadSegMax pins; inb(p) counts are
// added to pinb.
void launch_part_table_thread(const int32_t *hoff, const uint32_t *hpin, int32_t E, const int32_t *rho, int32_t *pt,
                              uint32_t *ptc, int32_t *lam, uint8_t *solo, int32_t *pinb, int32_t n_parts,
                              hipStream_t s);
// list[0 .. *count) = the hedges with lo < |e| <= hi (default: the wave
// part-table kernel's range kThreadSegMax < |e| <= kWaveSegMax).
void launch_mid_hedges(const int32_t *hoff, int32_t E, int32_t *list, int32_t *count, hipStream_t s,
                       int32_t lo = kThreadSegMax, int32_t hi = kWaveSegMax);
// Coarse pins of every hedge of at most kWaveSegMax pins: short hedges by one
// thread each, the others by one wave each over a list built here in
// list_buf (E + 1 ints, count first; reused by launch_pack_split).
void launch_contract_split(const int32_t *hoff, const uint32_t *hpin, int32_t E, const int32_t *map, uint32_t *out,
                           int32_t *cnt, int32_t *list_buf, hipStream_t s);
void launch_pack_split(const int32_t *old_off, const int32_t *new_off, int32_t E, const uint32_t *src, uint32_t *dst,
                       const int32_t *list_buf, hipStream_t s);
// list[0 .. count[0]) = hedges longer than kWaveSegMax; count[1] = the
// longest hedge's length.
void launch_big_hedges(const int32_t *hoff, int32_t E, int32_t *list, int32_t *count, hipStream_t s);

void launch_check_range(const int32_t *a, int64_t n, int32_t lo, int32_t hi, int32_t *err, hipStream_t s);
void launch_check_level(const int32_t *hoff, const uint32_t *hpin, int32_t E, int32_t n, int32_t *err,
                        hipStream_t s);


// device scalars of a refinement round (RoundBufs::scal)
// (SC_ERR: the error bits, copied there at the end of the round so that they
// are read back with the round's result)
enum { SC_S = 0, SC_EVENTS = 1, SC_ISTAR = 2, SC_GSTAR = 3, SC_INVALID0 = 4, SC_HEAVY = 5, SC_PHEAVY = 6, SC_GMAX = 7,
       SC_ERR = 8, SC_COUNT = 9 };

// (pins, pins_in) of part p in the sorted part table of a hedge: part ids
// pt[b .. b+len), counts ptc (pins | pins_in << 16).
__device__ __forceinline__ int2 pt_lookup(const int32_t *__restrict__ pt, const uint32_t *__restrict__ ptc, int b,
                                          int len, int p) {
  int lo = 0, hi = len;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (pt[b + mid] < p) lo = mid + 1;
    else hi = mid;
  }
  if (lo < len && pt[b + lo] == p) return make_int2((int)(ptc[b + lo] & 0xffffu), (int)(ptc[b + lo] >> 16));
  return make_int2(0, 0);
}

int bits_for(int64_t x);  // smallest b with 2^b > x
// ascending sort of n 64-bit keys over their low `bits` bits
void sort_keys(uint64_t *keys, uint64_t *alt, int64_t n, int bits, DevBuf &sort_tmp, hipStream_t s);
// 32-bit keys by bits [lo, bits) (the small-input path sorts by all bits);
// keys equal on those bits end in any order.
void sort_keys32(uint32_t *keys, uint32_t *alt, int64_t n, int bits, DevBuf &sort_tmp, hipStream_t s, int lo = 0);

// --- refine.hip ---
struct RoundBufs {
  // part table (oversized: one slot per pin, at the hedge's pin offset)
  int32_t *pt = nullptr;       // [P] part ids, ascending per hedge
  uint32_t *ptc = nullptr;     // [P] pins(p,e) | pins_in(p,e) << 16 (both <= kSegCap)
  int32_t *lam = nullptr;      // [E] entries per hedge
  uint8_t *solo = nullptr;     // [P] 1 if the pin is the only pin of its part in its hedge
  int32_t *psize = nullptr;    // [n_parts]
  int32_t *pinb = nullptr;     // [n_parts]
  int32_t *dest = nullptr;     // [n]
  int32_t *gain = nullptr;     // [n]
  int32_t *pos = nullptr;      // [n] 1-based sequence position, 0 if not moving
  int32_t *flag = nullptr;     // [n] scratch
  int32_t *seq = nullptr;      // [n]
  uint64_t *keys = nullptr;    // [cap_events]
  uint64_t *keys2 = nullptr;   // [cap_events]
  int32_t *gp = nullptr;       // [n+1] in-sequence gain per position
  int32_t *vdelta = nullptr;   // [n+1] violation deltas per position
  int64_t *G = nullptr;        // [n+1]
  int32_t *viol = nullptr;     // [n+1]
  int64_t *scal = nullptr;     // [SC_COUNT] device scalars: S, events, istar, Gstar, init_invalid, heavy hedges,
                               // heavy nodes, max gain, error bits
  int32_t *heavy = nullptr;    // [E] hedges queued for the workgroup event kernel
  int64_t *evoff = nullptr;    // [E + 1] inbound-count events per hedge, then their offsets
  int2 *contrib = nullptr;     // [P] per moving pin: in-sequence gain terms (source, destination role)
  int64_t *tile_e = nullptr;   // [cap_tiles] per tile of sorted events: size-sum aggregate
  int32_t *tile_i = nullptr;   // [2 cap_tiles] inbound-sum aggregate, then the part-start flags
  DevBuf *partial = nullptr;   // per-workgroup inb(p) rows of the part-table kernel
  int64_t *hbox = nullptr;     // pinned host words for the round's read-backs
  int64_t cap_events = 0;
  int64_t cap_tiles = 0;
};
constexpr int kEventTile = 2048;  // sorted events per tile of the transition pass

void launch_part_table(const LevelView &L, const int32_t *rho, int32_t n_parts, RoundBufs &B, int32_t *err,
                       hipStream_t s);
// Proposals for every node, or for list[0 .. *count) when list is non-null.
void launch_propose(const LevelView &L, const int32_t *total, const int32_t *rho, int32_t n_parts, int32_t omega,
                    RoundBufs &B, hipStream_t s, const int32_t *list = nullptr, const int64_t *count = nullptr);
// Zeroes the round's device scalars (see k_round_reset); first launch of a
// refinement round.
void launch_round_reset(RoundBufs &B, int32_t E, int64_t *cnt, hipStream_t s);
// *cnt must be zero (launch_round_reset).
void launch_prop_gather(int32_t n, const int32_t *match, const int32_t *gamma, const int32_t *cdest,
                        const int32_t *cgain, RoundBufs &B, int32_t *list, int64_t *cnt, hipStream_t s);
// Builds the sequence; returns |S| (host sync).
int64_t build_sequence(const LevelView &L, RoundBufs &B, DevBuf &scan_tmp, DevBuf &sort_tmp, hipStream_t s);
// In-sequence gains, validity, best prefix; returns (istar, Gstar) and the
// device error bits *err (into *err_bits) in one host sync.
void evaluate_sequence(const LevelView &L, const int32_t *rho, int32_t n_parts, int32_t omega, int32_t delta,
                       int64_t S, RoundBufs &B, int32_t *err, DevBuf &scan_tmp, DevBuf &sort_tmp, hipStream_t s,
                       int64_t *istar, int64_t *gstar, int32_t *err_bits);
void launch_apply(int32_t *rho, RoundBufs &B, int64_t istar, hipStream_t s);
void launch_project(const int32_t *gamma, const int32_t *rho_coarse, int32_t n, int32_t *rho_fine, hipStream_t s);
// Eq. 1 from a part table; result in *conn_dev (device int64).
void launch_connectivity(const LevelView &L, const RoundBufs &B, int64_t *conn_dev, hipStream_t s);
void launch_compact_parts(const int32_t *rho, int32_t n, int32_t n_parts, int32_t *used, int32_t *part_out,
                          int32_t *np_dev, DevBuf &scan_tmp, hipStream_t s);

void launch_cluster_size_sum(const int32_t *gamma, const int32_t *size, int32_t n, int32_t *out, hipStream_t s);
void launch_widen(const int32_t *dest, const int32_t *gain, int32_t n, int32_t *d2, int64_t *g2, hipStream_t s);

}  // namespace hgp
