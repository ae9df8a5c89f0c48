// Host driver of the multilevel scheme (Sec. II-B) and the C-ABI of libhgp.
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <algorithm>
#include <atomic>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>

#include "../../include/hgp.h"
#include "coarsen.hpp"
#include "learned.hpp"
#include "tail.hpp"

namespace hgp {

static thread_local std::string g_last_error;

// HGP_LOG=1 prints one line per level and per refinement round to stderr.
// HGP_LOG_BATCH=1 prints one line per finished graph of a batch and per
// schedule the tuner times.
static bool log_batch_on() {
  static const bool on = [] {
    const char *v = std::getenv("HGP_LOG_BATCH");
    return v && v[0] && v[0] != '0';
  }();
  return on;
}

static bool log_on() {
  static const bool on = [] {
    const char *v = std::getenv("HGP_LOG");
    return v && v[0] && v[0] != '0';
  }();
  return on;
}

// Bytes of coarse levels a context keeps for refinement: HGP_LEVEL_CACHE_GB
// (default 48; 0 disables).  Batch workers keep none.
static int64_t level_cache_default() {
  static const int64_t v = [] {
    const char *e = std::getenv("HGP_LEVEL_CACHE_GB");
    const double gb = e && e[0] ? std::atof(e) : 48.0;
    return (int64_t)(gb > 0 ? gb * (double)(int64_t(1) << 30) : 0.0);
  }();
  return v;
}

// A coarse level kept in HBM between coarsening and refinement (its hedge
// CSR and incidence), so refinement need not rebuild it from level 0.  Its
// arrays lie in one range of the workspace's level ring.
struct CachedLevel {
  int lvl = -1;
  int32_t n = 0;
  int64_t P = 0;
  size_t off = 0, bytes = 0;  // range in the ring
  int32_t *hoff = nullptr, *ioff = nullptr, *indeg = nullptr, *total = nullptr;
  uint32_t *hpin = nullptr, *inc = nullptr, *perm = nullptr;
};

// The kept levels share one device allocation used as a ring: a new level
// goes right after the newest one (back to the start when it would run past
// the end) and evicts the oldest levels it overlaps, so the most recent
// levels within the budget stay.  The allocation is made once and reused by
// every run (it grows between runs when the last run wanted more): a level
// costs a copy of its hedge CSR (its incidence is built in place), never a
// device allocation or free, each of which would synchronise the device.
struct LevelRing {
  DevBuf arena;
  std::deque<CachedLevel> kept;  // oldest first
  size_t head = 0;               // end of the newest level
  int64_t want = 0;              // bytes of every coarse level of the current run
  int64_t want_last = 0;         // ... of the previous run
  int64_t kept_bytes() const {
    int64_t b = 0;
    for (const CachedLevel &c : kept) b += (int64_t)c.bytes;
    return b;
  }
};

struct Workspace {
  DevBuf err, sums, scal2;
  DevBuf hpin0, hoffA, hoffB, hpinA, hpinB, hoffR, hpinR, tmp_pins, cnt;
  DevBuf ioff, inc, indeg, total, work, tkey, tkey2, tval, tval2, perm;
  DevBuf pair, score, best, up, match, rep;
  DevBuf rhoA, rhoB, used, conn;
  DevBuf heavy, evoff, maxin, pt, ptc, lam, solo, psize, pinb, dest, gain, pos, flag, seq, keys, keys2, gp, vdelta, G, viol, scal;
  DevBuf contrib, tile_e, tile_i, pt_partial;
  DevBuf scan_tmp, sort_tmp;
  DevBuf in_off, in_pins, in_nsrc, in_hw, in_nw, in_part;  // staging of host inputs
  DevBuf ones_e, ones_n;
  std::vector<DevBuf> lv_size, lv_gamma, lv_Gamma;
  std::vector<int32_t> lv_n;
  std::vector<int32_t> lv_bigb;  // per level: bound of its long-hedge count (BigHedges::bound)
  KTimer timer;
  DevBuf units_dev;
  HostBox hbox;  // pinned words for read-backs
  // incremental late levels
  DevBuf tkA_key, tkA_c, tkA_cnt, tkA_kap, tkB_key, tkB_c, tkB_cnt, tkB_kap, newc, row_slot, nflag, rerate, dev_cnt;
  DevBuf split, cdest, cgain, maxbits, biglist, midlist, longlist, huge_k, huge_i, tail_acc;
  DevBuf dp_nchild, dp_arrived, dp_g, dp_key, dp_f, dp_root;  // exact matching
  DevBuf gk, gka, gv, gva, gpos, goff, gcnt, gscr;             // grouped ratings
  bool group_on = true;        // grouped ratings still pay in this run
  bool group_pending = false;  // a grouped rating's counts await the next read-back
  // learned proposal
  hgp_trace *trace = nullptr;  // set for the duration of a traced run
  // coarse levels kept for refinement: the most recent, within the budget
  LevelRing ring;
  int64_t lcache_budget = level_cache_default();
  int rate_tile = 1024;        // rating workgroup size (schedule knob; same result)
  DevBuf tr_xq, tr_prm, tr_mom, tr_part, tr_perm, tr_loss, tr_grad;
  DevBuf mlp, ck, cc, ccnt, coff32, ctot, ckey, ckey2, cval, cval2, cflag, cnm, csrc, cs, ccoff, ppair, pscore,
      pmatch, pgam;
  std::vector<DevBuf> lv_match;

  void release_level_cache() {
    ring.kept.clear();
    ring.head = 0;
    ring.arena.release();
  }

  // Per-level buffers (sizes, cluster maps, matches) are kept for the next
  // run: it reuses them level by level, growing only those that are too small
  // (thousands of levels would otherwise cost a hipFree and a hipMalloc each).
  void clear_levels() { lv_n.clear(); }

  void release_levels() {
    for (auto *v : {&lv_size, &lv_gamma, &lv_Gamma, &lv_match}) {
      for (auto &b : *v) b.release();
      v->clear();
    }
    lv_n.clear();
  }

  void release_all() {
    DevBuf *all[] = {&err,  &sums,  &scal2,  &hpin0,  &hoffA,    &hoffB,  &hpinA,  &hpinB,   &hoffR,   &hpinR,
                     &tmp_pins, &cnt, &ioff, &inc,  &indeg,    &total,  &work, &tkey, &tkey2, &tval, &tval2, &perm,   &pair,    &score,   &best,
                     &up,   &match, &rep,    &rhoA,   &rhoB,     &used,   &conn,   &pt,      &ptc,     &lam, &heavy, &evoff, &maxin, &solo,
                     &psize, &pinb, &dest,   &gain,   &pos,      &flag,   &seq,    &keys,    &keys2,   &gp,
                     &vdelta, &contrib, &tile_e, &tile_i, &pt_partial, &G,     &viol,   &scal,     &scan_tmp, &sort_tmp, &in_off, &in_pins,
                     &in_nsrc, &in_hw, &in_nw, &in_part, &ones_e, &ones_n};
    for (DevBuf *b : all) b->release();
    units_dev.release();
    hbox.release();
    release_level_cache();
    DevBuf *inc_bufs[] = {&tkA_key, &tkA_c, &tkA_cnt, &tkA_kap, &tkB_key, &tkB_c, &tkB_cnt, &tkB_kap, &newc, &row_slot,
                          &nflag, &rerate, &dev_cnt, &split, &cdest, &cgain, &maxbits, &biglist, &midlist, &longlist, &huge_k, &huge_i, &dp_nchild, &dp_arrived, &dp_g, &dp_key, &dp_f, &dp_root, &gk, &gka, &gv, &gva, &gpos, &goff, &gcnt, &gscr, &tr_xq, &tr_prm, &tr_mom, &tr_part, &tr_perm, &tr_loss, &tr_grad, &mlp, &ck, &cc, &ccnt, &coff32, &ctot, &ckey, &ckey2, &cval, &cval2, &cflag, &cnm, &csrc, &cs, &ccoff, &ppair, &pscore, &pmatch, &pgam, &tail_acc};
    for (DevBuf *b : inc_bufs) b->release();
    timer.destroy();
    release_levels();
  }
};

}  // namespace hgp


// Merge trace of one plain run (see hgp_partition_traced).
struct hgp_trace {
  std::vector<int32_t> xq, level, node, cand;
  std::vector<float> label;
  std::vector<std::vector<int32_t>> gammas;  // per level, filled during the run
};

struct hgp_ctx {
  int device = 0;
  void *noalloc_scratch = nullptr;  // device address of the scoring scratch on `device`
  hgp::Workspace ws;
  // batch workers: one workspace and one stream each
  std::vector<std::unique_ptr<hgp::Workspace>> pool;
  std::vector<hipStream_t> pool_streams;
  hgp_batch_sched tuned{};  // zero until hgp_batch_tune ran
  hgp::DevBuf batch_stamps;  // device clock at each batch graph's start and end
  ~hgp_ctx() {
    ws.release_all();
    batch_stamps.release();
    for (auto &w : pool) w->release_all();
    for (hipStream_t st : pool_streams) (void)hipStreamDestroy(st);
  }
};

namespace hgp {

template <class T>
static T *need(DevBuf &b, int64_t n) {
  b.reserve((size_t)(n > 0 ? n : 1) * sizeof(T));
  return b.as<T>();
}

static int map_err(int32_t bits, const char **msg) {
  if (bits & (kErrCsr | kErrPin | kErrNsrc)) {
    *msg = (bits & kErrCsr) ? "hedge offsets are not monotone from 0"
                            : (bits & kErrPin) ? "pin id out of range" : "n_src outside [0, |e|]";
    return HGP_EBADCSR;
  }
  if (bits & kErrWeight) {
    *msg = "hedge or node weight below 1";
    return HGP_EINVAL;
  }
  if (bits & kErrDup) {
    *msg = "duplicate pin within a hedge";
    return HGP_EBADCSR;
  }
  if (bits & kErrBigHedge) {
    *msg = "hedge with more than 4096 pins (unsupported)";
    return HGP_EUNSUPPORTED;
  }
  if (bits & kErrInfeasible) {
    *msg = "a node alone exceeds Omega or Delta";
    return HGP_EINFEASIBLE;
  }
  if (bits & kErrInternal) {
    *msg = "internal consistency check failed";
    return HGP_EINTERNAL;
  }
  *msg = "";
  return HGP_OK;
}

static int32_t read_i32(const int32_t *dptr, hipStream_t s) {
  int32_t v = 0;
  HGP_HIP(hipMemcpyAsync(&v, dptr, sizeof v, hipMemcpyDeviceToHost, s));
  HGP_HIP(hipStreamSynchronize(s));
  return v;
}

// As read_i32, through the workspace's pinned words (the per-level reads).
static int32_t read_i32(Workspace &W, const int32_t *dptr, hipStream_t s) {
  int32_t *h = reinterpret_cast<int32_t *>(W.hbox.get());
  HGP_HIP(hipMemcpyAsync(h, dptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HGP_HIP(hipStreamSynchronize(s));
  return h[0];
}

static void raise_err(int32_t bits) {
  const char *msg = "";
  const int rc = map_err(bits, &msg);
  if (rc != HGP_OK) throw Error(rc, msg);
}

static void check_err(Workspace &W, hipStream_t s, int32_t mask = -1) {
  raise_err(read_i32(W, W.err.as<int32_t>(), s) & mask);
}

// The error word buffer (W.err): word 0 holds the error bits, the words after
// it the per-level scalars that are read back with them in one copy.
constexpr int kErrWords = 16;
constexpr int kErrNnext = 4;     // matching: nodes of the next level (learned, plain pairs)
constexpr int kErrContract = 8;  // contraction: pins of the next level, long hedges
constexpr int kErrGroups = 12;   // grouped rating: groups, rated nodes

// err[0 .. n) in one round trip; throws on an error.
static const int32_t *read_err_words(Workspace &W, int n, hipStream_t s) {
  int32_t *v = reinterpret_cast<int32_t *>(W.hbox.get());
  HGP_HIP(hipMemcpyAsync(v, W.err.ptr, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
  HGP_HIP(hipStreamSynchronize(s));
  raise_err(v[0]);
  return v;
}

__global__ void k_pick2(int32_t *__restrict__ dst, const int32_t *__restrict__ a, const int32_t *__restrict__ b) {
  if (threadIdx.x == 0) {
    dst[0] = *a;
    dst[1] = *b;
  }
}

static void check_scalars(const hgp_hypergraph *g, int32_t omega, int32_t delta) {
  if (!g) throw Error(HGP_EINVAL, "hypergraph is NULL");
  if (g->n_nodes < 0 || g->n_hedges < 0) throw Error(HGP_EINVAL, "negative count");
  if (omega < 1 || delta < 0) throw Error(HGP_EINVAL, "Omega < 1 or Delta < 0");
  if (!g->hedge_off) throw Error(HGP_EINVAL, "hedge_off is NULL");
  if (g->n_nodes >= (1 << 30)) throw Error(HGP_EUNSUPPORTED, "more than 2^30 - 1 nodes");
}

// Hedges of `hoff` longer than kWaveSegMax pins (list kept in W.biglist),
// and the global scratch of the workgroup kernels when some hedge is longer
// than kSegCap (sized for the P pins of the level it is found on: coarser
// levels only have fewer).
static BigHedges find_big(Workspace &W, const int32_t *hoff, int32_t E, hipStream_t s, int64_t P = -1) {
  BigHedges b;
  int32_t *list = need<int32_t>(W.biglist, (int64_t)E + 2);
  launch_big_hedges(hoff, E, list + 2, list, s);
  int32_t hdr[2];
  HGP_HIP(hipMemcpyAsync(hdr, list, sizeof hdr, hipMemcpyDeviceToHost, s));
  HGP_HIP(hipStreamSynchronize(s));
  b.n = hdr[0];
  b.max_len = hdr[1];
  b.list = list + 2;
  if (b.max_len > kSegCap) {
    if (P < 0) P = read_i32(hoff + E, s);
    b.huge_k = need<uint64_t>(W.huge_k, 4 * P + 16);
    b.huge_i = need<int32_t>(W.huge_i, 2 * P + 16);
  }
  return b;
}

struct Ingest {
  int64_t P = 0;
  BigHedges big;  // level-0 long hedges (a superset for every coarser level)
  int64_t wsum_nodes = 0;
  const int32_t *hw = nullptr;
  const int32_t *nw = nullptr;
  uint32_t *hpin0 = nullptr;
};

// Validate a device hypergraph (Sec. II-C layout) and build its canonical
// level-0 pins: per hedge, ids ascending with the destination flag in bit 31.
static Ingest ingest(Workspace &W, const hgp_hypergraph *g, int32_t omega, int32_t delta, hipStream_t s,
                     int32_t role = HGP_INBOUND) {
  check_scalars(g, omega, delta);
  Ingest I;
  const int32_t N = g->n_nodes, E = g->n_hedges;
  int32_t *err = need<int32_t>(W.err, kErrWords);
  fill_i32(err, 1, 0, s);
  launch_check_offsets(g->hedge_off, E, err, s);
  const int32_t P32 = read_i32(g->hedge_off + E, s);
  check_err(W, s, kErrCsr | kErrBigHedge);
  I.P = P32;
  if (I.P > 0 && !g->pins) throw Error(HGP_EINVAL, "pins is NULL");
  I.hpin0 = need<uint32_t>(W.hpin0, I.P);
  unsigned long long *sums = need<unsigned long long>(W.sums, 2);
  fill_i64(reinterpret_cast<int64_t *>(sums), 2, 0, s);
  launch_check_weights(g->hedge_w, E, g->node_w, N, err, sums, s);
  I.big = find_big(W, g->hedge_off, E, s, I.P);
  launch_canon(g->hedge_off, g->pins, g->n_src, E, N, role, err, I.hpin0,
               reinterpret_cast<uint32_t *>(I.big.huge_i), s);
  unsigned long long hs[2] = {0, 0};
  HGP_HIP(hipMemcpyAsync(hs, sums, sizeof hs, hipMemcpyDeviceToHost, s));
  check_err(W, s, kErrCsr | kErrPin | kErrNsrc | kErrWeight);
  if (hs[0] > 2147483647ull || hs[1] > 2147483647ull)
    throw Error(HGP_EUNSUPPORTED, "total hedge or node weight exceeds 2^31-1");
  check_err(W, s);
  I.wsum_nodes = (int64_t)hs[1];
  if (g->hedge_w) {
    I.hw = g->hedge_w;
  } else {
    int32_t *o = need<int32_t>(W.ones_e, E);
    fill_i32(o, E, 1, s);
    I.hw = o;
  }
  if (g->node_w) {
    I.nw = g->node_w;
  } else {
    int32_t *o = need<int32_t>(W.ones_n, N);
    fill_i32(o, N, 1, s);
    I.nw = o;
  }
  return I;
}


// Makes v[i] exist (per-level buffers are reused across runs).
static void level_slot(std::vector<DevBuf> &v, size_t i) {
  if (v.size() <= i) v.resize(i + 1);
}

// Scratch of the exact matching for n nodes.
static MatchScratch match_scratch(Workspace &W, int32_t n) {
  MatchScratch m;
  m.nchild = need<int32_t>(W.dp_nchild, n);
  m.arrived = need<int32_t>(W.dp_arrived, n);
  m.gsum = need<unsigned long long>(W.dp_g, n);
  m.dkey = need<unsigned long long>(W.dp_key, n);
  m.f = need<int64_t>(W.dp_f, n);
  m.root = need<uint8_t>(W.dp_root, n);
  return m;
}

// The level's hedges for the wave part-table kernel (list kept in W.midlist,
// count on the device): built once per level, used by every round.
static void set_mid(Workspace &W, LevelView &V, hipStream_t s) {
  int32_t *buf = need<int32_t>(W.midlist, 2 * ((int64_t)V.E + 1));
  int32_t *bbuf = buf + V.E + 1;
  launch_mid_hedges(V.hoff, V.E, buf + 1, buf, s);
  V.mid.list = buf + 1;
  V.mid.count = buf;
  if (V.big.n > 0 && V.big.bound > 0) {
    // the level's own long hedges (the level-0 list is only a superset)
    launch_mid_hedges(V.hoff, V.E, bbuf + 1, bbuf, s, kWaveSegMax, 0x7fffffff);
    V.mid.big_list = bbuf + 1;
    V.mid.big_count = bbuf;
  }
}

// `size_cap` is the element capacity of the buffer behind `size` (checked).
// The level's incidence is built in the workspace, or in the ring range of
// `keep` when the level is kept.
static LevelView make_view(Workspace &W, int32_t n, int32_t E, const int32_t *hoff, const uint32_t *hpin,
                           int64_t P, const int32_t *size, size_t size_cap, const int32_t *hw, const BigHedges &big,
                           hipStream_t s, const CachedLevel *keep = nullptr) {
  if ((size_t)n > size_cap) throw Error(HGP_EINTERNAL, "node-size buffer smaller than the level");
  if (keep && (keep->n != n || keep->P != P)) throw Error(HGP_EINTERNAL, "kept level shape");
  int32_t *ioff = keep ? keep->ioff : need<int32_t>(W.ioff, (int64_t)n + 1);
  uint32_t *inc = keep ? keep->inc : need<uint32_t>(W.inc, P);
  int32_t *indeg = keep ? keep->indeg : need<int32_t>(W.indeg, n);
  int32_t *total = keep ? keep->total : need<int32_t>(W.total, n);
  uint32_t *tkey = need<uint32_t>(W.tkey, P);
  uint32_t *tkey2 = need<uint32_t>(W.tkey2, P);
  uint64_t *tval = need<uint64_t>(W.tval, P);
  uint64_t *tval2 = need<uint64_t>(W.tval2, P);
  uint32_t *perm = keep ? keep->perm : need<uint32_t>(W.perm, P);
  build_incidence(hoff, hpin, E, n, P, hw, ioff, inc, perm, indeg, total, tkey, tkey2, tval, tval2, W.sort_tmp, s);
  add_units(HGP_K_INCIDENCE, P);
  int32_t *maxin = need<int32_t>(W.maxin, 1);  // the ratings' test of whether Delta can bind
  launch_max_i32(indeg, n, maxin, s);
  LevelView L;
  L.n = n;
  L.E = E;
  L.hoff = hoff;
  L.hpin = hpin;
  L.ioff = ioff;
  L.inc = inc;
  L.perm = perm;
  L.size = size;
  L.indeg = indeg;
  L.total = total;
  L.maxin = maxin;
  L.hw = hw;
  L.big = big;
  return L;
}

// Grouped ratings (launch_rate_topk_grouped) for levels of at least
// HGP_GROUP_MIN nodes (default 16384; negative: never), until one of at
// least 4096 rated nodes finds groups of fewer than two nodes on average:
// then the rest of the run rates node by node (the groups of a level only
// ever shrink as clusters merge).
static int64_t group_min() {
  const char *e = std::getenv("HGP_GROUP_MIN");
  return e && e[0] ? std::atoll(e) : 16384;
}

// Re-rating lists are grouped when they hold at least HGP_GROUP_LIST_MIN
// nodes (default 65536; HGP_GROUP_LISTS=1 groups every list): small lists
// have small groups, and on conv302k grouping every list was slower than
// rating them node by node (3.04 against 2.96 s), grouping lists of 65536
// nodes or more faster (2.92 s).
static int64_t group_list_min() {
  const char *a = std::getenv("HGP_GROUP_LISTS");
  if (a && a[0] == '1') return 0;
  const char *e = std::getenv("HGP_GROUP_LIST_MIN");
  return e && e[0] ? std::atoll(e) : 65536;
}

static bool grouping(Workspace &W, int32_t n) {
  const int64_t m = group_min();
  return W.group_on && m >= 0 && n >= m;
}

// Top-K rating of list[0 .. *count) (every node when list is null; bound: a
// host bound of the count), grouped when grouping(W, n).
static void rate_topk(Workspace &W, const LevelView &L, int32_t omega, int32_t delta, const int32_t *list,
                      const int64_t *count, int64_t bound, int32_t *pair, int64_t *score, TopK &tk, hipStream_t s) {
  if (!grouping(W, L.n) || bound <= 0 || (list && bound < group_list_min())) {
    launch_rate_topk(L, L.total, omega, delta, list, count, bound, pair, score, tk, s);
    return;
  }
  if (list) {
    const int64_t lmin = group_list_min();
    if (lmin > 0) {
      // the list's length decides (one read-back)
      HGP_HIP(hipMemcpyAsync(W.hbox.get(), count, sizeof(int64_t), hipMemcpyDeviceToHost, s));
      HGP_HIP(hipStreamSynchronize(s));
      if (*W.hbox.get() < lmin) {
        launch_rate_topk(L, L.total, omega, delta, list, count, bound, pair, score, tk, s);
        return;
      }
    }
  }
  GroupBufs G;
  G.keys = need<uint32_t>(W.gk, bound);
  G.alt = need<uint32_t>(W.gka, bound);
  G.vals = need<uint32_t>(W.gv, bound);
  G.valt = need<uint32_t>(W.gva, bound);
  G.pos = need<int32_t>(W.gpos, bound);
  G.goff = need<int32_t>(W.goff, bound + 1);
  G.groups = need<int32_t>(W.gcnt, 1);
  G.tmp = &W.sort_tmp;
  G.scan_tmp = &W.scan_tmp;
  launch_group_order(L, list, count, bound, G, s);
  if (!list) {
    // a full rating reads the group count first: without groups (random
    // networks) it rates node by node, and the run stops grouping
    int32_t *h = reinterpret_cast<int32_t *>(W.hbox.get());
    HGP_HIP(hipMemcpyAsync(h, G.groups, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HGP_HIP(hipStreamSynchronize(s));
    if (2 * (int64_t)h[0] > bound) {
      W.group_on = false;
      launch_rate_topk(L, L.total, omega, delta, nullptr, nullptr, bound, pair, score, tk, s);
      return;
    }
  }
  G.scratch = need<uint32_t>(W.gscr, group_scratch_words(L.n));  // only once groups pay
  launch_rate_topk_grouped(L, L.total, omega, delta, count, bound, pair, score, tk, G,
                           need<int32_t>(W.err, kErrWords) + kErrGroups, s);
  W.group_pending = true;
}

// After a read-back of the error words: a grouped rating of at least 4096
// nodes with groups of fewer than two nodes on average ends grouping.
static void group_decide(Workspace &W, const int32_t *v) {
  if (!W.group_pending) return;
  W.group_pending = false;
  const int64_t groups = v[kErrGroups], rated = v[kErrGroups + 1];
  if (rated >= 4096 && 2 * groups > rated) W.group_on = false;
}

static RoundBufs round_bufs(Workspace &W, int32_t n, int32_t E, int64_t P, int32_t n_parts) {
  RoundBufs B;
  B.pt = need<int32_t>(W.pt, P);
  B.ptc = need<uint32_t>(W.ptc, P);
  B.lam = need<int32_t>(W.lam, E);
  B.solo = need<uint8_t>(W.solo, P);
  B.psize = need<int32_t>(W.psize, n_parts);
  B.pinb = need<int32_t>(W.pinb, n_parts);
  B.dest = need<int32_t>(W.dest, n);
  B.gain = need<int32_t>(W.gain, n);
  B.pos = need<int32_t>(W.pos, n);
  B.flag = need<int32_t>(W.flag, n);
  B.seq = need<int32_t>(W.seq, n);
  B.cap_events = 2 * P + 2 * (int64_t)n + 16;
  B.keys = need<uint64_t>(W.keys, B.cap_events);
  B.keys2 = need<uint64_t>(W.keys2, B.cap_events);
  B.gp = need<int32_t>(W.gp, (int64_t)n + 1);
  B.vdelta = need<int32_t>(W.vdelta, (int64_t)n + 1);
  B.contrib = need<int2>(W.contrib, P);
  B.cap_tiles = B.cap_events / kEventTile + 1;
  B.tile_e = need<int64_t>(W.tile_e, B.cap_tiles);
  B.tile_i = need<int32_t>(W.tile_i, 2 * B.cap_tiles);
  B.partial = &W.pt_partial;
  B.G = need<int64_t>(W.G, (int64_t)n + 1);
  B.viol = need<int32_t>(W.viol, (int64_t)n + 1);
  B.scal = need<int64_t>(W.scal, SC_COUNT);
  B.heavy = need<int32_t>(W.heavy, E);
  B.evoff = need<int64_t>(W.evoff, (int64_t)E + 1);
  B.hbox = W.hbox.get();
  return B;
}

struct RoundResult {
  int64_t S = 0, istar = -1, gstar = 0;
  bool applied = false;
};

// One refinement round (Sec. IV) on rho, in place.
// Proposals carried from the next coarser level (see k_prop_gather).
struct Carry {
  const int32_t *match = nullptr;  // level match (n)
  const int32_t *gamma = nullptr;  // level cluster map (n)
};

static RoundResult refine_round(Workspace &W, const LevelView &L, int64_t P, int32_t *rho, int32_t n_parts,
                                int32_t omega, int32_t delta, hipStream_t s, RoundBufs *out_bufs = nullptr,
                                const Carry *carry = nullptr) {
  RoundBufs B = round_bufs(W, L.n, L.E, P, n_parts);
  int32_t *err = W.err.as<int32_t>();
  int64_t *cnt = carry ? need<int64_t>(W.dev_cnt, 4) : nullptr;
  launch_round_reset(B, L.E, cnt, s);
  launch_part_table(L, rho, n_parts, B, err, s);
  add_units(HGP_K_PARTTABLE, P);
  if (carry) {
    int32_t *list = need<int32_t>(W.split, L.n);
    launch_prop_gather(L.n, carry->match, carry->gamma, W.cdest.as<int32_t>(), W.cgain.as<int32_t>(), B, list, cnt,
                       s);
    launch_propose(L, L.total, rho, n_parts, omega, B, s, list, cnt);
  } else {
    launch_propose(L, L.total, rho, n_parts, omega, B, s);
  }
  RoundResult R;
  R.S = build_sequence(L, B, W.scan_tmp, W.sort_tmp, s);
  if (R.S > 0) add_units(HGP_K_SEQEVENTS, 4 * P);  // 4 B per pin scanned (+16 B per event, counted with the events)
  int32_t err_bits = 0;
  evaluate_sequence(L, rho, n_parts, omega, delta, R.S, B, err, W.scan_tmp, W.sort_tmp, s, &R.istar, &R.gstar,
                    &err_bits);
  raise_err(err_bits);
  if (R.istar >= 0 && R.gstar > 0) {
    launch_apply(rho, B, R.istar, s);
    R.applied = true;
  }
  if (out_bufs) *out_bufs = B;
  return R;
}

struct RunStats {
  int64_t conn = 0;
  int32_t n_parts = 0, n_levels = 0, n_rounds = 0, n_fallback = 0, n_kept = 0;
  double ms_coarsen = 0, ms_refine = 0;
  double ms_kernel[HGP_NKERNEL] = {};
  int64_t n_kernel[HGP_NKERNEL] = {};
  int64_t units_kernel[HGP_NKERNEL] = {};
};

// Installs the context's kernel timer for the duration of one call.
struct TimerGuard {
  Workspace &W;
  TimerGuard(Workspace &w, bool on, hipStream_t s, int32_t classes = 0) : W(w) {
    W.timer.reset();
    W.timer.on = on;
    W.timer.mask = classes ? (uint32_t)classes : ~0u;
    g_ktimer = &W.timer;
    if (on) {
      W.units_dev.reserve(HGP_NKERNEL * sizeof(int64_t));
      fill_i64(W.units_dev.as<int64_t>(), HGP_NKERNEL, 0, s);
      W.timer.units_dev = W.units_dev.as<unsigned long long>();
    } else {
      W.timer.units_dev = nullptr;
    }
  }
  void collect(RunStats &st, hipStream_t s) {
    if (!W.timer.on) return;
    HGP_HIP(hipStreamSynchronize(s));
    W.timer.resolve(st.ms_kernel, st.n_kernel);
    int64_t dev[HGP_NKERNEL];
    HGP_HIP(hipMemcpy(dev, W.units_dev.ptr, sizeof dev, hipMemcpyDeviceToHost));
    for (int c = 0; c < HGP_NKERNEL; ++c) st.units_kernel[c] = W.timer.units[c] + dev[c];
  }
  ~TimerGuard() {
    W.timer.on = false;
    g_ktimer = nullptr;
  }
};

// Learned-level buffers for n nodes; pair/score are the caller's arrays.
static CandBufs cand_bufs(Workspace &W, int32_t n, int32_t *pair, int64_t *score) {
  CandBufs B;
  const int64_t nk = (int64_t)n * kCandK, m = 2 * nk;
  B.ck = need<uint64_t>(W.ck, nk);
  B.cc = need<int32_t>(W.cc, nk);
  B.ccnt = need<int32_t>(W.ccnt, n);
  B.coff32 = need<int32_t>(W.coff32, n);
  B.tot32 = need<int32_t>(W.ctot, 4);
  B.key = need<uint64_t>(W.ckey, m);
  B.key2 = need<uint64_t>(W.ckey2, m);
  B.val = need<uint32_t>(W.cval, m);
  B.val2 = need<uint32_t>(W.cval2, m);
  B.flag = need<int32_t>(W.cflag, m);
  B.cnm = need<uint64_t>(W.cnm, m);
  B.csrc = need<uint32_t>(W.csrc, m);
  B.cs = need<int32_t>(W.cs, m);
  B.coff = need<int64_t>(W.ccoff, (int64_t)n + 1);
  B.pair = pair;
  B.score = score;
  B.ppair = need<int32_t>(W.ppair, n);
  B.pscore = need<int64_t>(W.pscore, n);
  B.best = need<unsigned long long>(W.best, n);  // the matching refills it
  B.hbox = W.hbox.get();
  return B;
}

// Records the unordered candidate pairs {n < m} of level `lvl` and their codes.
static void trace_level(Workspace &W, const LevelView &L, int lvl, int32_t omega, int32_t delta, int32_t *pair,
                        int64_t *score, hipStream_t s) {
  const int32_t n = L.n;
  if (n <= 0) return;
  CandBufs CB = cand_bufs(W, n, pair, score);
  const int64_t C = build_candidates(L, L.total, omega, delta, kCandK, CB, W.scan_tmp, W.sort_tmp, s);
  if (C <= 0) return;
  int32_t *xq = need<int32_t>(W.tr_xq, C * kMlpF);
  launch_cand_codes(L, omega, delta, lvl, CB, C, xq, s);
  std::vector<uint64_t> nm((size_t)C);
  std::vector<int32_t> codes((size_t)C * kMlpF);
  HGP_HIP(hipMemcpyAsync(nm.data(), CB.cnm, sizeof(uint64_t) * (size_t)C, hipMemcpyDeviceToHost, s));
  HGP_HIP(hipMemcpyAsync(codes.data(), xq, sizeof(int32_t) * (size_t)C * kMlpF, hipMemcpyDeviceToHost, s));
  HGP_HIP(hipStreamSynchronize(s));
  const int idbits = std::max(1, bits_for(n - 1));
  const uint64_t mask = (1ull << idbits) - 1ull;
  hgp_trace &T = *W.trace;
  for (int64_t i = 0; i < C; ++i) {
    const int32_t a = (int32_t)(nm[(size_t)i] >> idbits), b = (int32_t)(nm[(size_t)i] & mask);
    if (a >= b) continue;
    T.node.push_back(a);
    T.cand.push_back(b);
    T.level.push_back(lvl);
    T.xq.insert(T.xq.end(), codes.begin() + i * kMlpF, codes.begin() + (i + 1) * kMlpF);
  }
}

// Labels of the recorded pairs from the cluster maps and the final parts.
static void trace_label(hgp_trace &T, int32_t N, const int32_t *part) {
  std::vector<std::vector<int32_t>> rep(1);
  rep[0].resize((size_t)N);
  for (int32_t v = 0; v < N; ++v) rep[0][(size_t)v] = v;
  int maxl = 0;
  for (int32_t l : T.level) maxl = std::max(maxl, l);
  for (int l = 0; l < maxl; ++l) {
    const std::vector<int32_t> &g = T.gammas.at((size_t)l);
    int32_t nn = 0;
    for (int32_t c : g) nn = std::max(nn, c + 1);
    std::vector<int32_t> r((size_t)nn, INT32_MAX);
    for (size_t v = 0; v < g.size(); ++v) r[(size_t)g[v]] = std::min(r[(size_t)g[v]], rep[(size_t)l][v]);
    rep.push_back(std::move(r));
  }
  T.label.resize(T.node.size());
  for (size_t i = 0; i < T.node.size(); ++i) {
    const std::vector<int32_t> &r = rep[(size_t)T.level[i]];
    T.label[i] = part[r[(size_t)T.node[i]]] == part[r[(size_t)T.cand[i]]] ? 1.0f : 0.0f;
  }
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Ring size of a batch worker in level-0 sizes: the coarse levels of the
// random networks add up to about 35 times level 0 (their hedges barely
// shrink), those of the layered ones to about 7 times.
constexpr int64_t kBatchRingLevels = 40;

// Ring bytes of a level with n nodes, E hedges and P pins: hoff, hpin, ioff,
// inc, perm, indeg and total, each starting on a 256-byte boundary.
static size_t level_bytes(int32_t n, int32_t E, int64_t P) {
  const size_t pb = align256(4 * (size_t)P), nb = align256(4 * ((size_t)n + 1));
  return align256(4 * ((size_t)E + 1)) + 3 * pb + 3 * nb;
}

// Starts a run's level cache: the ring is emptied and, if the previous run
// wanted more than it holds (or, on a first run, 32 times level 0's size),
// reallocated at up to the budget (halving on failure).
static void ring_begin(Workspace &W, int32_t N, int32_t E, int64_t P) {
  LevelRing &R = W.ring;
  if (R.want > 0) R.want_last = R.want;
  R.kept.clear();
  R.head = 0;
  R.want = 0;
  const int64_t budget = std::max<int64_t>(W.lcache_budget, 0);
  int64_t desired = std::min<int64_t>(budget, std::max<int64_t>(R.want_last, 32 * (int64_t)level_bytes(N, E, P)));
  desired &= ~int64_t(255);  // within the budget
  if ((int64_t)R.arena.bytes > budget) R.arena.release();
  if ((int64_t)R.arena.bytes >= desired) return;
  R.arena.release();
  while (desired >= (int64_t(1) << 20)) {
    try {
      R.arena.reserve((size_t)desired);
      return;
    } catch (const Error &e) {
      if (e.code != HGP_ENOMEM) throw;
      desired = (desired / 2) & ~int64_t(255);
    }
  }
}

// Places level `lvl` (n nodes, E hedges, P pins) in the ring, evicting the
// oldest kept levels in its way; nullptr (nothing evicted) if the level is
// larger than the ring.  Coarsening reads a level's incidence only until the
// next level's is built, so the level just before may be evicted too.
static const CachedLevel *ring_place(Workspace &W, int lvl, int32_t n, int32_t E, int64_t P) {
  LevelRing &R = W.ring;
  const size_t b = level_bytes(n, E, P);
  R.want += (int64_t)b;
  if (b > R.arena.bytes) return nullptr;
  size_t off = R.head;
  if (off + b > R.arena.bytes) {
    // wrap: the levels between the head and the end are the oldest
    while (!R.kept.empty() && R.kept.front().off >= R.head) R.kept.pop_front();
    off = 0;
  }
  while (!R.kept.empty() && R.kept.front().off < off + b && R.kept.front().off + R.kept.front().bytes > off)
    R.kept.pop_front();
  CachedLevel c;
  c.lvl = lvl;
  c.n = n;
  c.P = P;
  c.off = off;
  c.bytes = b;
  char *p = R.arena.as<char>() + off;
  const size_t pb = align256(4 * (size_t)P), nb = align256(4 * ((size_t)n + 1));
  c.hoff = reinterpret_cast<int32_t *>(p);
  p += align256(4 * ((size_t)E + 1));
  c.hpin = reinterpret_cast<uint32_t *>(p);
  c.inc = reinterpret_cast<uint32_t *>(p + pb);
  c.perm = reinterpret_cast<uint32_t *>(p + 2 * pb);
  p += 3 * pb;
  c.ioff = reinterpret_cast<int32_t *>(p);
  c.indeg = reinterpret_cast<int32_t *>(p + nb);
  c.total = reinterpret_cast<int32_t *>(p + 2 * nb);
  R.head = off + b;
  R.kept.push_back(c);
  return &R.kept.back();
}

static const CachedLevel *cached_level(const Workspace &W, int lvl) {
  for (const CachedLevel &c : W.ring.kept)
    if (c.lvl == lvl) return &c;
  return nullptr;
}

static double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// The multilevel scheme of Sec. II-B on a device hypergraph.  Coarsening
// (Sec. III) repeats rate, match and contract until a matching leaves at most
// T clusters (T = k, or ceil(sum w / Omega)) or matches nothing; those
// clusters (or the nodes) are the initial parts.  Refinement (Sec. IV) then
// runs from the coarsest level down, projecting through the cluster maps.
// Coarse levels are not kept: level l is rebuilt from level 0 by the composed
// cluster map when refinement reaches it.
static RunStats run_partition(Workspace &W, const hgp_hypergraph *g, int32_t omega, int32_t delta,
                              const hgp_options &opt, hipStream_t s, int32_t *part_out) {
  RunStats st;
  const int64_t allocs0 = g_dev_allocs.load(), frees0 = g_dev_frees.load();
  struct AllocLog {
    int64_t a0, f0;
    ~AllocLog() {
      if (log_on())
        fprintf(stderr, "[hgp] partition: %lld device allocations, %lld frees\n",
                (long long)(g_dev_allocs.load() - a0), (long long)(g_dev_frees.load() - f0));
    }
  } alloc_log{allocs0, frees0};
  if (opt.k < 0 || opt.max_refine_rounds < 0) throw Error(HGP_EINVAL, "k < 0 or max_refine_rounds < 0");
  if (opt.proposal != HGP_PLAIN && opt.proposal != HGP_LEARNED) throw Error(HGP_EINVAL, "unknown proposal");
  const bool learned = opt.proposal == HGP_LEARNED;
  if (learned) check_mlp(opt.mlp);
  const bool exact = (opt.flags & HGP_FLAG_EXACT_MATCHING) != 0;
  if (exact && learned) throw Error(HGP_EINVAL, "exact matching applies to the plain proposal");
  const double t0 = now_ms();
  if (opt.constraint != HGP_INBOUND && opt.constraint != HGP_OUTBOUND && opt.constraint != HGP_INCIDENT)
    throw Error(HGP_EINVAL, "unknown constraint");
  Ingest I = ingest(W, g, omega, delta, s, opt.constraint);
  const int32_t N = g->n_nodes, E = g->n_hedges;
  const int64_t P = I.P;
  const int32_t *hoff0 = g->hedge_off;
  const uint32_t *hpin0 = I.hpin0;
  const int32_t *hw = I.hw;
  const int32_t *mlp_params = learned ? upload_mlp(W.mlp, opt.mlp, s) : nullptr;
  W.clear_levels();
  W.group_on = true;
  W.group_pending = false;
  level_slot(W.lv_size, 0);
  W.lv_n.push_back(N);
  int32_t *size0 = need<int32_t>(W.lv_size[0], N);
  if (N > 0)
    HGP_HIP(hipMemcpyAsync(size0, I.nw, sizeof(int32_t) * (size_t)N, hipMemcpyDeviceToDevice, s));
  BigHedges big = I.big;  // coarse hedges only shrink: valid for every level
  big.bound = big.n;
  W.lv_bigb.assign(1, big.bound);
  LevelView L = make_view(W, N, E, hoff0, hpin0, P, size0, W.lv_size[0].bytes / 4, hw, big, s);
  launch_feasible(size0, L.indeg, N, omega, delta, W.err.as<int32_t>(), s);
  check_err(W, s);
  st.n_levels = 1;
  if (N == 0) {
    // the single (empty) level still runs one refinement round that finds no move
    st.n_rounds = opt.max_refine_rounds > 0 ? 1 : 0;
    return st;
  }
  const int64_t T = opt.k > 0 ? (int64_t)opt.k : (I.wsum_nodes + omega - 1) / omega;

  int32_t *pair = need<int32_t>(W.pair, N);
  int64_t *score = need<int64_t>(W.score, N);
  unsigned long long *best = need<unsigned long long>(W.best, N);
  uint8_t *up = need<uint8_t>(W.up, N);
  int32_t *match = need<int32_t>(W.match, N);
  int32_t *rep = need<int32_t>(W.rep, N);
  int32_t *nnext_dev = need<int32_t>(W.err, kErrWords) + kErrNnext;
  int32_t *rho = need<int32_t>(W.rhoA, N);
  int32_t *rho2 = need<int32_t>(W.rhoB, N);
  need<int32_t>(W.hoffA, (int64_t)E + 1);
  need<int32_t>(W.hoffB, (int64_t)E + 1);
  need<uint32_t>(W.hpinA, P);
  need<uint32_t>(W.hpinB, P);
  need<uint32_t>(W.tmp_pins, P);
  need<int32_t>(W.cnt, E);
  // after the level-0 buffers, which the ring must not crowd out
  ring_begin(W, N, E, P);

  // ---- coarsening ----
  // Late levels that merge few pairs are rated incrementally (tail.hip):
  // lists of the exact top candidates per node are carried between levels,
  // new clusters are rated in full and offered to their neighbours.
  const bool incremental = (opt.flags & HGP_FLAG_NO_INCREMENTAL) == 0;
  int32_t n_parts = 0;
  int lvl = 0;
  const int32_t *cur_hoff = hoff0;
  const uint32_t *cur_hpin = hpin0;
  int64_t cur_P = P;
  int ping = 0;
  TopK tk_cur, tk_nxt;
  tk_cur.key = need<uint64_t>(W.tkA_key, (int64_t)N * kTopK);
  tk_cur.c = need<int32_t>(W.tkA_c, (int64_t)N * kTopK);
  tk_cur.cnt = need<int32_t>(W.tkA_cnt, N);
  tk_cur.kappa = need<uint64_t>(W.tkA_kap, N);
  tk_nxt.key = need<uint64_t>(W.tkB_key, (int64_t)N * kTopK);
  tk_nxt.c = need<int32_t>(W.tkB_c, (int64_t)N * kTopK);
  tk_nxt.cnt = need<int32_t>(W.tkB_cnt, N);
  tk_nxt.kappa = need<uint64_t>(W.tkB_kap, N);
  int32_t *newc = need<int32_t>(W.newc, N);
  int32_t *row_slot = need<int32_t>(W.row_slot, N);
  int32_t *nflag = need<int32_t>(W.nflag, N);
  int32_t *rerate = need<int32_t>(W.rerate, N);
  int64_t *dcnt = need<int64_t>(W.dev_cnt, 8);  // [4..7]: re-rating diagnostics (HGP_LOG)
  bool have_pairs = false;  // pair/score of the current level already computed
  bool lists_ok = false;    // tk_cur holds exact lists for the current level
  bool lists_fresh = false; // ... carried to it incrementally (learned: first k entries certain)
  bool tail = false;        // the previous matching merged few pairs
  const char *path = "plain";
  while (true) {
    const int32_t n = L.n;
    if (!have_pairs) {
      path = "plain";
      if (learned) {
        path = "learned";
        CandBufs CB = cand_bufs(W, n, pair, score);
        if (lists_fresh || incremental) {
          // candidate lists from the top-K lists (rated in full here unless
          // carried from the previous level); every level keeps lists so
          // that the next one can be rated incrementally (on the layered
          // networks the top-K rating is also faster than the candidate
          // rating of k_rate_cand: conv302k 3.65 to 3.27 s per partition)
          if (!lists_fresh) {
            path = "learned, topk";
            rate_topk(W, L, omega, delta, nullptr, nullptr, n, pair, score, tk_cur, s);
            lists_ok = true;
          } else {
            path = "learned, incremental";
          }
          {
            KScope ks(HGP_K_RATE, s);
            launch_cand_from_lists(n, opt.mlp->k, tk_cur, CB.ck, CB.cc, CB.ccnt, s);
          }
          const int64_t Cb = candidate_sets_dev(L, CB, opt.mlp->k, W.scan_tmp, W.sort_tmp, s);
          score_and_select(L, omega, delta, lvl, mlp_params, CB, Cb, s);
        } else {
          learned_candidates(L, L.total, omega, delta, lvl, opt.mlp->k, mlp_params, CB, W.scan_tmp,
                             W.sort_tmp, s);
          lists_ok = false;
        }
        lists_fresh = false;
      } else if (incremental && tail) {
        path = "topk";
        rate_topk(W, L, omega, delta, nullptr, nullptr, n, pair, score, tk_cur, s);
        lists_ok = true;
      } else {
        launch_rate(L, L.total, omega, delta, pair, score, need<int32_t>(W.maxin, 1), s,
                    W.rate_tile);
        lists_ok = false;
      }
    }
    have_pairs = false;
    if (W.trace) trace_level(W, L, lvl, omega, delta, pair, score, s);
    level_slot(W.lv_gamma, (size_t)lvl);
    level_slot(W.lv_match, (size_t)lvl);
    int32_t *gam = need<int32_t>(W.lv_gamma[lvl], n);
    int32_t *lmatch = need<int32_t>(W.lv_match[lvl], n);
    if (exact)
      launch_match_exact(pair, score, n, match_scratch(W, n), best, up, lmatch, gam, rep, nnext_dev,
                         W.err.as<int32_t>(), W.scan_tmp, s);
    else
      launch_match(pair, score, n, best, up, lmatch, gam, rep, nnext_dev, W.err.as<int32_t>(), W.scan_tmp, s);
    int32_t n_next = 0;
    if (!learned) {
      const int32_t *v = read_err_words(W, kErrWords, s);
      group_decide(W, v);
      n_next = v[kErrNnext];
    } else {
      // fallback: the plain pairs' matching, used if it merges over twice as
      // many pairs (both counts read back together)
      int32_t *pm = need<int32_t>(W.pmatch, n);
      int32_t *pg = need<int32_t>(W.pgam, n);
      launch_match(W.ppair.as<int32_t>(), W.pscore.as<int64_t>(), n, best, up, pm, pg, rep, nnext_dev + 1,
                   W.err.as<int32_t>(), W.scan_tmp, s);
      const int32_t *v = read_err_words(W, kErrWords, s);
      group_decide(W, v);
      n_next = v[kErrNnext];
      const int32_t n_next_p = v[kErrNnext + 1];
      if (2 * (int64_t)(n - n_next) < (int64_t)(n - n_next_p)) {
        HGP_HIP(hipMemcpyAsync(lmatch, pm, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
        HGP_HIP(hipMemcpyAsync(gam, pg, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
        n_next = n_next_p;
        ++st.n_fallback;
        path = "learned, plain fallback";
      }
    }
    if (W.trace) {
      W.trace->gammas.emplace_back((size_t)n);
      HGP_HIP(hipMemcpyAsync(W.trace->gammas.back().data(), gam, sizeof(int32_t) * (size_t)n,
                             hipMemcpyDeviceToHost, s));
      HGP_HIP(hipStreamSynchronize(s));
    }
    if (log_on())
      fprintf(stderr, "[hgp] level %d n=%d pins=%lld merged=%d rating=%s at %.1f ms\n", lvl, n, (long long)cur_P,
              n - n_next, path, now_ms());
    if (n_next == n) {
      iota_i32(rho, n, s);
      n_parts = n;
      break;
    }
    if ((int64_t)n_next <= T) {
      HGP_HIP(hipMemcpyAsync(rho, gam, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
      n_parts = n_next;
      break;
    }
    const int32_t M = n - n_next;
    level_slot(W.lv_size, (size_t)lvl + 1);
    W.lv_n.push_back(n_next);
    int32_t *csize = need<int32_t>(W.lv_size[lvl + 1], n_next);
    launch_cluster_size(lmatch, gam, W.lv_size[lvl].as<int32_t>(), n, csize, s);
    level_slot(W.lv_Gamma, (size_t)lvl);  // lv_Gamma[k]: level 0 -> level k+1
    int32_t *Gm = need<int32_t>(W.lv_Gamma[lvl], N);
    if (lvl == 0)
      HGP_HIP(hipMemcpyAsync(Gm, gam, sizeof(int32_t) * (size_t)N, hipMemcpyDeviceToDevice, s));
    else
      launch_project(W.lv_Gamma[lvl - 1].as<int32_t>(), gam, N, Gm, s);
    // the contracted level (at most cur_P pins) goes to the other ping-pong pair
    DevBuf &hoff_buf = ping ? W.hoffB : W.hoffA;
    DevBuf &hpin_buf = ping ? W.hpinB : W.hpinA;
    int32_t *nh = need<int32_t>(hoff_buf, (int64_t)E + 1);
    uint32_t *npin = need<uint32_t>(hpin_buf, cur_P);
    int32_t *longlist = need<int32_t>(W.longlist, 2 * ((int64_t)E + 1));
    launch_contract(cur_hoff, cur_hpin, E, gam, W.tmp_pins.as<uint32_t>(), W.cnt.as<int32_t>(), nh, npin, big,
                    W.scan_tmp, longlist, W.err.as<int32_t>(), s);
    add_units(HGP_K_CONTRACT, cur_P);
    {
      // the contracted pin count, and this level's count of long hedges:
      // a bound for the next level's
      k_pick2<<<1, 64, 0, s>>>(W.err.as<int32_t>() + kErrContract, nh + E, longlist + E + 1);
      HGP_LAUNCH_CHECK();
      const int32_t *h = read_err_words(W, kErrContract + 2, s) + kErrContract;
      cur_P = h[0];
      big.bound = std::min(big.bound, h[1]);
    }
    W.lv_bigb.push_back(big.bound);
    cur_hoff = nh;
    cur_hpin = npin;
    ping ^= 1;
    ++lvl;
    const CachedLevel *keep = ring_place(W, lvl, n_next, E, cur_P);
    if (keep) {
      HGP_HIP(hipMemcpyAsync(keep->hoff, cur_hoff, 4 * ((size_t)E + 1), hipMemcpyDeviceToDevice, s));
      if (cur_P > 0)
        HGP_HIP(hipMemcpyAsync(keep->hpin, cur_hpin, 4 * (size_t)cur_P, hipMemcpyDeviceToDevice, s));
    }
    L = make_view(W, n_next, E, cur_hoff, cur_hpin, cur_P, csize, W.lv_size[lvl].bytes / 4, hw, big, s, keep);
    tail = (int64_t)M * kTailRatio <= (int64_t)n;
    if (incremental && lists_ok && tail && (int64_t)M * n_next <= kRowBudget) {
      // rate level lvl incrementally from the lists of level lvl-1
      launch_new_clusters(lmatch, gam, n, n_next, nflag, newc, row_slot, W.scan_tmp, s);
      fill_i64(dcnt, 1, M, s);
      const uint64_t *rows = launch_rate_topk_rows(L, L.total, omega, delta, newc, dcnt, M, row_slot,
                                                   pair, score, tk_nxt, W.tail_acc, s);
      if (log_on()) fill_i64(dcnt + 4, 4, 0, s);
      // re-rated nodes: flags in nflag (free after the new clusters' list),
      // count in dcnt[1] (dcnt[2] holds the scan total)
      launch_rate_update(n, lmatch, gam, tk_cur, M, newc, rows, n_next, L.size, L.indeg, omega, delta,
                         learned ? opt.mlp->k : 1, tk_nxt, pair,
                         score, nflag, rerate, dcnt + 1, W.scan_tmp, s, log_on() ? dcnt + 4 : nullptr);
      rate_topk(W, L, omega, delta, rerate, dcnt + 1, n_next, pair, score, tk_nxt, s);
      have_pairs = !learned;
      lists_fresh = learned;
      lists_ok = true;
      path = "incremental";
      if (log_on()) {
        int64_t rr[8] = {};
        HGP_HIP(hipMemcpyAsync(rr, dcnt, sizeof rr, hipMemcpyDeviceToHost, s));
        HGP_HIP(hipStreamSynchronize(s));
        fprintf(stderr,
                "[hgp]   level %d: %d new clusters rated, %lld nodes re-rated (hist-only bound %lld, short list "
                "%lld, need-th key at or below the bound %lld; bound's node merged at %lld nodes)\n",
                lvl, M, (long long)rr[1], (long long)rr[4], (long long)rr[5], (long long)rr[6], (long long)rr[7]);
      }
    } else {
      lists_ok = false;
    }
    std::swap(tk_cur, tk_nxt);
  }
  const int Lmax = lvl;
  st.n_levels = Lmax + 1;
  HGP_HIP(hipStreamSynchronize(s));
  const double t1 = now_ms();

  // ---- refinement, coarsest level first ----
  // A level whose last round applied no move hands its proposals to the next
  // finer level: only the nodes of split clusters are proposed again there.
  int rounds = 0;
  LevelView V0;  // level 0, built by the last iteration
  bool carry_ok = false;
  need<int32_t>(W.cdest, N);
  need<int32_t>(W.cgain, N);
  for (int lv = Lmax; lv >= 0; --lv) {
    const int32_t n = W.lv_n[lv];
    LevelView V;
    int64_t Pl = 0;
    if (lv == Lmax) {
      V = L;
      Pl = cur_P;
    } else {
      // rho_lv(v) = rho_{lv+1}(gamma_lv(v))
      launch_project(W.lv_gamma[lv].as<int32_t>(), rho, n, rho2, s);
      std::swap(rho, rho2);
      const int32_t *h = nullptr;
      const uint32_t *p = nullptr;
      const CachedLevel *c = lv > 0 ? cached_level(W, lv) : nullptr;
      BigHedges vbig = I.big;  // level 0's long hedges, bounded by this level's count
      vbig.bound = W.lv_bigb[(size_t)lv];
      if (log_on())
        fprintf(stderr, "[hgp] refine level %d view %s (%zu levels kept, %.2f GB)\n", lv, c ? "kept" : "rebuilt",
                W.ring.kept.size(), W.ring.kept_bytes() / 1e9);
      if (c) {
        ++st.n_kept;
        V.n = n;
        V.E = E;
        V.hoff = c->hoff;
        V.hpin = c->hpin;
        V.ioff = c->ioff;
        V.inc = c->inc;
        V.perm = c->perm;
        V.indeg = c->indeg;
        V.total = c->total;
        V.size = W.lv_size[lv].as<int32_t>();
        V.hw = hw;
        V.big = vbig;
        Pl = c->P;
        if (c->n != n) throw Error(HGP_EINTERNAL, "cached level size");
      } else if (lv == 0) {
        h = hoff0;
        p = hpin0;
        Pl = P;
      } else {
        int32_t *rh = need<int32_t>(W.hoffR, (int64_t)E + 1);
        uint32_t *rp = need<uint32_t>(W.hpinR, P);
        launch_contract(hoff0, hpin0, E, W.lv_Gamma[lv - 1].as<int32_t>(), W.tmp_pins.as<uint32_t>(),
                        W.cnt.as<int32_t>(), rh, rp, I.big, W.scan_tmp, need<int32_t>(W.longlist, 2 * ((int64_t)E + 1)),
                        W.err.as<int32_t>(), s);
        add_units(HGP_K_CONTRACT, P);
        Pl = read_i32(W, rh + E, s);
        h = rh;
        p = rp;
      }
      if (!c) V = make_view(W, n, E, h, p, Pl, W.lv_size[lv].as<int32_t>(), W.lv_size[lv].bytes / 4, hw, vbig, s);
    }
    set_mid(W, V, s);
    bool last_applied = false;
    int ran = 0;
    for (int r = 0; r < opt.max_refine_rounds; ++r) {
      ++rounds;
      ++ran;
      Carry c;
      const bool use_carry = incremental && r == 0 && carry_ok && lv < Lmax;
      if (use_carry) {
        c.match = W.lv_match[lv].as<int32_t>();
        c.gamma = W.lv_gamma[lv].as<int32_t>();
      }
      RoundBufs B;
      RoundResult R = refine_round(W, V, Pl, rho, n_parts, omega, delta, s, &B, use_carry ? &c : nullptr);
      last_applied = R.applied;
      if (log_on())
        fprintf(stderr, "[hgp] refine level %d round %d n=%d moves=%lld i*=%lld G=%lld applied=%d carried=%d\n", lv,
                r, n, (long long)R.S, (long long)R.istar, (long long)R.gstar, R.applied ? 1 : 0, use_carry ? 1 : 0);
      if (!R.applied) {
        // the state is unchanged: these proposals hold for it
        if (incremental && n > 0) {
          // the round's proposal buffers become the carried ones (B.dest and
          // B.gain are W.dest and W.gain)
          if (B.dest != W.dest.as<int32_t>() || B.gain != W.gain.as<int32_t>())
            throw Error(HGP_EINTERNAL, "proposal buffers");
          std::swap(W.cdest, W.dest);
          std::swap(W.cgain, W.gain);
        }
        break;
      }
    }
    carry_ok = ran > 0 && !last_applied;
    if (lv == 0) V0 = V;
  }
  st.n_rounds = rounds;

  // ---- output: Eq. 1 and compact part ids ----
  {
    if (V0.n != N || V0.hoff != hoff0 || V0.hpin != hpin0) throw Error(HGP_EINTERNAL, "level-0 view");
    RoundBufs B = round_bufs(W, N, E, P, n_parts);
    launch_part_table(V0, rho, n_parts, B, W.err.as<int32_t>(), s);
    int64_t *conn = need<int64_t>(W.conn, 2);
    launch_connectivity(V0, B, conn, s);
    int32_t *used = need<int32_t>(W.used, (int64_t)n_parts + 1);
    launch_compact_parts(rho, N, n_parts, used, part_out, reinterpret_cast<int32_t *>(conn + 1), W.scan_tmp, s);
    int64_t h[2];
    HGP_HIP(hipMemcpyAsync(h, conn, sizeof h, hipMemcpyDeviceToHost, s));
    HGP_HIP(hipStreamSynchronize(s));
    check_err(W, s);
    st.conn = h[0];
    st.n_parts = (int32_t)(h[1] & 0xffffffff);
  }
  const double t2 = now_ms();
  st.ms_coarsen = t1 - t0;
  st.ms_refine = t2 - t1;
  return st;
}

// ---------------------------------------------------------------------------
// ABI plumbing
// ---------------------------------------------------------------------------
template <class F>
static int guarded(F &&f) {
  try {
    f();
    g_last_error.clear();
    return HGP_OK;
  } catch (const Error &e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return HGP_ENOMEM;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return HGP_EINTERNAL;
  } catch (...) {
    g_last_error = "unknown failure";
    return HGP_EINTERNAL;
  }
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    HGP_HIP(hipGetDevice(&prev));
    if (prev != dev) HGP_HIP(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && prev >= 0 && cur != prev) (void)hipSetDevice(prev);
  }
};

static hgp_options opts_or_default(const hgp_options *o) {
  hgp_options d;
  hgp_options_default(&d);
  return o ? *o : d;
}

static void fill_result(hgp_result *res, const RunStats &st) {
  if (!res) return;
  std::memset(res, 0, sizeof *res);
  res->connectivity = st.conn;
  res->n_parts = st.n_parts;
  res->n_levels = st.n_levels;
  res->n_rounds = st.n_rounds;
  res->n_fallback = st.n_fallback;
  res->n_kept = st.n_kept;
  res->ms_coarsen = st.ms_coarsen;
  res->ms_refine = st.ms_refine;
  for (int c = 0; c < HGP_NKERNEL; ++c) {
    res->ms_kernel[c] = st.ms_kernel[c];
    res->n_kernel[c] = st.n_kernel[c];
    res->units_kernel[c] = st.units_kernel[c];
  }
}

static LevelView level_view_from(Workspace &W, const hgp_level *lv, hipStream_t s, int64_t *P_out) {
  if (!lv || lv->n_nodes < 0 || lv->n_hedges < 0 || !lv->hoff || !lv->size || !lv->hedge_w)
    throw Error(HGP_EINVAL, "bad level");
  if (lv->n_nodes >= (1 << 30)) throw Error(HGP_EUNSUPPORTED, "more than 2^30 - 1 nodes");
  const int64_t P = read_i32(lv->hoff + lv->n_hedges, s);
  if (P > 0 && !lv->hpin) throw Error(HGP_EINVAL, "bad level");
  *P_out = P;
  int32_t *err = need<int32_t>(W.err, kErrWords);
  fill_i32(err, 1, 0, s);
  launch_check_offsets(lv->hoff, lv->n_hedges, err, s);
  check_err(W, s);
  launch_check_level(lv->hoff, reinterpret_cast<const uint32_t *>(lv->hpin), lv->n_hedges, lv->n_nodes, err, s);
  check_err(W, s);
  const BigHedges big = find_big(W, lv->hoff, lv->n_hedges, s);
  LevelView V = make_view(W, lv->n_nodes, lv->n_hedges, lv->hoff, reinterpret_cast<const uint32_t *>(lv->hpin), P,
                          lv->size, (size_t)lv->n_nodes, lv->hedge_w, big, s);
  set_mid(W, V, s);
  return V;
}

}  // namespace hgp

using namespace hgp;

extern "C" {

void hgp_options_default(hgp_options *opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof *opt);
  opt->k = 0;
  opt->max_refine_rounds = 8;
  opt->seed = 0;
  opt->proposal = HGP_PLAIN;
}

const char *hgp_strerror(int code) {
  switch (code) {
    case HGP_OK: return "success";
    case HGP_EINVAL: return "invalid argument";
    case HGP_EBADCSR: return "malformed CSR hypergraph";
    case HGP_EINFEASIBLE: return "infeasible: a node alone exceeds Omega or Delta";
    case HGP_ENOMEM: return "out of memory";
    case HGP_EDEVICE: return "HIP device error";
    case HGP_EUNSUPPORTED: return "unsupported input";
    case HGP_EIO: return "checkpoint file input/output error";
    case HGP_EFORMAT: return "not a valid checkpoint file";
    case HGP_EINTERNAL: return "internal error";
    default: return "unknown error";
  }
}

const char *hgp_last_error(void) { return g_last_error.c_str(); }

int hgp_ctx_create(hgp_ctx **ctx, int device) {
  if (!ctx) {
    g_last_error = "ctx is NULL";
    return HGP_EINVAL;
  }
  *ctx = nullptr;
  return guarded([&] {
    int count = 0;
    HGP_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) throw Error(HGP_EINVAL, "no such device");
    DeviceGuard dg(device);
    HGP_HIP(hipFree(nullptr));
    void *scratch = noalloc_scratch_init(device);
    hgp_ctx *c = new hgp_ctx();
    c->device = device;
    c->noalloc_scratch = scratch;
    *ctx = c;
  });
}

int hgp_set_level_cache(hgp_ctx *ctx, int64_t bytes, int64_t *held) {
  if (!ctx) {
    g_last_error = "ctx is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    ctx->ws.lcache_budget = bytes < 0 ? level_cache_default() : bytes;
    if ((int64_t)ctx->ws.ring.arena.bytes > ctx->ws.lcache_budget) {
      HGP_HIP(hipDeviceSynchronize());  // a partition on another stream may still read the levels
      ctx->ws.release_level_cache();
    }
    if (held) *held = (int64_t)ctx->ws.ring.arena.bytes;
  });
}

void hgp_ctx_destroy(hgp_ctx *ctx) {
  if (!ctx) return;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  delete ctx;
  if (prev >= 0) (void)hipSetDevice(prev);
}

int hgp_partition_device(hgp_ctx *ctx, const hgp_hypergraph *g, int32_t omega, int32_t delta,
                         const hgp_options *opt, void *stream, int32_t *part_out, hgp_result *res) {
  if (!ctx) {
    g_last_error = "ctx is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (g && g->n_nodes > 0 && !part_out) throw Error(HGP_EINVAL, "part_out is NULL");
    const hgp_options o = opts_or_default(opt);
    TimerGuard tg(ctx->ws, (o.flags & HGP_FLAG_TIME_KERNELS) != 0, s, o.time_classes);
    RunStats st = run_partition(ctx->ws, g, omega, delta, o, s, part_out);
    tg.collect(st, s);
    HGP_HIP(hipStreamSynchronize(s));
    fill_result(res, st);
  });
}

// Copies a host hypergraph into the workspace's input buffers (validated
// later, on the device, by ingest()); returns the device view.
static hgp_hypergraph upload_host(Workspace &W, const hgp_hypergraph *g, hipStream_t s) {
  const int32_t N = g->n_nodes, E = g->n_hedges;
  for (int32_t e = 0; e < E; ++e)
    if (g->hedge_off[e + 1] < g->hedge_off[e]) throw Error(HGP_EBADCSR, "hedge offsets are not monotone from 0");
  if (g->hedge_off[0] != 0) throw Error(HGP_EBADCSR, "hedge offsets are not monotone from 0");
  const int64_t P = g->hedge_off[E];
  if (P > 0 && !g->pins) throw Error(HGP_EINVAL, "pins is NULL");
  hgp_hypergraph d = *g;
  int32_t *off = need<int32_t>(W.in_off, (int64_t)E + 1);
  HGP_HIP(hipMemcpyAsync(off, g->hedge_off, sizeof(int32_t) * ((size_t)E + 1), hipMemcpyHostToDevice, s));
  d.hedge_off = off;
  if (P > 0) {
    int32_t *pp = need<int32_t>(W.in_pins, P);
    HGP_HIP(hipMemcpyAsync(pp, g->pins, sizeof(int32_t) * (size_t)P, hipMemcpyHostToDevice, s));
    d.pins = pp;
  }
  if (g->n_src && E > 0) {
    int32_t *q = need<int32_t>(W.in_nsrc, E);
    HGP_HIP(hipMemcpyAsync(q, g->n_src, sizeof(int32_t) * (size_t)E, hipMemcpyHostToDevice, s));
    d.n_src = q;
  }
  if (g->hedge_w && E > 0) {
    int32_t *q = need<int32_t>(W.in_hw, E);
    HGP_HIP(hipMemcpyAsync(q, g->hedge_w, sizeof(int32_t) * (size_t)E, hipMemcpyHostToDevice, s));
    d.hedge_w = q;
  }
  if (g->node_w && N > 0) {
    int32_t *q = need<int32_t>(W.in_nw, N);
    HGP_HIP(hipMemcpyAsync(q, g->node_w, sizeof(int32_t) * (size_t)N, hipMemcpyHostToDevice, s));
    d.node_w = q;
  }
  return d;
}

static int partition_host_impl(hgp_ctx *ctx, const hgp_hypergraph *g, int32_t omega, int32_t delta,
                               const hgp_options *opt, int32_t *part_out, hgp_result *res, hgp_trace *trace) {
  if (!ctx) {
    g_last_error = "ctx is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    check_scalars(g, omega, delta);
    Workspace &W = ctx->ws;
    const int32_t N = g->n_nodes;
    if (N > 0 && !part_out) throw Error(HGP_EINVAL, "part_out is NULL");
    hipStream_t s = nullptr;
    hgp_hypergraph d = upload_host(W, g, s);
    int32_t *po = need<int32_t>(W.in_part, N);
    const hgp_options o = opts_or_default(opt);
    if (trace && o.proposal != HGP_PLAIN) throw Error(HGP_EINVAL, "traces record the plain method");
    TimerGuard tg(W, (o.flags & HGP_FLAG_TIME_KERNELS) != 0, s, o.time_classes);
    struct TraceGuard {
      Workspace &W;
      ~TraceGuard() { W.trace = nullptr; }
    } trg{W};
    if (trace) *trace = hgp_trace();
    W.trace = trace;
    RunStats st = run_partition(W, &d, omega, delta, o, s, po);
    W.trace = nullptr;
    tg.collect(st, s);
    if (N > 0) HGP_HIP(hipMemcpyAsync(part_out, po, sizeof(int32_t) * (size_t)N, hipMemcpyDeviceToHost, s));
    HGP_HIP(hipStreamSynchronize(s));
    if (trace) trace_label(*trace, N, part_out);
    fill_result(res, st);
  });
}

int hgp_partition(hgp_ctx *ctx, const hgp_hypergraph *g, int32_t omega, int32_t delta, const hgp_options *opt,
                  int32_t *part_out, hgp_result *res) {
  return partition_host_impl(ctx, g, omega, delta, opt, part_out, res, nullptr);
}

int hgp_partition_traced(hgp_ctx *ctx, const hgp_hypergraph *g, int32_t omega, int32_t delta,
                         const hgp_options *opt, hgp_trace *t, int32_t *part_out, hgp_result *res) {
  if (!t) {
    g_last_error = "trace is NULL";
    return HGP_EINVAL;
  }
  return partition_host_impl(ctx, g, omega, delta, opt, part_out, res, t);
}

int hgp_trace_create(hgp_trace **t) {
  if (!t) {
    g_last_error = "t is NULL";
    return HGP_EINVAL;
  }
  *t = new (std::nothrow) hgp_trace();
  return *t ? HGP_OK : HGP_ENOMEM;
}

void hgp_trace_destroy(hgp_trace *t) { delete t; }

int64_t hgp_trace_rows(const hgp_trace *t) { return t ? (int64_t)t->node.size() : -1; }

int hgp_trace_read(const hgp_trace *t, int32_t *xq, float *label, int32_t *level, int32_t *node, int32_t *cand) {
  if (!t) {
    g_last_error = "t is NULL";
    return HGP_EINVAL;
  }
  const size_t r = t->node.size();
  if (xq && r) std::memcpy(xq, t->xq.data(), sizeof(int32_t) * r * kMlpF);
  if (label && r) std::memcpy(label, t->label.data(), sizeof(float) * r);
  if (level && r) std::memcpy(level, t->level.data(), sizeof(int32_t) * r);
  if (node && r) std::memcpy(node, t->node.data(), sizeof(int32_t) * r);
  if (cand && r) std::memcpy(cand, t->cand.data(), sizeof(int32_t) * r);
  return HGP_OK;
}

void hgp_mlp_init(hgp_mlp_f32 *w, uint64_t seed) {
  if (w) mlp_init(w, seed);
}

int hgp_mlp_grad(hgp_ctx *ctx, const hgp_mlp_f32 *w, const int32_t *xq, const float *y, int64_t n,
                 hgp_mlp_f32 *grad, double *loss, void *stream) {
  if (!ctx) {
    g_last_error = "ctx is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    if (!w || !grad || !loss || n < 1 || !xq || !y) throw Error(HGP_EINVAL, "bad arguments");
    Workspace &W = ctx->ws;
    mlp_grad(w, xq, y, n, W.tr_prm, W.tr_part, W.tr_grad, W.tr_loss, grad, loss, static_cast<hipStream_t>(stream));
  });
}

int hgp_mlp_train(hgp_ctx *ctx, hgp_mlp_f32 *w, const int32_t *xq, const float *y, int64_t n,
                  const hgp_train_opts *opt, float *loss_epochs, void *stream) {
  if (!ctx) {
    g_last_error = "ctx is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    if (!w || !opt || n < 1 || !xq || !y) throw Error(HGP_EINVAL, "bad arguments");
    if (opt->epochs < 0 || opt->batch < 1 || !(opt->lr > 0) || !(opt->eps > 0)) throw Error(HGP_EINVAL, "bad options");
    Workspace &W = ctx->ws;
    hgp_train_state st;
    train_state_init(&st, w, opt->seed);
    mlp_train(&st, xq, y, n, *opt, opt->epochs, W.tr_prm, W.tr_mom, W.tr_part, W.tr_perm, W.tr_loss, loss_epochs,
              static_cast<hipStream_t>(stream));
    *w = st.w;
  });
}

int hgp_mlp_save(const char *path, const hgp_train_state *st, const hgp_mlp *q, int32_t score_shift) {
  return guarded([&] { ckpt_save(path, st, q, score_shift); });
}

int hgp_mlp_load(const char *path, hgp_train_state *st, hgp_mlp *q, int32_t *score_shift) {
  return guarded([&] { ckpt_load(path, st, q, score_shift); });
}

void hgp_train_state_init(hgp_train_state *st, const hgp_mlp_f32 *w, const hgp_train_opts *opt) {
  if (st && w) train_state_init(st, w, opt ? opt->seed : 0);
}

int hgp_mlp_train_state(hgp_ctx *ctx, hgp_train_state *st, const int32_t *xq, const float *y, int64_t n,
                        const hgp_train_opts *opt, int32_t epochs, float *loss_epochs, void *stream) {
  if (!ctx) {
    g_last_error = "ctx is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    if (!st || !opt || n < 1 || !xq || !y || epochs < 0) throw Error(HGP_EINVAL, "bad arguments");
    if (opt->batch < 1 || !(opt->lr > 0) || !(opt->eps > 0)) throw Error(HGP_EINVAL, "bad options");
    if (st->step < 0 || st->epoch < 0 || st->step > 0x7fffffff - (int64_t)epochs * ((n + opt->batch - 1) / opt->batch))
      throw Error(HGP_EINVAL, "bad training state");
    Workspace &W = ctx->ws;
    mlp_train(st, xq, y, n, *opt, epochs, W.tr_prm, W.tr_mom, W.tr_part, W.tr_perm, W.tr_loss, loss_epochs,
              static_cast<hipStream_t>(stream));
  });
}

int hgp_mlp_quantize(const hgp_mlp_f32 *w, const int32_t *xq, int64_t n, int32_t k, hgp_mlp *out,
                     int32_t *score_shift) {
  return guarded([&] {
    if (!w || !out || n < 0 || (n > 0 && !xq)) throw Error(HGP_EINVAL, "bad arguments");
    if (k < 1 || k > kCandK) throw Error(HGP_EINVAL, "k outside 1..8");
    for (int64_t i = 0; i < n * kMlpF; ++i)
      if (xq[i] < 0 || xq[i] > 255) throw Error(HGP_EINVAL, "code outside 0..255");
    mlp_quantize(w, xq, n, k, out, score_shift);
    check_mlp(out);
  });
}


// Eq. 1 for a partition of a device hypergraph (both validated on the device).
static int64_t connectivity_impl(Workspace &W, const hgp_hypergraph *g, const int32_t *part, hipStream_t s) {
  Ingest I = ingest(W, g, 1, 0x7fffffff, s);
  const int32_t N = g->n_nodes, E = g->n_hedges;
  // part ids must be valid indices: bound them by the node count (ids >= 0 checked on device)
  const int32_t np = N > 0 ? N : 1;
  launch_check_range(part, N, 0, np, W.err.as<int32_t>(), s);
  check_err(W, s);
  LevelView V;
  V.n = N;
  V.E = E;
  V.hoff = g->hedge_off;
  V.hpin = I.hpin0;
  V.hw = I.hw;
  V.size = I.nw;
  V.big = I.big;
  set_mid(W, V, s);
  RoundBufs B = round_bufs(W, N, E, I.P, np);
  launch_part_table(V, part, np, B, W.err.as<int32_t>(), s);
  int64_t *conn = need<int64_t>(W.conn, 2);
  launch_connectivity(V, B, conn, s);
  int64_t out = 0;
  HGP_HIP(hipMemcpyAsync(&out, conn, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  HGP_HIP(hipStreamSynchronize(s));
  return out;
}

int hgp_connectivity_device(hgp_ctx *ctx, const hgp_hypergraph *g, const int32_t *part, void *stream,
                            int64_t *out) {
  if (!ctx || !out) {
    g_last_error = "ctx or out is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    if (g && g->n_nodes > 0 && !part) throw Error(HGP_EINVAL, "part is NULL");
    *out = connectivity_impl(ctx->ws, g, part, static_cast<hipStream_t>(stream));
  });
}

int hgp_connectivity(hgp_ctx *ctx, const hgp_hypergraph *g, const int32_t *part, int64_t *out) {
  if (!ctx || !out) {
    g_last_error = "ctx or out is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    check_scalars(g, 1, 0x7fffffff);
    const int32_t N = g->n_nodes;
    if (N > 0 && !part) throw Error(HGP_EINVAL, "part is NULL");
    Workspace &W = ctx->ws;
    hipStream_t s = nullptr;
    hgp_hypergraph d = upload_host(W, g, s);
    int32_t *pd = need<int32_t>(W.in_part, N);
    if (N > 0) HGP_HIP(hipMemcpyAsync(pd, part, sizeof(int32_t) * (size_t)N, hipMemcpyHostToDevice, s));
    *out = connectivity_impl(W, &d, pd, s);
  });
}

int hgp_level_canonical(hgp_ctx *ctx, const hgp_hypergraph *g, int32_t omega, int32_t delta, void *stream,
                        int32_t *hoff_out, int32_t *hpin_out) {
  if (!ctx || !hoff_out) {
    g_last_error = "ctx or hoff_out is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace &W = ctx->ws;
    Ingest I = ingest(W, g, omega, delta, s);
    const int32_t N = g->n_nodes, E = g->n_hedges;
    if (I.P > 0 && !hpin_out) throw Error(HGP_EINVAL, "hpin_out is NULL");
    int32_t *size0 = need<int32_t>(W.rhoB, N);
    if (N > 0) HGP_HIP(hipMemcpyAsync(size0, I.nw, sizeof(int32_t) * (size_t)N, hipMemcpyDeviceToDevice, s));
    LevelView L = make_view(W, N, E, g->hedge_off, I.hpin0, I.P, size0, W.rhoB.bytes / 4, I.hw, I.big, s);
    launch_feasible(size0, L.indeg, N, omega, delta, W.err.as<int32_t>(), s);
    check_err(W, s);
    HGP_HIP(hipMemcpyAsync(hoff_out, g->hedge_off, sizeof(int32_t) * ((size_t)E + 1), hipMemcpyDeviceToDevice, s));
    if (I.P > 0)
      HGP_HIP(hipMemcpyAsync(hpin_out, I.hpin0, sizeof(int32_t) * (size_t)I.P, hipMemcpyDeviceToDevice, s));
    HGP_HIP(hipStreamSynchronize(s));
  });
}

int hgp_level_rate(hgp_ctx *ctx, const hgp_level *lv, int32_t omega, int32_t delta, void *stream,
                   int32_t *pair_out, int64_t *score_out) {
  if (!ctx) {
    g_last_error = "ctx is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (omega < 1 || delta < 0) throw Error(HGP_EINVAL, "Omega < 1 or Delta < 0");
    if (lv && lv->n_nodes > 0 && (!pair_out || !score_out)) throw Error(HGP_EINVAL, "output is NULL");
    int64_t P = 0;
    LevelView L = level_view_from(ctx->ws, lv, s, &P);
    launch_rate(L, ctx->ws.total.as<int32_t>(), omega, delta, pair_out, score_out, need<int32_t>(ctx->ws.maxin, 1),
                s);
    HGP_HIP(hipStreamSynchronize(s));
  });
}

static int level_match_impl(hgp_ctx *ctx, int32_t n, const int32_t *pair, const int64_t *score, int32_t rule,
                            void *stream, int32_t *match_out, int32_t *gamma_out, int32_t *n_next) {
  if (!ctx || !n_next) {
    g_last_error = "ctx or n_next is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (n < 0) throw Error(HGP_EINVAL, "negative count");
    if (rule != HGP_MATCH_TRAVERSAL && rule != HGP_MATCH_EXACT) throw Error(HGP_EINVAL, "unknown matching rule");
    if (n > 0 && (!pair || !score || !match_out || !gamma_out)) throw Error(HGP_EINVAL, "NULL array");
    Workspace &W = ctx->ws;
    if (n == 0) {
      *n_next = 0;
      return;
    }
    need<int32_t>(W.err, kErrWords);
    fill_i32(W.err.as<int32_t>(), 1, 0, s);
    unsigned long long *best = need<unsigned long long>(W.best, n);
    uint8_t *up = need<uint8_t>(W.up, n);
    int32_t *rep = need<int32_t>(W.rep, n);
    int32_t *nn = need<int32_t>(W.scal2, 4);
    launch_check_range(pair, n, -1, n, W.err.as<int32_t>(), s);
    check_err(W, s);
    if (rule == HGP_MATCH_EXACT)
      launch_match_exact(pair, score, n, match_scratch(W, n), best, up, match_out, gamma_out, rep, nn,
                         W.err.as<int32_t>(), W.scan_tmp, s);
    else
      launch_match(pair, score, n, best, up, match_out, gamma_out, rep, nn, W.err.as<int32_t>(), W.scan_tmp, s);
    *n_next = read_i32(nn, s);
    check_err(W, s);
  });
}

int hgp_level_match(hgp_ctx *ctx, int32_t n, const int32_t *pair, const int64_t *score, void *stream,
                    int32_t *match_out, int32_t *gamma_out, int32_t *n_next) {
  return level_match_impl(ctx, n, pair, score, HGP_MATCH_TRAVERSAL, stream, match_out, gamma_out, n_next);
}

int hgp_level_match_ex(hgp_ctx *ctx, int32_t n, const int32_t *pair, const int64_t *score, int32_t rule,
                       void *stream, int32_t *match_out, int32_t *gamma_out, int32_t *n_next) {
  return level_match_impl(ctx, n, pair, score, rule, stream, match_out, gamma_out, n_next);
}

int hgp_level_contract(hgp_ctx *ctx, const hgp_level *lv, const int32_t *gamma, int32_t n_next, void *stream,
                       int32_t *hoff_out, int32_t *hpin_out, int32_t *size_out) {
  if (!ctx) {
    g_last_error = "ctx is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!lv || !hoff_out || lv->n_nodes < 0 || lv->n_hedges < 0 || n_next < 0) throw Error(HGP_EINVAL, "bad args");
    if (lv->n_nodes > 0 && (!gamma || !size_out || !lv->size)) throw Error(HGP_EINVAL, "NULL array");
    Workspace &W = ctx->ws;
    const int32_t E = lv->n_hedges;
    const int64_t P = read_i32(lv->hoff + E, s);
    if (P > 0 && (!hpin_out || !lv->hpin)) throw Error(HGP_EINVAL, "NULL array");
    int32_t *err = need<int32_t>(W.err, kErrWords);
    fill_i32(err, 1, 0, s);
    launch_check_offsets(lv->hoff, E, err, s);
    check_err(W, s);
    launch_check_level(lv->hoff, reinterpret_cast<const uint32_t *>(lv->hpin), E, lv->n_nodes, err, s);
    launch_check_range(gamma, lv->n_nodes, 0, n_next, err, s);
    check_err(W, s);
    uint32_t *tmp = need<uint32_t>(W.tmp_pins, P);
    int32_t *cnt = need<int32_t>(W.cnt, E);
    const BigHedges big = find_big(W, lv->hoff, E, s);
    launch_contract(lv->hoff, reinterpret_cast<const uint32_t *>(lv->hpin), E, gamma, tmp, cnt, hoff_out,
                    reinterpret_cast<uint32_t *>(hpin_out), big, W.scan_tmp, need<int32_t>(W.longlist, 2 * ((int64_t)E + 1)),
                    W.err.as<int32_t>(), s);
    // cluster sizes: sum of member sizes (atomics over the fine nodes)
    fill_i32(size_out, n_next, 0, s);
    launch_cluster_size_sum(gamma, lv->size, lv->n_nodes, size_out, s);
    HGP_HIP(hipStreamSynchronize(s));
  });
}

int hgp_level_refine_round(hgp_ctx *ctx, const hgp_level *lv, const int32_t *rho, int32_t n_parts, int32_t omega,
                           int32_t delta, void *stream, int32_t *pdest, int64_t *pgain, int32_t *seq, int64_t *gsum,
                           int32_t *viol, int32_t *rho_out, int64_t *info) {
  if (!ctx || !info) {
    g_last_error = "ctx or info is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (omega < 1 || delta < 0 || n_parts < 0) throw Error(HGP_EINVAL, "bad scalar");
    if (lv && lv->n_nodes > 0 && (!rho || !pdest || !pgain || !seq || !gsum || !viol || !rho_out))
      throw Error(HGP_EINVAL, "NULL array");
    Workspace &W = ctx->ws;
    int64_t P = 0;
    LevelView L = level_view_from(W, lv, s, &P);
    const int32_t n = L.n;
    launch_check_range(rho, n, 0, n_parts, W.err.as<int32_t>(), s);
    check_err(W, s);
    if (n > 0)
      HGP_HIP(hipMemcpyAsync(rho_out, rho, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    RoundBufs B;
    RoundResult R = refine_round(W, L, P, rho_out, n_parts, omega, delta, s, &B);
    if (n > 0) {
      launch_widen(B.dest, B.gain, n, pdest, pgain, s);
      if (R.S > 0) HGP_HIP(hipMemcpyAsync(seq, B.seq, sizeof(int32_t) * (size_t)R.S, hipMemcpyDeviceToDevice, s));
      HGP_HIP(hipMemcpyAsync(gsum, B.G, sizeof(int64_t) * (size_t)(R.S + 1), hipMemcpyDeviceToDevice, s));
      HGP_HIP(hipMemcpyAsync(viol, B.viol, sizeof(int32_t) * (size_t)(R.S + 1), hipMemcpyDeviceToDevice, s));
    }
    HGP_HIP(hipStreamSynchronize(s));
    info[0] = R.S;
    info[1] = R.istar;
    info[2] = R.gstar;
    info[3] = R.applied ? 1 : 0;
  });
}

int hgp_level_learned(hgp_ctx *ctx, const hgp_level *lv, int32_t level, int32_t omega, int32_t delta,
                      const hgp_mlp *mlp, void *stream, int64_t cap, int64_t *coff, int32_t *cand, int32_t *xq,
                      int64_t *cscore, int32_t *pair, int64_t *score, int32_t *ppair, int64_t *count) {
  if (!ctx || !count) {
    g_last_error = "ctx or count is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (omega < 1 || delta < 0 || level < 0 || cap < 0) throw Error(HGP_EINVAL, "bad scalar");
    check_mlp(mlp);
    if (lv && lv->n_nodes > 0 && (!coff || !cscore || !pair || !score || !ppair || (cap > 0 && !cand)))
      throw Error(HGP_EINVAL, "NULL array");
    Workspace &W = ctx->ws;
    int64_t P = 0;
    LevelView L = level_view_from(W, lv, s, &P);
    const int32_t n = L.n;
    *count = 0;
    if (n == 0) {
      if (coff) fill_i64(coff, 1, 0, s);
      HGP_HIP(hipStreamSynchronize(s));
      return;
    }
    const int32_t *params = upload_mlp(W.mlp, mlp, s);
    int32_t *lp = need<int32_t>(W.pair, n);
    int64_t *ls = need<int64_t>(W.score, n);
    CandBufs B = cand_bufs(W, n, lp, ls);
    const int64_t C = learned_candidates(L, L.total, omega, delta, level, mlp->k, params, B,
                                         W.scan_tmp, W.sort_tmp, s);
    if (C > cap) throw Error(HGP_EINVAL, "candidate capacity too small");
    HGP_HIP(hipMemcpyAsync(coff, B.coff, sizeof(int64_t) * ((size_t)n + 1), hipMemcpyDeviceToDevice, s));
    launch_cand_ids(B, C, n, cand, s);
    if (xq) launch_cand_codes(L, omega, delta, level, B, C, xq, s);
    launch_widen_scores(B.cs, C, cscore, s);
    HGP_HIP(hipMemcpyAsync(pair, lp, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    launch_unkey(lp, ls, n, score, s);
    HGP_HIP(hipMemcpyAsync(ppair, B.ppair, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    HGP_HIP(hipStreamSynchronize(s));
    *count = C;
  });
}

int hgp_mlp_score_device(hgp_ctx *ctx, const hgp_mlp *mlp, const int32_t *xq, int64_t n, int64_t *score,
                         void *stream) {
  if (!ctx) {
    g_last_error = "ctx is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (n < 0 || (n > 0 && (!xq || !score))) throw Error(HGP_EINVAL, "bad arguments");
    check_mlp(mlp);
    if (n == 0) return;
    Workspace &W = ctx->ws;
    const int32_t *params = upload_mlp(W.mlp, mlp, s);
    int32_t *tmp = need<int32_t>(W.cs, n);
    launch_mlp_score_codes(xq, n, params, tmp, s);
    launch_widen_scores(tmp, n, score, s);
  });
}

int hgp_mlp_score_device_noalloc(hgp_ctx *ctx, const hgp_mlp *mlp, const int32_t *xq, int64_t n, int64_t *score,
                                 void *stream) {
  if (!ctx) {
    g_last_error = "ctx is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    if (n < 0 || (n > 0 && (!xq || !score))) throw Error(HGP_EINVAL, "bad arguments");
    check_mlp(mlp);
    if (n > HGP_NOALLOC_MAX_ROWS)
      throw Error(HGP_EUNSUPPORTED, "more than HGP_NOALLOC_MAX_ROWS rows for the allocation-free scoring");
    mlp_score_noalloc(ctx->noalloc_scratch, mlp, xq, n, score, static_cast<hipStream_t>(stream));
  });
}

// ---------------------------------------------------------------------------
// batches of independent hypergraphs
// ---------------------------------------------------------------------------
static hgp_batch_sched sched_resolve(const hgp_ctx *ctx, const hgp_batch_sched *sc) {
  hgp_batch_sched r{};
  if (sc) r = *sc;
  const hgp_batch_sched &t = ctx->tuned;
  if (r.workers == 0) r.workers = t.workers ? t.workers : 4;
  if (r.order == 0) r.order = t.order ? t.order : HGP_ORDER_LPT;
  if (r.rate_tile == 0) r.rate_tile = t.rate_tile ? t.rate_tile : 1024;
  if (r.late_levels == 0) r.late_levels = t.late_levels ? t.late_levels : HGP_LATE_INCREMENTAL;
  if (r.workers < 1 || r.workers > 16) throw Error(HGP_EINVAL, "workers outside 1..16");
  if (r.order != HGP_ORDER_LPT && r.order != HGP_ORDER_INPUT) throw Error(HGP_EINVAL, "unknown order");
  if (r.rate_tile != 256 && r.rate_tile != 512 && r.rate_tile != 1024)
    throw Error(HGP_EINVAL, "rate_tile must be 256, 512 or 1024");
  if (r.late_levels != HGP_LATE_INCREMENTAL && r.late_levels != HGP_LATE_FULL)
    throw Error(HGP_EINVAL, "unknown late-level schedule");
  return r;
}

static int64_t pins_of(const hgp_hypergraph &g, hipStream_t s) {
  if (g.n_hedges <= 0) return 0;
  return read_i32(g.hedge_off + g.n_hedges, s);
}

// Device wall-clock stamp (the constant-rate counter read by wall_clock64).
__global__ void k_stamp(unsigned long long *slot) { *slot = (unsigned long long)wall_clock64(); }

// Runs every graph once on `sc.workers` concurrent streams (one workspace
// each), taking graphs in the schedule's order.  Each graph's start and end
// are stamped on its stream by the device clock; times are ms from a stamp
// taken on the caller's stream before any graph starts.
static void run_batch(hgp_ctx *ctx, int32_t n, const hgp_hypergraph *graphs, const int32_t *omega,
                      const int32_t *delta, const hgp_options &opt, const hgp_batch_sched &sc, hipStream_t caller,
                      int32_t *const *part_out, hgp_result *res, double *t_start, double *t_end) {
  while ((int)ctx->pool.size() < sc.workers) {
    ctx->pool.emplace_back(new Workspace());
    hipStream_t st = nullptr;
    HGP_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    ctx->pool_streams.push_back(st);
  }
  HGP_HIP(hipStreamSynchronize(caller));
  std::vector<int64_t> pins((size_t)n);
  int64_t ring_need = 0;
  for (int32_t i = 0; i < n; ++i) {
    pins[(size_t)i] = pins_of(graphs[i], caller);
    ring_need = std::max<int64_t>(
        ring_need, kBatchRingLevels * (int64_t)level_bytes(graphs[i].n_nodes, graphs[i].n_hedges, pins[(size_t)i]));
  }
  // Each worker keeps its graphs' coarse levels in a ring sized once for the
  // largest graph of the batch (a share of the context's budget), so no
  // worker reallocates it mid-batch: a hipFree would stall every worker.
  const int64_t share = std::max<int64_t>(ctx->ws.lcache_budget, 0) / std::max(sc.workers, 1);
  for (int w = 0; w < sc.workers; ++w) {
    Workspace &W = *ctx->pool[(size_t)w];
    W.lcache_budget = std::min(share, ring_need);
    W.ring.want_last = std::max(W.ring.want_last, W.lcache_budget);
  }
  unsigned long long *stamps = need<unsigned long long>(ctx->batch_stamps, 2 * (int64_t)n + 1);
  int khz = 0;
  HGP_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device));
  if (khz <= 0) throw Error(HGP_EDEVICE, "device wall-clock rate unknown");
  k_stamp<<<1, 1, 0, caller>>>(stamps + 2 * (int64_t)n);
  HGP_HIP(hipGetLastError());
  HGP_HIP(hipStreamSynchronize(caller));
  std::vector<int32_t> order((size_t)n);
  std::iota(order.begin(), order.end(), 0);
  if (sc.order == HGP_ORDER_LPT)
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return pins[(size_t)a] > pins[(size_t)b]; });
  hgp_options o = opt;
  if (sc.late_levels == HGP_LATE_FULL) o.flags |= HGP_FLAG_NO_INCREMENTAL;
  std::atomic<int32_t> next{0};
  std::atomic<bool> failed{false};
  std::mutex mu;
  int err_code = HGP_OK;
  std::string err_msg;
  const double t0 = now_ms();
  auto work = [&](int w) {
    try {
      HGP_HIP(hipSetDevice(ctx->device));
      Workspace &W = *ctx->pool[(size_t)w];
      W.rate_tile = sc.rate_tile;
      hipStream_t s = ctx->pool_streams[(size_t)w];
      while (!failed.load()) {
        const int32_t i = next.fetch_add(1);
        if (i >= n) break;
        const int32_t g = order[(size_t)i];
        k_stamp<<<1, 1, 0, s>>>(stamps + 2 * (int64_t)g);
        HGP_HIP(hipGetLastError());
        TimerGuard tg(W, (o.flags & HGP_FLAG_TIME_KERNELS) != 0, s, o.time_classes);
        RunStats st = run_partition(W, &graphs[g], omega[g], delta[g], o, s, part_out[g]);
        tg.collect(st, s);
        k_stamp<<<1, 1, 0, s>>>(stamps + 2 * (int64_t)g + 1);
        HGP_HIP(hipGetLastError());
        HGP_HIP(hipStreamSynchronize(s));
        if (log_batch_on())
          fprintf(stderr, "[hgp] batch graph %d (n=%d) done at %.0f ms (host) by worker %d\n", g, graphs[g].n_nodes,
                  now_ms() - t0, w);
        if (res) fill_result(&res[g], st);
      }
    } catch (const Error &e) {
      std::lock_guard<std::mutex> lk(mu);
      if (!failed.exchange(true)) {
        err_code = e.code;
        err_msg = e.what();
      }
    } catch (const std::exception &e) {
      std::lock_guard<std::mutex> lk(mu);
      if (!failed.exchange(true)) {
        err_code = HGP_EINTERNAL;
        err_msg = e.what();
      }
    }
  };
  std::vector<std::thread> th;
  for (int w = 0; w < sc.workers; ++w) th.emplace_back(work, w);
  for (auto &t : th) t.join();
  if (failed.load()) throw Error(err_code, err_msg);
  if (n > 0 && (t_start || t_end)) {
    std::vector<unsigned long long> h(2 * (size_t)n + 1);
    HGP_HIP(hipMemcpy(h.data(), stamps, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost));
    const unsigned long long base = h[2 * (size_t)n];
    const double per_ms = (double)khz;  // ticks per ms
    for (int32_t g = 0; g < n; ++g) {
      if (t_start) t_start[g] = (double)(long long)(h[2 * (size_t)g] - base) / per_ms;
      if (t_end) t_end[g] = (double)(long long)(h[2 * (size_t)g + 1] - base) / per_ms;
    }
  }
}

static void check_batch_args(int32_t n, const hgp_hypergraph *graphs, const int32_t *omega, const int32_t *delta,
                             int32_t *const *part_out) {
  if (n < 0) throw Error(HGP_EINVAL, "n_graphs < 0");
  if (n > 0 && (!graphs || !omega || !delta || !part_out)) throw Error(HGP_EINVAL, "NULL array");
  for (int32_t i = 0; i < n; ++i) {
    check_scalars(&graphs[i], omega[i], delta[i]);
    if (graphs[i].n_nodes > 0 && !part_out[i]) throw Error(HGP_EINVAL, "part_out[i] is NULL");
  }
}

int hgp_partition_batch_device(hgp_ctx *ctx, int32_t n_graphs, const hgp_hypergraph *graphs, const int32_t *omega,
                               const int32_t *delta, const hgp_options *opt, const hgp_batch_sched *sched,
                               void *stream, int32_t *const *part_out, hgp_result *res, double *t_start_ms,
                               double *t_end_ms) {
  if (!ctx) {
    g_last_error = "ctx is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    check_batch_args(n_graphs, graphs, omega, delta, part_out);
    const hgp_batch_sched sc = sched_resolve(ctx, sched);
    run_batch(ctx, n_graphs, graphs, omega, delta, opts_or_default(opt), sc, static_cast<hipStream_t>(stream),
              part_out, res, t_start_ms, t_end_ms);
  });
}

int hgp_batch_tune(hgp_ctx *ctx, int32_t n_graphs, const hgp_hypergraph *graphs, const int32_t *omega,
                   const int32_t *delta, const hgp_options *opt, void *stream, int32_t *const *part_out,
                   hgp_batch_sched *best, double *best_ms) {
  if (!ctx) {
    g_last_error = "ctx is NULL";
    return HGP_EINVAL;
  }
  return guarded([&] {
    DeviceGuard dg(ctx->device);
    check_batch_args(n_graphs, graphs, omega, delta, part_out);
    const hgp_options o = opts_or_default(opt);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // coordinate search: workers first (the dominant knob), then each other
    // knob in turn with the best setting so far; every candidate runs the
    // whole batch once after one warm-up of the largest worker count
    hgp_batch_sched cur{};
    cur.workers = 4;
    cur.order = HGP_ORDER_LPT;
    cur.rate_tile = 1024;
    cur.late_levels = HGP_LATE_INCREMENTAL;
    auto time_of = [&](const hgp_batch_sched &c) {
      const double a = now_ms();
      run_batch(ctx, n_graphs, graphs, omega, delta, o, c, s, part_out, nullptr, nullptr, nullptr);
      const double t = now_ms() - a;
      if (log_batch_on())
        fprintf(stderr, "[hgp] tune workers=%d order=%d tile=%d late=%d: %.0f ms\n", c.workers, c.order,
                c.rate_tile, c.late_levels, t);
      return t;
    };
    {
      hgp_batch_sched warm = cur;
      warm.workers = 16;
      (void)time_of(warm);
    }
    double best_t = 1e300;
    for (int w : {1, 2, 4, 8, 16}) {
      hgp_batch_sched c = cur;
      c.workers = w;
      const double t = time_of(c);
      if (t < best_t) {
        best_t = t;
        cur = c;
      }
    }
    {
      hgp_batch_sched c = cur;
      c.order = HGP_ORDER_INPUT;
      const double t = time_of(c);
      if (t < best_t) {
        best_t = t;
        cur = c;
      }
    }
    for (int tile : {512, 256}) {
      hgp_batch_sched c = cur;
      c.rate_tile = tile;
      const double t = time_of(c);
      if (t < best_t) {
        best_t = t;
        cur = c;
      }
    }
    {
      hgp_batch_sched c = cur;
      c.late_levels = HGP_LATE_FULL;
      const double t = time_of(c);
      if (t < best_t) {
        best_t = t;
        cur = c;
      }
    }
    ctx->tuned = cur;
    if (best) *best = cur;
    if (best_ms) *best_ms = best_t;
  });
}

}  // extern "C"
