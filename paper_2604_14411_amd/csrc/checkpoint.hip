// Checkpoint files of the learned proposal's network and the check of an
// integer network's domain (host code only).
//
// Layout (little-endian), version 1:
//   header, 48 bytes: magic "HGPMLP\0\0", u32 version, u32 header size,
//     u32 inputs, u32 hidden units, u32 parameter count, u32 section bits
//     (1: training state, 2: integer network), i32 score shift, u32 reserved,
//     u64 payload bytes;
//   payload: training state (weights, first moments, second moments as
//     kNPar floats each in hgp_mlp_f32 order; i64 step, i64 epoch, u64 rng),
//     then the integer network (hgp_mlp as laid out in the header file);
//   trailer: CRC-32 of header and payload.
// The CRC is the IEEE 802.3 one (reflected polynomial 0xEDB88320, initial
// value and final xor 0xFFFFFFFF), computed bit by bit.
#include <cstdio>
#include <cstring>
#include <memory>
#include <vector>

#include "learned.hpp"

namespace hgp {

static_assert(__BYTE_ORDER__ == __ORDER_LITTLE_ENDIAN__, "checkpoint files are written in host byte order");

namespace {

constexpr char kMagic[8] = {'H', 'G', 'P', 'M', 'L', 'P', '\0', '\0'};
constexpr uint32_t kVersion = 1;
constexpr uint32_t kSecState = 1, kSecInt = 2;
constexpr uint32_t kNParams = (uint32_t)(sizeof(hgp_mlp_f32) / sizeof(float));

struct Header {
  char magic[8];
  uint32_t version;
  uint32_t header_bytes;
  uint32_t inputs;
  uint32_t hidden;
  uint32_t n_params;
  uint32_t sections;
  int32_t score_shift;
  uint32_t reserved;
  uint64_t payload_bytes;
};
static_assert(sizeof(Header) == 48, "checkpoint header is 48 bytes");

constexpr size_t kStateBytes = 3 * sizeof(hgp_mlp_f32) + 3 * sizeof(int64_t);

uint32_t crc32_update(uint32_t crc, const unsigned char *p, size_t n) {
  for (size_t i = 0; i < n; ++i) {
    crc ^= p[i];
    for (int b = 0; b < 8; ++b) crc = (crc >> 1) ^ (0xEDB88320u & (0u - (crc & 1u)));
  }
  return crc;
}

void put(std::vector<unsigned char> &buf, const void *p, size_t n) {
  const unsigned char *c = static_cast<const unsigned char *>(p);
  buf.insert(buf.end(), c, c + n);
}

struct FileCloser {
  void operator()(FILE *f) const {
    if (f) std::fclose(f);
  }
};

}  // namespace

// The integer network's domain (see hgp_mlp): the ranges that keep every
// partial sum exact in FP32 on the MFMA path.
void check_mlp(const hgp_mlp *q) {
  if (!q) throw Error(HGP_EINVAL, "learned proposal without a network");
  if (q->k < 1) throw Error(HGP_EINVAL, "network k < 1");
  if (q->k > kCandK) throw Error(HGP_EUNSUPPORTED, "network k > 8");
  if (q->r1 < 0 || q->r1 > 30 || q->r2 < 0 || q->r2 > 30) throw Error(HGP_EINVAL, "shift outside 0..30");
  const int64_t bmax = int64_t(1) << 22;
  for (int i = 0; i < kMlpF * kMlpH; ++i)
    if (q->w1[i] < -255 || q->w1[i] > 255) throw Error(HGP_EINVAL, "w1 outside -255..255");
  for (int i = 0; i < kMlpH * kMlpH; ++i)
    if (q->w2[i] < -255 || q->w2[i] > 255) throw Error(HGP_EINVAL, "w2 outside -255..255");
  for (int i = 0; i < kMlpH; ++i) {
    if (q->w3[i] < -255 || q->w3[i] > 255) throw Error(HGP_EINVAL, "w3 outside -255..255");
    if (q->b1[i] < -bmax || q->b1[i] > bmax || q->b2[i] < -bmax || q->b2[i] > bmax)
      throw Error(HGP_EINVAL, "bias outside -2^22..2^22");
  }
  if (q->b3 < -bmax || q->b3 > bmax) throw Error(HGP_EINVAL, "bias outside -2^22..2^22");
}

void ckpt_save(const char *path, const hgp_train_state *st, const hgp_mlp *q, int32_t score_shift) {
  if (!path) throw Error(HGP_EINVAL, "path is NULL");
  if (!st && !q) throw Error(HGP_EINVAL, "nothing to save");
  if (q) check_mlp(q);
  std::vector<unsigned char> pay;
  if (st) {
    put(pay, &st->w, sizeof st->w);
    put(pay, &st->m, sizeof st->m);
    put(pay, &st->v, sizeof st->v);
    put(pay, &st->step, sizeof st->step);
    put(pay, &st->epoch, sizeof st->epoch);
    put(pay, &st->rng, sizeof st->rng);
  }
  if (q) put(pay, q, sizeof *q);
  Header h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, kMagic, sizeof kMagic);
  h.version = kVersion;
  h.header_bytes = sizeof(Header);
  h.inputs = kMlpF;
  h.hidden = kMlpH;
  h.n_params = kNParams;
  h.sections = (st ? kSecState : 0u) | (q ? kSecInt : 0u);
  h.score_shift = score_shift;
  h.payload_bytes = pay.size();
  uint32_t crc = crc32_update(0xFFFFFFFFu, reinterpret_cast<const unsigned char *>(&h), sizeof h);
  crc = crc32_update(crc, pay.data(), pay.size()) ^ 0xFFFFFFFFu;
  std::unique_ptr<FILE, FileCloser> f(std::fopen(path, "wb"));
  if (!f) throw Error(HGP_EIO, std::string("cannot open for writing: ") + path);
  bool ok = std::fwrite(&h, sizeof h, 1, f.get()) == 1;
  ok = ok && (pay.empty() || std::fwrite(pay.data(), pay.size(), 1, f.get()) == 1);
  ok = ok && std::fwrite(&crc, sizeof crc, 1, f.get()) == 1;
  ok = (std::fclose(f.release()) == 0) && ok;
  if (!ok) throw Error(HGP_EIO, std::string("write failed: ") + path);
}

void ckpt_load(const char *path, hgp_train_state *st, hgp_mlp *q, int32_t *score_shift) {
  if (!path) throw Error(HGP_EINVAL, "path is NULL");
  std::unique_ptr<FILE, FileCloser> f(std::fopen(path, "rb"));
  if (!f) throw Error(HGP_EIO, std::string("cannot open: ") + path);
  std::vector<unsigned char> all;
  unsigned char chunk[65536];
  size_t got;
  while ((got = std::fread(chunk, 1, sizeof chunk, f.get())) > 0) {
    all.insert(all.end(), chunk, chunk + got);
    if (all.size() > (size_t(1) << 24)) throw Error(HGP_EFORMAT, "file too large for a checkpoint");
  }
  if (std::ferror(f.get())) throw Error(HGP_EIO, std::string("read failed: ") + path);
  if (all.size() < sizeof(Header) + sizeof(uint32_t)) throw Error(HGP_EFORMAT, "file shorter than a checkpoint");
  Header h;
  std::memcpy(&h, all.data(), sizeof h);
  if (std::memcmp(h.magic, kMagic, sizeof kMagic) != 0) throw Error(HGP_EFORMAT, "not a checkpoint (magic)");
  if (h.version != kVersion) throw Error(HGP_EFORMAT, "unsupported checkpoint version");
  if (h.header_bytes != sizeof(Header) || h.inputs != (uint32_t)kMlpF || h.hidden != (uint32_t)kMlpH ||
      h.n_params != kNParams || h.reserved != 0)
    throw Error(HGP_EFORMAT, "checkpoint shapes differ from this library's network");
  if (h.sections == 0 || (h.sections & ~(kSecState | kSecInt)) != 0) throw Error(HGP_EFORMAT, "bad section bits");
  const uint64_t want = ((h.sections & kSecState) ? kStateBytes : 0) + ((h.sections & kSecInt) ? sizeof(hgp_mlp) : 0);
  if (h.payload_bytes != want || all.size() != sizeof(Header) + want + sizeof(uint32_t))
    throw Error(HGP_EFORMAT, "checkpoint size does not match its header");
  uint32_t stored;
  std::memcpy(&stored, all.data() + sizeof(Header) + want, sizeof stored);
  const uint32_t crc = crc32_update(0xFFFFFFFFu, all.data(), sizeof(Header) + want) ^ 0xFFFFFFFFu;
  if (crc != stored) throw Error(HGP_EFORMAT, "checkpoint CRC mismatch");
  if (st && !(h.sections & kSecState)) throw Error(HGP_EFORMAT, "checkpoint has no training state");
  if (q && !(h.sections & kSecInt)) throw Error(HGP_EFORMAT, "checkpoint has no integer network");
  const unsigned char *p = all.data() + sizeof(Header);
  if (h.sections & kSecState) {
    if (st) {
      std::memcpy(&st->w, p, sizeof st->w);
      std::memcpy(&st->m, p + sizeof(hgp_mlp_f32), sizeof st->m);
      std::memcpy(&st->v, p + 2 * sizeof(hgp_mlp_f32), sizeof st->v);
      std::memcpy(&st->step, p + 3 * sizeof(hgp_mlp_f32), sizeof st->step);
      std::memcpy(&st->epoch, p + 3 * sizeof(hgp_mlp_f32) + 8, sizeof st->epoch);
      std::memcpy(&st->rng, p + 3 * sizeof(hgp_mlp_f32) + 16, sizeof st->rng);
    }
    p += kStateBytes;
  }
  if ((h.sections & kSecInt) && q) {
    hgp_mlp tmp;
    std::memcpy(&tmp, p, sizeof tmp);
    try {
      check_mlp(&tmp);
    } catch (const Error &e) {
      throw Error(HGP_EFORMAT, std::string("stored network invalid: ") + e.what());
    }
    *q = tmp;
  }
  if (score_shift) *score_shift = h.score_shift;
}

}  // namespace hgp
