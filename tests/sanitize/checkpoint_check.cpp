// Runs the library's host-side checkpoint code (what hgp_mlp_save and
// hgp_mlp_load call, and the integer network's checks) under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_sanitize_cpu.py): a round
// trip, every single-byte corruption of a small file, truncations and bad
// networks.  No device is needed.  Exit status 0 when every call returned
// its expected code.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../paper_2604_14411_amd/csrc/learned.hpp"

static int failures = 0;

// The C-ABI entry points return the code of the error the call threw.
static int save(const char *path, const hgp_train_state *st, const hgp_mlp *q, int32_t shift) {
  try {
    hgp::ckpt_save(path, st, q, shift);
  } catch (const hgp::Error &e) {
    return e.code;
  }
  return HGP_OK;
}

static int load(const char *path, hgp_train_state *st, hgp_mlp *q, int32_t *shift) {
  try {
    hgp::ckpt_load(path, st, q, shift);
  } catch (const hgp::Error &e) {
    return e.code;
  }
  return HGP_OK;
}

static void expect(int got, int want, const char *what) {
  if (got != want) {
    std::fprintf(stderr, "%s: rc %d, expected %d\n", what, got, want);
    ++failures;
  }
}

int main(int argc, char **argv) {
  const std::string dir = argc > 1 ? argv[1] : ".";
  const std::string path = dir + "/ck.bin", bad = dir + "/bad.bin";
  static hgp_mlp q;
  std::memset(&q, 0, sizeof q);
  q.k = 8;
  q.r1 = 3;
  q.r2 = 4;
  for (int i = 0; i < HGP_MLP_F * HGP_MLP_H; ++i) q.w1[i] = (i * 7) % 511 - 255;
  static hgp_train_state st;
  std::memset(&st, 0, sizeof st);
  st.step = 7;
  st.epoch = 2;
  st.rng = 12345;
  st.w.b3 = 0.5f;
  expect(save(path.c_str(), &st, &q, -3), HGP_OK, "save");
  static hgp_train_state st2;
  static hgp_mlp q2;
  int32_t sh = 0;
  expect(load(path.c_str(), &st2, &q2, &sh), HGP_OK, "load");
  if (std::memcmp(&q, &q2, sizeof q) != 0 || st2.step != 7 || sh != -3) ++failures;
  // read the file back and damage it
  std::vector<unsigned char> raw;
  if (FILE *f = std::fopen(path.c_str(), "rb")) {
    int c;
    while ((c = std::fgetc(f)) != EOF) raw.push_back((unsigned char)c);
    std::fclose(f);
  }
  auto write = [&](const std::vector<unsigned char> &d) {
    FILE *f = std::fopen(bad.c_str(), "wb");
    if (!f) return;
    if (!d.empty()) std::fwrite(d.data(), 1, d.size(), f);
    std::fclose(f);
  };
  for (size_t i = 0; i < raw.size(); i += 53) {
    std::vector<unsigned char> d = raw;
    d[i] ^= 0x5a;
    write(d);
    expect(load(bad.c_str(), &st2, &q2, &sh), HGP_EFORMAT, "flipped byte");
  }
  for (size_t n : {(size_t)0, (size_t)10, (size_t)47, (size_t)48, raw.size() - 1}) {
    write(std::vector<unsigned char>(raw.begin(), raw.begin() + (long)n));
    expect(load(bad.c_str(), &st2, &q2, &sh), HGP_EFORMAT, "truncated");
  }
  q.w2[5] = 300;
  expect(save(bad.c_str(), nullptr, &q, 0), HGP_EINVAL, "bad network");
  expect(load((dir + "/missing.bin").c_str(), &st2, nullptr, nullptr), HGP_EIO, "missing file");
  expect(save(nullptr, &st, nullptr, 0), HGP_EINVAL, "null path");
  std::printf("checkpoint code under sanitizers: %d failures\n", failures);
  return failures ? 1 : 0;
}
