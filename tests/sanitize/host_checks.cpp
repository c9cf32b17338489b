// Host-only code of the library (MBR schedule and GPS ordering, SAO and
// RANSAC on host threads) and the C oracle, exercised under AddressSanitizer
// and UndefinedBehaviorSanitizer on the CPU (tests/test_host_sanitizers.py
// builds and runs this).  Seeded random inputs, valid and invalid; every
// check failure prints a line and makes the exit status nonzero.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "chm.h"

// The library's error reporting (chm_host.cpp needs the HIP runtime, so the
// sanitizer build supplies its own).
namespace chm {
chm_status fail(chm_status st, const char*, ...) { return st; }
void clear_error() {}
bool hip_fault_due() { return false; }
}  // namespace chm

extern "C" {
typedef struct orc_image {
  const uint8_t* desc;
  const uint32_t* codes;
  const uint8_t* ids;
  const int32_t* offsets;
  const int32_t* members;
  int64_t n;
} orc_image;
void orc_set_threads(int n);
void orc_hash(const uint8_t* X, int64_t n, const uint16_t* W, const uint8_t* mu, int32_t L, int32_t m,
              uint32_t* codes, uint8_t* ids);
void orc_tables(const uint8_t* ids, int64_t n, int32_t L, int32_t m, int32_t* offsets, int32_t* members);
int64_t orc_match_pairs(const orc_image* images, const int32_t* pairs, int64_t P, const int64_t* out_offsets,
                        int32_t L, int32_t m, int32_t K, int32_t ra, int32_t rb, int32_t single, int32_t whole,
                        int32_t* out, uint32_t* topk);
void orc_bruteforce(const uint8_t* Xq, int64_t nq, const uint8_t* Xd, int64_t nd, int32_t ra, int32_t rb,
                    int32_t* out);
}

static int g_bad = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::printf("check failed %s:%d: %s\n", __FILE__, __LINE__, #c); \
      ++g_bad;                                                     \
    }                                                              \
  } while (0)

static void schedules(std::mt19937& rng) {
  // grid view graph with oblique links, several caps and block sizes
  for (int rows : {3, 7}) {
    const int cols = 13, n = rows * cols;
    std::vector<int32_t> pairs;
    for (int r = 0; r < rows; ++r)
      for (int c = 0; c < cols; ++c)
        for (int dr = -1; dr <= 1; ++dr)
          for (int dc = -2; dc <= 2; ++dc) {
            const int r2 = r + dr, c2 = c + dc;
            if ((dr || dc) && r2 >= 0 && r2 < rows && c2 >= 0 && c2 < cols) {
              pairs.push_back(r * cols + c);
              pairs.push_back(r2 * cols + c2);
            }
          }
    for (int i = 0; i < n / 4; ++i) {
      pairs.push_back((int)(rng() % n));
      pairs.push_back((int)(rng() % n));
    }
    const int P = (int)pairs.size() / 2;
    std::vector<uint64_t> bytes(n);
    for (auto& b : bytes) b = 1000 + rng() % 3000;
    for (uint64_t cap : {(uint64_t)8000, (uint64_t)20000, (uint64_t)1u << 30})
      for (int blk : {1, 4, 16}) {
        chm_schedule* s = nullptr;
        const chm_status st = chm_schedule_mbr(n, pairs.data(), P, bytes.data(), cap, blk, &s);
        CHECK(st == CHM_OK);
        if (st != CHM_OK) continue;
        std::set<int> resident;
        std::vector<int> seen(P, 0);
        for (int k = 0; k < chm_schedule_num_steps(s); ++k) {
          const int32_t *ev, *ld, *pp;
          int32_t nev, nld, npp;
          CHECK(chm_schedule_step(s, k, &ev, &nev, &ld, &nld, &pp, &npp) == CHM_OK);
          for (int i = 0; i < nev; ++i) resident.erase(ev[i]);
          for (int i = 0; i < nld; ++i) resident.insert(ld[i]);
          uint64_t used = 0;
          for (int i : resident) used += bytes[i];
          CHECK(used <= cap);
          for (int i = 0; i < npp; ++i) {
            CHECK(pp[i] >= 0 && pp[i] < P);
            if (pp[i] < 0 || pp[i] >= P) continue;
            ++seen[pp[i]];
            CHECK(resident.count(pairs[2 * pp[i]]) && resident.count(pairs[2 * pp[i] + 1]));
          }
        }
        for (int p = 0; p < P; ++p) CHECK(seen[p] == 1);
        int32_t iters = 0, fb = 0;
        const int32_t *dims = nullptr, *bws = nullptr;
        CHECK(chm_schedule_info(s, &iters, &fb, &dims, &bws) == CHM_OK);
        chm_schedule_free(s);
      }
    std::vector<int32_t> nodes(n), order(n);
    for (int i = 0; i < n; ++i) nodes[i] = i;
    CHECK(chm_gps_order(n, pairs.data(), P, nodes.data(), n, order.data()) == CHM_OK);
    std::set<int> perm(order.begin(), order.end());
    CHECK((int)perm.size() == n);
  }
  // invalid arguments are rejected
  chm_schedule* s = nullptr;
  int32_t bad_pair[2] = {0, 5};
  uint64_t one[1] = {10};
  CHECK(chm_schedule_mbr(1, bad_pair, 1, one, 100, 1, &s) != CHM_OK);
  CHECK(chm_schedule_mbr(-1, nullptr, 0, nullptr, 100, 1, &s) != CHM_OK);
  CHECK(chm_gps_order(2, nullptr, 1, nullptr, 0, nullptr) != CHM_OK);
}

static void outlier_removal(std::mt19937& rng) {
  const int n_img = 4, nf = 300;
  std::vector<std::vector<int32_t>> kp(n_img, std::vector<int32_t>(2 * nf));
  for (auto& k : kp)
    for (auto& v : k) v = (int32_t)(rng() % 50000);
  const int32_t* kps[n_img] = {kp[0].data(), kp[1].data(), kp[2].data(), kp[3].data()};
  const int32_t feats[n_img] = {nf, nf, nf, nf};
  const int32_t pairs[6] = {0, 1, 1, 2, 3, 0};
  const int64_t offs[4] = {0, nf, 2 * nf, 3 * nf};
  std::vector<int32_t> match(3 * nf), out(3 * nf), ced(3 * nf), best(3);
  for (int i = 0; i < 3 * nf; ++i) match[i] = rng() % 3 ? (int32_t)(rng() % nf) : -1;
  for (int nn : {1, 6, 32})
    CHECK(chm_sao_filter(3, pairs, kps, feats, n_img, offs, match.data(), nn, 1, 2, 3, out.data(), ced.data()) ==
          CHM_OK);
  std::vector<uint32_t> words(3 * 16 * 2);
  for (auto& w : words) w = (uint32_t)rng();
  for (auto& k : kp)
    for (auto& v : k) v %= (1 << 18);
  CHECK(chm_ransac_filter(3, pairs, kps, feats, n_img, offs, match.data(), words.data(), 16, 40, 4, 3, out.data(),
                          best.data()) == CHM_OK);
  // a db row out of range is rejected
  match[5] = nf + 3;
  CHECK(chm_sao_filter(3, pairs, kps, feats, n_img, offs, match.data(), 6, 1, 2, 2, out.data(), nullptr) !=
        CHM_OK);
  CHECK(chm_ransac_filter(3, pairs, kps, feats, n_img, offs, match.data(), words.data(), 16, 40, 4, 2, out.data(),
                          nullptr) != CHM_OK);
}

static void oracle(std::mt19937& rng) {
  const int L = 6, m = 8, R = 128 + L * m;
  std::vector<uint16_t> W(R * 128);
  std::normal_distribution<float> nd(0.f, 1.f);
  for (auto& w : W) {
    float f = nd(rng);
    uint32_t u;
    std::memcpy(&u, &f, 4);
    w = (uint16_t)(u >> 16);
    if ((w & 0x7F80) < 0x3780) w = 0;  // below 2^-16: zero
  }
  std::vector<uint8_t> mu(128, 60);
  const int sizes[4] = {0, 1, 257, 700};
  std::vector<std::vector<uint8_t>> X(4), ids(4);
  std::vector<std::vector<uint32_t>> codes(4);
  std::vector<std::vector<int32_t>> offs(4), mem(4);
  std::vector<orc_image> img(4);
  for (int i = 0; i < 4; ++i) {
    const int n = sizes[i];
    X[i].resize((size_t)n * 128 + 1);
    for (auto& v : X[i]) v = (uint8_t)(rng() % 120);
    codes[i].resize((size_t)n * 4 + 1);
    ids[i].resize((size_t)n * L + 1);
    offs[i].resize(L * ((1 << m) + 1));
    mem[i].resize((size_t)L * n + 1);
    orc_hash(X[i].data(), n, W.data(), mu.data(), L, m, codes[i].data(), ids[i].data());
    orc_tables(ids[i].data(), n, L, m, offs[i].data(), mem[i].data());
    img[i] = orc_image{X[i].data(), codes[i].data(), ids[i].data(), offs[i].data(), mem[i].data(), n};
  }
  const int32_t pairs[] = {3, 2, 2, 3, 3, 3, 0, 3, 3, 0, 1, 3, 3, 1};
  const int P = 7;
  std::vector<int64_t> o(P + 1, 0);
  for (int p = 0; p < P; ++p) o[p + 1] = o[p] + sizes[pairs[2 * p]];
  std::vector<int32_t> out(o[P] + 1);
  std::vector<uint32_t> topk((o[P] + 1) * 8);
  for (int threads : {1, 4})
    for (int whole : {0, 1}) {
      orc_set_threads(threads);
      orc_match_pairs(img.data(), pairs, P, o.data(), L, m, 8, 4, 5, whole, whole, out.data(), topk.data());
    }
  orc_bruteforce(X[3].data(), 700, X[2].data(), 257, 99, 100, out.data());
}

int main() {
  std::mt19937 rng(12345);
  schedules(rng);
  outlier_removal(rng);
  oracle(rng);
  std::printf("host checks: %d failures\n", g_bad);
  return g_bad ? 1 : 0;
}
