// RANSAC global verification (Sec. 2.3.3) of each pair's matches on host
// threads, with a 2D similarity as the two-view model.
//
// Hypothesis t of a pair draws its two matches from two caller-supplied
// random words: i = u mod M, j = v mod (M - 1), plus one when j >= i.  With
// dp = p_j - p_i, dq = q_j - q_i, D = |dp|^2 and w = dq * conj(dp) (complex
// notation), the similarity through the two matches is q = q_i + (w / D)
// (p - p_i), and match k is an inlier when |D (q_k - q_i) - w (p_k - p_i)|^2
// <= D^2 thr^2.  For coordinates below 2^19 and thr below 2^20 every term
// fits a signed 128-bit integer, so the test is exact.  The best hypothesis
// (most inliers, the earlier one on ties) verifies the pair when its count
// reaches min_inliers; its inliers are the verified matches.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "chm.h"
#include "chm_host.h"

namespace {

using i128 = __int128;
constexpr int64_t kRansacCoordLimit = int64_t(1) << 19;
constexpr int64_t kRansacThrLimit = int64_t(1) << 20;

struct Job {
  const int32_t* idx;       // job entry p is pair idx[p] of the lists below (null: p)
  const int32_t* pairs;
  const int32_t* const* kp;
  const int32_t* n_feats;
  const int64_t* offs;
  const int32_t* match;
  const uint32_t* words;
  int32_t iterations;
  int64_t thr;
  int32_t min_inliers;
  int32_t* out;
  int32_t* best_counts;
};

struct Sim {
  int64_t pix, piy, qix, qiy, D, wr, wi;
};

inline bool make_sim(const std::vector<int64_t>& P, const std::vector<int64_t>& Q, int i, int j, Sim* s) {
  s->pix = P[2 * i];
  s->piy = P[2 * i + 1];
  s->qix = Q[2 * i];
  s->qiy = Q[2 * i + 1];
  const int64_t dpx = P[2 * j] - s->pix, dpy = P[2 * j + 1] - s->piy;
  const int64_t dqx = Q[2 * j] - s->qix, dqy = Q[2 * j + 1] - s->qiy;
  s->D = dpx * dpx + dpy * dpy;
  s->wr = dqx * dpx + dqy * dpy;
  s->wi = dqy * dpx - dqx * dpy;
  return s->D != 0;
}

inline bool inlier(const Sim& s, const std::vector<int64_t>& P, const std::vector<int64_t>& Q, int k, i128 lim) {
  const int64_t ex = P[2 * k] - s.pix, ey = P[2 * k + 1] - s.piy;
  const int64_t fx = Q[2 * k] - s.qix, fy = Q[2 * k + 1] - s.qiy;
  const i128 rx = (i128)s.D * fx - ((i128)s.wr * ex - (i128)s.wi * ey);
  const i128 ry = (i128)s.D * fy - ((i128)s.wr * ey + (i128)s.wi * ex);
  return rx * rx + ry * ry <= lim;
}

std::string run_pair(const Job& J, int32_t e) {
  const int32_t p = J.idx ? J.idx[e] : e;
  const int32_t qi = J.pairs[2 * p], di = J.pairs[2 * p + 1];
  const int32_t nq = J.n_feats[qi], nd = J.n_feats[di];
  const int64_t o = J.offs[p];
  std::vector<int32_t> rows;
  std::vector<int64_t> P, Q;
  for (int32_t r = 0; r < nq; ++r) {
    const int32_t m = J.match[o + r];
    if (m < 0) continue;
    if (m >= nd) return "pair " + std::to_string(p) + ": db row out of range";
    const int64_t v[4] = {J.kp[qi][2 * (size_t)r], J.kp[qi][2 * (size_t)r + 1], J.kp[di][2 * (size_t)m],
                          J.kp[di][2 * (size_t)m + 1]};
    for (int64_t c : v)
      if (c <= -kRansacCoordLimit || c >= kRansacCoordLimit)
        return "pair " + std::to_string(p) + ": keypoint coordinate out of range";
    rows.push_back(r);
    P.push_back(v[0]);
    P.push_back(v[1]);
    Q.push_back(v[2]);
    Q.push_back(v[3]);
  }
  const int M = (int)rows.size();
  std::vector<int32_t> res((size_t)nq, -1);
  int best = -1, bi = -1, bj = -1;
  if (M >= 2) {
    const uint32_t* w = J.words + (size_t)p * (size_t)J.iterations * 2;
    for (int32_t t = 0; t < J.iterations; ++t) {
      const int i = (int)(w[2 * t] % (uint32_t)M);
      int j = (int)(w[2 * t + 1] % (uint32_t)(M - 1));
      if (j >= i) ++j;
      Sim s;
      if (!make_sim(P, Q, i, j, &s)) continue;
      const i128 lim = (i128)s.D * s.D * J.thr * J.thr;
      int c = 0;
      for (int k = 0; k < M; ++k) c += inlier(s, P, Q, k, lim) ? 1 : 0;
      if (c > best) {
        best = c;
        bi = i;
        bj = j;
      }
    }
  }
  if (bi >= 0 && best >= J.min_inliers) {
    Sim s;
    make_sim(P, Q, bi, bj, &s);
    const i128 lim = (i128)s.D * s.D * J.thr * J.thr;
    for (int k = 0; k < M; ++k)
      if (inlier(s, P, Q, k, lim)) res[(size_t)rows[(size_t)k]] = J.match[o + rows[(size_t)k]];
  }
  std::copy(res.begin(), res.end(), J.out + o);
  if (J.best_counts) J.best_counts[p] = std::max(best, 0);
  return std::string();
}

std::string run_jobs(const Job& J, int32_t n_pairs, int32_t n_threads);

}  // namespace

using chm::clear_error;
using chm::fail;

extern "C" chm_status chm_ransac_filter(int32_t n_pairs, const int32_t* h_pairs, const int32_t* const* h_kp,
                                        const int32_t* h_n_feats, int32_t n_images, const int64_t* h_offs,
                                        const int32_t* h_match, const uint32_t* h_words, int32_t iterations,
                                        int32_t thr, int32_t min_inliers, int32_t n_threads, int32_t* h_out,
                                        int32_t* h_best_counts) {
  clear_error();
  if (n_pairs < 0 || n_images < 0 || iterations < 0) return fail(CHM_E_INVALID_ARG, "negative count");
  if (n_pairs == 0) return CHM_OK;
  if (!h_pairs || !h_kp || !h_n_feats || !h_offs || !h_match || !h_out || (iterations > 0 && !h_words))
    return fail(CHM_E_INVALID_ARG, "NULL array");
  if (thr < 0 || thr >= kRansacThrLimit) return fail(CHM_E_INVALID_ARG, "thr must be 0..2^20-1");
  for (int32_t p = 0; p < n_pairs; ++p) {
    const int32_t q = h_pairs[2 * p], d = h_pairs[2 * p + 1];
    if (q < 0 || q >= n_images || d < 0 || d >= n_images)
      return fail(CHM_E_INVALID_ARG, "pair %d names an image outside 0..%d", p, n_images - 1);
    if (h_n_feats[q] < 0 || h_n_feats[d] < 0) return fail(CHM_E_INVALID_ARG, "negative row count");
    if ((h_n_feats[q] > 0 && !h_kp[q]) || (h_n_feats[d] > 0 && !h_kp[d]))
      return fail(CHM_E_INVALID_ARG, "pair %d: NULL keypoints", p);
    if (h_offs[p] < 0 || h_offs[p + 1] - h_offs[p] != h_n_feats[q])
      return fail(CHM_E_INVALID_ARG, "pair %d: offsets do not span the query image's rows", p);
  }
  const Job J{nullptr, h_pairs, h_kp, h_n_feats, h_offs, h_match, h_words, iterations, thr, min_inliers, h_out,
              h_best_counts};
  const std::string err = run_jobs(J, n_pairs, n_threads);
  if (!err.empty()) return fail(CHM_E_INVALID_ARG, "%s", err.c_str());
  return CHM_OK;
}

std::string chm::ransac_pairs(int32_t n, const int32_t* idx, const int32_t* h_pairs, const int32_t* const* h_kp,
                              const int32_t* h_n_feats, const int64_t* h_starts, const int32_t* h_match,
                              const uint32_t* h_words, int32_t iterations, int32_t thr, int32_t min_inliers,
                              int32_t n_threads, int32_t* h_out) {
  const Job J{idx, h_pairs, h_kp, h_n_feats, h_starts, h_match, h_words, iterations, thr, min_inliers, h_out,
              nullptr};
  return run_jobs(J, n, n_threads);
}

namespace {
std::string run_jobs(const Job& J, int32_t n_pairs, int32_t n_threads) {
  int T = n_threads > 0 ? n_threads : (int)std::thread::hardware_concurrency();
  T = std::max(1, std::min(T, n_pairs));
  std::atomic<int32_t> next{0};
  std::mutex mu;
  std::string err;
  auto worker = [&]() {
    for (;;) {
      const int32_t p = next.fetch_add(1);
      if (p >= n_pairs) return;
      std::string e = run_pair(J, p);
      if (!e.empty()) {
        std::lock_guard<std::mutex> lk(mu);
        if (err.empty()) err = e;
      }
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < T; ++t) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
  return err;
}
}  // namespace
