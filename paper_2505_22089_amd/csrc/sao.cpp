// SAO local geometric constraint (Sec. 2.3.3, Fig. 4) on host threads.
//
// For an initial match i -> m(i) of a directed pair, the N nearest other
// matches around its keypoint in the query image and around m(i)'s keypoint
// in the db image are put in angular order; the cyclic edit distance between
// the two orders (as sequences of match labels, the query rows) divided by N
// is the match's dissimilarity.  Matches whose neighbourhoods are laid out
// alike in both images score low.
//
// Neighbours come from a uniform grid over the pair's matched keypoints in
// each image (about two points per cell), searched ring by ring until no
// unvisited cell can hold a nearer point.  Distances, angular comparisons
// (half-plane, then the sign of the cross product) and the edit distance are
// exact integer arithmetic, so the result does not depend on the search
// order.  The cyclic edit distance rotates one sequence only: the least
// distance over rotations of both equals the least over rotations of one
// (Maes, 1990).  Pairs are dealt to worker threads through an atomic counter.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "chm.h"
#include "chm_host.h"

namespace {

constexpr int kMaxNeighbors = 32;
constexpr int64_t kCoordLimit = int64_t(1) << 30;
constexpr int64_t kSqrtInt64Max = 3037000499LL;  // floor(sqrt(2^63 - 1))

struct Pt {
  int64_t x, y;
  int32_t label;
};

struct Near {
  int64_t d2;
  int32_t label;
  int32_t idx;
};

inline bool near_less(const Near& a, const Near& b) {
  return a.d2 != b.d2 ? a.d2 < b.d2 : a.label < b.label;
}

class Grid {
 public:
  void build(const std::vector<Pt>& pts) {
    pts_ = &pts;
    const int64_t M = (int64_t)pts.size();
    int64_t x1 = INT64_MIN, y1 = INT64_MIN;
    x0_ = y0_ = INT64_MAX;
    for (const Pt& p : pts) {
      x0_ = std::min(x0_, p.x);
      y0_ = std::min(y0_, p.y);
      x1 = std::max(x1, p.x);
      y1 = std::max(y1, p.y);
    }
    if (M == 0) x0_ = y0_ = x1 = y1 = 0;
    const double w = double(x1 - x0_) + 1.0, h = double(y1 - y0_) + 1.0;
    cell_ = std::max<int64_t>(1, (int64_t)std::ceil(std::sqrt(w * h * 2.0 / double(std::max<int64_t>(M, 1)))));
    for (;;) {  // thin or sparse layouts: coarser cells until their count is O(M)
      nx_ = (x1 - x0_) / cell_ + 1;
      ny_ = (y1 - y0_) / cell_ + 1;
      if ((double)nx_ * (double)ny_ <= 4.0 * (double)M + 64.0) break;
      cell_ *= 2;
    }
    start_.assign((size_t)(nx_ * ny_ + 1), 0);
    std::vector<int64_t> cell_of(pts.size());
    for (size_t k = 0; k < pts.size(); ++k) {
      cell_of[k] = ((pts[k].y - y0_) / cell_) * nx_ + (pts[k].x - x0_) / cell_;
      ++start_[(size_t)cell_of[k] + 1];
    }
    for (size_t c = 1; c < start_.size(); ++c) start_[c] += start_[c - 1];
    order_.resize(pts.size());
    std::vector<int32_t> fill(start_.begin(), start_.end() - 1);
    for (size_t k = 0; k < pts.size(); ++k) order_[(size_t)fill[(size_t)cell_of[k]]++] = (int32_t)k;
  }

  // The n nearest points to (x, y), one of the grid's points, other than
  // those labelled `own`, ascending by (squared distance, label).
  void nearest(int64_t x, int64_t y, int32_t own, int n, std::vector<Near>& best) const {
    best.clear();
    if (n <= 0) return;
    const int64_t ix = (x - x0_) / cell_, iy = (y - y0_) / cell_;
    const int64_t rmax = std::max(std::max(ix, nx_ - 1 - ix), std::max(iy, ny_ - 1 - iy));
    for (int64_t r = 0; r <= rmax; ++r) {
      for (int64_t j = iy - r; j <= iy + r; ++j) {
        if (j < 0 || j >= ny_) continue;
        if (r == 0 || j == iy - r || j == iy + r) {
          for (int64_t i = std::max<int64_t>(0, ix - r); i <= std::min(nx_ - 1, ix + r); ++i)
            scan(i, j, x, y, own, n, best);
        } else {
          if (ix - r >= 0) scan(ix - r, j, x, y, own, n, best);
          if (ix + r < nx_) scan(ix + r, j, x, y, own, n, best);
        }
      }
      // every point outside rings 0..r is farther than r cells from (x, y)
      if ((int)best.size() == n) {
        const int64_t lb = r * cell_;
        if (lb > kSqrtInt64Max || lb * lb >= best.back().d2) break;
      }
    }
  }

 private:
  void scan(int64_t i, int64_t j, int64_t x, int64_t y, int32_t own, int n,
            std::vector<Near>& best) const {
    const size_t c = (size_t)(j * nx_ + i);
    for (int32_t k = start_[c]; k < start_[c + 1]; ++k) {
      const Pt& p = (*pts_)[(size_t)order_[(size_t)k]];
      if (p.label == own) continue;
      const int64_t dx = p.x - x, dy = p.y - y;
      const Near cand{dx * dx + dy * dy, p.label, order_[(size_t)k]};
      if ((int)best.size() == n && !near_less(cand, best.back())) continue;
      if ((int)best.size() == n) best.pop_back();
      best.insert(std::upper_bound(best.begin(), best.end(), cand, near_less), cand);
    }
  }

  const std::vector<Pt>* pts_ = nullptr;
  int64_t x0_ = 0, y0_ = 0, cell_ = 1, nx_ = 1, ny_ = 1;
  std::vector<int32_t> start_, order_;
};

struct Polar {
  int64_t dx, dy, d2;
  int32_t label;
};

inline int half_plane(const Polar& v) {
  if (v.dx == 0 && v.dy == 0) return -1;
  return (v.dy > 0 || (v.dy == 0 && v.dx > 0)) ? 0 : 1;
}

// counter-clockwise from +x; the centre itself first; then distance, label
inline bool angle_less(const Polar& u, const Polar& v) {
  const int hu = half_plane(u), hv = half_plane(v);
  if (hu != hv) return hu < hv;
  if (hu >= 0) {
    const int64_t cross = u.dx * v.dy - u.dy * v.dx;
    if (cross != 0) return cross > 0;
  }
  if (u.d2 != v.d2) return u.d2 < v.d2;
  return u.label < v.label;
}

// Levenshtein distance (unit costs) of two sequences of length n.
inline int levenshtein(const int32_t* a, const int32_t* b, int n) {
  int row[kMaxNeighbors + 1];
  for (int j = 0; j <= n; ++j) row[j] = j;
  for (int i = 1; i <= n; ++i) {
    int diag = row[0];
    row[0] = i;
    for (int j = 1; j <= n; ++j) {
      const int up = row[j];
      row[j] = std::min(std::min(up + 1, row[j - 1] + 1), diag + (a[i - 1] != b[j - 1] ? 1 : 0));
      diag = up;
    }
  }
  return row[n];
}

inline int cyclic_edit_distance(const int32_t* a, const int32_t* b, int n) {
  if (n == 0) return 0;
  int32_t bb[2 * kMaxNeighbors];
  for (int k = 0; k < n; ++k) bb[k] = bb[k + n] = b[k];
  int best = n;
  for (int s = 0; s < n && best > 0; ++s) best = std::min(best, levenshtein(a, bb + s, n));
  return best;
}

struct Job {
  int32_t n_pairs;
  const int32_t* pairs;
  const int32_t* const* kp;
  const int32_t* n_feats;
  const int64_t* offs;
  const int32_t* match;
  int n_neighbors;
  int64_t num, den;
  int32_t* out;
  int32_t* ced;
};

// Neighbour labels of point a in angular order around it.
void ordered_neighbours(const Grid& g, const std::vector<Pt>& pts, size_t a, int n,
                        std::vector<Near>& tmp, std::vector<Polar>& pol, int32_t* labels) {
  g.nearest(pts[a].x, pts[a].y, pts[a].label, n, tmp);
  pol.clear();
  for (const Near& e : tmp) {
    const Pt& p = pts[(size_t)e.idx];
    pol.push_back({p.x - pts[a].x, p.y - pts[a].y, e.d2, e.label});
  }
  std::sort(pol.begin(), pol.end(), angle_less);
  for (size_t k = 0; k < pol.size(); ++k) labels[k] = pol[k].label;
}

// One pair; returns an empty string or what was wrong with its input.
std::string run_pair(const Job& J, int32_t p) {
  const int32_t qi = J.pairs[2 * p], di = J.pairs[2 * p + 1];
  const int32_t nq = J.n_feats[qi], nd = J.n_feats[di];
  const int32_t* kq = J.kp[qi];
  const int32_t* kd = J.kp[di];
  const int64_t o = J.offs[p];
  std::vector<int32_t> rows;
  for (int32_t i = 0; i < nq; ++i) {
    const int32_t m = J.match[o + i];
    if (m < 0) continue;
    if (m >= nd) return "pair " + std::to_string(p) + ": db row out of range";
    rows.push_back(i);
  }
  std::vector<Pt> P(rows.size()), Q(rows.size());
  for (size_t a = 0; a < rows.size(); ++a) {
    const int32_t i = rows[a], m = J.match[o + i];
    P[a] = {kq[2 * (size_t)i], kq[2 * (size_t)i + 1], i};
    Q[a] = {kd[2 * (size_t)m], kd[2 * (size_t)m + 1], i};
    for (const Pt* t : {&P[a], &Q[a]})
      if (t->x <= -kCoordLimit || t->x >= kCoordLimit || t->y <= -kCoordLimit || t->y >= kCoordLimit)
        return "pair " + std::to_string(p) + ": keypoint coordinate out of range";
  }
  const int M = (int)rows.size();
  const int N = M > 0 ? std::min(J.n_neighbors, M - 1) : 0;
  Grid gp, gq;
  gp.build(P);
  gq.build(Q);
  std::vector<int32_t> res_out((size_t)nq, -1), res_ced((size_t)nq, -1);
  std::vector<Near> tmp;
  std::vector<Polar> pol;
  int32_t la[kMaxNeighbors], lb[kMaxNeighbors];
  for (size_t a = 0; a < rows.size(); ++a) {
    int c = 0;
    if (N > 0) {
      ordered_neighbours(gp, P, a, N, tmp, pol, la);
      ordered_neighbours(gq, Q, a, N, tmp, pol, lb);
      c = cyclic_edit_distance(la, lb, N);
    }
    const int32_t i = rows[a];
    res_ced[(size_t)i] = c;
    if ((int64_t)c * J.den <= J.num * N) res_out[(size_t)i] = J.match[o + i];
  }
  std::copy(res_out.begin(), res_out.end(), J.out + o);
  if (J.ced) std::copy(res_ced.begin(), res_ced.end(), J.ced + o);
  return std::string();
}

}  // namespace

using chm::clear_error;
using chm::fail;

extern "C" chm_status chm_sao_filter(int32_t n_pairs, const int32_t* h_pairs, const int32_t* const* h_kp,
                                     const int32_t* h_n_feats, int32_t n_images, const int64_t* h_offs,
                                     const int32_t* h_match, int32_t n_neighbors, int32_t score_num,
                                     int32_t score_den, int32_t n_threads, int32_t* h_out,
                                     int32_t* h_ced) {
  clear_error();
  if (n_pairs < 0 || n_images < 0) return fail(CHM_E_INVALID_ARG, "negative count");
  if (n_pairs == 0) return CHM_OK;
  if (!h_pairs || !h_kp || !h_n_feats || !h_offs || !h_match || !h_out)
    return fail(CHM_E_INVALID_ARG, "NULL array");
  if (n_neighbors < 1 || n_neighbors > kMaxNeighbors)
    return fail(CHM_E_INVALID_ARG, "n_neighbors must be 1..%d", kMaxNeighbors);
  if (score_num < 0 || score_den <= 0) return fail(CHM_E_INVALID_ARG, "bad score threshold");
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
  const Job J{n_pairs, h_pairs, h_kp, h_n_feats, h_offs, h_match, n_neighbors,
              score_num, score_den, h_out, h_ced};
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
  if (!err.empty()) return fail(CHM_E_INVALID_ARG, "%s", err.c_str());
  return CHM_OK;
}
