// MBR block schedule on the host (Sec. 2.2 steps (1)-(5), Algorithm 1,
// Gibbs-Poole-Stockmeyer ordering of Appendix A, Algorithm 2).
//
// Readings where the paper is silent:
//  - GPS runs per connected component (components in order of their
//    smallest id); self pairs are not edges of the ordering graph.
//  - Pseudo-peripheral pair: u = minimum (degree, id); v = minimum
//    (degree, id) of the last level of L(u); restart from v while L(v) is
//    deeper.
//  - Combined level structure: (i, j) = (level in L(u), depth - level in
//    L(v)); i == j fixes the level; the other nodes' components, largest
//    first (ties: smallest id), go wholly to their L(u) or reversed L(v)
//    levels, whichever gives the smaller maximum width over the levels they
//    add to (ties: the structure of smaller width, then L(u)).
//  - Numbering level by level: level 0 by (degree, id), level i by (smallest
//    number of a neighbour in level i-1, degree, id).
//  - Size_blk counts images; a segment closes early before it would exceed
//    half the cap; block row r is the window of segments r.. that fits the
//    cap and processes the remaining pairs with one end in segment r and the
//    other in the window; images load when first needed and everything
//    outside the window is freed first; an iteration that processes nothing
//    falls back to one pair per step.
#include <algorithm>
#include <climits>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <vector>

#include "chm.h"
#include "chm_host.h"

using namespace chm;

namespace {

typedef std::vector<std::vector<int>> Adj;

struct Levels {
  std::vector<std::vector<int>> lv;
};

Levels level_structure(const Adj& adj, int root, std::vector<int>& mark, int stamp) {
  Levels L;
  L.lv.push_back({root});
  mark[root] = stamp;
  for (;;) {
    std::vector<int> nxt;
    for (int w : L.lv.back())
      for (int x : adj[w])
        if (mark[x] != stamp) {
          mark[x] = stamp;
          nxt.push_back(x);
        }
    if (nxt.empty()) break;
    L.lv.push_back(std::move(nxt));
  }
  for (auto& l : L.lv) std::sort(l.begin(), l.end());
  return L;
}

int argmin_deg(const Adj& adj, const std::vector<int>& nodes) {
  int best = nodes[0];
  for (int w : nodes)
    if (adj[w].size() < adj[best].size() || (adj[w].size() == adj[best].size() && w < best)) best = w;
  return best;
}

size_t width(const Levels& L) {
  size_t w = 0;
  for (auto& l : L.lv) w = std::max(w, l.size());
  return w;
}

// Orders one connected component (comp sorted ascending, size >= 2).
void gps_component(const Adj& adj, const std::vector<int>& comp, std::vector<int>& mark,
                   int& stamp, std::vector<int>& number, std::vector<int>& order) {
  int u = argmin_deg(adj, comp);
  Levels Lu = level_structure(adj, u, mark, ++stamp);
  Levels Lv;
  for (;;) {
    const int v = argmin_deg(adj, Lu.lv.back());
    Lv = level_structure(adj, v, mark, ++stamp);
    if (Lv.lv.size() > Lu.lv.size()) {
      u = v;
      Lu = Lv;
      continue;
    }
    break;
  }
  const int k = (int)Lu.lv.size() - 1;
  std::map<int, int> li, lj;
  for (int i = 0; i <= k; ++i)
    for (int w : Lu.lv[i]) li[w] = i;
  for (int i = 0; i < (int)Lv.lv.size(); ++i)
    for (int w : Lv.lv[i]) lj[w] = k - i;
  std::vector<int> widthv(k + 1, 0);
  std::map<int, int> level;
  for (int w : comp)
    if (li[w] == lj[w]) {
      level[w] = li[w];
      widthv[li[w]] += 1;
    }
  std::vector<int> rest;
  for (int w : comp)
    if (!level.count(w)) rest.push_back(w);
  std::set<int> rest_set(rest.begin(), rest.end());
  std::vector<std::vector<int>> comps;
  std::set<int> seen;
  for (int s : rest) {
    if (seen.count(s)) continue;
    seen.insert(s);
    std::vector<int> c;
    std::deque<int> dq{s};
    while (!dq.empty()) {
      const int w = dq.front();
      dq.pop_front();
      c.push_back(w);
      for (int x : adj[w])
        if (rest_set.count(x) && !seen.count(x)) {
          seen.insert(x);
          dq.push_back(x);
        }
    }
    std::sort(c.begin(), c.end());
    comps.push_back(std::move(c));
  }
  std::stable_sort(comps.begin(), comps.end(), [](const std::vector<int>& a, const std::vector<int>& b) {
    if (a.size() != b.size()) return a.size() > b.size();
    return a[0] < b[0];
  });
  const size_t wu = width(Lu), wv = width(Lv);
  for (auto& c : comps) {
    std::vector<int> ai(k + 1, 0), aj(k + 1, 0);
    for (int w : c) {
      ai[li[w]] += 1;
      aj[lj[w]] += 1;
    }
    int h0 = -1, l0 = -1;
    for (int i = 0; i <= k; ++i) {
      if (ai[i] > 0) h0 = std::max(h0, widthv[i] + ai[i]);
      if (aj[i] > 0) l0 = std::max(l0, widthv[i] + aj[i]);
    }
    const bool use_u = h0 < l0 || (h0 == l0 && wu <= wv);
    for (int w : c) {
      const int lv = use_u ? li[w] : lj[w];
      level[w] = lv;
      widthv[lv] += 1;
    }
  }
  std::vector<std::vector<int>> levels(k + 1);
  for (int w : comp) levels[level[w]].push_back(w);
  for (int i = 0; i <= k; ++i) {
    std::vector<int>& lev = levels[i];
    if (i == 0) {
      std::sort(lev.begin(), lev.end(), [&](int a, int b) {
        if (adj[a].size() != adj[b].size()) return adj[a].size() < adj[b].size();
        return a < b;
      });
    } else {
      std::set<int> prev(levels[i - 1].begin(), levels[i - 1].end());
      std::map<int, int> key;
      for (int w : lev) {
        int best = INT_MAX;
        for (int x : adj[w])
          if (prev.count(x)) best = std::min(best, number[x]);
        key[w] = best;
      }
      std::sort(lev.begin(), lev.end(), [&](int a, int b) {
        if (key[a] != key[b]) return key[a] < key[b];
        if (adj[a].size() != adj[b].size()) return adj[a].size() < adj[b].size();
        return a < b;
      });
    }
    for (int w : lev) {
      number[w] = (int)order.size();
      order.push_back(w);
    }
  }
}

// GPS order of `nodes` (any order) in the graph given by adj (restricted to nodes).
std::vector<int> gps_order(int n, const Adj& full, std::vector<int> nodes) {
  std::sort(nodes.begin(), nodes.end());
  nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
  std::vector<char> in(n, 0);
  for (int w : nodes) in[w] = 1;
  Adj adj(n);
  for (int w : nodes)
    for (int x : full[w])
      if (in[x]) adj[w].push_back(x);
  std::vector<int> mark(n, 0), number(n, -1), order;
  int stamp = 0;
  std::vector<char> seen(n, 0);
  for (int s : nodes) {
    if (seen[s]) continue;
    std::vector<int> comp{s};
    seen[s] = 1;
    std::deque<int> dq{s};
    while (!dq.empty()) {
      const int w = dq.front();
      dq.pop_front();
      for (int x : adj[w])
        if (!seen[x]) {
          seen[x] = 1;
          comp.push_back(x);
          dq.push_back(x);
        }
    }
    std::sort(comp.begin(), comp.end());
    if (comp.size() == 1) {
      number[comp[0]] = (int)order.size();
      order.push_back(comp[0]);
      continue;
    }
    gps_component(adj, comp, mark, stamp, number, order);
  }
  return order;
}

Adj adjacency(int n, const std::vector<std::pair<int, int>>& edges) {
  std::vector<std::set<int>> nb(n);
  for (auto& e : edges)
    if (e.first != e.second) {
      nb[e.first].insert(e.second);
      nb[e.second].insert(e.first);
    }
  Adj adj(n);
  for (int i = 0; i < n; ++i) adj[i].assign(nb[i].begin(), nb[i].end());
  return adj;
}

}  // namespace

struct chm_schedule {
  std::vector<std::vector<int32_t>> evict, load, pairs;
  std::vector<int32_t> dims, bws;
  int32_t iterations = 0;
  int32_t fallback = 0;
};

extern "C" chm_status chm_gps_order(int32_t n, const int32_t* edges, int32_t n_edges,
                                    const int32_t* nodes, int32_t n_nodes, int32_t* order_out) {
  clear_error();
  if (n < 0 || n_edges < 0 || n_nodes < 0) return fail(CHM_E_INVALID_ARG, "negative size");
  if ((n_edges && !edges) || (n_nodes && (!nodes || !order_out)))
    return fail(CHM_E_INVALID_ARG, "NULL argument");
  std::vector<std::pair<int, int>> e;
  for (int i = 0; i < n_edges; ++i) {
    const int a = edges[2 * i], b = edges[2 * i + 1];
    if (a < 0 || a >= n || b < 0 || b >= n) return fail(CHM_E_INVALID_ARG, "edge %d out of range", i);
    e.push_back({a, b});
  }
  std::vector<int> nd(nodes, nodes + n_nodes);
  std::set<int> uniq;
  for (int w : nd) {
    if (w < 0 || w >= n) return fail(CHM_E_INVALID_ARG, "node %d out of range", w);
    if (!uniq.insert(w).second) return fail(CHM_E_INVALID_ARG, "node %d listed twice", w);
  }
  const std::vector<int> ord = gps_order(n, adjacency(n, e), nd);
  std::copy(ord.begin(), ord.end(), order_out);
  return CHM_OK;
}

extern "C" chm_status chm_schedule_mbr(int32_t n_images, const int32_t* pairs, int32_t P,
                                       const uint64_t* image_bytes, uint64_t cap, int32_t blk,
                                       chm_schedule** out) {
  clear_error();
  if (!out) return fail(CHM_E_INVALID_ARG, "out is NULL");
  if (n_images < 0 || P < 0 || (P && !pairs) || (n_images && !image_bytes))
    return fail(CHM_E_INVALID_ARG, "bad arguments");
  if (blk < 1) return fail(CHM_E_INVALID_ARG, "blk_images must be >= 1");
  for (int p = 0; p < P; ++p) {
    const int a = pairs[2 * p], b = pairs[2 * p + 1];
    if (a < 0 || a >= n_images || b < 0 || b >= n_images)
      return fail(CHM_E_INVALID_ARG, "pair %d references an image out of range", p);
    const uint64_t need = image_bytes[a] + (a != b ? image_bytes[b] : 0);
    if (need > cap) return fail(CHM_E_CAPACITY, "pair %d does not fit in the cap", p);
  }
  chm_schedule* S = new chm_schedule();
  std::map<std::pair<int, int>, std::vector<int32_t>> cell_pairs;
  for (int p = 0; p < P; ++p) {
    const int a = pairs[2 * p], b = pairs[2 * p + 1];
    cell_pairs[{std::min(a, b), std::max(a, b)}].push_back(p);
  }
  std::set<std::pair<int, int>> remaining;
  for (auto& c : cell_pairs) remaining.insert(c.first);
  std::vector<int> resident;
  std::vector<int> pos(n_images, -1);

  while (!remaining.empty()) {
    S->iterations += 1;
    std::set<int> act;
    for (auto& c : remaining) {
      act.insert(c.first);
      act.insert(c.second);
    }
    std::vector<int> active(act.begin(), act.end());
    S->dims.push_back((int32_t)active.size());
    std::vector<std::pair<int, int>> edges(remaining.begin(), remaining.end());
    const Adj adj = adjacency(n_images, edges);
    const std::vector<int> order = gps_order(n_images, adj, active);
    std::fill(pos.begin(), pos.end(), -1);
    for (int i = 0; i < (int)order.size(); ++i) pos[order[i]] = i;
    int bw = 0;
    for (auto& c : edges) bw = std::max(bw, std::abs(pos[c.first] - pos[c.second]));
    S->bws.push_back(bw);

    std::vector<std::pair<int, int>> seg;
    std::vector<int> seg_of(order.size());
    {
      int start = 0;
      uint64_t nbytes = 0;
      for (int i = 0; i < (int)order.size(); ++i) {
        const uint64_t b = image_bytes[order[i]];
        if (i > start && (i - start == blk || 2 * (nbytes + b) > cap)) {
          seg.push_back({start, i});
          start = i;
          nbytes = 0;
        }
        nbytes += b;
      }
      seg.push_back({start, (int)order.size()});
    }
    std::vector<uint64_t> seg_bytes(seg.size(), 0);
    for (size_t si = 0; si < seg.size(); ++si)
      for (int i = seg[si].first; i < seg[si].second; ++i) {
        seg_bytes[si] += image_bytes[order[i]];
        seg_of[i] = (int)si;
      }
    std::vector<std::vector<std::pair<int, int>>> by_seg(seg.size());
    for (auto& c : edges) by_seg[seg_of[std::min(pos[c.first], pos[c.second])]].push_back(c);

    int processed = 0;
    for (size_t r = 0; r < seg.size(); ++r) {
      size_t e = r;
      uint64_t tot = seg_bytes[r];
      while (e + 1 < seg.size() && tot + seg_bytes[e + 1] <= cap) {
        ++e;
        tot += seg_bytes[e];
      }
      const int lo = seg[r].first, hi = seg[e].second;
      std::vector<std::pair<int, int>> cells;
      for (auto& c : by_seg[r])
        if (pos[c.first] >= lo && pos[c.first] < hi && pos[c.second] >= lo && pos[c.second] < hi)
          cells.push_back(c);
      if (cells.empty()) continue;
      std::vector<int> keep, ev;
      for (int w : resident) {
        if (pos[w] >= lo && pos[w] < hi) keep.push_back(w);
        else ev.push_back(w);
      }
      std::sort(ev.begin(), ev.end());
      std::set<int> need;
      for (auto& c : cells) {
        need.insert(c.first);
        need.insert(c.second);
      }
      std::set<int> kset(keep.begin(), keep.end());
      std::vector<int32_t> ld;
      for (int w : need)
        if (!kset.count(w)) ld.push_back(w);
      resident = keep;
      resident.insert(resident.end(), ld.begin(), ld.end());
      std::vector<int32_t> pp;
      for (auto& c : cells)
        for (int32_t p : cell_pairs[c]) pp.push_back(p);
      std::sort(pp.begin(), pp.end());
      S->evict.push_back(std::vector<int32_t>(ev.begin(), ev.end()));
      S->load.push_back(ld);
      S->pairs.push_back(pp);
      for (auto& c : cells) remaining.erase(c);
      processed += (int)cells.size();
    }
    if (processed == 0) {
      for (auto& c : remaining) {
        std::set<int> need{c.first, c.second};
        std::vector<int> keep, ev;
        for (int w : resident) {
          if (need.count(w)) keep.push_back(w);
          else ev.push_back(w);
        }
        std::sort(ev.begin(), ev.end());
        std::set<int> kset(keep.begin(), keep.end());
        std::vector<int32_t> ld;
        for (int w : need)
          if (!kset.count(w)) ld.push_back(w);
        resident = keep;
        resident.insert(resident.end(), ld.begin(), ld.end());
        std::vector<int32_t> pp = cell_pairs[c];
        std::sort(pp.begin(), pp.end());
        S->fallback += (int32_t)pp.size();
        S->evict.push_back(std::vector<int32_t>(ev.begin(), ev.end()));
        S->load.push_back(ld);
        S->pairs.push_back(pp);
      }
      remaining.clear();
    }
  }
  *out = S;
  return CHM_OK;
}

extern "C" chm_status chm_schedule_from_steps(int32_t n_images, int32_t n_pairs, const int32_t* pairs,
                                              const uint64_t* image_bytes, uint64_t cap_bytes, int32_t n_steps,
                                              const int32_t* evict_offs, const int32_t* evict_ids,
                                              const int32_t* load_offs, const int32_t* load_ids,
                                              const int32_t* pair_offs, const int32_t* pair_ids,
                                              chm_schedule** out) {
  clear_error();
  if (n_images < 0 || n_pairs < 0 || n_steps < 0) return fail(CHM_E_INVALID_ARG, "negative size");
  if (!out || !evict_offs || !load_offs || !pair_offs || (n_pairs && !pairs) || (n_images && !image_bytes))
    return fail(CHM_E_INVALID_ARG, "NULL argument");
  if (evict_offs[0] != 0 || load_offs[0] != 0 || pair_offs[0] != 0)
    return fail(CHM_E_INVALID_ARG, "step offsets must start at 0");
  for (int k = 0; k < n_steps; ++k)
    if (evict_offs[k + 1] < evict_offs[k] || load_offs[k + 1] < load_offs[k] || pair_offs[k + 1] < pair_offs[k])
      return fail(CHM_E_INVALID_ARG, "step %d: decreasing offsets", k);
  if ((evict_offs[n_steps] && !evict_ids) || (load_offs[n_steps] && !load_ids) || (pair_offs[n_steps] && !pair_ids))
    return fail(CHM_E_INVALID_ARG, "NULL argument");
  for (int p = 0; p < n_pairs; ++p)
    if (pairs[2 * p] < 0 || pairs[2 * p] >= n_images || pairs[2 * p + 1] < 0 || pairs[2 * p + 1] >= n_images)
      return fail(CHM_E_INVALID_ARG, "pair %d names an image outside 0..%d", p, n_images - 1);
  // replay the residency: evictions of resident images, loads of absent
  // ones, the cap after each step's loads, every pair once with both images
  // resident
  std::vector<char> res(n_images, 0), done(n_pairs, 0);
  uint64_t used = 0;
  chm_schedule* S = new chm_schedule();
  for (int k = 0; k < n_steps; ++k) {
    std::vector<int32_t> ev(evict_ids + evict_offs[k], evict_ids + evict_offs[k + 1]);
    std::vector<int32_t> ld(load_ids + load_offs[k], load_ids + load_offs[k + 1]);
    std::vector<int32_t> pp(pair_ids + pair_offs[k], pair_ids + pair_offs[k + 1]);
    const char* err = nullptr;
    int bad = -1;
    for (int32_t i : ev) {
      if (i < 0 || i >= n_images || !res[i]) {
        err = "evicts an image that is not resident";
        bad = i;
        break;
      }
      res[i] = 0;
      used -= image_bytes[i];
    }
    for (size_t x = 0; !err && x < ld.size(); ++x) {
      const int32_t i = ld[x];
      if (i < 0 || i >= n_images || res[i]) {
        err = "loads an image that is resident or out of range";
        bad = i;
        break;
      }
      res[i] = 1;
      used += image_bytes[i];
    }
    if (!err && used > cap_bytes) err = "exceeds the cap";
    for (size_t x = 0; !err && x < pp.size(); ++x) {
      const int32_t p = pp[x];
      if (p < 0 || p >= n_pairs || done[p]) {
        err = "lists a pair out of range or twice";
        bad = p;
      } else if (!res[pairs[2 * p]] || !res[pairs[2 * p + 1]]) {
        err = "lists a pair whose images are not resident";
        bad = p;
      } else {
        done[p] = 1;
      }
    }
    if (err) {
      delete S;
      return fail(CHM_E_INVALID_ARG, "step %d %s (%d)", k, err, bad);
    }
    S->evict.push_back(std::move(ev));
    S->load.push_back(std::move(ld));
    S->pairs.push_back(std::move(pp));
  }
  for (int p = 0; p < n_pairs; ++p)
    if (!done[p]) {
      delete S;
      return fail(CHM_E_INVALID_ARG, "pair %d is in no step", p);
    }
  *out = S;
  return CHM_OK;
}

extern "C" int32_t chm_schedule_num_steps(const chm_schedule* s) {
  return s ? (int32_t)s->pairs.size() : 0;
}

extern "C" chm_status chm_schedule_step(const chm_schedule* s, int32_t k, const int32_t** ev,
                                        int32_t* nev, const int32_t** ld, int32_t* nld,
                                        const int32_t** pp, int32_t* np) {
  clear_error();
  if (!s || k < 0 || k >= (int32_t)s->pairs.size()) return fail(CHM_E_INVALID_ARG, "bad step");
  if (ev) *ev = s->evict[k].data();
  if (nev) *nev = (int32_t)s->evict[k].size();
  if (ld) *ld = s->load[k].data();
  if (nld) *nld = (int32_t)s->load[k].size();
  if (pp) *pp = s->pairs[k].data();
  if (np) *np = (int32_t)s->pairs[k].size();
  return CHM_OK;
}

extern "C" chm_status chm_schedule_info(const chm_schedule* s, int32_t* iterations,
                                        int32_t* fallback, const int32_t** dims,
                                        const int32_t** bws) {
  clear_error();
  if (!s) return fail(CHM_E_INVALID_ARG, "schedule is NULL");
  if (iterations) *iterations = s->iterations;
  if (fallback) *fallback = s->fallback;
  if (dims) *dims = s->dims.data();
  if (bws) *bws = s->bws.data();
  return CHM_OK;
}

extern "C" void chm_schedule_free(chm_schedule* s) { delete s; }
