// Host planner: greedy elimination orders on the line graph (Section V-A)
// and the step-dependent slicing search (Section VI-C, VI-D).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <limits>
#include <random>
#include <thread>

#include "qt_internal.h"

namespace qt {
namespace {

// Line graph with bitset rows: vertex = variable, tensor = clique.
struct Graph {
  int V = 0, W = 0;
  std::vector<uint64_t> adj;  // V rows of W words
  std::vector<char> alive;
  std::vector<int> deg;

  uint64_t* row(int v) { return adj.data() + (size_t)v * W; }
  const uint64_t* row(int v) const { return adj.data() + (size_t)v * W; }
  bool has(int u, int v) const { return (row(u)[v >> 6] >> (v & 63)) & 1; }

  void init(int nv) {
    V = nv;
    W = (nv + 63) / 64;
    adj.assign((size_t)V * W, 0);
    alive.assign(V, 1);
    deg.assign(V, 0);
  }
  void add_clique(const std::vector<int32_t>& vs) {
    for (int a : vs)
      for (int b : vs)
        if (a != b) row(a)[b >> 6] |= 1ull << (b & 63);
  }
  void recount() {
    for (int v = 0; v < V; ++v) deg[v] = alive[v] ? count(v) : 0;
  }
  int count(int v) const {
    int c = 0;
    const uint64_t* r = row(v);
    for (int w = 0; w < W; ++w) c += __builtin_popcountll(r[w]);
    return c;
  }
  template <class F>
  void for_nbrs(int v, F f) const {
    const uint64_t* r = row(v);
    for (int w = 0; w < W; ++w) {
      uint64_t m = r[w];
      while (m) {
        int b = __builtin_ctzll(m);
        m &= m - 1;
        f(w * 64 + b);
      }
    }
  }
  // Vertex elimination: connect the neighbours, remove v (Section IV-B).
  void eliminate(int v) {
    std::vector<int> nb;
    for_nbrs(v, [&](int u) { nb.push_back(u); });
    const uint64_t* rv = row(v);
    for (int u : nb) {
      uint64_t* ru = row(u);
      for (int w = 0; w < W; ++w) ru[w] |= rv[w];
      ru[u >> 6] &= ~(1ull << (u & 63));
      ru[v >> 6] &= ~(1ull << (v & 63));
      deg[u] = count(u);
    }
    std::memset(row(v), 0, sizeof(uint64_t) * W);
    alive[v] = 0;
    deg[v] = 0;
  }
  // Deletion without fill (slicing a variable, Section VI-C).
  void remove(int v) {
    for_nbrs(v, [&](int u) {
      row(u)[v >> 6] &= ~(1ull << (v & 63));
      deg[u] -= 1;
    });
    std::memset(row(v), 0, sizeof(uint64_t) * W);
    alive[v] = 0;
    deg[v] = 0;
  }
  // Number of edges missing among the neighbours of v.
  int64_t fill(int v) const {
    const uint64_t* rv = row(v);
    int64_t d = deg[v];
    int64_t inside = 0;
    for_nbrs(v, [&](int u) {
      const uint64_t* ru = row(u);
      for (int w = 0; w < W; ++w) inside += __builtin_popcountll(ru[w] & rv[w]);
    });
    return d * (d - 1) / 2 - inside / 2;
  }
};

Graph build_graph(const qt_network& net) {
  Graph g;
  g.init(net.n_vars());
  for (const auto& l : net.leaves) g.add_clique(l.vars);
  g.recount();
  return g;
}

// Greedy order of the alive vertices; returns the neighbour count of each
// vertex at its elimination (its step width).
void greedy(Graph g, int algo, double tau, uint64_t seed, std::vector<int32_t>& order,
            std::vector<int32_t>& widths) {
  order.clear();
  widths.clear();
  std::vector<int64_t> fl;
  std::vector<char> dirty;
  if (algo == QT_ORDER_MIN_FILL) {
    fl.assign(g.V, 0);
    for (int v = 0; v < g.V; ++v)
      if (g.alive[v]) fl[v] = g.fill(v);
    dirty.assign(g.V, 0);
  }
  std::mt19937_64 rng(seed);
  std::vector<double> wts;
  std::vector<int> cand;
  int n_alive = 0;
  for (int v = 0; v < g.V; ++v) n_alive += g.alive[v];
  for (int it = 0; it < n_alive; ++it) {
    int best = -1;
    if (algo == QT_ORDER_MIN_DEGREE) {
      for (int v = 0; v < g.V; ++v)
        if (g.alive[v] && (best < 0 || g.deg[v] < g.deg[best])) best = v;
    } else if (algo == QT_ORDER_MIN_FILL) {
      for (int v = 0; v < g.V; ++v) {
        if (!g.alive[v]) continue;
        if (best < 0 || fl[v] < fl[best] || (fl[v] == fl[best] && g.deg[v] < g.deg[best])) best = v;
      }
    } else {
      // Boltzmann weights exp(-N(v)/tau) (Section V-A2), shifted by the
      // minimum degree for range.
      int dmin = std::numeric_limits<int>::max();
      for (int v = 0; v < g.V; ++v)
        if (g.alive[v]) dmin = std::min(dmin, g.deg[v]);
      cand.clear();
      wts.clear();
      double tot = 0;
      for (int v = 0; v < g.V; ++v)
        if (g.alive[v]) {
          double w = std::exp(-(g.deg[v] - dmin) / tau);
          cand.push_back(v);
          wts.push_back(w);
          tot += w;
        }
      double r = std::uniform_real_distribution<double>(0.0, tot)(rng);
      best = cand.back();
      for (size_t i = 0; i < cand.size(); ++i) {
        r -= wts[i];
        if (r < 0) {
          best = cand[i];
          break;
        }
      }
    }
    order.push_back(best);
    widths.push_back(g.deg[best]);
    if (algo == QT_ORDER_MIN_FILL) {
      std::vector<int> nb;
      g.for_nbrs(best, [&](int u) { nb.push_back(u); });
      g.eliminate(best);
      for (int u : nb) {
        dirty[u] = 1;
        g.for_nbrs(u, [&](int w) { dirty[w] = 1; });
      }
      for (int v = 0; v < g.V; ++v)
        if (dirty[v]) {
          dirty[v] = 0;
          if (g.alive[v]) fl[v] = g.fill(v);
        }
    } else {
      g.eliminate(best);
    }
  }
}

int max_of(const std::vector<int32_t>& w, size_t b, size_t e) {
  int m = 0;
  for (size_t i = b; i < e; ++i) m = std::max(m, (int)w[i]);
  return m;
}

void best_greedy(const Graph& g, int algo, double tau, int repeats, uint64_t seed,
                 std::vector<int32_t>& order, std::vector<int32_t>& widths) {
  if (algo != QT_ORDER_RGREEDY) {
    greedy(g, algo, tau, seed, order, widths);
    return;
  }
  std::vector<int32_t> o, w;
  int best = std::numeric_limits<int>::max();
  for (int r = 0; r < std::max(1, repeats); ++r) {
    greedy(g, algo, tau, seed + 0x9E3779B97F4A7C15ull * (r + 1), o, w);
    int c = max_of(w, 0, w.size());
    if (c < best) {
      best = c;
      order = o;
      widths = w;
    }
  }
}

double step_cost(const std::vector<int32_t>& w, size_t b, size_t e) {
  double c = 0;
  for (size_t i = b; i < e; ++i) c += std::ldexp(1.0, w[i] + 1);
  return c;
}

}  // namespace
}  // namespace qt

using namespace qt;

extern "C" qt_status qt_order_greedy(const qt_network* net, int32_t algo, const int32_t* exclude,
                                     int32_t n_exclude, double tau, int32_t repeats, uint64_t seed,
                                     int32_t* order_out, int32_t* n_order_out, int32_t* width_out) {
  try {
    if (!net || !order_out || !n_order_out || !width_out || (n_exclude > 0 && !exclude))
      return fail(QT_EINVAL, "qt_order_greedy: null argument");
    if (algo < 0 || algo > 2) return fail(QT_EINVAL, "qt_order_greedy: unknown algo");
    if (algo == QT_ORDER_RGREEDY && !(tau > 0)) return fail(QT_EINVAL, "qt_order_greedy: tau must be > 0");
    Graph g = build_graph(*net);
    for (int i = 0; i < n_exclude; ++i) {
      int e = exclude[i];
      if (e < 0 || e >= net->n_vars_ext || net->int_of[e] < 0)
        return fail(QT_EINVAL, "qt_order_greedy: exclude id not a variable of the network");
      if (g.alive[net->int_of[e]]) g.remove(net->int_of[e]);
    }
    std::vector<int32_t> order, widths;
    best_greedy(g, algo, tau, repeats, seed, order, widths);
    for (size_t i = 0; i < order.size(); ++i) order_out[i] = net->ext_of[order[i]];
    *n_order_out = (int32_t)order.size();
    *width_out = max_of(widths, 0, widths.size());
    return QT_OK;
  } catch (const std::exception& ex) {
    return fail(QT_ENOMEM, std::string("qt_order_greedy: ") + ex.what());
  }
}

namespace qt {
namespace {

// One step-dependent slicing search (Section VI-C, VI-D) on graph g0 for
// k variables: the candidate steps up to the peak of g0's order, each
// eliminating that prefix, deleting the k highest-degree vertices (degrees
// recomputed after each deletion, ties to the smallest id) and ordering the
// rest afresh; the narrowest candidate wins (ties: cost, then step).
struct Sweep {
  int s = 0, width = 0, pw = 0, sw = 0, unsliced = 0, peak = 0;
  double pre_cost = 0, post_cost = 0;
  std::vector<int32_t> pre, post, sl;
  std::vector<int> cands, cand_width;
};

qt_status sweep(const Graph& g0, int k, const qt_slicing_opts& opts, Sweep& out) {
  std::vector<int32_t> order0, w0;
  best_greedy(g0, opts.algo, opts.tau, opts.repeats, opts.seed, order0, w0);
  const int unsliced = max_of(w0, 0, w0.size());
  int peak = 0;
  while (peak < (int)w0.size() && w0[peak] != unsliced) ++peak;
  std::vector<int> cands;
  if (k == 0) {
    cands.push_back(0);
  } else if (opts.max_candidates <= 0 || opts.max_candidates >= peak + 1) {
    for (int s = 0; s <= peak; ++s) cands.push_back(s);
  } else {
    int m = opts.max_candidates;
    for (int i = 0; i < m; ++i) cands.push_back((int)((int64_t)i * peak / std::max(1, m - 1)));
    cands.erase(std::unique(cands.begin(), cands.end()), cands.end());
  }
  struct Eval {
    int width = std::numeric_limits<int>::max(), pw = 0, sw = 0;
    double cost = 0, post_cost = 0;
    std::vector<int32_t> post, sl;
  };
  std::vector<Eval> evals(cands.size());
  auto run = [&](size_t ci) {
    const int s = cands[ci];
    Graph g = g0;
    for (int i = 0; i < s; ++i) g.eliminate(order0[i]);
    Eval& e = evals[ci];
    for (int j = 0; j < k; ++j) {
      int best = -1;
      for (int v = 0; v < g.V; ++v)
        if (g.alive[v] && (best < 0 || g.deg[v] > g.deg[best])) best = v;
      if (best < 0) break;
      e.sl.push_back(best);
      g.remove(best);
    }
    std::vector<int32_t> w;
    best_greedy(g, opts.algo, opts.tau, opts.repeats, opts.seed + 1000003ull * (s + 1), e.post, w);
    e.pw = max_of(w0, 0, s);
    e.sw = max_of(w, 0, w.size());
    e.width = std::max(e.pw, e.sw);
    e.post_cost = step_cost(w, 0, w.size());
    e.cost = step_cost(w0, 0, s) + std::ldexp(e.post_cost, k);
  };
  int nt = opts.threads > 0 ? opts.threads : (int)std::thread::hardware_concurrency();
  nt = std::max(1, std::min({nt, 16, (int)cands.size()}));
  std::atomic<size_t> next{0};
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&] {
      for (size_t i = next++; i < cands.size(); i = next++) run(i);
    });
  for (auto& th : pool) th.join();
  size_t bi = 0;
  for (size_t i = 1; i < evals.size(); ++i) {
    const Eval &a = evals[i], &b = evals[bi];
    if (a.width < b.width || (a.width == b.width && a.cost < b.cost)) bi = i;
  }
  Eval& be = evals[bi];
  if ((int)be.sl.size() != k) return fail(QT_EPLAN, "qt_plan_slicing: not enough vertices to slice");
  out.s = cands[bi];
  out.width = be.width;
  out.pw = be.pw;
  out.sw = be.sw;
  out.unsliced = unsliced;
  out.peak = peak;
  out.pre.assign(order0.begin(), order0.begin() + out.s);
  out.pre_cost = step_cost(w0, 0, out.s);
  out.post_cost = be.post_cost;
  out.post = std::move(be.post);
  out.sl = std::move(be.sl);
  out.cands = cands;
  out.cand_width.clear();
  for (const Eval& e : evals) out.cand_width.push_back(e.width);
  return QT_OK;
}

}  // namespace
}  // namespace qt

extern "C" qt_status qt_plan_slicing(const qt_network* net, const qt_slicing_opts* opts,
                                     int32_t* order_out, int32_t* n_order_out,
                                     int32_t* slice_vars_out, qt_slicing_result* result,
                                     int32_t* width_by_step) {
  try {
    if (!net || !opts || !order_out || !n_order_out || !result || (opts->n_slice_vars > 0 && !slice_vars_out) ||
        (opts->n_exclude > 0 && !opts->exclude))
      return fail(QT_EINVAL, "qt_plan_slicing: null argument");
    if (opts->algo < 0 || opts->algo > 2) return fail(QT_EINVAL, "qt_plan_slicing: unknown algo");
    const int k = opts->n_slice_vars;
    const int V = net->n_vars();
    if (k < 0 || k >= V || k > 40) return fail(QT_EINVAL, "qt_plan_slicing: n_slice_vars out of range");
    const int r = opts->group_size <= 0 || opts->group_size >= k ? k : opts->group_size;
    if (k > 0 && (k + r - 1) / r > QT_MAX_SLICE_GROUPS)
      return fail(QT_EINVAL, "qt_plan_slicing: more than QT_MAX_SLICE_GROUPS groups");
    Graph g = build_graph(*net);
    for (int i = 0; i < opts->n_exclude; ++i) {  // held (open) variables: deleted without fill
      const int e = opts->exclude[i];
      if (e < 0 || e >= net->n_vars_ext || net->int_of[e] < 0)
        return fail(QT_EINVAL, "qt_plan_slicing: exclude id not a variable of the network");
      if (g.alive[net->int_of[e]]) g.remove(net->int_of[e]);
    }
    // Section VI-D: r variables at a time, each group at its own best step
    // of the expression sliced by the groups before it.
    int n = 0, nsl = 0, left = k, cum = 0, pw = 0, sw = 0, ng = 0;
    double cost = 0;
    Sweep first;
    do {
      const int rg = std::min(r, left);
      Sweep S;
      QT_TRY(sweep(g, rg, *opts, S));
      if (ng == 0) first = S;
      for (int v : S.pre) {
        g.eliminate(v);
        order_out[n++] = net->ext_of[v];
      }
      for (int v : S.sl) {
        g.remove(v);
        slice_vars_out[nsl++] = net->ext_of[v];
      }
      cost += std::ldexp(S.pre_cost, k - left);
      cum += S.s;
      pw = std::max(pw, S.pw);
      if (rg > 0) {
        result->group_step[ng] = cum;
        result->group_len[ng] = rg;
        ++ng;
      }
      left -= rg;
      if (left == 0) {
        for (int v : S.post) order_out[n++] = net->ext_of[v];
        sw = S.sw;
        cost += std::ldexp(S.post_cost, k);
      }
    } while (left > 0);
    *n_order_out = n;
    result->n_groups = ng;
    result->step = ng ? result->group_step[0] : 0;
    result->width = std::max(pw, sw);
    result->prefix_width = pw;
    result->slice_width = sw;
    result->unsliced_width = first.unsliced;
    result->peak_step = first.peak;
    result->cost = cost;
    if (width_by_step) {
      for (int i = 0; i <= V; ++i) width_by_step[i] = -1;
      for (size_t i = 0; i < first.cands.size(); ++i) width_by_step[first.cands[i]] = first.cand_width[i];
    }
    return QT_OK;
  } catch (const std::exception& ex) {
    return fail(QT_ENOMEM, std::string("qt_plan_slicing: ") + ex.what());
  }
}
