// Network ingest and plan compilation: the symbolic half of Algorithm 1.
//
// qt_load_plan runs the bucket assignment of Algorithm 1 on shapes only:
// every tensor goes to the bucket of its earliest variable under the order,
// every bucket becomes one step (its product and the sum over its
// variable), and every result goes to the bucket of its earliest remaining
// variable or, when nothing is left, into the list of scalar factors whose
// product is the value ("result <- result * R").  With step-dependent
// slicing (Section VI-C, VI-D) the first s steps form the prefix, run once
// per point; the remaining steps run per slice, batched over slices, and
// see the slice variables of prefix tensors as fixed bits.
//
// Storage layout: a global key orders all variables -- eliminated variables
// by their position in the order, slice variables above all of them, the
// first slice variable highest.  Every tensor stores its variables in key
// order with the lowest key in the least significant bit.  Consequences the
// kernels rely on:
//   * the variable eliminated by a bucket is bit 0 of every tensor in it;
//   * an input's remaining variables are a subset of the output's, in the
//     same relative order, so its index is a pext of the output index;
//   * slice variables are the top bits, so fixing them picks a contiguous
//     block of a prefix tensor.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cstring>
#include <numeric>

#include "qt_internal.h"

namespace qt {

static thread_local std::string g_error;

void set_error(const std::string& msg) { g_error = msg; }
qt_status fail(qt_status code, const std::string& msg) {
  g_error = msg;
  return code;
}

namespace {

int expected_rank(int kind) {
  switch (kind) {
    case QT_T_VEC_PLUS:
    case QT_T_BRA_BIT:
      return 1;
    case QT_T_ZZ:
    case QT_T_RX:
    case QT_T_ZZ_DAG:
    case QT_T_RX_DAG:
    case QT_T_OBS_CUT:
      return 2;
    default:
      return -1;
  }
}

constexpr int kMaxDenseRank = 24;

}  // namespace

// Offline first-fit placement of buffers live over closed time intervals:
// largest first, each at the lowest offset free over its whole interval.
int64_t place_intervals(std::vector<Interval>& iv, std::vector<int64_t>& off_out) {
  std::sort(iv.begin(), iv.end(), [](const Interval& a, const Interval& b) {
    if (a.size != b.size) return a.size > b.size;
    return a.start < b.start;
  });
  struct Placed {
    int64_t off, size;
    int32_t start, end;
  };
  std::vector<Placed> placed;
  int64_t total = 0;
  std::vector<std::pair<int64_t, int64_t>> busy;
  for (const auto& it : iv) {
    busy.clear();
    for (const auto& p : placed)
      if (p.start <= it.end && it.start <= p.end) busy.emplace_back(p.off, p.off + p.size);
    std::sort(busy.begin(), busy.end());
    int64_t off = 0;
    for (const auto& b : busy) {
      if (b.first >= off + it.size) break;
      off = std::max(off, b.second);
    }
    placed.push_back({off, it.size, it.start, it.end});
    off_out[it.t] = off;
    total = std::max(total, off + it.size);
  }
  return total;
}

}  // namespace qt

using namespace qt;

extern "C" const char* qt_last_error(void) { return g_error.c_str(); }

extern "C" qt_status qt_load_network(const qt_network_desc* d, qt_network** out) {
  try {
    if (!d || !out) return fail(QT_EINVAL, "qt_load_network: null argument");
    *out = nullptr;
    if (d->n_vars <= 0 || d->n_tensors < 0 || (d->n_tensors > 0 && !d->tensors) || d->p < 0 || d->p > 64)
      return fail(QT_EINVAL, "qt_load_network: bad sizes");
    auto net = std::make_unique<qt_network>();
    net->n_vars_ext = d->n_vars;
    net->p = d->p;
    std::vector<char> used(d->n_vars, 0);
    for (int t = 0; t < d->n_tensors; ++t) {
      const qt_tensor_desc& td = d->tensors[t];
      const std::string where = "qt_load_network: tensor " + std::to_string(t) + ": ";
      if (td.kind < QT_T_VEC_PLUS || td.kind > QT_T_DENSE) return fail(QT_EINVAL, where + "unknown kind");
      const int want = expected_rank(td.kind);
      if (want > 0 && td.rank != want) return fail(QT_EINVAL, where + "rank does not match kind");
      if (td.kind == QT_T_DENSE && (td.rank < 1 || td.rank > kMaxDenseRank || !td.dense))
        return fail(QT_EINVAL, where + "dense tensor needs 1 <= rank <= 24 and values");
      if (!td.vars) return fail(QT_EINVAL, where + "null vars");
      if (td.kind == QT_T_ZZ || td.kind == QT_T_RX || td.kind == QT_T_ZZ_DAG || td.kind == QT_T_RX_DAG) {
        if (td.layer < 1 || td.layer > d->p) return fail(QT_EINVAL, where + "layer out of 1..p");
      }
      if (td.kind == QT_T_BRA_BIT && td.layer != 0 && td.layer != 1)
        return fail(QT_EINVAL, where + "BRA_BIT bit must be 0 or 1");
      for (int i = 0; i < td.rank; ++i) {
        const int v = td.vars[i];
        if (v < 0 || v >= d->n_vars) return fail(QT_EINVAL, where + "variable id out of range");
        for (int j = 0; j < i; ++j)
          if (td.vars[j] == v) return fail(QT_EINVAL, where + "repeated variable");
        used[v] = 1;
      }
    }
    net->int_of.assign(d->n_vars, -1);
    for (int v = 0; v < d->n_vars; ++v)
      if (used[v]) {
        net->int_of[v] = (int32_t)net->ext_of.size();
        net->ext_of.push_back(v);
      }
    net->leaves.resize(d->n_tensors);
    for (int t = 0; t < d->n_tensors; ++t) {
      const qt_tensor_desc& td = d->tensors[t];
      Leaf& L = net->leaves[t];
      L.kind = td.kind;
      L.layer = td.layer;
      for (int i = 0; i < td.rank; ++i) L.vars.push_back(net->int_of[td.vars[i]]);
      if (td.kind == QT_T_DENSE) L.dense.assign(td.dense, td.dense + 2 * ((size_t)1 << td.rank));
    }
    *out = net.release();
    return QT_OK;
  } catch (const std::exception& ex) {
    return fail(QT_ENOMEM, std::string("qt_load_network: ") + ex.what());
  }
}

extern "C" void qt_free_network(qt_network* net) { delete net; }

extern "C" qt_status qt_load_plan(const qt_network* net, const qt_plan_desc* d, qt_plan** out) {
  try {
    if (!net || !d || !out) return fail(QT_EINVAL, "qt_load_plan: null argument");
    *out = nullptr;
    if (d->precision < QT_C128 || d->precision > QT_C64_SCALED_MFMA_BF16X3)
      return fail(QT_EINVAL, "qt_load_plan: unknown precision");
    if (d->n_order < 0 || (d->n_order > 0 && !d->order)) return fail(QT_EINVAL, "qt_load_plan: bad order");
    if (d->n_groups < 0 || d->n_groups > 64 || (d->n_groups > 0 && (!d->group_step || !d->group_len)))
      return fail(QT_EINVAL, "qt_load_plan: bad groups");
    if (d->slice_batch < 0) return fail(QT_EINVAL, "qt_load_plan: negative slice_batch");
    if (d->gemm_min_rank != 0 && (d->gemm_min_rank < 4 || d->gemm_min_rank > kGemmMaxRank))
      return fail(QT_EINVAL, "qt_load_plan: gemm_min_rank must be 0 or 4.." + std::to_string(kGemmMaxRank));
    if (d->n_open < 0 || d->n_open > kMaxOpen || (d->n_open > 0 && !d->open_vars))
      return fail(QT_EINVAL, "qt_load_plan: n_open out of 0.." + std::to_string(kMaxOpen) + " or null open_vars");

    auto plan = std::make_unique<qt_plan>();
    static std::atomic<uint64_t> next_serial{1};
    plan->serial = next_serial++;
    plan->net = *net;
    plan->precision = d->precision;
    plan->slice_batch_req = d->slice_batch;
    plan->flags = d->flags;
    const int V = net->n_vars();
    std::vector<int> role(V, -1);
    auto internal = [&](int ext, int& iv) -> bool {
      if (ext < 0 || ext >= net->n_vars_ext) return false;
      iv = net->int_of[ext];
      return iv >= 0;
    };
    for (int i = 0; i < d->n_order; ++i) {
      int iv;
      if (!internal(d->order[i], iv)) return fail(QT_EPLAN, "qt_load_plan: order names a variable not in the network");
      if (role[iv] >= 0) return fail(QT_EPLAN, "qt_load_plan: order repeats a variable");
      role[iv] = 0;
      plan->order.push_back(iv);
    }
    // Slice groups: variables concatenated group by group (the slice id's
    // bits, first variable most significant); all are fixed at the last
    // group's step.
    int k = 0, s = d->n_order, prev_step = 0;
    for (int gi = 0; gi < d->n_groups; ++gi) {
      const int kg = d->group_len[gi], sg = d->group_step[gi];
      if (kg < 0 || k + kg > 30 || (kg > 0 && !d->slice_vars))
        return fail(QT_EPLAN, "qt_load_plan: slice variables out of 0..30 in total");
      if (sg < 0 || sg > d->n_order) return fail(QT_EPLAN, "qt_load_plan: group step out of [0, n_order]");
      if (sg < prev_step) return fail(QT_EPLAN, "qt_load_plan: group steps must be non-decreasing");
      prev_step = sg;
      for (int j = 0; j < kg; ++j) {
        int iv;
        if (!internal(d->slice_vars[k + j], iv))
          return fail(QT_EPLAN, "qt_load_plan: slice variable not in the network");
        if (role[iv] >= 0) return fail(QT_EPLAN, "qt_load_plan: slice variable repeated or also in the order");
        role[iv] = 1;
        plan->slice_vars.push_back(iv);
      }
      k += kg;
      s = sg;
    }
    plan->n_groups = d->n_groups;
    if (k == 0) s = d->n_order;
    const int a = d->n_open;
    for (int q = 0; q < a; ++q) {
      int iv;
      if (!internal(d->open_vars[q], iv)) return fail(QT_EPLAN, "qt_load_plan: open variable not in the network");
      if (role[iv] >= 0) return fail(QT_EPLAN, "qt_load_plan: open variable repeated, ordered or sliced");
      role[iv] = 2;
      plan->open_vars.push_back(iv);
    }
    for (int v = 0; v < V; ++v)
      if (role[v] < 0)
        return fail(QT_EPLAN, "qt_load_plan: variable " + std::to_string(net->ext_of[v]) +
                                  " neither ordered, sliced nor open");
    const int n_order = d->n_order;
    plan->n_order = n_order;
    plan->slice_step = s;

    // Global key: order position; open variable q gets n_order + (a-1-q)
    // (its bit in the output index); slice variable j gets
    // n_order + a + (k-1-j), above everything else.
    auto& key = plan->key;
    key.assign(V, 0);
    std::vector<int> slice_index(V, -1);
    for (int i = 0; i < n_order; ++i) key[plan->order[i]] = i;
    for (int q = 0; q < a; ++q) key[plan->open_vars[q]] = n_order + (a - 1 - q);
    for (int j = 0; j < k; ++j) {
      key[plan->slice_vars[j]] = n_order + a + (k - 1 - j);
      slice_index[plan->slice_vars[j]] = j;
    }
    auto by_key = [&](int a, int b) { return key[a] < key[b]; };

    auto& T = plan->tensors;
    auto& steps = plan->steps;
    std::vector<std::vector<int>> buckets(n_order);
    // Leaves (level 0).
    for (size_t l = 0; l < net->leaves.size(); ++l) {
      SymTensor st;
      st.vars = net->leaves[l].vars;
      std::sort(st.vars.begin(), st.vars.end(), by_key);
      st.level = 0;
      st.leaf = (int)l;
      st.rank = (int)st.vars.size();
      T.push_back(st);
    }
    auto place = [&](int t) {
      int mk = INT_MAX;
      for (int v : T[t].vars) mk = std::min(mk, key[v]);
      if (T[t].vars.empty() || mk >= n_order) {
        T[t].consumer = -2;
        plan->finals.push_back(t);
      } else {
        buckets[mk].push_back(t);
      }
    };
    for (int t = 0; t < (int)T.size(); ++t) place(t);

    // Effective variables of tensor t in a phase: slice variables drop out
    // of level-0 tensors once the slice step is reached.
    auto eff = [&](int t, bool post) {
      std::vector<int> e;
      for (int v : T[t].vars)
        if (!(post && slice_index[v] >= 0)) e.push_back(v);
      return e;
    };

    auto emit = [&](const std::vector<int>& ins, bool sum, int v, bool post) -> qt_status {
      std::vector<int> U;
      for (int t : ins) {
        auto e = eff(t, post);
        U.insert(U.end(), e.begin(), e.end());
      }
      std::sort(U.begin(), U.end(), by_key);
      U.erase(std::unique(U.begin(), U.end()), U.end());
      std::vector<int> outv = U;
      if (sum) {
        if (U.empty() || U[0] != v) return fail(QT_EPLAN, "qt_load_plan: internal: bucket variable is not lowest");
        outv.erase(outv.begin());
      }
      if ((int)outv.size() > kMaxRank)
        return fail(QT_EUNSUPPORTED, "qt_load_plan: intermediate of rank " + std::to_string(outv.size()) + " exceeds 31");
      SymTensor o;
      o.vars = outv;
      o.level = post ? 1 : 0;
      o.rank = (int)outv.size();
      o.producer = (int)steps.size();
      const int ot = (int)T.size();
      T.push_back(o);
      SymStep st;
      st.out = ot;
      st.level = o.level;
      st.rank = o.rank;
      st.sum = sum ? 1 : 0;
      st.var = sum ? v : -1;
      st.nbr = sum ? (int)outv.size() : -1;
      double in_elems = 0;
      for (int t : ins) {
        auto e = eff(t, post);
        SymIn si{};
        si.tensor = t;
        si.has_v = (sum && !e.empty() && e[0] == v) ? 1 : 0;
        size_t pos = 0;
        int matched = 0;
        for (size_t i = 0; i < outv.size(); ++i) {
          if (std::find(e.begin(), e.end(), outv[i]) != e.end()) {
            si.mask |= 1u << i;
            ++matched;
          }
        }
        (void)pos;
        if (matched + si.has_v != (int)e.size())
          return fail(QT_EPLAN, "qt_load_plan: internal: input variables not covered by the output");
        if (post && T[t].level == 0) {
          for (int x : T[t].vars)
            if (slice_index[x] >= 0) si.smask |= 1u << (k - 1 - slice_index[x]);
          si.slow = (int)e.size();
        }
        in_elems += std::ldexp(1.0, (int)e.size());
        T[t].consumer = (int)steps.size();
        st.ins.push_back(si);
      }
      const double out_elems = std::ldexp(1.0, st.rank);
      const int m = (int)ins.size();
      st.bytes_c64 = 8.0 * (in_elems + out_elems);
      st.flops = out_elems * (sum ? (12.0 * (m - 1) + 2.0) : 6.0 * (m - 1));
      steps.push_back(std::move(st));
      place(ot);
      return QT_OK;
    };

    // Fused GEMM bucket (MFMA precisions).  When the two largest tensors A
    // and B of the bucket of v share variables that no other live tensor
    // holds (apart from vectors on them), summing v and those variables at
    // once is one contraction C[b, m, n] = sum_k A[b, m, k] B[b, n, k]
    // (b: shared kept variables, m / n: variables of A / B only); the
    // summed variables' buckets are then empty.  The bucket's other tensors
    // and the vectors on summed variables are first multiplied into A or B
    // (product steps), so the result is that of eliminating the same
    // variables one by one, with a smaller intermediate.
    const bool mfma = d->precision == QT_C64_SCALED_MFMA_FP32 || d->precision == QT_C64_SCALED_MFMA_BF16X3;
    const int gemm_min_rank = d->gemm_min_rank > 0 ? d->gemm_min_rank : env_int("QT_GEMM_MIN_RANK", 12);
    auto subset = [](const std::vector<int>& a, const std::vector<int>& b) {
      for (int x : a)
        if (std::find(b.begin(), b.end(), x) == b.end()) return false;
      return true;
    };
    auto contains = [](const std::vector<int>& a, int x) { return std::find(a.begin(), a.end(), x) != a.end(); };
    // Multiplies the tensors of grp into one (product steps).  The small
    // tensors are multiplied among themselves first, so the big one (grp[0])
    // is read and rewritten once.
    auto fold = [&](std::vector<int> grp, int v, bool post, int& res) -> qt_status {
      auto take_product = [&](const std::vector<int>& g) -> int {
        const int id = (int)T.size();  // emit appends the product as the next tensor
        if (emit(g, false, v, post) != QT_OK) return -1;
        for (auto& bk : buckets) {
          auto it = std::find(bk.begin(), bk.end(), id);
          if (it != bk.end()) {
            bk.erase(it);
            break;
          }
        }
        return id;
      };
      std::vector<int> small(grp.begin() + 1, grp.end());
      while (small.size() > 1) {
        std::vector<int> g(small.begin(), small.begin() + std::min<size_t>(kMaxIn, small.size()));
        small.erase(small.begin(), small.begin() + g.size());
        const int t = take_product(g);
        if (t < 0) return fail(QT_EPLAN, "qt_load_plan: internal: product of small tensors failed");
        small.insert(small.begin(), t);
      }
      res = grp[0];
      if (!small.empty()) {
        res = take_product({grp[0], small[0]});
        if (res < 0) return fail(QT_EPLAN, "qt_load_plan: internal: product failed");
      }
      return QT_OK;
    };
    auto try_fuse = [&](int i, int v, const std::vector<int>& ins, bool post, bool& fused) -> qt_status {
      fused = false;
      if (!mfma || ins.size() < 2) return QT_OK;
      std::vector<int> srt = ins;
      std::stable_sort(srt.begin(), srt.end(),
                       [&](int a, int b) { return eff(a, post).size() > eff(b, post).size(); });
      const int A = srt[0], B = srt[1];
      const std::vector<int> SA = eff(A, post), SB = eff(B, post);
      if (SA.size() < 4 || SB.size() < 4) return QT_OK;
      std::vector<int> U;
      for (int t : ins)
        for (int x : eff(t, post))
          if (!contains(U, x)) U.push_back(x);
      if ((int)U.size() - 1 < gemm_min_rank) return QT_OK;
      // the other tensors go to the smaller operand that holds their variables
      const bool a_small = SA.size() <= SB.size();
      std::vector<int> toA = {A}, toB = {B};
      auto assign = [&](int t) {
        const auto e = eff(t, post);
        const bool inA = subset(e, SA), inB = subset(e, SB);
        if (inA && inB) (a_small ? toA : toB).push_back(t);
        else if (inA) toA.push_back(t);
        else if (inB) toB.push_back(t);
        else return false;
        return true;
      };
      for (int t : ins)
        if (t != A && t != B && !assign(t)) return QT_OK;
      std::vector<int> K = {v};
      std::vector<std::pair<int, int>> vecs;  // (bucket, tensor) of vectors on summed variables
      for (int u : SA) {
        if (u == v || !contains(SB, u) || key[u] >= n_order) continue;
        bool excl = true;
        std::vector<std::pair<int, int>> uv;
        for (int j = i + 1; j < n_order && excl; ++j)
          for (int t : buckets[j]) {
            const auto e = eff(t, post);
            if (!contains(e, u)) continue;
            if (e.size() == 1) uv.emplace_back(j, t);
            else {
              excl = false;
              break;
            }
          }
        if (!excl) continue;
        K.push_back(u);
        vecs.insert(vecs.end(), uv.begin(), uv.end());
      }
      int nm = 0, nn = 0, nb = 0;
      for (int x : SA) nm += !contains(SB, x);
      for (int x : SB) nn += !contains(SA, x);
      for (int x : SA) nb += contains(SB, x) && !contains(K, x);
      const int nk = (int)K.size();
      if (nk < 3 || nm < 4 || nn < 4 || nb + nm + nn > kGemmMaxRank || nb + nm + nk > kGemmMaxRank ||
          nb + nn + nk > kGemmMaxRank)
        return QT_OK;
      for (const auto& jt : vecs) {
        auto& bk = buckets[jt.first];
        bk.erase(std::find(bk.begin(), bk.end(), jt.second));
        (a_small ? toA : toB).push_back(jt.second);  // summed variables are in both
      }
      int Ap = -1, Bp = -1;
      qt_status st = fold(toA, v, post, Ap);
      if (st != QT_OK) return st;
      st = fold(toB, v, post, Bp);
      if (st != QT_OK) return st;
      std::sort(K.begin(), K.end(), by_key);
      std::vector<int> outv;
      for (int x : eff(Ap, post))
        if (!contains(K, x)) outv.push_back(x);
      for (int x : eff(Bp, post))
        if (!contains(K, x) && !contains(outv, x)) outv.push_back(x);
      std::sort(outv.begin(), outv.end(), by_key);
      SymTensor o;
      o.vars = outv;
      o.level = post ? 1 : 0;
      o.rank = (int)outv.size();
      o.producer = (int)steps.size();
      const int ot = (int)T.size();
      T.push_back(o);
      SymStep gs;
      gs.out = ot;
      gs.level = o.level;
      gs.rank = o.rank;
      gs.sum = 1;
      gs.var = v;
      gs.nbr = o.rank;
      gs.gemm = 1;
      gs.kvars = K;
      double in_elems = 0;
      for (int t : {Ap, Bp}) {
        const auto e = eff(t, post);
        SymIn si{};
        si.tensor = t;
        for (size_t q = 0; q < outv.size(); ++q)
          if (contains(e, outv[q])) si.mask |= 1u << q;
        if (post && T[t].level == 0) {
          for (int x : T[t].vars)
            if (slice_index[x] >= 0) si.smask |= 1u << (k - 1 - slice_index[x]);
          si.slow = (int)e.size();
        }
        in_elems += std::ldexp(1.0, (int)e.size());
        T[t].consumer = (int)steps.size();
        gs.ins.push_back(si);
      }
      gs.bytes_c64 = 8.0 * (in_elems + std::ldexp(1.0, o.rank));
      gs.flops = 8.0 * std::ldexp(1.0, nb + nm + nn + (int)K.size());
      steps.push_back(std::move(gs));
      place(ot);
      fused = true;
      return QT_OK;
    };

    // With QT_PLAN_FOLD_PREFIX every step runs per slice (slice variables
    // fixed from the start).
    const int s_exec = (k > 0 && (d->flags & QT_PLAN_FOLD_PREFIX)) ? 0 : s;
    for (int i = 0; i < n_order; ++i) {
      const bool post = k > 0 && i >= s_exec;
      const int v = plan->order[i];
      std::vector<int> ins = std::move(buckets[i]);
      buckets[i].clear();
      if (ins.empty()) continue;
      bool fused = false;
      qt_status fs = try_fuse(i, v, ins, post, fused);
      if (fs != QT_OK) return fs;
      if (fused) {
        if (!post) plan->n_prefix_steps = (int)steps.size();
        continue;
      }
      while ((int)ins.size() > kMaxIn) {
        std::stable_sort(ins.begin(), ins.end(),
                         [&](int a, int b) { return eff(a, post).size() < eff(b, post).size(); });
        std::vector<int> grp(ins.begin(), ins.begin() + kMaxIn);
        ins.erase(ins.begin(), ins.begin() + kMaxIn);
        // the product keeps v; it lands back in this bucket
        qt_status st = emit(grp, false, v, post);
        if (st != QT_OK) return st;
        if (buckets[i].empty()) return fail(QT_EPLAN, "qt_load_plan: internal: product left its bucket");
        ins.push_back(buckets[i].back());
        buckets[i].pop_back();
      }
      qt_status st = emit(ins, true, v, post);
      if (st != QT_OK) return st;
      if (!post) plan->n_prefix_steps = (int)steps.size();
    }
    for (const auto& b : buckets)
      if (!b.empty()) return fail(QT_EPLAN, "qt_load_plan: internal: bucket left unprocessed");

    // A product step (no summed variable) one of whose inputs holds all of
    // its output's variables and is an intermediate consumed only there,
    // produced at the same level by a step that is not a fused GEMM, is
    // merged with that producer: the producer moves to the product's place
    // (its output has no other reader, and its inputs exist by then) and
    // takes the product's other inputs without the summed variable (they
    // multiply both of its v-products alike), so its output is the product.
    // The product's output's reader reads it instead.  Same arithmetic up
    // to rounding order, one pass over the large tensor fewer.  The plain
    // path keeps every step.
    if (!(d->flags & QT_PLAN_PLAIN)) {
      for (int pi = 0; pi < (int)steps.size(); ++pi) {
        const SymStep& P = steps[pi];
        if (P.sum || P.gemm || P.ins.size() < 2) continue;
        const uint32_t all = P.rank >= 32 ? ~0u : ((1u << P.rank) - 1u);
        int cover = -1;
        for (size_t j = 0; j < P.ins.size(); ++j) {
          const SymIn& in = P.ins[j];
          const SymTensor& X = T[in.tensor];
          if (X.leaf < 0 && X.producer >= 0 && X.consumer == pi && X.rank == P.rank && in.mask == all && !in.smask) {
            cover = (int)j;
            break;
          }
        }
        if (cover < 0) continue;
        const int t = P.ins[cover].tensor;
        const int si = T[t].producer;
        if (steps[si].gemm || steps[si].level != P.level || steps[si].ins.size() + P.ins.size() - 1 > (size_t)kMaxIn)
          continue;
        SymStep merged = steps[si];
        double extra_elems = 0;
        std::vector<int> extra;
        for (size_t j = 0; j < P.ins.size(); ++j) {
          if ((int)j == cover) continue;
          SymIn in = P.ins[j];
          in.has_v = 0;
          merged.ins.push_back(in);
          extra.push_back(in.tensor);
          extra_elems += std::ldexp(1.0, T[in.tensor].rank - __builtin_popcount(in.smask));
        }
        const int m = (int)merged.ins.size();
        merged.bytes_c64 += 8.0 * extra_elems;
        merged.flops = std::ldexp(1.0, merged.rank) * (merged.sum ? (12.0 * (m - 1) + 2.0) : 6.0 * (m - 1));
        const int o = P.out, oc = T[o].consumer;
        steps[pi] = std::move(merged);  // the merged step at the product's place ...
        for (const SymIn& in : steps[pi].ins) T[in.tensor].consumer = pi;
        T[t].producer = pi;
        T[t].consumer = oc;
        if (oc == -2) {
          for (auto& f : plan->finals)
            if (f == o) f = t;
        } else if (oc >= 0) {
          for (SymIn& in : steps[oc].ins)
            if (in.tensor == o) in.tensor = t;
        }
        T[o].producer = -1;
        T[o].consumer = -1;
        steps.erase(steps.begin() + si);  // ... and the producer's old place gone
        for (auto& X : T) {
          if (X.producer > si) --X.producer;
          if (X.consumer > si) --X.consumer;
        }
        if (si < plan->n_prefix_steps) --plan->n_prefix_steps;
        pi = si - 1;  // steps from the producer's old place on have moved
      }
    }

    // Widths and algorithmic counts.
    for (const auto& st : steps) {
      if (st.sum) {
        if (st.level == 0) plan->prefix_width = std::max(plan->prefix_width, st.nbr);
        else plan->slice_width = std::max(plan->slice_width, st.nbr);
      }
      if (st.level == 0) {
        plan->prefix_bytes += st.bytes_c64;
        plan->prefix_flops += st.flops;
      } else {
        plan->slice_bytes += st.bytes_c64;
        plan->slice_flops += st.flops;
      }
    }
    plan->width = std::max(plan->prefix_width, plan->slice_width);

    // Leaves: one block per point; DENSE values permuted to storage order.
    int32_t off = 0;
    for (size_t t = 0; t < net->leaves.size(); ++t) {
      const Leaf& L = net->leaves[t];
      DevLeaf dl{};
      dl.kind = L.kind;
      dl.layer = L.layer;
      dl.rank = (int)L.vars.size();
      dl.off = off;
      if (L.kind == QT_T_VEC_PLUS) plan->log2_const -= 0.5;
      if (L.kind == QT_T_DENSE) {
        dl.dense_off = (int32_t)(plan->dense_table.size() / 2);
        const auto& sv = T[t].vars;  // storage order, bit i = sv[i]
        const int r = dl.rank;
        for (int64_t y = 0; y < (1ll << r); ++y) {
          int64_t u = 0;
          for (int i = 0; i < r; ++i) {
            const int bit = (y >> i) & 1;
            const int j = (int)(std::find(L.vars.begin(), L.vars.end(), sv[i]) - L.vars.begin());
            u |= (int64_t)bit << (r - 1 - j);
          }
          plan->dense_table.push_back(L.dense[2 * u]);
          plan->dense_table.push_back(L.dense[2 * u + 1]);
        }
      }
      off += 1 << dl.rank;
      plan->dev_leaves.push_back(dl);
    }
    plan->leaf_block = (off + 1) & ~1;
    if (plan->dense_table.empty()) plan->dense_table.push_back(0.0);

    // Exponent slots of intermediates: per point (level 0) or per point and
    // slice item (level 1).  Device arenas are laid out at run time, once
    // the launch schedule is known.
    for (auto& st : T) {
      if (st.leaf >= 0) continue;
      st.exp_slot = st.level == 0 ? plan->n_exp0++ : plan->n_exp1++;
    }

    qt_plan_info& in = plan->info;
    in.n_steps = (int)steps.size();
    in.n_prefix_steps = plan->n_prefix_steps;
    in.width = plan->width;
    in.prefix_width = plan->prefix_width;
    in.slice_width = plan->slice_width;
    in.n_slice_vars = k;
    in.n_slices = 1ll << k;
    in.prefix_bytes = plan->prefix_bytes;
    in.slice_bytes = plan->slice_bytes;
    in.prefix_flops = plan->prefix_flops;
    in.slice_flops = plan->slice_flops;
    in.element_bytes = d->precision == QT_C128 ? 16 : 8;
    in.n_open = a;
    in.n_groups = d->n_groups;
    *out = plan.release();
    return QT_OK;
  } catch (const std::exception& ex) {
    return fail(QT_ENOMEM, std::string("qt_load_plan: ") + ex.what());
  }
}

extern "C" qt_status qt_plan_get_info(const qt_plan* plan, qt_plan_info* out) {
  if (!plan || !out) return fail(QT_EINVAL, "qt_plan_get_info: null argument");
  *out = plan->info;
  return QT_OK;
}
