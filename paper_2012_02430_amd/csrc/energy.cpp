// QAOA MaxCut energy from per-edge lightcone networks (Section III-B: the
// energy is one amplitude of a duplicated expression; Section III-A:
// lightcone optimisation), every edge and point in one launch of the
// multi-program LDS executor, then a fixed-order FP64 sum over edges.
//
// Each lightcone plan becomes one program: all its bucket steps in
// dependency levels, every intermediate in LDS (first-fit over level
// intervals), its closing scalars kept in LDS until the epilogue.  Jobs
// (the uploaded programs of one list of plans) are cached by plan serial
// numbers and dropped when a plan is freed.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>

#include "qt_internal.h"

namespace qt {
namespace {



struct Program {
  bool fits = true;
  std::vector<XStep> steps;
  std::vector<XRev> revs;
  std::vector<uint2> units;
  std::vector<int32_t> levels;
  std::vector<XFinal> finals;
  std::vector<int32_t> rec_off;  // gradient programs: 2p + 1 record offsets
  std::vector<std::vector<int>> lsteps;  // forward programs: steps of each level
  int n_levels = 0, n_slots = 0, n_recs = 0, lds_elems = 0;
  int dropped = 0, recomputed = 0;
  double log2_const = 0, cost = 0, bytes_c64 = 0, flops = 0;
};

// Operand location of a tensor for one use: LDS element offset and scale slot.
struct Loc {
  uint32_t off;
  int32_t slot;
};

int gate_offset(const qt_plan& plan, int t) {
  const Leaf& L = plan.net.leaves[plan.tensors[t].leaf];
  return x_gate_off(L.kind, L.layer);
}

// Descriptor of bucket step s writing (out) and reading its inputs where
// loc(tensor) says (gate leaves read the gate table).
template <class LocFn>
qt_status fill_xstep(const qt_plan& plan, int s, int elt, Loc out, LocFn loc, XStep& xs) {
  const SymStep& st = plan.steps[s];
  std::memset(&xs, 0, sizeof(xs));
  xs.out.ptr = nullptr;
  xs.out.lds_off = out.off;
  xs.out.slot_kind = 1;
  xs.out.slot = out.slot;
  xs.r = st.rank;
  xs.sum = st.sum;
  xs.n_in = (int)st.ins.size();  // exact; operands up to the class (2, 4, 8) are identities
  const int epu = x_epu(st.rank, (int)st.ins.size(), elt);
  for (size_t j = 0; j < st.ins.size(); ++j) {
    const SymIn& si = st.ins[j];
    XOp& x = xs.in[j];
    x.slot = -1;
    if (plan.tensors[si.tensor].leaf >= 0) {
      const int g = gate_offset(plan, si.tensor);
      if (g < 0) return fail(QT_EUNSUPPORTED, "qt_energy_grad: dense tensors are not supported in lightcones");
      x.lds_off = (uint32_t)g;
    } else {
      const Loc l = loc(si.tensor);
      x.lds_off = l.off;
      x.slot = l.slot;
    }
    x.has_v = si.has_v;
    int32_t nr = 0;
    if (!make_runs(si.mask, kXRuns, x.run_lo, x.run_len, x.run_dst, nr))
      return fail(QT_EUNSUPPORTED, "qt_energy_grad: index map too fragmented");
    x.lane_runs = x_lane_runs(x.run_lo, x.run_len, x.run_dst, nr, x.has_v);
    for (int e = 0; e < 4; ++e) {
      uint32_t r = 0;
      if (e < epu)
        for (int q = 0; q < nr; ++q)
          r |= (((uint32_t)(64 * e) >> x.run_lo[q]) & ((1u << x.run_len[q]) - 1u)) << x.run_dst[q];
      x.ep[e] = r << x.has_v;
    }
  }
  for (int j = (int)st.ins.size(); j < x_nin_class(xs.n_in); ++j) {
    XOp& id = xs.in[j];  // identity operand
    std::memset(&id, 0, sizeof(id));
    id.has_v = 1;
    id.slot = -1;
  }
  return QT_OK;
}

void push_step_units(const qt_plan& plan, int s, int xs_index, int elt, std::vector<uint2>& units) {
  const int r = plan.steps[s].rank;
  const int64_t chunks = std::max<int64_t>(1, (1ll << r) / x_unit_elems(r, (int)plan.steps[s].ins.size(), elt));
  for (int64_t c = 0; c < chunks; ++c) units.push_back(make_uint2((uint32_t)xs_index, (uint32_t)c));
}

// Units of a forward program run for P points per workgroup, level by
// level: a step with fewer than 64 outputs takes 64 / 2^r points per unit
// (unit index: the block of points); a larger one takes P x chunks units of
// its per-point size (unit index: point x chunks + chunk).  With P = 1 these
// are the per-point units.
void pts_units(const Program& pg, int P, int elt, std::vector<uint2>& units, std::vector<int32_t>& levels) {
  for (const auto& lv : pg.lsteps) {
    levels.push_back((int32_t)(units.size()));
    for (int xs : lv) {
      const int r = pg.steps[xs].r;
      if (r < 6) {
        const int per = 64 >> r;
        for (int b = 0; b < (P + per - 1) / per; ++b) units.push_back(make_uint2((uint32_t)xs, (uint32_t)b));
      } else {
        const int64_t chunks = std::max<int64_t>(1, (1ll << r) / x_unit_elems(r, pg.steps[xs].n_in, elt));
        for (int q = 0; q < P; ++q)
          for (int64_t c = 0; c < chunks; ++c) units.push_back(make_uint2((uint32_t)xs, (uint32_t)(q * chunks + c)));
      }
    }
  }
  levels.push_back((int32_t)units.size());
}

// The gradient schedule's units for P points per workgroup: each forward
// or recomputation step's units as in pts_units, emitted where its first
// per-point unit stood; reverse operations and the closing-scalar unit as
// they are (a reverse unit runs every point of the workgroup in turn).
void grad_pts_units(const Program& pg, int P, int elt, std::vector<uint2>& units, std::vector<int32_t>& levels) {
  for (int L = 0; L < pg.n_levels; ++L) {
    levels.push_back((int32_t)units.size());
    for (int u = pg.levels[L]; u < pg.levels[L + 1]; ++u) {
      const uint2 un = pg.units[u];
      const uint32_t kind = un.x & ~kXUnitIndex, idx = un.x & kXUnitIndex;
      if (kind == 0) {
        if (un.y != 0) continue;  // emitted with the step's first unit
        const int r = pg.steps[idx].r;
        if (r < 6) {
          const int per = 64 >> r;
          for (int b = 0; b < (P + per - 1) / per; ++b) units.push_back(make_uint2(un.x, (uint32_t)b));
        } else {
          const int64_t chunks = std::max<int64_t>(1, (1ll << r) / x_unit_elems(r, pg.steps[idx].n_in, elt));
          for (int q = 0; q < P; ++q)
            for (int64_t c = 0; c < chunks; ++c) units.push_back(make_uint2(un.x, (uint32_t)(q * chunks + c)));
        }
      } else {  // reverse operations run every point in their unit; the closing-scalar unit takes a lane per point
        units.push_back(un);
      }
    }
  }
  levels.push_back((int32_t)units.size());
}

int count_intermediates(const qt_plan& plan) {
  int n = 0;
  for (const SymTensor& T : plan.tensors) n += T.leaf < 0;
  return n;
}

// Forward-only program: every intermediate in LDS over its level interval.
bool has_gemm(const qt_plan& plan) {
  for (const SymStep& st : plan.steps)
    if (st.gemm) return true;
  return false;
}

qt_status build_program(const qt_plan& plan, int elt, int64_t cap_elems, Program& pg) {
  if (!plan.slice_vars.empty()) return fail(QT_EINVAL, "qt_energy_grad: lightcone plans take no slicing");
  if (has_gemm(plan)) return fail(QT_EUNSUPPORTED, "qt_energy_grad: lightcone plans with GEMM buckets are not supported");
  const int nsteps = (int)plan.steps.size();
  const int ntens = (int)plan.tensors.size();
  std::vector<int> depth(nsteps, 0);
  for (int i = 0; i < nsteps; ++i) {
    for (const SymIn& in : plan.steps[i].ins) {
      const int pr = plan.tensors[in.tensor].producer;
      if (pr >= 0) depth[i] = std::max(depth[i], depth[pr] + 1);
    }
    pg.n_levels = std::max(pg.n_levels, depth[i] + 1);
  }
  std::vector<Interval> iv;
  for (int t = 0; t < ntens; ++t) {
    const SymTensor& T = plan.tensors[t];
    if (T.leaf >= 0) continue;
    const int end = T.consumer >= 0 ? depth[T.consumer] : pg.n_levels;
    iv.push_back({t, std::max<int64_t>(2, 1ll << T.rank), depth[T.producer], end});
  }
  std::vector<int64_t> off(ntens, -1);
  const int64_t top = place_intervals(iv, off);
  if (top > cap_elems) {
    pg.fits = false;  // contracted through the general schedule instead
    return QT_OK;
  }
  std::vector<int> slot(ntens, -1);
  for (const Interval& it : iv) slot[it.t] = pg.n_slots++;
  const int tbase = x_tensor_base(plan.net.p);
  pg.lds_elems = (int)top + tbase;
  pg.log2_const = plan.log2_const;
  auto loc = [&](int t) { return Loc{(uint32_t)(off[t] + tbase), slot[t]}; };
  pg.steps.assign(nsteps, XStep{});
  for (int i = 0; i < nsteps; ++i) {
    const SymStep& st = plan.steps[i];
    QT_TRY(fill_xstep(plan, i, elt, loc(st.out), loc, pg.steps[i]));
    pg.cost += std::ldexp(1.0, st.rank) * (double)st.ins.size();
    pg.bytes_c64 += st.bytes_c64;
    pg.flops += st.flops;
  }
  pg.lsteps.assign(pg.n_levels, {});
  for (int L = 0; L < pg.n_levels; ++L) {
    pg.levels.push_back((int32_t)pg.units.size());
    for (int i = 0; i < nsteps; ++i)
      if (depth[i] == L) {
        push_step_units(plan, i, i, elt, pg.units);
        pg.lsteps[L].push_back(i);
      }
  }
  pg.levels.push_back((int32_t)pg.units.size());
  for (int t : plan.finals) {
    if (plan.tensors[t].leaf >= 0) return fail(QT_EPLAN, "qt_energy_grad: internal: leaf as closing scalar");
    pg.finals.push_back({loc(t).off, loc(t).slot});
  }
  return QT_OK;
}

// ---------------------------------------------------------------- adjoint
// Reverse bucket elimination.  Every tensor of a bucket-elimination plan has
// exactly one consumer (a step, or the closing product), so the reverse
// pass visits the steps in reverse order and each input's adjoint is formed
// once, by its consumer's reverse operation; no accumulation is needed.
//
// Checkpointing: a subset C of the intermediates keeps its forward value
// until its consumer's reverse operation; the others are dropped after
// their forward use and recomputed, by their step re-run in the reverse
// schedule once the adjoint of their nearest kept ancestor exists.  The
// schedule (forward levels, the closing adjoints, recomputation and reverse
// levels) and the LDS intervals follow from C; C starts as every
// intermediate and loses one tensor at a time, the one whose loss gives the
// smallest LDS peak, until the program fits.
struct GradSched {
  std::vector<int> lf, lr, lb;  // forward, recompute (-1: none), reverse level per step
  int lfa = 0, n_levels = 0;
  std::vector<Interval> iv;     // interval ids 3 t + {0: value, 1: recomputed value, 2: adjoint}
  std::vector<int64_t> off;
  int64_t top = 0;
  double recompute = 0;
};

void grad_schedule(const qt_plan& plan, const std::vector<char>& keep, GradSched& g) {
  const auto& T = plan.tensors;
  const auto& S = plan.steps;
  const int ns = (int)S.size(), nt = (int)T.size();
  g.lf.assign(ns, 0);
  g.lr.assign(ns, -1);
  g.lb.assign(ns, -1);
  for (int s = 0; s < ns; ++s)
    for (const SymIn& in : S[s].ins)
      if (T[in.tensor].leaf < 0) g.lf[s] = std::max(g.lf[s], g.lf[T[in.tensor].producer] + 1);
  g.lfa = 0;
  for (int t : plan.finals) g.lfa = std::max(g.lfa, g.lf[T[t].producer] + 1);
  auto radj = [&](int t) { return T[t].consumer == -2 ? g.lfa : g.lb[T[t].consumer]; };
  // level at which intermediate t's value is available to the reverse pass
  std::function<int(int)> avail = [&](int t) -> int {
    const int q = T[t].producer;
    if (keep[t]) return g.lf[q];
    if (g.lr[q] < 0) {
      int u = t;
      while (!keep[u]) u = S[T[u].consumer].out;
      int l = radj(u);
      for (const SymIn& in : S[q].ins)
        if (T[in.tensor].leaf < 0) l = std::max(l, avail(in.tensor) + 1);
      g.lr[q] = l;
    }
    return g.lr[q];
  };
  for (int s = ns - 1; s >= 0; --s) {
    int l = radj(S[s].out);
    for (const SymIn& in : S[s].ins)
      if (T[in.tensor].leaf < 0) l = std::max(l, avail(in.tensor));
    g.lb[s] = l + 1;
  }
  g.n_levels = g.lfa + 1;
  g.recompute = 0;
  for (int s = 0; s < ns; ++s) {
    g.n_levels = std::max({g.n_levels, g.lf[s] + 1, g.lr[s] + 1, g.lb[s] + 1});
    if (g.lr[s] >= 0) g.recompute += std::ldexp(1.0, S[s].rank) * (double)S[s].ins.size();
  }
  g.iv.clear();
  for (int t = 0; t < nt; ++t) {
    if (T[t].leaf >= 0) continue;
    const int64_t size = std::max<int64_t>(2, 1ll << T[t].rank);
    const int q = T[t].producer, c = T[t].consumer;
    int end;
    if (c == -2) end = g.n_levels - 1;
    else if (keep[t]) end = std::max({g.lf[c], g.lr[c], g.lb[c]});
    else end = g.lf[c];
    g.iv.push_back({3 * t, size, g.lf[q], end});
    if (!keep[t]) g.iv.push_back({3 * t + 1, size, g.lr[q], std::max(g.lr[c], g.lb[c])});
    g.iv.push_back({3 * t + 2, size, radj(t), g.lb[q]});
  }
  g.off.assign(3 * (size_t)nt, -1);
  std::vector<Interval> iv = g.iv;
  g.top = place_intervals(iv, g.off);
}

bool add_run_pairs(const std::vector<std::pair<int, int>>& pairs, uint8_t* lo, uint8_t* len, uint8_t* dst) {
  int n = 0;
  for (size_t i = 0; i < pairs.size();) {
    size_t e = i + 1;
    while (e < pairs.size() && pairs[e].first == pairs[e - 1].first + 1 && pairs[e].second == pairs[e - 1].second + 1)
      ++e;
    if (n == kXRuns) return false;
    lo[n] = (uint8_t)pairs[i].first;
    len[n] = (uint8_t)(e - i);
    dst[n] = (uint8_t)pairs[i].second;
    ++n;
    i = e;
  }
  return true;
}

// Maps the y (bits of zj) and c (bits of zc) counters onto an operand whose
// element index is the compaction of the z bits in zo.
bool fill_rop(uint64_t zj, uint64_t zc, uint64_t zo, XROp& op) {
  std::vector<std::pair<int, int>> py, pc;
  int iy = 0, ic = 0, io = 0;
  for (int b = 0; b < 64; ++b) {
    const bool inj = (zj >> b) & 1u, inc = (zc >> b) & 1u, ino = (zo >> b) & 1u;
    if (ino) {
      if (inj) py.emplace_back(iy, io);
      if (inc) pc.emplace_back(ic, io);
    }
    iy += inj;
    ic += inc;
    io += ino;
  }
  return add_run_pairs(py, op.y_lo, op.y_len, op.y_dst) && add_run_pairs(pc, op.c_lo, op.c_len, op.c_dst);
}

uint32_t runs_pext(uint64_t x, const uint8_t* lo, const uint8_t* len, const uint8_t* dst) {
  uint32_t r = 0;
  for (int i = 0; i < kXRuns; ++i)
    if (len[i]) r |= (uint32_t)(((x >> lo[i]) & ((1ull << len[i]) - 1ull)) << dst[i]);
  return r;
}

// Per-lane-bit weights of a reverse operand's maps (XROp::lw, iw) for an
// adjoint of ry bits.
void rop_weights(int ry, XROp& op) {
  const bool wide = ry >= 6;
  const uint64_t G = wide ? 1u : (64u >> ry);
  for (int b = 0; b < 6; ++b) {
    op.lw[b] = (wide || b < ry) ? runs_pext(1ull << b, op.y_lo, op.y_len, op.y_dst)
                                : runs_pext(1ull << (b - ry), op.c_lo, op.c_len, op.c_dst);
    op.iw[b] = runs_pext(G << b, op.c_lo, op.c_len, op.c_dst);
  }
}

int gate_deriv_kind(int kind) {
  switch (kind) {
    case QT_T_ZZ: return 0;
    case QT_T_ZZ_DAG: return 1;
    case QT_T_RX: return 2;
    case QT_T_RX_DAG: return 3;
    default: return -1;
  }
}

int count_records(const qt_plan& plan) {
  int n = 0;
  for (const SymStep& st : plan.steps)
    for (const SymIn& in : st.ins) {
      const SymTensor& T = plan.tensors[in.tensor];
      if (T.leaf >= 0 && gate_deriv_kind(plan.net.leaves[T.leaf].kind) >= 0) ++n;
    }
  return n;
}

qt_status build_grad_program(const qt_plan& plan, int elt, int64_t cap_elems, int prog_id, Program& pg) {
  if (!plan.slice_vars.empty()) return fail(QT_EINVAL, "qt_energy_grad: lightcone plans take no slicing");
  if (has_gemm(plan)) return fail(QT_EUNSUPPORTED, "qt_energy_grad: lightcone plans with GEMM buckets are not supported");
  const auto& T = plan.tensors;
  const auto& S = plan.steps;
  const int ns = (int)S.size(), nt = (int)T.size(), p = plan.net.p;
  for (int t : plan.finals)
    if (T[t].leaf >= 0 || T[t].rank != 0) return fail(QT_EPLAN, "qt_energy_grad: internal: closing tensor is not a scalar");
  std::vector<char> keep(nt, 0);
  for (int t = 0; t < nt; ++t) keep[t] = T[t].leaf < 0;
  GradSched g;
  grad_schedule(plan, keep, g);
  while (g.top > cap_elems) {
    int best = -1;
    GradSched bg;
    for (int t = 0; t < nt; ++t) {
      if (!keep[t] || T[t].consumer == -2) continue;
      keep[t] = 0;
      GradSched h;
      grad_schedule(plan, keep, h);
      keep[t] = 1;
      if (best < 0 || h.top < bg.top || (h.top == bg.top && h.recompute < bg.recompute)) {
        best = t;
        bg = std::move(h);
      }
    }
    if (best < 0) break;
    keep[best] = 0;
    ++pg.dropped;
    g = std::move(bg);
  }
  if (g.top > cap_elems) {
    if (env_int("QT_DEBUG_GRAD_SCHEDULE", 0))
      std::fprintf(stderr, "[qt grad] program %d: needs %lld tensor elements after %d drops, %lld available\n", prog_id,
                   (long long)g.top, pg.dropped, (long long)cap_elems);
    pg.fits = false;
    return QT_OK;
  }
  const int tbase = x_tensor_base(p);
  pg.lds_elems = (int)g.top + tbase;
  pg.log2_const = plan.log2_const;
  pg.n_levels = g.n_levels;
  // scale slots: forward value (shared by its recomputation), then adjoint
  std::vector<int> sf(nt, -1), sb(nt, -1);
  for (int t = 0; t < nt; ++t)
    if (T[t].leaf < 0) {
      sf[t] = pg.n_slots++;
      sb[t] = pg.n_slots++;
    }
  auto at = [&](int id) { return (uint32_t)(g.off[id] + tbase); };
  auto val = [&](int t) { return Loc{at(3 * t), sf[t]}; };
  auto rval = [&](int t) { return keep[t] ? val(t) : Loc{at(3 * t + 1), sf[t]}; };
  auto adj = [&](int t) { return Loc{at(3 * t + 2), sb[t]}; };

  // forward steps keep their indices; recomputation steps follow
  pg.steps.assign(ns, XStep{});
  std::vector<int> rstep(ns, -1);
  for (int s = 0; s < ns; ++s) {
    QT_TRY(fill_xstep(plan, s, elt, val(S[s].out), val, pg.steps[s]));
    pg.cost += std::ldexp(1.0, S[s].rank) * (double)S[s].ins.size();
    pg.bytes_c64 += S[s].bytes_c64;
    pg.flops += S[s].flops;
  }
  for (int s = 0; s < ns; ++s)
    if (g.lr[s] >= 0) {
      XStep xs;
      QT_TRY(fill_xstep(plan, s, elt, rval(S[s].out), rval, xs));
      rstep[s] = (int)pg.steps.size();
      pg.steps.push_back(xs);
      ++pg.recomputed;
      pg.cost += std::ldexp(1.0, S[s].rank) * (double)S[s].ins.size();
    }

  // reverse operations, gate records grouped by parameter
  struct RecRef {
    int param, rev;
  };
  std::vector<RecRef> recs;
  std::vector<std::vector<int>> revs_of(ns);
  for (int s = 0; s < ns; ++s) {
    const SymStep& st = S[s];
    const int zs = st.sum ? 1 : 0;
    const int nz = st.rank + zs;
    const uint64_t full = (nz >= 64 ? ~0ull : ((1ull << nz) - 1ull));
    auto zmask = [&](const SymIn& in) { return ((uint64_t)in.mask << zs) | (uint64_t)(in.has_v ? 1 : 0); };
    const uint64_t zr = (((1ull << st.rank) - 1ull) << zs);
    for (size_t j = 0; j < st.ins.size(); ++j) {
      const int tj = st.ins[j].tensor;
      int gk = -1, param = -1;
      if (T[tj].leaf >= 0) {
        const Leaf& L = plan.net.leaves[T[tj].leaf];
        gk = gate_deriv_kind(L.kind);
        if (gk < 0) continue;  // constant leaf
        param = (gk < 2 ? 0 : p) + L.layer - 1;
      }
      XRev rv;
      std::memset(&rv, 0, sizeof(rv));
      const uint64_t zj = zmask(st.ins[j]);
      const uint64_t zc = full & ~zj;
      rv.ry = __builtin_popcountll(zj);
      rv.nc = __builtin_popcountll(zc);
      rv.n_ops = (int)st.ins.size();  // the adjoint R-bar and the step's other inputs
      rv.gate = gk;
      rv.param = param;
      rv.rec = -1;
      if (gk < 0) {
        const Loc a = adj(tj);
        rv.out_off = a.off;
        rv.out_slot = a.slot;
      } else {
        rv.out_off = (uint32_t)gate_offset(plan, tj);  // the gate's table block (read for its derivative)
        rv.out_slot = -1;
      }
      int o = 0;
      const Loc ar = adj(st.out);
      rv.op[o].lds_off = ar.off;
      rv.op[o].slot = ar.slot;
      if (!fill_rop(zj, zc, zr, rv.op[o])) return fail(QT_EUNSUPPORTED, "qt_energy_grad: index map too fragmented");
      ++o;
      for (size_t i = 0; i < st.ins.size(); ++i) {
        if (i == j) continue;
        const int ti = st.ins[i].tensor;
        XROp& op = rv.op[o++];
        if (T[ti].leaf >= 0) {
          const int goff = gate_offset(plan, ti);
          if (goff < 0) return fail(QT_EUNSUPPORTED, "qt_energy_grad: dense tensors are not supported in lightcones");
          op.lds_off = (uint32_t)goff;
          op.slot = -1;
        } else {
          const Loc l = rval(ti);
          op.lds_off = l.off;
          op.slot = l.slot;
        }
        if (!fill_rop(zj, zc, zmask(st.ins[i]), op))
          return fail(QT_EUNSUPPORTED, "qt_energy_grad: index map too fragmented");
      }
      for (; o < kMaxIn; ++o) rv.op[o].slot = -1;  // unused operands: identity (element 0, no runs)
      for (int q = 0; q < kMaxIn; ++q) rop_weights(rv.ry, rv.op[q]);
      if (gk >= 0) recs.push_back({param, (int)pg.revs.size()});
      revs_of[s].push_back((int)pg.revs.size());
      pg.revs.push_back(rv);
    }
  }
  std::stable_sort(recs.begin(), recs.end(), [](const RecRef& a, const RecRef& b) { return a.param < b.param; });
  pg.rec_off.assign(2 * p + 1, 0);
  for (size_t r = 0; r < recs.size(); ++r) {
    pg.revs[recs[r].rev].rec = (int32_t)r;
    pg.rec_off[recs[r].param + 1] = (int32_t)(r + 1);
  }
  for (int q = 1; q <= 2 * p; ++q) pg.rec_off[q] = std::max(pg.rec_off[q], pg.rec_off[q - 1]);
  pg.n_recs = (int)recs.size();

  for (int L = 0; L < g.n_levels; ++L) {
    pg.levels.push_back((int32_t)pg.units.size());
    for (int s = 0; s < ns; ++s) {
      if (g.lf[s] == L) push_step_units(plan, s, s, elt, pg.units);
      if (g.lr[s] == L) push_step_units(plan, s, rstep[s], elt, pg.units);
    }
    if (g.lfa == L) pg.units.push_back(make_uint2(kXUnitFinal, 0));
    for (int s = 0; s < ns; ++s) {
      if (g.lb[s] != L) continue;
      for (int r : revs_of[s]) {
        const int ry = pg.revs[r].ry;
        const uint32_t chunks = ry >= 6 ? (1u << ry) / 64u : 1u;
        for (uint32_t c = 0; c < chunks; ++c) pg.units.push_back(make_uint2(kXUnitRev | (uint32_t)r, c));
      }
    }
  }
  pg.levels.push_back((int32_t)pg.units.size());
  for (int t : plan.finals) pg.finals.push_back({val(t).off, val(t).slot});
  for (int t : plan.finals) pg.finals.push_back({adj(t).off, adj(t).slot});
  if (env_int("QT_DEBUG_GRAD_SCHEDULE", 0))
    std::fprintf(stderr,
                 "[qt grad] program %d: %d steps, %d levels, %d reverse ops, %d records, %d dropped, %d recomputed, "
                 "%d LDS elements\n",
                 prog_id, ns, pg.n_levels, (int)pg.revs.size(), pg.n_recs, pg.dropped, pg.recomputed, pg.lds_elems);
  return QT_OK;
}

uint32_t run_max(const uint8_t* lo, const uint8_t* len, const uint8_t* dst, uint64_t all) {
  uint32_t r = 0;
  for (int i = 0; i < kXRuns; ++i)
    if (len[i]) r |= (uint32_t)(((all >> lo[i]) & ((1ull << len[i]) - 1ull)) << dst[i]);
  return r;
}

// Every LDS element, scale slot and record a program's descriptors can
// touch lies inside its areas.
qt_status check_program(const Program& pg, int p) {
  const uint32_t gate_end = (uint32_t)(kXGate + x_gate_elems(p));
  auto in_range = [&](uint32_t off, uint64_t extent) { return (uint64_t)off + extent <= (uint64_t)pg.lds_elems; };
  auto bad = [](const char* what) { return fail(QT_EPLAN, std::string("qt_energy_grad: internal: ") + what); };
  for (const XStep& xs : pg.steps) {
    if (!in_range(xs.out.lds_off, 1ull << xs.r) || xs.out.slot >= pg.n_slots) return bad("step output out of range");
    for (int j = 0; j < xs.n_in; ++j) {
      const XOp& x = xs.in[j];
      const uint64_t all = (1ull << xs.r) - 1ull;
      const uint64_t hi = ((uint64_t)run_max(x.run_lo, x.run_len, x.run_dst, all) << x.has_v) + x.has_v;
      if (!in_range(x.lds_off, hi + 1) || x.slot >= pg.n_slots) return bad("step operand out of range");
      if (x.slot < 0 && x.lds_off >= 2 && x.lds_off + hi >= gate_end) return bad("gate operand out of range");
    }
  }
  for (const XRev& rv : pg.revs) {
    if (rv.ry > 16 || rv.nc > 20) return bad("reverse operation too large");
    if (rv.gate < 0 && (!in_range(rv.out_off, 1ull << rv.ry) || rv.out_slot < 0 || rv.out_slot >= pg.n_slots))
      return bad("adjoint output out of range");
    if (rv.gate >= 0 && (rv.rec < 0 || rv.rec >= pg.n_recs || rv.param < 0 || rv.param >= 2 * p ||
                         rv.out_off < (uint32_t)kXGate || rv.out_off + 4 > gate_end))
      return bad("gradient record out of range");
    for (int o = 0; o < rv.n_ops; ++o) {
      const XROp& op = rv.op[o];
      const uint64_t hi = (uint64_t)run_max(op.y_lo, op.y_len, op.y_dst, (1ull << rv.ry) - 1ull) +
                          run_max(op.c_lo, op.c_len, op.c_dst, (1ull << rv.nc) - 1ull);
      if (!in_range(op.lds_off, hi + 1) || op.slot >= pg.n_slots) return bad("reverse operand out of range");
    }
  }
  for (const XFinal& f : pg.finals)
    if (!in_range(f.lds_off, 1) || f.slot >= pg.n_slots) return bad("closing scalar out of range");
  for (const uint2& u : pg.units) {
    const uint32_t kind = u.x & ~kXUnitIndex, idx = u.x & kXUnitIndex;
    if ((kind == 0 && idx >= pg.steps.size()) || (kind == kXUnitRev && idx >= pg.revs.size()))
      return bad("unit names no descriptor");
  }
  return QT_OK;
}

// Largest element area of a forward program run from global scratch in the
// batched launch (one workgroup per item); larger lightcones take the
// general per-step schedule, whose launches spread one step over the chip.
constexpr int64_t kMaxGlobalElems = int64_t(1) << 22;

struct EnergyJob {
  std::vector<uint64_t> serials;
  int np = 0, precision = 0, p = 0;
  bool grad = false;
  bool wide = false;  // complex128 elements (c128 plans, and every gradient job)
  int64_t budget = 0, lds_cap = 0;
  int n_progs = 0;
  void* tables = nullptr;
  double* params = nullptr;
  double* out = nullptr;     // [np][n_progs][3]
  double* sums = nullptr;    // [np][3]
  double* reals = nullptr;   // [np] energies then [np][n_progs] per edge
  double* gout = nullptr;    // gradient jobs: [np][n_progs][2p]
  double* gsum = nullptr;    // [np][2p]
  double* weights = nullptr; // [n_progs]: per-edge weights of the sums (weighted calls)
  char* scratch = nullptr;   // areas of the programs run from global scratch
  XMulti multi{};
  int n_items = 0;           // programs of the batched launch
  int n_blocks = 0;          // forward launch: workgroups (program, group of points)
  size_t smem = 0;           // forward launch: LDS bytes per workgroup
  int n_fit = 0, n_global = 0;
  std::vector<int> big;      // forward programs beyond kMaxGlobalElems
  double bytes_c64 = 0, flops = 0;
  // graph of the device sequence per argument set (QT_PLAN_GRAPH)
  struct Graph {
    const void* key[7];
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
  std::mutex run_mu;  // one enqueue at a time per job (buffers are shared)
  ~EnergyJob() {
    for (Graph& g : graphs) {
      (void)hipGraphExecDestroy(g.exec);
      (void)hipGraphDestroy(g.graph);
    }
    for (void* q : {tables, (void*)params, (void*)out, (void*)sums, (void*)reals, (void*)gout, (void*)gsum,
                    (void*)weights, (void*)scratch})
      if (q) (void)hipFree(q);
  }
};

std::mutex g_mu;
std::vector<std::shared_ptr<EnergyJob>> g_jobs;

template <class T>
qt_status alloc(T** p, size_t count) {
  if (hipMalloc((void**)p, std::max<size_t>(1, count) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QT_ENOMEM, "qt_energy_grad: device allocation failed");
  }
  return QT_OK;
}

// One batched launch runs every (program, point) item.  Programs whose
// tensors fit in lds_cap bytes of LDS keep them there; the launch's
// workgroups are sized for the largest of them.  The others run the same
// schedule from a global scratch area of their own per point (the gradient
// pass for every size; the forward pass up to kMaxGlobalElems).  Items are
// dispatched in order of blockIdx, so the order is the launch's work queue:
// global-scratch programs first, then by decreasing cost, so the tail of
// the launch is made of short items.
qt_status build_job(qt_plan* const* plans, int n, int np, bool grad, int64_t lds_bytes, int64_t lds_cap,
                    EnergyJob& job) {
  // The gradient pass runs in complex128 for every precision: a derivative
  // is a sum of per-gate terms of the size of the edge energy that cancel
  // down to a much smaller value near stationary points, so FP32 arithmetic
  // does not hold the complex64 tolerance there, while FP64 costs the same
  // VALU issue rate as unpacked FP32 on this hardware.
  const bool wide = plans[0]->precision == QT_C128 || grad;
  const int elt = wide ? 16 : 8;
  const int p = plans[0]->net.p;
  // the launch shares the largest slot and record areas: size every
  // program's tensor area against them
  int max_slots = 0, max_recs = 0;
  for (int e = 0; e < n; ++e) {
    const int ni = count_intermediates(*plans[e]);
    max_slots = std::max(max_slots, grad ? 2 * ni : ni);
    if (grad) max_recs = std::max(max_recs, count_records(*plans[e]));
  }
  const int64_t fixed = 8 * (int64_t)((max_slots + 3) & ~3) + 8 * (int64_t)((max_recs + 1) & ~1);
  const int64_t cap_elems = (lds_bytes - fixed) / elt - 1 - x_tensor_base(p);  // - 1: the odd point stride
  std::vector<Program> progs(n);
  std::vector<char> global(n, 0);
  auto smem_of = [&](const Program& pg) {
    return grad ? lds_grad_smem_bytes(pg.n_slots, pg.n_recs, pg.lds_elems, elt == 16)
                : lds_exec_smem_bytes(pg.n_slots, pg.lds_elems, elt == 16);
  };
  // Forward programs in LDS: per point, the scale slots (max and exponent)
  // and the tensor area, whose stride is odd so that the points' copies of
  // an element fall in different LDS banks.
  auto slot_stride = [](const Program& pg) { return (pg.n_slots + 3) & ~3; };
  auto rec_stride = [](const Program& pg) { return (pg.n_recs + 1) & ~1; };
  auto pt_stride = [](const Program& pg) { return pg.lds_elems | 1; };
  auto pt_bytes = [&](const Program& pg) {
    return 8ll * slot_stride(pg) + 8ll * rec_stride(pg) + (int64_t)pt_stride(pg) * elt;
  };
  int p_max = 1;  // points per workgroup: a power of two, at most 64 and the points' count rounded up
  while (p_max < 64 && p_max < np) p_max *= 2;
  for (int e = 0; e < n; ++e) {
    if (grad) QT_TRY(build_grad_program(*plans[e], elt, cap_elems, e, progs[e]));
    else QT_TRY(build_program(*plans[e], elt, cap_elems, progs[e]));
    if (progs[e].fits && pt_bytes(progs[e]) > lds_cap) global[e] = 1;
    if (!progs[e].fits) {  // every intermediate kept, in global scratch
      progs[e] = Program{};
      if (grad) QT_TRY(build_grad_program(*plans[e], elt, int64_t(1) << 40, e, progs[e]));
      else QT_TRY(build_program(*plans[e], elt, int64_t(1) << 40, progs[e]));
      if (grad || progs[e].lds_elems <= kMaxGlobalElems) global[e] = 1;
      else progs[e].fits = false;
    }
    if (progs[e].fits) QT_TRY(check_program(progs[e], p));
  }
  std::vector<XProg> xp(n);
  std::vector<XStep> steps;
  std::vector<XRev> revs;
  std::vector<uint2> units;
  std::vector<int32_t> levels, rec_off;
  std::vector<XFinal> finals;
  int max_lds = 0;
  max_slots = max_recs = 0;
  int64_t scratch_bytes = 0, smem_multi = 16, max_pt_bytes = 0;
  std::vector<int> n_pts(n, 1);
  for (int e = 0; e < n; ++e) {
    const Program& pg = progs[e];
    XProg& x = xp[e];
    std::memset(&x, 0, sizeof(x));
    x.steps_off = (int32_t)steps.size();
    x.units_off = (int32_t)units.size();
    x.levels_off = (int32_t)levels.size();
    x.n_levels = pg.n_levels;
    x.n_slots = pg.n_slots;
    x.finals_off = (int32_t)finals.size();
    x.n_finals = (int32_t)(grad ? pg.finals.size() / 2 : pg.finals.size());
    x.revs_off = (int32_t)revs.size();
    x.recs_off = (int32_t)rec_off.size();
    x.n_recs = pg.n_recs;
    x.log2_const = pg.log2_const;
    x.area_elems = pg.lds_elems;
    x.scratch_off = -1;
    x.n_pts = 1;
    steps.insert(steps.end(), pg.steps.begin(), pg.steps.end());
    revs.insert(revs.end(), pg.revs.begin(), pg.revs.end());
    if (pg.fits && !global[e]) {
      // as many points as the LDS cap holds
      const int64_t b = pt_bytes(pg);
      int P = p_max;
      while (P > 1 && P * b > lds_cap) P /= 2;
      n_pts[e] = x.n_pts = P;
      x.pt_stride = pt_stride(pg);
      x.slot_stride = slot_stride(pg);
      x.rec_stride = rec_stride(pg);
      smem_multi = std::max<int64_t>(smem_multi, P * b);
      max_pt_bytes = std::max(max_pt_bytes, b);
      std::vector<uint2> pu;
      std::vector<int32_t> pl;
      if (grad) grad_pts_units(pg, P, elt, pu, pl);
      else pts_units(pg, P, elt, pu, pl);
      units.insert(units.end(), pu.begin(), pu.end());
      levels.insert(levels.end(), pl.begin(), pl.end());
    } else {
      units.insert(units.end(), pg.units.begin(), pg.units.end());
      levels.insert(levels.end(), pg.levels.begin(), pg.levels.end());
    }
    finals.insert(finals.end(), pg.finals.begin(), pg.finals.end());
    rec_off.insert(rec_off.end(), pg.rec_off.begin(), pg.rec_off.end());
    if (global[e]) {
      x.scratch_off = scratch_bytes;
      x.scratch_stride = multi_scratch_bytes(pg.n_slots, grad ? pg.n_recs : 0, pg.lds_elems, wide);
      scratch_bytes += (int64_t)np * x.scratch_stride;
    } else if (pg.fits) {
      max_lds = std::max(max_lds, pg.lds_elems);
      max_slots = std::max(max_slots, pg.n_slots);
      max_recs = std::max(max_recs, pg.n_recs);
    }
    job.bytes_c64 += pg.bytes_c64;
    job.flops += pg.flops;
  }
  std::vector<int32_t> order;
  for (int e = 0; e < n; ++e) {
    if (global[e]) ++job.n_global;
    else if (progs[e].fits) ++job.n_fit;
    if (progs[e].fits) order.push_back(e);
    else job.big.push_back(e);
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (global[a] != global[b]) return global[a] > global[b];
    return progs[a].cost > progs[b].cost;
  });
  job.n_items = (int)order.size();
  // forward launch: one workgroup per (program, group of its points)
  std::vector<int2> items;
  for (int e : order)
    for (int pt = 0; pt < np; pt += n_pts[e]) items.push_back(make_int2(e, pt));
  job.n_blocks = (int)items.size();
  job.smem = (size_t)smem_multi;
  auto pad = [](size_t b) { return (b + 255) & ~(size_t)255; };
  struct Part {
    const void* src;
    size_t bytes;
  };
  const Part parts[] = {{xp.data(), xp.size() * sizeof(XProg)},
                        {steps.data(), steps.size() * sizeof(XStep)},
                        {units.data(), units.size() * sizeof(uint2)},
                        {levels.data(), levels.size() * sizeof(int32_t)},
                        {finals.data(), finals.size() * sizeof(XFinal)},
                        {order.data(), order.size() * sizeof(int32_t)},
                        {revs.data(), revs.size() * sizeof(XRev)},
                        {rec_off.data(), rec_off.size() * sizeof(int32_t)},
                        {items.data(), items.size() * sizeof(int2)}};
  constexpr int kParts = sizeof(parts) / sizeof(parts[0]);
  size_t at[kParts], total = 0;
  for (int i = 0; i < kParts; ++i) {
    at[i] = total;
    total += pad(std::max<size_t>(1, parts[i].bytes));
  }
  std::vector<char> host(total, 0);
  for (int i = 0; i < kParts; ++i)
    if (parts[i].bytes) std::memcpy(host.data() + at[i], parts[i].src, parts[i].bytes);
  QT_TRY(alloc((char**)&job.tables, total));
  QT_HIP_CHECK(hipMemcpy(job.tables, host.data(), total, hipMemcpyHostToDevice));
  QT_TRY(alloc(&job.params, (size_t)np * 2 * std::max(1, p)));
  QT_TRY(alloc(&job.out, (size_t)np * n * 3));
  QT_TRY(alloc(&job.sums, (size_t)np * 3));
  QT_TRY(alloc(&job.reals, (size_t)np * (n + 1)));
  QT_TRY(alloc(&job.weights, (size_t)n));
  if (grad) {
    QT_TRY(alloc(&job.gout, (size_t)np * n * 2 * std::max(1, p)));
    QT_TRY(alloc(&job.gsum, (size_t)np * 2 * std::max(1, p)));
  }
  if (scratch_bytes) QT_TRY(alloc(&job.scratch, (size_t)scratch_bytes));
  char* base = (char*)job.tables;
  XMulti& m = job.multi;
  m.progs = (const XProg*)(base + at[0]);
  m.steps = (const XStep*)(base + at[1]);
  m.units = (const uint2*)(base + at[2]);
  m.level_off = (const int32_t*)(base + at[3]);
  m.finals = (const XFinal*)(base + at[4]);
  m.item_prog = (const int32_t*)(base + at[5]);
  m.revs = (const XRev*)(base + at[6]);
  m.rec_off = (const int32_t*)(base + at[7]);
  m.items = (const int2*)(base + at[8]);
  m.gam = job.params;
  m.bet = job.params + p;
  m.pstride = 2 * p;
  m.out = job.out;
  m.gout = job.gout;
  m.n_points = np;
  m.n_progs = n;
  m.p = p;
  m.lds_elems = max_lds;
  m.n_slots = max_slots;
  m.n_recs = max_recs;
  m.scratch = job.scratch;
  job.np = np;
  job.n_progs = n;
  job.p = p;
  job.grad = grad;
  job.wide = wide;
  job.budget = lds_bytes;
  job.lds_cap = lds_cap;
  job.precision = plans[0]->precision;
  for (int e = 0; e < n; ++e) job.serials.push_back(plans[e]->serial);
  if (env_int("QT_DEBUG_GRAD_SCHEDULE", 0))
    std::fprintf(stderr,
                 "[qt grad] job: %d of %d programs in LDS, %zu bytes of LDS per workgroup, %d from global scratch, "
                 "%lld scratch bytes, %d by steps, %lld bytes per point\n",
                 job.n_fit, n, job.smem, job.n_global, (long long)scratch_bytes, (int)job.big.size(),
                 (long long)max_pt_bytes);
  return QT_OK;
}

qt_status copy_out(double* dst, const double* src, size_t n, hipStream_t stream) {
  if (!dst) return QT_OK;
  return copy_2d(dst, n * sizeof(double), src, n * sizeof(double), n * sizeof(double), 1, stream);
}

}  // namespace

void energy_forget(uint64_t serial) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_jobs.erase(std::remove_if(g_jobs.begin(), g_jobs.end(),
                              [&](const std::shared_ptr<EnergyJob>& j) {
                                return std::find(j->serials.begin(), j->serials.end(), serial) != j->serials.end();
                              }),
               g_jobs.end());
}

}  // namespace qt

using namespace qt;

namespace {

qt_status energy_grad(qt_plan* const* lightcones, int32_t n_edges, const double* weights, int32_t n_points,
                      const double* gammas, const double* betas, double* energy, double* dE_dgamma, double* dE_dbeta,
                      double* per_edge, void* hip_stream) {
  try {
    if (!lightcones || n_edges <= 0 || n_points <= 0 || !energy)
      return fail(QT_EINVAL, "qt_energy_grad: bad arguments");
    const int p = lightcones[0] ? lightcones[0]->net.p : 0;
    if (p > 0 && (!gammas || !betas)) return fail(QT_EINVAL, "qt_energy_grad: null parameters");
    for (int e = 0; e < n_edges; ++e) {
      if (!lightcones[e]) return fail(QT_EINVAL, "qt_energy_grad: null plan");
      if (lightcones[e]->net.p != p || lightcones[e]->precision != lightcones[0]->precision)
        return fail(QT_EINVAL, "qt_energy_grad: plans differ in p or precision");
      if (!lightcones[e]->open_vars.empty() || !lightcones[e]->slice_vars.empty())
        return fail(QT_EINVAL, "qt_energy_grad: lightcone plans take no slicing and no open variables");
    }
    const bool w_dev = weights && is_device_ptr(weights);
    if (weights && !w_dev)
      for (int e = 0; e < n_edges; ++e)
        if (!(weights[e] >= 0.0)) return fail(QT_EINVAL, "qt_energy_grad_weighted: negative or NaN weight");
    const bool grad = dE_dgamma || dE_dbeta;
    const qt_tuning& tu = lightcones[0]->tuning;
    const int64_t lds_bytes = std::min<int64_t>(160 * 1024, env_int("QT_LDS_BYTES", 160 * 1024));
    const int64_t budget = grad ? std::min<int64_t>(lds_bytes, env_int("QT_GRAD_LDS_BYTES", (int)lds_bytes)) : lds_bytes;
    // Default LDS per workgroup (the autotuner searches this tunable): a few
    // points of a lightcone per workgroup with several workgroups per
    // compute unit; the time follows the points per wavefront, so the
    // default pairs 32 KiB with four wavefronts (measured on the 1000-node
    // p = 3 energy and the 200-node p = 2 gradient).
    const int dflt_cap = (!grad && lightcones[0]->precision == QT_C128) ? 65536 : 32768;
    const int64_t lds_cap = std::min<int64_t>(budget, grad ? tuned(tu.grad_lds_cap, "QT_GRAD_LDS_CAP", dflt_cap)
                                                           : tuned(tu.multi_lds_cap, "QT_MULTI_LDS_CAP", dflt_cap));
    hipStream_t stream = (hipStream_t)hip_stream;
    std::shared_ptr<EnergyJob> job;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      for (auto& j : g_jobs) {
        if (j->np != n_points || (int)j->serials.size() != n_edges || j->grad != grad || j->budget != budget ||
            j->lds_cap != lds_cap)
          continue;
        bool same = true;
        for (int e = 0; e < n_edges && same; ++e) same = j->serials[e] == lightcones[e]->serial;
        if (same) {
          job = j;
          break;
        }
      }
      if (!job) {
        auto nj = std::make_shared<EnergyJob>();
        QT_TRY(build_job(lightcones, n_edges, n_points, grad, budget, lds_cap, *nj));
        if (g_jobs.size() >= 16) g_jobs.erase(g_jobs.begin());
        g_jobs.push_back(nj);
        job = nj;
      }
    }
    const int waves = std::max(1, std::min(kXMaxThreads / 64, grad ? tuned(tu.grad_waves, "QT_LDS_WAVES_GRAD", 4)
                                                                    : tuned(tu.multi_waves, "QT_LDS_WAVES_MULTI", 4)));
    std::lock_guard<std::mutex> run_lk(job->run_mu);
    // The device sequence: parameters in, the batched launch, the FP64 sums
    // over edges and the results out.
    auto enqueue = [&](hipStream_t s) -> qt_status {
      EnergyJob& J = *job;
      // parameters in device memory are read where they are; host ones go
      // to the job's buffer ([points][2p])
      XMulti m = J.multi;
      if (p > 0 && is_device_ptr(gammas) && is_device_ptr(betas)) {
        m.gam = gammas;
        m.bet = betas;
        m.pstride = p;
      } else {
        QT_TRY(upload_params_to(J.params, n_points, p, gammas, betas, s));
      }
      if (grad) QT_HIP_CHECK(launch_lds_grad(m, J.n_blocks, J.smem, waves, s));
      else QT_HIP_CHECK(launch_lds_multi(m, J.n_blocks, J.smem, waves, J.wide, !J.wide, s));
      for (int e : J.big) {
        const double* sums = nullptr;
        QT_TRY(run_plan_points(*lightcones[e], n_points, gammas, betas, s, &sums));
        QT_HIP_CHECK(hipMemcpy2DAsync(J.out + 3 * e, (size_t)n_edges * 3 * sizeof(double), sums, 3 * sizeof(double),
                                      3 * sizeof(double), n_points, hipMemcpyDeviceToDevice, s));
      }
      // device weights and results are read and written where they are
      const double* w = nullptr;
      if (weights && is_device_ptr(weights)) {
        w = weights;
      } else if (weights) {
        const size_t wb = sizeof(double) * n_edges;
        QT_TRY(copy_2d(J.weights, wb, weights, wb, wb, 1, s));
        w = J.weights;
      }
      QT_HIP_CHECK(launch_slice_sum(J.out, n_points, n_edges, J.sums, s, w));
      if (energy && is_device_ptr(energy)) {
        QT_HIP_CHECK(launch_amp_to_real(J.sums, n_points, energy, s));
      } else {
        QT_HIP_CHECK(launch_amp_to_real(J.sums, n_points, J.reals, s));
        QT_TRY(copy_out(energy, J.reals, n_points, s));
      }
      if (per_edge && is_device_ptr(per_edge)) {
        QT_HIP_CHECK(launch_amp_to_real(J.out, (int64_t)n_points * n_edges, per_edge, s));
      } else if (per_edge) {
        QT_HIP_CHECK(launch_amp_to_real(J.out, (int64_t)n_points * n_edges, J.reals + n_points, s));
        QT_TRY(copy_out(per_edge, J.reals + n_points, (size_t)n_points * n_edges, s));
      }
      if (grad && p > 0) {
        QT_HIP_CHECK(launch_rows_sum(J.gout, n_points, n_edges, 2 * p, J.gsum, s, w));
        const size_t row = p * sizeof(double), pitch = 2 * p * sizeof(double);
        if (dE_dgamma) QT_TRY(copy_2d(dE_dgamma, row, J.gsum, pitch, row, n_points, s));
        if (dE_dbeta) QT_TRY(copy_2d(dE_dbeta, row, J.gsum + p, pitch, row, n_points, s));
      }
      return QT_OK;
    };
    // QT_PLAN_GRAPH on lightcones[0]: with every argument in device memory
    // and no lightcone on the per-step schedule, capture the sequence once
    // per argument set and replay it (kernels and device copies only).
    auto dev = [](const void* q) { return !q || is_device_ptr(q); };
    const bool graph = (lightcones[0]->flags & QT_PLAN_GRAPH) && job->big.empty() && (p == 0 || (dev(gammas) && dev(betas))) &&
                       dev(energy) && dev(dE_dgamma) && dev(dE_dbeta) && dev(per_edge) && dev(weights);
    if (!graph) return enqueue(stream);
    const void* key[7] = {gammas, betas, weights, energy, dE_dgamma, dE_dbeta, per_edge};
    EnergyJob::Graph* hit = nullptr;
    for (auto& g : job->graphs)
      if (std::equal(key, key + 7, g.key)) hit = &g;
    if (!hit) {
      if (job->graphs.size() >= 8) {
        for (auto& g : job->graphs) {
          (void)hipGraphExecDestroy(g.exec);
          (void)hipGraphDestroy(g.graph);
        }
        job->graphs.clear();
      }
      hipStream_t cs = nullptr;
      QT_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      qt_status st = QT_OK;
      if (e == hipSuccess) {
        st = enqueue(cs);
        e = hipStreamEndCapture(cs, &g);
      }
      (void)hipStreamDestroy(cs);
      if (st != QT_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return fail(QT_EHIP, std::string("qt_energy_grad: graph capture: ") + hipGetErrorString(e));
      hipGraphExec_t x = nullptr;
      e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(QT_EHIP, std::string("qt_energy_grad: graph instantiation: ") + hipGetErrorString(e));
      }
      EnergyJob::Graph ng;
      std::copy(key, key + 7, ng.key);
      ng.graph = g;
      ng.exec = x;
      job->graphs.push_back(ng);
      hit = &job->graphs.back();
    }
    QT_HIP_CHECK(hipGraphLaunch(hit->exec, stream));
    return QT_OK;
  } catch (const std::exception& ex) {
    return fail(QT_ENOMEM, std::string("qt_energy_grad: ") + ex.what());
  }
}

}  // namespace

extern "C" qt_status qt_energy_grad(qt_plan* const* lightcones, int32_t n_edges, int32_t n_points,
                                    const double* gammas, const double* betas, double* energy, double* dE_dgamma,
                                    double* dE_dbeta, double* per_edge, void* hip_stream) {
  return energy_grad(lightcones, n_edges, nullptr, n_points, gammas, betas, energy, dE_dgamma, dE_dbeta, per_edge,
                     hip_stream);
}

extern "C" qt_status qt_energy_grad_weighted(qt_plan* const* lightcones, const double* edge_weights, int32_t n_edges,
                                             int32_t n_points, const double* gammas, const double* betas,
                                             double* energy, double* dE_dgamma, double* dE_dbeta, double* per_edge,
                                             void* hip_stream) {
  if (!edge_weights) return fail(QT_EINVAL, "qt_energy_grad_weighted: null weights");
  return energy_grad(lightcones, n_edges, edge_weights, n_points, gammas, betas, energy, dE_dgamma, dE_dbeta,
                     per_edge, hip_stream);
}
