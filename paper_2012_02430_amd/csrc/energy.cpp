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
#include <cstring>
#include <mutex>

#include "qt_internal.h"

namespace qt {
namespace {

struct Program {
  bool fits = true;
  std::vector<XStep> steps;
  std::vector<uint2> units;
  std::vector<int32_t> levels;
  std::vector<XFinal> finals;
  int n_levels = 0, n_slots = 0, lds_elems = 0;
  double log2_const = 0, cost = 0, bytes_c64 = 0, flops = 0;
};

qt_status build_program(const qt_plan& plan, int elt, int64_t lds_bytes, Program& pg) {
  if (!plan.slice_vars.empty()) return fail(QT_EINVAL, "qt_energy_grad: lightcone plans take no slicing");
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
  const int tbase = x_tensor_base(plan.net.p);
  const int64_t cap = (lds_bytes - 8 * (int64_t)(iv.size() + 4)) / elt - tbase;
  if (top > cap) {
    pg.fits = false;  // contracted through the general schedule instead
    return QT_OK;
  }
  std::vector<int> slot(ntens, -1);
  for (const Interval& it : iv) slot[it.t] = pg.n_slots++;
  pg.lds_elems = (int)top + tbase;
  pg.log2_const = plan.log2_const;

  pg.steps.assign(nsteps, XStep{});
  for (int i = 0; i < nsteps; ++i) {
    const SymStep& st = plan.steps[i];
    XStep& xs = pg.steps[i];
    std::memset(&xs, 0, sizeof(xs));
    xs.out.ptr = nullptr;
    xs.out.lds_off = (uint32_t)(off[st.out] + tbase);
    xs.out.slot_kind = 1;
    xs.out.slot = slot[st.out];
    xs.r = st.rank;
    xs.sum = st.sum;
    xs.n_in = x_nin_class((int)st.ins.size());
    const int epu = x_epu(st.rank, (int)st.ins.size(), elt);
    for (size_t j = 0; j < st.ins.size(); ++j) {
      const SymIn& si = st.ins[j];
      const SymTensor& T = plan.tensors[si.tensor];
      XOp& x = xs.in[j];
      x.slot = -1;
      if (T.leaf >= 0) {
        const Leaf& L = plan.net.leaves[T.leaf];
        const int g = x_gate_off(L.kind, L.layer);
        if (g < 0) return fail(QT_EUNSUPPORTED, "qt_energy_grad: dense tensors are not supported in lightcones");
        x.lds_off = (uint32_t)g;
      } else {
        x.lds_off = (uint32_t)(off[si.tensor] + tbase);
        x.slot = slot[si.tensor];
      }
      x.has_v = si.has_v;
      int32_t nr = 0;
      if (!make_runs(si.mask, kXRuns, x.run_lo, x.run_len, x.run_dst, nr))
        return fail(QT_EUNSUPPORTED, "qt_energy_grad: index map too fragmented");
      for (int e = 0; e < 4; ++e) {
        uint32_t r = 0;
        if (e < epu)
          for (int q = 0; q < nr; ++q)
            r |= (((uint32_t)(64 * e) >> x.run_lo[q]) & ((1u << x.run_len[q]) - 1u)) << x.run_dst[q];
        x.ep[e] = r;
      }
    }
    for (int j = (int)st.ins.size(); j < xs.n_in; ++j) {
      XOp& id = xs.in[j];  // identity operand
      std::memset(&id, 0, sizeof(id));
      id.has_v = 1;
      id.slot = -1;
    }
    pg.cost += std::ldexp(1.0, st.rank) * (double)st.ins.size();
    pg.bytes_c64 += st.bytes_c64;
    pg.flops += st.flops;
  }
  for (int L = 0; L < pg.n_levels; ++L) {
    pg.levels.push_back((int32_t)pg.units.size());
    for (int i = 0; i < nsteps; ++i)
      if (depth[i] == L) {
        const int r = plan.steps[i].rank;
        const int64_t chunks = std::max<int64_t>(1, (1ll << r) / x_unit_elems(r, (int)plan.steps[i].ins.size(), elt));
        for (int64_t c = 0; c < chunks; ++c) pg.units.push_back(make_uint2((uint32_t)i, (uint32_t)c));
      }
  }
  pg.levels.push_back((int32_t)pg.units.size());
  for (int t : plan.finals) {
    if (plan.tensors[t].leaf >= 0) return fail(QT_EPLAN, "qt_energy_grad: internal: leaf as closing scalar");
    pg.finals.push_back({(uint32_t)(off[t] + tbase), slot[t]});
  }
  return QT_OK;
}

struct EnergyJob {
  std::vector<uint64_t> serials;
  int np = 0, precision = 0, p = 0;
  int n_progs = 0;
  void* tables = nullptr;
  double* params = nullptr;
  double* out = nullptr;     // [np][n_progs][3]
  double* sums = nullptr;    // [np][3]
  double* reals = nullptr;   // [np] energies then [np][n_progs] per edge
  XMulti multi{};
  int n_fit = 0;
  std::vector<int> big;  // programs that do not fit in LDS
  double bytes_c64 = 0, flops = 0;
  ~EnergyJob() {
    for (void* q : {tables, (void*)params, (void*)out, (void*)sums, (void*)reals})
      if (q) (void)hipFree(q);
  }
};

std::mutex g_mu;
std::vector<std::unique_ptr<EnergyJob>> g_jobs;

template <class T>
qt_status alloc(T** p, size_t count) {
  if (hipMalloc((void**)p, std::max<size_t>(1, count) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QT_ENOMEM, "qt_energy_grad: device allocation failed");
  }
  return QT_OK;
}

#define QT_TRY(expr)            \
  do {                          \
    qt_status _s = (expr);      \
    if (_s != QT_OK) return _s; \
  } while (0)

qt_status build_job(qt_plan* const* plans, int n, int np, EnergyJob& job) {
  const int elt = plans[0]->precision == QT_C128 ? 16 : 8;
  const int64_t lds_bytes = std::min(160 * 1024, env_int("QT_LDS_BYTES", 160 * 1024));
  std::vector<Program> progs(n);
  for (int e = 0; e < n; ++e) QT_TRY(build_program(*plans[e], elt, lds_bytes, progs[e]));
  std::vector<XProg> xp(n);
  std::vector<XStep> steps;
  std::vector<uint2> units;
  std::vector<int32_t> levels;
  std::vector<XFinal> finals;
  int max_lds = 0, max_slots = 0;
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
    x.n_finals = (int32_t)pg.finals.size();
    x.log2_const = pg.log2_const;
    steps.insert(steps.end(), pg.steps.begin(), pg.steps.end());
    units.insert(units.end(), pg.units.begin(), pg.units.end());
    levels.insert(levels.end(), pg.levels.begin(), pg.levels.end());
    finals.insert(finals.end(), pg.finals.begin(), pg.finals.end());
    max_lds = std::max(max_lds, pg.lds_elems);
    max_slots = std::max(max_slots, pg.n_slots);
    job.bytes_c64 += pg.bytes_c64;
    job.flops += pg.flops;
  }
  // longest programs first, so the tail of the launch is made of short ones;
  // programs that do not fit in LDS run separately
  std::vector<int32_t> order;
  for (int e = 0; e < n; ++e) {
    if (progs[e].fits) order.push_back(e);
    else job.big.push_back(e);
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return progs[a].cost > progs[b].cost; });
  job.n_fit = (int)order.size();
  auto pad = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t b0 = pad(xp.size() * sizeof(XProg)), b1 = pad(steps.size() * sizeof(XStep)),
               b2 = pad(units.size() * sizeof(uint2)), b3 = pad(levels.size() * sizeof(int32_t)),
               b4 = pad(std::max<size_t>(1, finals.size()) * sizeof(XFinal)), b5 = pad(order.size() * sizeof(int32_t));
  const size_t total = b0 + b1 + b2 + b3 + b4 + std::max<size_t>(b5, 256);
  std::vector<char> host(total, 0);
  size_t o = 0;
  auto put = [&](const void* src, size_t bytes, size_t span) {
    if (bytes) std::memcpy(host.data() + o, src, bytes);
    const size_t at = o;
    o += span;
    return at;
  };
  const size_t o0 = put(xp.data(), xp.size() * sizeof(XProg), b0);
  const size_t o1 = put(steps.data(), steps.size() * sizeof(XStep), b1);
  const size_t o2 = put(units.data(), units.size() * sizeof(uint2), b2);
  const size_t o3 = put(levels.data(), levels.size() * sizeof(int32_t), b3);
  const size_t o4 = put(finals.data(), finals.size() * sizeof(XFinal), b4);
  const size_t o5 = put(order.data(), order.size() * sizeof(int32_t), b5);
  QT_TRY(alloc((char**)&job.tables, total));
  QT_HIP_CHECK(hipMemcpy(job.tables, host.data(), total, hipMemcpyHostToDevice));
  const int p = plans[0]->net.p;
  QT_TRY(alloc(&job.params, (size_t)np * 2 * std::max(1, p)));
  QT_TRY(alloc(&job.out, (size_t)np * n * 3));
  QT_TRY(alloc(&job.sums, (size_t)np * 3));
  QT_TRY(alloc(&job.reals, (size_t)np * (n + 1)));
  char* base = (char*)job.tables;
  XMulti& m = job.multi;
  m.progs = (const XProg*)(base + o0);
  m.steps = (const XStep*)(base + o1);
  m.units = (const uint2*)(base + o2);
  m.level_off = (const int32_t*)(base + o3);
  m.finals = (const XFinal*)(base + o4);
  m.item_prog = (const int32_t*)(base + o5);
  m.params = job.params;
  m.out = job.out;
  m.n_points = np;
  m.n_progs = n;
  m.p = p;
  m.lds_elems = max_lds;
  m.n_slots = max_slots;
  job.np = np;
  job.n_progs = n;
  job.p = p;
  job.precision = plans[0]->precision;
  for (int e = 0; e < n; ++e) job.serials.push_back(plans[e]->serial);
  return QT_OK;
}

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

qt_status copy_out(double* dst, const double* src, size_t n, hipStream_t stream) {
  if (!dst) return QT_OK;
  QT_HIP_CHECK(hipMemcpyAsync(dst, src, n * sizeof(double),
                              is_device_ptr(dst) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, stream));
  return QT_OK;
}

}  // namespace

void energy_forget(uint64_t serial) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_jobs.erase(std::remove_if(g_jobs.begin(), g_jobs.end(),
                              [&](const std::unique_ptr<EnergyJob>& j) {
                                return std::find(j->serials.begin(), j->serials.end(), serial) != j->serials.end();
                              }),
               g_jobs.end());
}

}  // namespace qt

using namespace qt;

extern "C" qt_status qt_energy_grad(qt_plan* const* lightcones, int32_t n_edges, int32_t n_points,
                                    const double* gammas, const double* betas, double* energy, double* dE_dgamma,
                                    double* dE_dbeta, double* per_edge, void* hip_stream) {
  try {
    if (!lightcones || n_edges <= 0 || n_points <= 0 || !energy)
      return fail(QT_EINVAL, "qt_energy_grad: bad arguments");
    const int p = lightcones[0] ? lightcones[0]->net.p : 0;
    if (p > 0 && (!gammas || !betas)) return fail(QT_EINVAL, "qt_energy_grad: null parameters");
    for (int e = 0; e < n_edges; ++e) {
      if (!lightcones[e]) return fail(QT_EINVAL, "qt_energy_grad: null plan");
      if (lightcones[e]->net.p != p || lightcones[e]->precision != lightcones[0]->precision)
        return fail(QT_EINVAL, "qt_energy_grad: plans differ in p or precision");
    }
    if (dE_dgamma || dE_dbeta) return fail(QT_EUNSUPPORTED, "qt_energy_grad: the gradient pass is not built yet");
    hipStream_t stream = (hipStream_t)hip_stream;
    EnergyJob* job = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      for (auto& j : g_jobs) {
        if (j->np != n_points || (int)j->serials.size() != n_edges) continue;
        bool same = true;
        for (int e = 0; e < n_edges && same; ++e) same = j->serials[e] == lightcones[e]->serial;
        if (same) {
          job = j.get();
          break;
        }
      }
      if (!job) {
        auto nj = std::make_unique<EnergyJob>();
        QT_TRY(build_job(lightcones, n_edges, n_points, *nj));
        if (g_jobs.size() >= 16) g_jobs.erase(g_jobs.begin());
        g_jobs.push_back(std::move(nj));
        job = g_jobs.back().get();
      }
    }
    const bool c128 = job->precision == QT_C128;
    if (p > 0) {
      const size_t pitch = 2 * p * sizeof(double);
      QT_HIP_CHECK(hipMemcpy2DAsync(job->params, pitch, gammas, p * sizeof(double), p * sizeof(double), n_points,
                                    hipMemcpyDefault, stream));
      QT_HIP_CHECK(hipMemcpy2DAsync(job->params + p, pitch, betas, p * sizeof(double), p * sizeof(double), n_points,
                                    hipMemcpyDefault, stream));
    }
    const int waves = std::max(1, std::min(kXMaxThreads / 64, env_int("QT_LDS_WAVES_MULTI", 4)));
    if (job->n_fit) {
      XMulti m = job->multi;
      m.n_progs = n_edges;  // output row length; items cover the fitting programs only
      QT_HIP_CHECK(launch_lds_multi(m, job->n_fit, waves, c128, !c128, stream));
    }
    for (int e : job->big) {
      const double* sums = nullptr;
      QT_TRY(run_plan_points(*lightcones[e], n_points, gammas, betas, stream, &sums));
      QT_HIP_CHECK(hipMemcpy2DAsync(job->out + 3 * e, (size_t)n_edges * 3 * sizeof(double), sums, 3 * sizeof(double),
                                    3 * sizeof(double), n_points, hipMemcpyDeviceToDevice, stream));
    }
    QT_HIP_CHECK(launch_slice_sum(job->out, n_points, n_edges, job->sums, stream));
    QT_HIP_CHECK(launch_amp_to_real(job->sums, n_points, job->reals, stream));
    QT_TRY(copy_out(energy, job->reals, n_points, stream));
    if (per_edge) {
      QT_HIP_CHECK(launch_amp_to_real(job->out, (int64_t)n_points * n_edges, job->reals + n_points, stream));
      QT_TRY(copy_out(per_edge, job->reals + n_points, (size_t)n_points * n_edges, stream));
    }
    if (!is_device_ptr(energy) || (per_edge && !is_device_ptr(per_edge))) QT_HIP_CHECK(hipStreamSynchronize(stream));
    return QT_OK;
  } catch (const std::exception& ex) {
    return fail(QT_ENOMEM, std::string("qt_energy_grad: ") + ex.what());
  }
}
