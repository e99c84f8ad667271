// Execution of compiled plans: workspace, step descriptors and the launch
// sequence of Algorithm 1 on one GPU -- gate tensors, the serial prefix,
// the per-slice steps batched over slices (the loop over ranks becomes a
// batch dimension), per-slice scalars, and the FP64 sum over slices.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <functional>

#include "qt_internal.h"

namespace qt {
namespace {

// Default device workspace budget for the per-slice arena.
constexpr int64_t kDefaultBudget = 64ll << 30;


int ilog2(int64_t x) {
  int r = 0;
  while ((1ll << r) < x) ++r;
  return r;
}

}  // namespace
}  // namespace qt

using namespace qt;

namespace qt {
int env_int(const char* name, int dflt) {
  const char* e = std::getenv(name);
  return e ? std::atoi(e) : dflt;
}

int tuned(int32_t value, const char* env, int dflt) { return value > 0 ? value : env_int(env, dflt); }

uint64_t next_ws_gen() {
  static std::atomic<uint64_t> g{1};
  return g++;
}

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof(a));
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

qt_status copy_2d(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width, size_t height,
                  hipStream_t stream) {
  if (!dst || !src || width == 0 || height == 0) return QT_OK;
  if (is_device_ptr(dst) && is_device_ptr(src)) {
    QT_HIP_CHECK(hipMemcpy2DAsync(dst, dpitch, src, spitch, width, height, hipMemcpyDeviceToDevice, stream));
    return QT_OK;
  }
  // host memory involved: drain the stream, then blocking 1-D copies with
  // an explicit direction (2-D copies to pageable memory were seen to leave
  // the destination unwritten)
  const bool dd = is_device_ptr(dst), sd = is_device_ptr(src);
  const hipMemcpyKind kind = dd ? hipMemcpyHostToDevice : (sd ? hipMemcpyDeviceToHost : hipMemcpyHostToHost);
  QT_HIP_CHECK(hipStreamSynchronize(stream));
  if (dpitch == width && spitch == width) {
    QT_HIP_CHECK(hipMemcpy(dst, src, width * height, kind));
  } else {
    for (size_t r = 0; r < height; ++r)
      QT_HIP_CHECK(hipMemcpy((char*)dst + r * dpitch, (const char*)src + r * spitch, width, kind));
  }
  return QT_OK;
}

qt_status upload_params_to(double* dev, int np, int p, const double* gammas, const double* betas,
                           hipStream_t stream) {
  if (p == 0) return QT_OK;
  const size_t row = (size_t)p * sizeof(double), pitch = 2 * row;
  if (is_device_ptr(gammas) && is_device_ptr(betas)) {
    QT_TRY(copy_2d(dev, pitch, gammas, row, row, np, stream));
    return copy_2d(dev + p, pitch, betas, row, row, np, stream);
  }
  // host parameters: interleave here, one blocking copy
  std::vector<double> h((size_t)np * 2 * p);
  for (int i = 0; i < np; ++i)
    for (int k = 0; k < p; ++k) {
      h[(size_t)i * 2 * p + k] = gammas[(size_t)i * p + k];
      h[(size_t)i * 2 * p + p + k] = betas[(size_t)i * p + k];
    }
  return copy_2d(dev, h.size() * sizeof(double), h.data(), h.size() * sizeof(double), h.size() * sizeof(double), 1,
                 stream);
}

bool make_runs(uint32_t mask, int max_runs, uint8_t* lo, uint8_t* len, uint8_t* dst, int32_t& nruns) {
  int n = 0, d = 0;
  for (int b = 0; b < 32;) {
    if (!((mask >> b) & 1u)) {
      ++b;
      continue;
    }
    int e = b;
    while (e < 32 && ((mask >> e) & 1u)) ++e;
    if (n == max_runs) return false;
    lo[n] = (uint8_t)b;
    len[n] = (uint8_t)(e - b);
    dst[n] = (uint8_t)d;
    d += e - b;
    ++n;
    b = e;
  }
  nruns = n;
  return true;
}

}  // namespace qt

struct qt_plan::Workspace {
  int np = 0;
  int64_t chunk = 0;
  void* leaves = nullptr;
  void* arena0 = nullptr;
  void* arena1 = nullptr;
  int* exps = nullptr;
  uint32_t* maxbits = nullptr;
  double* params = nullptr;
  DevLeaf* dleaves = nullptr;
  double* ddense = nullptr;
  DevIn* dfinal = nullptr;
  double* per_slice = nullptr;
  int64_t per_slice_cap = 0;
  double* sums = nullptr;
  int64_t bytes = 0;
  int64_t n_exp = 0, exp1_base = 0, exp1_count = 0;
  uint64_t gen = 0;  // changes whenever device buffers are (re)allocated
  std::vector<DevStep> steps;
  std::vector<DevGemm> gemms;  // per step (used by GEMM steps only)
  std::vector<int64_t> step_elems;
  std::vector<DevIn> finals;
  // Launch sequence: a streaming step (seg < 0, index `step`) or an LDS
  // segment (index `seg`), separately for the prefix and the per-slice part.
  struct Op {
    int step;
    int seg;
  };
  struct Segment {
    int level = 0;
    std::vector<int> steps;  // plan step ids, in plan order
    int n_levels = 0;
    int n_slots = 0;
    int lds_elems = 0;
    double bytes_c64 = 0, flops = 0;  // per item
    std::vector<XStep> xsteps;
    std::vector<XStep> ustep;  // per unit, level order
    std::vector<XCopy> copies;
    std::vector<uint2> units;
    std::vector<int32_t> level_off;
    XLaunch launch{};
  };
  std::vector<Op> prefix_ops, slice_ops;
  std::vector<Segment> segs;
  void* seg_tables = nullptr;
  int waves = 8;
  // schedule (independent of batch size): per step its segment and level,
  // per tensor its LDS offset/slot (-1: global) and global arena offset
  bool planned = false;
  std::vector<int> seg_of, depth;
  bool leaves_read = true;  // some launch reads the leaf tensors from global memory
  std::vector<int64_t> lds_off;
  std::vector<int> lds_slot;
  std::vector<int> staged_in;  // segment that stages the tensor into LDS, -1: none
  std::vector<int64_t> unit_off;
  int64_t arena0_units = 0, arena1_units = 0;
  // QT_DEBUG_LEVEL_TRACE: per-level clock of workgroup 0 of each segment launch
  bool trace_on = false;
  uint64_t* trace_buf = nullptr;
  // Buffers carved in order from a caller-provided device region instead of
  // allocated (ext_cap > 0); with `counting`, nothing is written or
  // uploaded and only ext_used is advanced (a sizing pass).
  char* ext = nullptr;
  int64_t ext_cap = 0, ext_used = 0;
  bool counting = false;

  void release() {
    if (ext_cap == 0)
      for (void* p : {leaves, arena0, arena1, (void*)exps, (void*)maxbits, (void*)params, (void*)dleaves,
                      (void*)ddense, (void*)dfinal, (void*)per_slice, (void*)sums, seg_tables, (void*)trace_buf})
        if (p) (void)hipFree(p);
    ext_used = 0;
    seg_tables = nullptr;
    trace_buf = nullptr;
    leaves = arena0 = arena1 = nullptr;
    exps = nullptr;
    maxbits = nullptr;
    params = ddense = per_slice = sums = nullptr;
    dleaves = nullptr;
    dfinal = nullptr;
    per_slice_cap = 0;
    bytes = 0;
  }
  ~Workspace() { release(); }
};

struct qt_plan::Profile {
  bool enabled = false;
  struct Rec {
    int kclass;
    int op;  // plan step (streaming, GEMM), LDS segment, or -1 (other kernels)
    double bytes, flops;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  qt_kernel_stats acc[QT_KCLASS_COUNT] = {};
  std::vector<qt_op_stats> ops;  // per (class, op), in order of first launch

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return e;
  }
  hipError_t drain() {
    for (auto& r : pending) {
      hipError_t e = hipEventSynchronize(r.b);
      if (e != hipSuccess) return e;
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, r.a, r.b);
      if (e != hipSuccess) return e;
      qt_kernel_stats& k = acc[r.kclass];
      k.launches += 1;
      k.ms += ms;
      k.bytes += r.bytes;
      k.flops += r.flops;
      qt_op_stats* o = nullptr;
      for (auto& x : ops)
        if (x.kclass == r.kclass && x.op == r.op) o = &x;
      if (!o) {
        ops.push_back(qt_op_stats{r.kclass, r.op, 0, 0.0, 0.0, 0.0});
        o = &ops.back();
      }
      o->launches += 1;
      o->ms += ms;
      o->bytes += r.bytes;
      o->flops += r.flops;
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
    return hipSuccess;
  }
  ~Profile() {
    (void)drain();
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

struct qt_plan::Graphs {
  struct Entry {
    int np;
    int64_t begin, end;
    const void *g, *b, *out, *per_slice;
    uint64_t gen;
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<Entry> entries;
  void clear() {
    for (auto& e : entries) {
      (void)hipGraphExecDestroy(e.exec);
      (void)hipGraphDestroy(e.graph);
    }
    entries.clear();
  }
  ~Graphs() { clear(); }
};

qt_plan::qt_plan() = default;
qt_plan::~qt_plan() = default;

namespace qt {
namespace {
// Records a HIP event pair around `launch` when profiling is on.
template <class F>
hipError_t timed(qt_plan& plan, hipStream_t stream, int kclass, int op, double bytes, double flops, F launch) {
  qt_plan::Profile* pr = plan.prof.get();
  if (!pr || !pr->enabled) return launch();
  hipEvent_t a = pr->get(), b = pr->get();
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, stream);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, stream);
  if (e != hipSuccess) return e;
  pr->pending.push_back({kclass, op, bytes, flops, a, b});
  return hipSuccess;
}
}  // namespace
}  // namespace qt

namespace qt {
namespace {

// A workspace buffer: allocated, or the next 256-byte-aligned piece of the
// workspace's external region.
template <class T>
qt_status dev_alloc(qt_plan::Workspace& ws, T** p, int64_t count, int64_t& bytes) {
  const size_t b = std::max<int64_t>(1, count) * sizeof(T);
  if (ws.ext_cap > 0) {
    const int64_t off = (ws.ext_used + 255) & ~(int64_t)255;
    if (!ws.counting && off + (int64_t)b > ws.ext_cap)
      return fail(QT_ENOMEM, "workspace exceeds the static scratch area");
    *p = reinterpret_cast<T*>(ws.ext + off);
    ws.ext_used = off + (int64_t)b;
  } else if (hipMalloc((void**)p, b) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QT_ENOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
  }
  bytes += (int64_t)b;
  return QT_OK;
}

// Host-to-device upload of workspace tables (skipped by a sizing pass).
qt_status ws_upload(const qt_plan::Workspace& ws, void* dst, const void* src, size_t bytes) {
  if (ws.counting || bytes == 0) return QT_OK;
  QT_HIP_CHECK(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
  return QT_OK;
}



constexpr int64_t kUnitAlign = 64;  // arena offsets in multiples of 64 elements
int64_t align_units(int64_t n) { return (n + kUnitAlign - 1) / kUnitAlign * kUnitAlign; }

bool build_in(const qt_plan& plan, const qt_plan::Workspace& ws, int t, uint32_t mask, int has_v, uint32_t smask,
              int slow, int elt, DevIn& d) {
  const SymTensor& st = plan.tensors[t];
  std::memset(&d, 0, sizeof(d));
  if (st.leaf >= 0) {
    d.ptr = (const char*)ws.leaves + (int64_t)plan.dev_leaves[st.leaf].off * elt;
    d.pt_stride = plan.leaf_block;
    d.sb_stride = 0;
    d.exp_base = -1;
  } else if (st.level == 0) {
    d.ptr = (const char*)ws.arena0 + ws.unit_off[t] * ws.np * elt;
    d.pt_stride = 1ll << st.rank;
    d.sb_stride = 0;
    d.exp_base = st.exp_slot;
    d.exp_pt = plan.n_exp0;
    d.exp_sb = 0;
  } else {
    d.ptr = (const char*)ws.arena1 + ws.unit_off[t] * ws.np * ws.chunk * elt;
    d.pt_stride = ws.chunk << st.rank;
    d.sb_stride = 1ll << st.rank;
    d.exp_base = (int32_t)(ws.exp1_base + st.exp_slot);
    d.exp_pt = (int32_t)(ws.chunk * plan.n_exp1);
    d.exp_sb = plan.n_exp1;
  }
  d.smask = smask;
  d.slow = slow;
  d.has_v = has_v;
  const int block_rank = st.rank - __builtin_popcount(smask);
  d.small_n = block_rank <= 10 ? (1 << block_rank) : 0;  // capped per step by x_small_cap
  if (!make_runs(mask, kMaxRuns, d.run_lo, d.run_len, d.run_dst, d.nruns)) return false;
  // tile part: the bits of x from 10 up, as runs over the tile index
  constexpr int kLgTile = 10;
  const uint32_t below = (uint32_t)__builtin_popcount(mask & ((1u << kLgTile) - 1u));
  if (!make_runs(mask >> kLgTile, kMaxRuns, d.t_lo, d.t_len, d.t_dst, d.t_nruns)) return false;
  for (int i = 0; i < d.t_nruns; ++i) d.t_dst[i] = (uint8_t)(d.t_dst[i] + below);
  for (uint32_t e = 0; e < 4; ++e) {
    uint32_t r = 0;
    for (int i = 0; i < d.nruns; ++i) r |= (((e << 8) >> d.run_lo[i]) & ((1u << d.run_len[i]) - 1u)) << d.run_dst[i];
    d.ep[e] = r;
  }
  return true;
}

// Launch schedule, independent of batch size and pointers:
//  * cuts the step list into LDS segments (maximal runs of consecutive steps
//    of one level whose outputs have rank <= max_rank) and streaming steps;
//  * groups each segment's steps into dependency levels;
//  * places every tensor produced and consumed inside a segment in LDS when
//    it fits (first-fit over level intervals, largest first);
//  * lays out the global arenas over schedule time (every launch is one
//    tick), so no two global buffers that one launch reads or writes share
//    memory.
qt_status plan_schedule(qt_plan& plan, qt_plan::Workspace& ws, int elt) {
  ws.prefix_ops.clear();
  ws.slice_ops.clear();
  ws.segs.clear();
  const bool plain = (plan.flags & QT_PLAN_PLAIN) != 0;
  const int max_rank = std::min(16, tuned(plan.tuning.lds_max_rank, "QT_LDS_MAX_RANK", 14));
  ws.waves = std::max(1, std::min(kXMaxThreads / 64, tuned(plan.tuning.lds_waves, "QT_LDS_WAVES", 16)));
  const int64_t lds_bytes = std::min(160 * 1024, env_int("QT_LDS_BYTES", 160 * 1024));
  const int nsteps = (int)plan.steps.size();
  const int ntens = (int)plan.tensors.size();
  ws.seg_of.assign(nsteps, -1);
  ws.depth.assign(nsteps, 0);
  ws.lds_off.assign(ntens, -1);
  ws.lds_slot.assign(ntens, -1);
  ws.staged_in.assign(ntens, -1);
  // Depth and LDS placement of a candidate segment (steps in plan order).
  // Returns false when some tensor produced and consumed inside does not
  // fit: a global buffer must never be written and read in the same launch
  // (the reader's vector L1 may hold the line from before the write).
  auto place = [&](const std::vector<int>& steps, qt_plan::Workspace::Segment& S, bool commit) -> bool {
    std::vector<char> in_seg(nsteps, 0);
    for (int i : steps) in_seg[i] = 1;
    std::vector<int> dep(nsteps, 0);
    int n_levels = 0;
    for (int i : steps) {
      for (const SymIn& in : plan.steps[i].ins) {
        const int pr = plan.tensors[in.tensor].producer;
        if (pr >= 0 && in_seg[pr]) dep[i] = std::max(dep[i], dep[pr] + 1);
      }
      n_levels = std::max(n_levels, dep[i] + 1);
    }
    std::vector<Interval> cands, ext;
    for (int i : steps) {
      const int t = plan.steps[i].out;
      const int c = plan.tensors[t].consumer;
      if (c >= 0 && in_seg[c]) cands.push_back({t, std::max<int64_t>(2, 1ll << plan.tensors[t].rank), dep[i], dep[c]});
      for (const SymIn& in : plan.steps[i].ins) {
        const SymTensor& T = plan.tensors[in.tensor];
        if (T.leaf >= 0 && x_gate_off(plan.net.leaves[T.leaf].kind, plan.net.leaves[T.leaf].layer) >= 0) continue;
        if (T.producer >= 0 && in_seg[T.producer]) continue;
        const int eff = in.smask ? in.slow : T.rank;
        ext.push_back({in.tensor, std::max<int64_t>(2, 1ll << eff), -1, dep[i]});
      }
    }
    auto by_size = [](const Interval& x, const Interval& y) {
      return x.size != y.size ? x.size > y.size : x.start < y.start;
    };
    std::sort(cands.begin(), cands.end(), by_size);
    std::sort(ext.begin(), ext.end(), by_size);
    cands.insert(cands.end(), ext.begin(), ext.end());
    const int64_t cap = (lds_bytes - 8 * (int64_t)(cands.size() + 4)) / elt - x_tensor_base(plan.net.p);
    struct Placed {
      int64_t off, size;
      int start, end;
    };
    std::vector<Placed> placed;
    std::vector<std::pair<int64_t, int64_t>> busy;
    std::vector<std::pair<int, int64_t>> where;
    int64_t top = 0;
    for (int ci = 0; ci < (int)cands.size(); ++ci) {
      const Interval& c = cands[ci];
      busy.clear();
      for (const auto& p : placed)
        if (p.start <= c.end && c.start <= p.end) busy.emplace_back(p.off, p.off + p.size);
      std::sort(busy.begin(), busy.end());
      int64_t off = 0;
      for (const auto& b : busy) {
        if (b.first >= off + c.size) break;
        off = std::max(off, b.second);
      }
      if (off + c.size > cap) return false;  // every operand of a segment lives in LDS
      placed.push_back({off, c.size, c.start, c.end});
      where.emplace_back(c.t, off);
      top = std::max(top, off + c.size);
    }
    if (!commit) return true;
    S.steps = steps;
    S.n_levels = n_levels;
    S.lds_elems = (int)top + x_tensor_base(plan.net.p);
    for (int i : steps) {
      ws.depth[i] = dep[i];
      S.bytes_c64 += plan.steps[i].bytes_c64;
      S.flops += plan.steps[i].flops;
    }
    for (const auto& w : where) {
      ws.lds_off[w.first] = w.second;
      if (plan.tensors[w.first].leaf < 0) ws.lds_slot[w.first] = S.n_slots++;
      const int pr = plan.tensors[w.first].producer;
      if (pr < 0 || !in_seg[pr]) ws.staged_in[w.first] = (int)ws.segs.size();  // copied in at launch start
    }
    return true;
  };
  // Recursive halving until every piece keeps its internal tensors in LDS.
  std::function<void(const std::vector<int>&, int, std::vector<qt_plan::Workspace::Op>&)> emit_run =
      [&](const std::vector<int>& steps, int level, std::vector<qt_plan::Workspace::Op>& ops) {
        qt_plan::Workspace::Segment S;
        S.level = level;
        if (place(steps, S, false)) {
          place(steps, S, true);
          ws.segs.push_back(std::move(S));
          const int si = (int)ws.segs.size() - 1;
          for (int i : ws.segs[si].steps) ws.seg_of[i] = si;
          ops.push_back({-1, si});
          return;
        }
        if (steps.size() == 1) {  // its operands do not fit: one streaming launch
          ops.push_back({steps[0], -1});
          return;
        }
        const size_t h = steps.size() / 2;
        emit_run(std::vector<int>(steps.begin(), steps.begin() + h), level, ops);
        emit_run(std::vector<int>(steps.begin() + h, steps.end()), level, ops);
      };
  std::vector<int> run;
  int run_level = -1;
  auto flush = [&]() {
    if (run.empty()) return;
    emit_run(run, run_level, run_level == 0 ? ws.prefix_ops : ws.slice_ops);
    run.clear();
  };
  for (int i = 0; i < nsteps; ++i) {
    const SymStep& st = plan.steps[i];
    if (plain || st.rank > max_rank || st.gemm) {
      flush();
      (st.level == 0 ? ws.prefix_ops : ws.slice_ops).push_back({i, -1});
      continue;
    }
    if (st.level != run_level) flush();
    run_level = st.level;
    run.push_back(i);
  }
  flush();
  for (int t = 0; t < ntens; ++t) {
    const SymTensor& st = plan.tensors[t];
    if (st.leaf < 0 && (ws.lds_off[t] < 0 || ws.staged_in[t] >= 0) && st.consumer >= 0 && ws.seg_of[st.producer] >= 0 &&
        ws.seg_of[st.producer] == ws.seg_of[st.consumer])
      return fail(QT_EPLAN, "internal: a global tensor is written and read inside one launch");
  }
  // Schedule time of every launch: one tick each.  The workgroups of a
  // launch do not run in step (with more items than fit the device at once,
  // later ones start after earlier ones have finished), so every global
  // tensor a launch reads or writes is live over its whole launch: a
  // segment's outputs must never share memory with the inputs it stages.
  std::vector<int> when(nsteps, 0);
  int clock = 0;
  for (auto* ops : {&ws.prefix_ops, &ws.slice_ops}) {
    for (const auto& op : *ops) {
      if (op.seg < 0) {
        when[op.step] = clock++;
      } else {
        for (int i : ws.segs[op.seg].steps) when[i] = clock;
        ++clock;
      }
    }
  }
  const int INF = 1 << 30;
  std::vector<Interval> iv0, iv1;
  for (int t = 0; t < ntens; ++t) {
    const SymTensor& st = plan.tensors[t];
    if (st.leaf >= 0 || (ws.lds_off[t] >= 0 && ws.staged_in[t] < 0)) continue;
    int end = st.consumer < 0 ? INF : when[st.consumer];
    if (st.level == 0 && st.consumer >= 0 && plan.steps[st.consumer].level == 1) end = INF;  // kept for every chunk
    Interval it{t, align_units(1ll << st.rank), when[st.producer], end};
    (st.level == 0 ? iv0 : iv1).push_back(it);
  }
  ws.unit_off.assign(ntens, 0);
  ws.arena0_units = place_intervals(iv0, ws.unit_off);
  ws.arena1_units = place_intervals(iv1, ws.unit_off);
  // leaves read from global memory: by streaming steps and GEMMs, staged
  // into a segment (all but the gate kinds, whose tables a segment builds
  // itself), or as closing factors
  ws.leaves_read = false;
  for (int i = 0; i < nsteps; ++i)
    for (const SymIn& in : plan.steps[i].ins) {
      const SymTensor& T = plan.tensors[in.tensor];
      if (T.leaf < 0) continue;
      if (ws.seg_of[i] < 0 || x_gate_off(plan.net.leaves[T.leaf].kind, plan.net.leaves[T.leaf].layer) < 0)
        ws.leaves_read = true;
    }
  for (int t : plan.finals)
    if (plan.tensors[t].leaf >= 0) ws.leaves_read = true;
  ws.planned = true;
  if (env_int("QT_DEBUG_SCHEDULE", 0)) {
    for (size_t si = 0; si < ws.segs.size(); ++si) {
      const auto& S = ws.segs[si];
      std::fprintf(stderr, "segment %zu level %d: %zu steps, %d levels, %d LDS slots, %d LDS elems\n", si, S.level,
                   S.steps.size(), S.n_levels, S.n_slots, S.lds_elems);
      for (int i : S.steps) {
        const SymStep& st = plan.steps[i];
        std::fprintf(stderr, "  step %d depth %d rank %d sum %d out t%d %s%lld", i, ws.depth[i], st.rank, st.sum, st.out,
                     ws.lds_off[st.out] >= 0 ? "lds@" : "glob@",
                     (long long)(ws.lds_off[st.out] >= 0 ? ws.lds_off[st.out] : ws.unit_off[st.out]));
        for (const SymIn& in : st.ins)
          std::fprintf(stderr, " | t%d r%d %s%lld m%x v%d s%x", in.tensor, plan.tensors[in.tensor].rank,
                       plan.tensors[in.tensor].leaf >= 0 ? "leaf" : (ws.lds_off[in.tensor] >= 0 ? "lds@" : "glob@"),
                       (long long)(ws.lds_off[in.tensor] >= 0 ? ws.lds_off[in.tensor] : ws.unit_off[in.tensor]),
                       in.mask, in.has_v, in.smask);
        std::fprintf(stderr, "\n");
      }
    }
  }
  return QT_OK;
}

// Device descriptors of the segments (needs the allocated buffers).
qt_status build_segment_tables(qt_plan& plan, qt_plan::Workspace& ws, int elt) {
  const int tbase = x_tensor_base(plan.net.p);
  // Operand: the gate table, a staged input or an internal tensor.
  auto to_op = [&](int t, const SymIn& si, int epu, XOp& x) -> bool {
    std::memset(&x, 0, sizeof(x));
    const SymTensor& T = plan.tensors[t];
    const int gate = T.leaf >= 0 ? x_gate_off(plan.net.leaves[T.leaf].kind, plan.net.leaves[T.leaf].layer) : -1;
    x.slot = -1;
    if (gate >= 0) {
      x.lds_off = (uint32_t)gate;
      x.smask = si.smask;  // a gate on a slice variable is read at the slice's bit
      x.slow = si.slow;
    } else if (ws.lds_off[t] >= 0) {
      x.lds_off = (uint32_t)(ws.lds_off[t] + tbase);  // staged inputs arrive with the slice already selected
      x.slot = ws.lds_slot[t];
    } else {
      return false;
    }
    x.has_v = si.has_v;
    int32_t nr = 0;
    if (!make_runs(si.mask, kXRuns, x.run_lo, x.run_len, x.run_dst, nr)) return false;
    x.lane_runs = x_lane_runs(x.run_lo, x.run_len, x.run_dst, nr, x.has_v);
    for (int e = 0; e < 4; ++e) {
      uint32_t r = 0;
      if (e < epu)
        for (int i = 0; i < nr; ++i)
          r |= (((uint32_t)(64 * e) >> x.run_lo[i]) & ((1u << x.run_len[i]) - 1u)) << x.run_dst[i];
      x.ep[e] = r << x.has_v;
    }
    return true;
  };
  auto to_out = [&](int t, XOut& x) {
    std::memset(&x, 0, sizeof(x));
    if (ws.lds_off[t] >= 0 && ws.staged_in[t] < 0) {  // internal: stays in LDS
      x.ptr = nullptr;
      x.lds_off = (uint32_t)(ws.lds_off[t] + tbase);
      x.slot_kind = 1;
      x.slot = ws.lds_slot[t];
      return;
    }
    DevIn d;
    build_in(plan, ws, t, 0, 0, 0, 0, elt, d);
    x.ptr = const_cast<void*>(d.ptr);
    x.pt_stride = d.pt_stride;
    x.sb_stride = d.sb_stride;
    x.slot_kind = d.exp_base >= 0 ? 2 : 0;
    x.slot = d.exp_base;
    x.exp_pt = d.exp_pt;
    x.exp_sb = d.exp_sb;
  };
  size_t total = 0;
  for (auto& S : ws.segs) {
    S.xsteps.assign(S.steps.size(), XStep{});
    std::vector<int> local(plan.steps.size(), -1);
    for (size_t a = 0; a < S.steps.size(); ++a) local[S.steps[a]] = (int)a;
    for (size_t a = 0; a < S.steps.size(); ++a) {
      const SymStep& st = plan.steps[S.steps[a]];
      XStep& xs = S.xsteps[a];
      std::memset(&xs, 0, sizeof(xs));
      to_out(st.out, xs.out);
      xs.r = st.rank;
      xs.sum = st.sum;
      xs.n_in = (int)st.ins.size();
      const int epu = x_epu(st.rank, (int)st.ins.size(), elt);
      for (size_t j = 0; j < st.ins.size(); ++j)
        if (!to_op(st.ins[j].tensor, st.ins[j], epu, xs.in[j]))
          return fail(QT_EPLAN, "internal: LDS segment operand not in LDS or index map too fragmented");
      for (int j = (int)st.ins.size(); j < x_nin_class(xs.n_in); ++j) {
        XOp& id = xs.in[j];  // identity operand: LDS elements 0 and 1 (1 + 0i), index 0
        std::memset(&id, 0, sizeof(id));
        id.has_v = 1;
        id.slot = -1;
      }
      // pairs: every operand (identities included) holds v, at an even
      // base: LDS offsets even, slice blocks above bit 0, lane and chunk
      // parts shifted by has_v
      xs.out.pairs = 1;
      for (int j = 0; j < x_nin_class(xs.n_in); ++j) {
        const XOp& o = xs.in[j];
        if (o.has_v != 1 || (o.lds_off & 1u) != 0 || (o.smask != 0 && o.slow < 1)) xs.out.pairs = 0;
      }
    }
    S.units.clear();
    S.level_off.clear();
    for (int L = 0; L < S.n_levels; ++L) {
      S.level_off.push_back((int32_t)S.units.size());
      for (size_t a = 0; a < S.steps.size(); ++a)
        if (ws.depth[S.steps[a]] == L) {
          const int r = plan.steps[S.steps[a]].rank;
          const int nin = (int)plan.steps[S.steps[a]].ins.size();
          const int64_t chunks = std::max<int64_t>(1, (1ll << r) / x_unit_elems(r, nin, elt));
          for (int64_t c = 0; c < chunks; ++c) S.units.push_back(make_uint2((uint32_t)a, (uint32_t)c));
        }
    }
    S.level_off.push_back((int32_t)S.units.size());
    // staging copies of external inputs
    S.copies.clear();
    for (int i : S.steps)
      for (const SymIn& in : plan.steps[i].ins) {
        const int t = in.tensor;
        if (ws.staged_in[t] < 0 || ws.seg_of[i] != ws.staged_in[t]) continue;
        DevIn d;
        build_in(plan, ws, t, 0, 0, in.smask, in.slow, elt, d);
        XCopy cp{};
        cp.ptr = d.ptr;
        cp.pt_stride = d.pt_stride;
        cp.sb_stride = d.sb_stride;
        cp.smask = d.smask;
        cp.slow = d.slow;
        cp.lds_off = (uint32_t)(ws.lds_off[t] + tbase);
        cp.n = 1u << (in.smask ? in.slow : plan.tensors[t].rank);
        cp.gslot = d.exp_base;
        cp.exp_pt = d.exp_pt;
        cp.exp_sb = d.exp_sb;
        cp.lslot = ws.lds_slot[t];
        S.copies.push_back(cp);
      }
    // per-unit descriptors: the unit's chunk in the chunk field, and the
    // chunk's part of every operand index folded into the operand's offset
    S.ustep.clear();
    for (const uint2& u : S.units) {
      XStep x = S.xsteps[u.x];
      x.chunk = (int32_t)u.y;
      const SymStep& st = plan.steps[S.steps[u.x]];
      const uint32_t cx = u.y * 64u * (uint32_t)x_epu(st.rank, (int)st.ins.size(), elt);
      for (size_t j = 0; j < st.ins.size(); ++j) {
        XOp& in = x.in[j];
        uint32_t r = 0;
        for (int i = 0; i < kXRuns && in.run_len[i]; ++i)
          r |= ((cx >> in.run_lo[i]) & ((1u << in.run_len[i]) - 1u)) << in.run_dst[i];
        in.lds_off += r << in.has_v;
      }
      S.ustep.push_back(x);
    }
    total += ((S.ustep.size() * sizeof(XStep) + 255) & ~(size_t)255) +
             ((S.copies.size() * sizeof(XCopy) + 255) & ~(size_t)255) +
             ((S.units.size() * sizeof(uint2) + 255) & ~(size_t)255) +
             ((S.level_off.size() * sizeof(int32_t) + 255) & ~(size_t)255);
  }
  if (!total) return QT_OK;
  QT_TRY(dev_alloc(ws, (char**)&ws.seg_tables, (int64_t)total, ws.bytes));
  std::vector<char> host(total);
  size_t off = 0;
  char* base = (char*)ws.seg_tables;
  auto put = [&](const void* src, size_t bytes) {
    std::memcpy(host.data() + off, src, bytes);
    const char* at = base + off;
    off = (off + bytes + 255) & ~(size_t)255;
    return at;
  };
  for (auto& S : ws.segs) {
    S.launch.steps = (const XStep*)put(S.ustep.data(), S.ustep.size() * sizeof(XStep));
    S.launch.units = (const uint2*)put(S.units.data(), S.units.size() * sizeof(uint2));
    S.launch.level_off = (const int32_t*)put(S.level_off.data(), S.level_off.size() * sizeof(int32_t));
    S.launch.copies = (const XCopy*)put(S.copies.data(), S.copies.size() * sizeof(XCopy));
    S.launch.n_copies = (int)S.copies.size();
    S.launch.gam = ws.params;
    S.launch.bet = ws.params + plan.net.p;
    S.launch.pstride = 2 * plan.net.p;
    S.launch.p = plan.net.p;
    S.launch.n_levels = S.n_levels;
    S.launch.n_slots = S.n_slots;
    S.launch.lds_elems = S.lds_elems;
  }
  return ws_upload(ws, ws.seg_tables, host.data(), total);
}

// Storage bits of the counter variables `counter` (key order) in a tensor
// with variables `vars` (key order): the counter's value enters the element
// index as a deposit into these bits, which must keep the counter's order.
bool counter_mask(const std::vector<int32_t>& counter, const std::vector<int32_t>& vars, uint32_t& mask) {
  mask = 0;
  int last = -1;
  for (int x : counter) {
    const int pos = (int)(std::find(vars.begin(), vars.end(), x) - vars.begin());
    if (pos >= (int)vars.size() || pos <= last || pos >= 32) return false;
    mask |= 1u << pos;
    last = pos;
  }
  return true;
}

uint32_t deposit(uint32_t x, uint32_t m) {
  uint32_t r = 0;
  for (; m; m &= m - 1, x >>= 1)
    if (x & 1u) r |= m & (0u - m);
  return r;
}

// Element numbering of a block whose bits are the low `bits[i]` bits of
// counters with storage masks `masks[i]` and LDS weights `lds[i]` (per
// counter unit): the block's bits sorted by storage position, each with its
// storage and LDS weight.
void number_block(std::initializer_list<std::pair<uint32_t, std::pair<int, uint32_t>>> parts, uint32_t* w,
                  uint32_t* l) {
  std::vector<std::pair<uint32_t, uint32_t>> bits;  // (storage weight, LDS weight)
  for (const auto& pt : parts)
    for (int i = 0; i < pt.second.first; ++i) bits.emplace_back(deposit(1u << i, pt.first), (1u << i) * pt.second.second);
  std::sort(bits.begin(), bits.end());
  for (int j = 0; j < kGBits; ++j) {
    w[j] = j < (int)bits.size() ? bits[j].first : 0u;
    l[j] = j < (int)bits.size() ? bits[j].second : 0u;
  }
}

// Tile shape of a fused GEMM bucket: (batch, m, n) tile bits with four
// 16 x 16 sub-tiles where possible.  A short-K product is output-bound:
// prefer the shape whose bits cover the longest run of C's low storage bits
// (a contiguous output block per tile).  A long-K product is operand-bound:
// prefer the largest m x n tile (most reuse of each loaded element), then
// the output run.  K stage: 64 deep for long sums (more operand bytes in
// flight per workgroup), else 16 (8 for K = 8).
void choose_gemm_tile(const qt_plan& plan, const SymStep& st, int32_t& tb_out, int32_t& tm_out, int32_t& tn_out,
                      int32_t& tk_out, int32_t& mode_out) {
  const auto& va = plan.tensors[st.ins[0].tensor].vars;
  const auto& vb = plan.tensors[st.ins[1].tensor].vars;
  const auto& vc = plan.tensors[st.out].vars;
  auto has = [](const std::vector<int32_t>& v, int x) { return std::find(v.begin(), v.end(), x) != v.end(); };
  std::vector<int32_t> cb, cm, cn;
  for (int x : vc) {
    const bool ia = has(va, x), ib = has(vb, x);
    if (ia && ib) cb.push_back(x);
    else if (ia) cm.push_back(x);
    else cn.push_back(x);
  }
  const int nb = (int)cb.size(), nm = (int)cm.size(), nn = (int)cn.size(), nk = (int)st.kvars.size();
  std::vector<char> kind(vc.size());  // counter of each C storage bit, with its index
  std::vector<int> idx(vc.size());
  for (size_t q = 0; q < vc.size(); ++q) {
    auto at = [&](const std::vector<int32_t>& v) { return (int)(std::find(v.begin(), v.end(), vc[q]) - v.begin()); };
    if (has(cb, vc[q])) kind[q] = 'b', idx[q] = at(cb);
    else if (has(cm, vc[q])) kind[q] = 'm', idx[q] = at(cm);
    else kind[q] = 'n', idx[q] = at(cn);
  }
  const int shapes[8][3] = {{0, 5, 5}, {1, 5, 4}, {1, 4, 5}, {2, 4, 4}, {0, 5, 4}, {0, 4, 5}, {1, 4, 4}, {0, 4, 4}};
  int best = 7, best_run = -1, best_subs = 0;
  for (int s = 0; s < 8; ++s) {
    const int tb = shapes[s][0], tm = shapes[s][1], tn = shapes[s][2];
    if (tb > nb || tm > nm || tn > nn) continue;
    int run = 0;
    while (run < (int)vc.size()) {
      const char k = kind[run];
      const int lim = k == 'b' ? tb : (k == 'm' ? tm : tn);
      if (idx[run] >= lim) break;
      ++run;
    }
    const int subs = 1 << (tb + tm + tn - 8);
    if (nk > 5) run += 64 * (tm + tn);  // reuse first
    if (run > best_run || (run == best_run && subs > best_subs)) {
      best = s;
      best_run = run;
      best_subs = subs;
    }
  }
  tb_out = shapes[best][0];
  tm_out = shapes[best][1];
  tn_out = shapes[best][2];
  tk_out = nk >= 6 ? 64 : (nk >= 4 ? 16 : 8);
  // split-BF16 products (32-deep stages) for K >= 32; shorter sums are
  // bound by their output, and keep the FP32 products
  mode_out = plan.precision == QT_C64_SCALED_MFMA_BF16X3 && nk >= 5 ? 1 : 0;
  if (mode_out == 1) tk_out = 32;
}

qt_status build_gemm(const qt_plan& plan, const qt_plan::Workspace& ws, const SymStep& st, int elt, int np,
                     int64_t chunk, DevGemm& g) {
  std::memset(&g, 0, sizeof(g));
  const int ta = st.ins[0].tensor, tb = st.ins[1].tensor;
  const auto& va = plan.tensors[ta].vars;
  const auto& vb = plan.tensors[tb].vars;
  const auto& vc = plan.tensors[st.out].vars;
  auto has = [](const std::vector<int32_t>& v, int x) { return std::find(v.begin(), v.end(), x) != v.end(); };
  std::vector<int32_t> cb, cm, cn;
  for (int x : vc) {
    const bool ia = has(va, x), ib = has(vb, x);
    if (ia && ib) cb.push_back(x);
    else if (ia) cm.push_back(x);
    else cn.push_back(x);
  }
  DevIn da, db, dc;
  build_in(plan, ws, ta, 0, 0, st.ins[0].smask, st.ins[0].slow, elt, da);
  build_in(plan, ws, tb, 0, 0, st.ins[1].smask, st.ins[1].slow, elt, db);
  build_in(plan, ws, st.out, 0, 0, 0, 0, elt, dc);
  g.a = da.ptr;
  g.b = db.ptr;
  g.c = const_cast<void*>(dc.ptr);
  g.a_pt = da.pt_stride;
  g.a_sb = da.sb_stride;
  g.b_pt = db.pt_stride;
  g.b_sb = db.sb_stride;
  g.c_pt = dc.pt_stride;
  g.c_sb = dc.sb_stride;
  g.a_smask = st.ins[0].smask;
  g.b_smask = st.ins[1].smask;
  g.a_slow = st.ins[0].slow;
  g.b_slow = st.ins[1].slow;
  g.lg_nsb = st.level == 1 ? ilog2(chunk) : 0;
  g.n_items = (int32_t)(np * (st.level == 1 ? chunk : 1));
  g.nb = (int)cb.size();
  g.nm = (int)cm.size();
  g.nn = (int)cn.size();
  g.nk = (int)st.kvars.size();
  g.a_exp_base = da.exp_base;
  g.a_exp_pt = da.exp_pt;
  g.a_exp_sb = da.exp_sb;
  g.b_exp_base = db.exp_base;
  g.b_exp_pt = db.exp_pt;
  g.b_exp_sb = db.exp_sb;
  g.c_exp_base = dc.exp_base;
  g.c_exp_pt = dc.exp_pt;
  g.c_exp_sb = dc.exp_sb;
  if (!counter_mask(cb, va, g.a_bm) || !counter_mask(cm, va, g.a_mm) || !counter_mask(st.kvars, va, g.a_km) ||
      !counter_mask(cb, vb, g.b_bm) || !counter_mask(cn, vb, g.b_nm) || !counter_mask(st.kvars, vb, g.b_km) ||
      !counter_mask(cb, vc, g.c_bm) || !counter_mask(cm, vc, g.c_mm) || !counter_mask(cn, vc, g.c_nm))
    return fail(QT_EPLAN, "internal: GEMM counter variables are not in key order in an operand");
  // each operand's counters cover distinct bits inside its rank (below its
  // slice bits), so every index stays in the tensor's block
  auto covers = [](std::initializer_list<uint32_t> masks, int bits, int rank) {
    uint32_t seen = 0;
    int total = 0;
    for (uint32_t m : masks) {
      if (seen & m) return false;
      seen |= m;
      total += __builtin_popcount(m);
    }
    return total == bits && (rank >= 32 || (seen >> rank) == 0);
  };
  const int ra = st.ins[0].smask ? st.ins[0].slow : (int)va.size();
  const int rb = st.ins[1].smask ? st.ins[1].slow : (int)vb.size();
  if (!covers({g.a_bm, g.a_mm, g.a_km}, g.nb + g.nm + g.nk, ra) || !covers({g.b_bm, g.b_nm, g.b_km}, g.nb + g.nn + g.nk, rb) ||
      !covers({g.c_bm, g.c_mm, g.c_nm}, g.nb + g.nm + g.nn, (int)vc.size()) || g.nm < 4 || g.nn < 4 || g.nk < 3 ||
      g.nb + g.nm + g.nk > kGemmMaxRank || g.nb + g.nn + g.nk > kGemmMaxRank || g.nb + g.nm + g.nn > kGemmMaxRank)
    return fail(QT_EPLAN, "internal: GEMM operand maps do not tile their tensors");
  choose_gemm_tile(plan, st, g.tb, g.tm, g.tn, g.tk, g.mode);
  const uint32_t pitch = g.mode == 1 ? 40u : (g.tk == 64 ? 68u : 17u);  // LDS row pitch of the kernel
  const int lg_tk = ilog2(g.tk);
  const uint32_t TM = 1u << g.tm, TN = 1u << g.tn;
  g.a_kh = g.a_km & ~deposit((uint32_t)g.tk - 1u, g.a_km);
  g.b_kh = g.b_km & ~deposit((uint32_t)g.tk - 1u, g.b_km);
  g.b_nh = g.b_nm & ~deposit(TN - 1u, g.b_nm);
  g.c_nh = g.c_nm & ~deposit(TN - 1u, g.c_nm);
  // LDS: operand row r = b * TM + m (or b * TN + n) at r * pitch + k; the
  // output staging row b * TM + m at pitch TN + 1
  number_block({{g.a_bm, {g.tb, TM * pitch}}, {g.a_mm, {g.tm, pitch}}, {g.a_km, {lg_tk, 1u}}}, g.aw, g.al);
  number_block({{g.b_bm, {g.tb, TN * pitch}}, {g.b_nm, {g.tn, pitch}}, {g.b_km, {lg_tk, 1u}}}, g.bw, g.bl);
  number_block({{g.c_bm, {g.tb, TM * (TN + 1u)}}, {g.c_mm, {g.tm, TN + 1u}}, {g.c_nm, {g.tn, 1u}}}, g.cw, g.cl);
  return QT_OK;
}

// Lays out (allocating, or carving from the workspace's external region)
// and uploads everything a run of `np` points over `n_range` slices needs,
// with `chunk` slices per launch (0: from slice_batch or the budget).
qt_status layout_workspace(qt_plan& plan, qt_plan::Workspace& ws, int np, int64_t n_range, int64_t chunk_req) {
  const bool c128 = plan.precision == QT_C128;
  const int elt = c128 ? 16 : 8;
  const int k = (int)plan.slice_vars.size();
  if (!ws.planned) QT_TRY(plan_schedule(plan, ws, elt));
  int64_t chunk = 1;
  if (chunk_req > 0) {
    chunk = chunk_req;
  } else if (k > 0) {
    const int64_t n_slices = 1ll << k;
    if (plan.slice_batch_req > 0) {
      chunk = 1;
      while (chunk * 2 <= std::min(plan.slice_batch_req, n_slices)) chunk *= 2;
    } else {
      int64_t budget = kDefaultBudget;
      if (const char* e = std::getenv("QT_WORKSPACE_BUDGET")) budget = std::max<int64_t>(1, std::atoll(e));
      const int64_t per = std::max<int64_t>(1, ws.arena1_units * np * elt);
      chunk = 1;
      while (chunk * 2 <= n_slices && chunk * 2 * per <= budget) chunk *= 2;
    }
  }
  if (ws.np != np || ws.chunk != chunk) {
    ws.release();
    ws.np = np;
    ws.chunk = chunk;
    ws.gen = next_ws_gen();
    int64_t& b = ws.bytes;
    QT_TRY(dev_alloc(ws, (char**)&ws.leaves, (int64_t)plan.leaf_block * np * elt, b));
    QT_TRY(dev_alloc(ws, (char**)&ws.arena0, std::max<int64_t>(1, ws.arena0_units) * np * elt, b));
    QT_TRY(dev_alloc(ws, (char**)&ws.arena1, std::max<int64_t>(1, ws.arena1_units) * np * chunk * elt, b));
    ws.exp1_base = (int64_t)np * plan.n_exp0;
    ws.exp1_count = (int64_t)np * chunk * plan.n_exp1;
    ws.n_exp = ws.exp1_base + ws.exp1_count;
    QT_TRY(dev_alloc(ws, &ws.exps, ws.n_exp, b));
    QT_TRY(dev_alloc(ws, &ws.maxbits, ws.n_exp, b));
    QT_TRY(dev_alloc(ws, &ws.params, (int64_t)np * 2 * std::max(1, plan.net.p), b));
    QT_TRY(dev_alloc(ws, &ws.dleaves, (int64_t)plan.dev_leaves.size(), b));
    QT_TRY(dev_alloc(ws, &ws.ddense, (int64_t)plan.dense_table.size(), b));
    QT_TRY(dev_alloc(ws, &ws.dfinal, (int64_t)plan.finals.size(), b));
    QT_TRY(dev_alloc(ws, &ws.sums, ((int64_t)np << plan.open_vars.size()) * 3, b));
    QT_TRY(ws_upload(ws, ws.dleaves, plan.dev_leaves.data(), plan.dev_leaves.size() * sizeof(DevLeaf)));
    QT_TRY(ws_upload(ws, ws.ddense, plan.dense_table.data(), plan.dense_table.size() * sizeof(double)));
    // streaming step descriptors
    ws.steps.clear();
    ws.gemms.assign(plan.steps.size(), DevGemm{});
    ws.step_elems.clear();
    for (const SymStep& st : plan.steps) {
      DevStep d;
      std::memset(&d, 0, sizeof(d));
      const SymTensor& ot = plan.tensors[st.out];
      ws.step_elems.push_back((int64_t)np * (st.level == 1 ? chunk : 1) << ot.rank);
      if (ws.seg_of[&st - plan.steps.data()] >= 0) {
        ws.steps.push_back(d);  // runs inside an LDS segment
        continue;
      }
      if (st.gemm) {
        ws.steps.push_back(d);
        QT_TRY(build_gemm(plan, ws, st, elt, np, chunk, ws.gemms[&st - plan.steps.data()]));
        continue;
      }
      DevIn od;
      build_in(plan, ws, st.out, 0, 0, 0, 0, elt, od);
      d.out = const_cast<void*>(od.ptr);
      d.r = st.rank;
      d.lg_nsb = st.level == 1 ? ilog2(chunk) : 0;
      d.sum = st.sum;
      d.n_in = (int)st.ins.size();
      d.out_exp_base = od.exp_base;
      d.out_exp_pt = od.exp_pt;
      d.out_exp_sb = od.exp_sb;
      for (size_t j = 0; j < st.ins.size(); ++j) {
        const SymIn& si = st.ins[j];
        if (ws.lds_off[si.tensor] >= 0 && ws.staged_in[si.tensor] < 0)
          return fail(QT_EPLAN, "internal: streaming step reads an LDS tensor");
        if (!build_in(plan, ws, si.tensor, si.mask, si.has_v, si.smask, si.slow, elt, d.in[j]))
          return fail(QT_EUNSUPPORTED, "input index map has more than 16 runs of bits");
      }
      // staging cap by the count of inputs the kernel indexes: a large
      // step's inputs read by no output bit are folded in once per item
      int n_idx = d.n_in;
      if (st.rank >= 10) {
        n_idx = 0;
        for (int j = 0; j < d.n_in; ++j) n_idx += d.in[j].nruns != 0;
        if (n_idx == 0) n_idx = d.n_in;
      }
      for (int j = 0; j < d.n_in; ++j)
        if (d.in[j].small_n > x_small_cap(n_idx)) d.in[j].small_n = 0;
      ws.steps.push_back(d);
    }
    ws.finals.clear();
    const int n_open = (int)plan.open_vars.size();
    for (int t : plan.finals) {
      const SymTensor& st = plan.tensors[t];
      // slice bits (a prefix tensor is read at the slice's block) and the
      // output bits of its open variables (key n_order + bit)
      uint32_t smask = 0, omask = 0;
      for (int x : st.vars) {
        const int kx = plan.key[x];
        if (kx >= plan.n_order && kx < plan.n_order + n_open) omask |= 1u << (kx - plan.n_order);
        if (st.level == 0)
          for (int j = 0; j < k; ++j)
            if (plan.slice_vars[j] == x) smask |= 1u << (k - 1 - j);
      }
      DevIn d;
      if (!build_in(plan, ws, t, omask, 0, smask, __builtin_popcount(omask), elt, d))
        return fail(QT_EUNSUPPORTED, "closing tensor index map too fragmented");
      ws.finals.push_back(d);
    }
    QT_TRY(ws_upload(ws, ws.dfinal, ws.finals.data(), ws.finals.size() * sizeof(DevIn)));
    QT_TRY(build_segment_tables(plan, ws, elt));
    ws.trace_on = env_int("QT_DEBUG_LEVEL_TRACE", 0) != 0;
    if (ws.trace_on) {
      int max_levels = 1;
      for (auto& S : ws.segs) max_levels = std::max(max_levels, S.n_levels + 1);
      QT_TRY(dev_alloc(ws, &ws.trace_buf, (int64_t)max_levels * (int64_t)ws.segs.size(), b));
    }
    plan.info.slice_batch = chunk;
  }
  const int64_t rows = (int64_t)np << plan.open_vars.size();  // (point, open output) rows of results
  if (ws.per_slice_cap < rows * n_range) {
    ws.gen = next_ws_gen();
    if (ws.per_slice && ws.ext_cap == 0) (void)hipFree(ws.per_slice);
    ws.per_slice = nullptr;
    ws.per_slice_cap = 0;
    int64_t dummy = 0;
    QT_TRY(dev_alloc(ws, &ws.per_slice, rows * n_range * 3, dummy));
    ws.per_slice_cap = rows * n_range;
  }
  plan.info.workspace_bytes = ws.bytes + ws.per_slice_cap * 24;
  return QT_OK;
}

qt_status ensure_workspace(qt_plan& plan, int np, int64_t n_range) {
  if (!plan.ws) plan.ws = std::make_unique<qt_plan::Workspace>();
  return layout_workspace(plan, *plan.ws, np, n_range, 0);
}


// Runs one plan at np points over slices [begin, end); leaves the per-slice
// values in ws.per_slice ([np][2^a][end - begin][3], a open output bits) and
// the sums in ws.sums ([np][2^a][3]).
// The workspace `ws` is laid out for np points and the slice range.
qt_status run_plan_ws(qt_plan& plan, qt_plan::Workspace& ws, int np, const double* gammas, const double* betas,
                      int64_t begin, int64_t end, int64_t stop, hipStream_t stream, double* sums_out = nullptr) {
  const bool c128 = plan.precision == QT_C128;
  const bool scaled = plan.precision != QT_C128;
  const int k = (int)plan.slice_vars.size();
  const int64_t n_range = end - begin;
  int launches = 0;
  // parameters in device memory go to the leaf launch, which lays them out
  // for the others; host parameters are uploaded first
  const int pp = plan.net.p;
  const bool dev_params = pp > 0 && is_device_ptr(gammas) && is_device_ptr(betas);
  // no launch reads the leaves from global memory: with device parameters
  // the segments read them where they are, and the leaf launch is skipped
  const bool direct = dev_params && !ws.leaves_read;
  if (!dev_params) QT_TRY(upload_params_to(ws.params, np, pp, gammas, betas, stream));
  const double eb = c128 ? 2.0 : 1.0;  // algorithmic byte counts are kept at 8 B per element
  // the leaf launch also clears the scale slots of the prefix and of the
  // first chunk
  const int64_t n_clear = scaled && !direct ? ws.exp1_base + (k > 0 ? ws.exp1_count : 0) : 0;
  if (!direct) {
    // leaves, and the device parameters laid out for the segments
    QT_HIP_CHECK(timed(plan, stream, QT_KCLASS_OTHER, -1, 0, 0, [&] {
      return launch_leaves(ws.dleaves, (int)plan.dev_leaves.size(), plan.leaf_block, ws.ddense, ws.params,
                           dev_params ? gammas : nullptr, dev_params ? betas : nullptr, pp, np, ws.leaves, c128,
                           stream, ws.maxbits, n_clear);
    }));
    ++launches;
  }
  if (scaled && ws.exp1_base && n_clear == 0) {
    QT_HIP_CHECK(timed(plan, stream, QT_KCLASS_OTHER, -1, 0, 0,
                       [&] { return launch_fill_u32(ws.maxbits, ws.exp1_base, 0u, stream); }));
    ++launches;
  }
  auto step = [&](const DevStep& d, int i) -> hipError_t {
    const SymStep& st = plan.steps[i];
    const double items = (double)(ws.step_elems[i] >> st.rank);
    const int kc = st.rank >= 10 ? QT_KCLASS_STEP_STREAM : QT_KCLASS_STEP_SMALL;
    return timed(plan, stream, kc, i, st.bytes_c64 * eb * items, st.flops * items, [&] {
      return launch_step(d, c128, scaled, ws.exps, ws.maxbits, ws.step_elems[i], stream, &launches, nullptr);
    });
  };
  const int step_lg_tpb =
      plan.tuning.step_tiles > 0 ? ilog2(plan.tuning.step_tiles) : std::max(0, env_int("QT_STEP_LG_TILES", 3));
  auto run_op = [&](const qt_plan::Workspace::Op& op, int64_t cb) -> hipError_t {
    if (op.seg < 0 && plan.steps[op.step].gemm) {
      DevGemm g = ws.gemms[op.step];
      g.chunk_base = cb;
      g.tiles = plan.tuning.gemm_tiles;
      const SymStep& st = plan.steps[op.step];
      ++launches;
      return timed(plan, stream, QT_KCLASS_GEMM, op.step, st.bytes_c64 * g.n_items, st.flops * g.n_items,
                   [&] { return launch_gemm(g, scaled, ws.exps, ws.maxbits, stream); });
    }
    if (op.seg < 0) {
      DevStep d = ws.steps[op.step];
      d.chunk_base = cb;
      d.lg_tpb = step_lg_tpb;
      return step(d, op.step);
    }
    auto& S = ws.segs[op.seg];
    XLaunch x = S.launch;
    x.chunk_base = cb;
    if (direct) {
      x.gam = gammas;
      x.bet = betas;
      x.pstride = pp;
    }
    int max_levels = 1;
    for (auto& T : ws.segs) max_levels = std::max(max_levels, T.n_levels + 1);
    x.trace = ws.trace_on ? ws.trace_buf + (int64_t)op.seg * max_levels : nullptr;
    x.lg_nsb = S.level == 1 ? ilog2(ws.chunk) : 0;
    const int64_t items = (int64_t)np * (S.level == 1 ? ws.chunk : 1);
    ++launches;
    return timed(plan, stream, QT_KCLASS_LDS, op.seg, S.bytes_c64 * eb * items, S.flops * items, [&] {
      return launch_lds_exec(x, items, ws.waves, c128, scaled, ws.exps, ws.maxbits, stream);
    });
  };
  for (const auto& op : ws.prefix_ops) QT_HIP_CHECK(run_op(op, 0));
  // the sums go into the caller's device array when given (no copy after);
  // a range of one slice has them formed by the final launch itself
  double* const sums = sums_out ? sums_out : ws.sums;
  // the final launch forms the sums itself for a range of one slice, or
  // for one point without open outputs whose whole range is one launch of
  // one workgroup
  int sum_mode = n_range == 1 ? 1 : 0;
  if (!sum_mode && k > 0 && np == 1 && plan.open_vars.empty()) {
    const int64_t C = ws.chunk, first = begin & ~(C - 1);
    if (first + C >= end && C <= 256) sum_mode = 2;
  }
  DevFinal f{};
  f.n_factors = (int)ws.finals.size();
  f.n_open = (int)plan.open_vars.size();
  f.slice_begin = begin;
  f.n_range = n_range;
  f.log2_const = plan.log2_const;
  if (k == 0) {
    f.lg_nsb = 0;
    f.chunk_base = 0;
    QT_HIP_CHECK(timed(plan, stream, QT_KCLASS_OTHER, -1, 0, 0, [&] {
      return launch_final(f, ws.dfinal, np, np, c128, scaled, ws.exps, ws.maxbits, ws.per_slice, end, stream, sums,
                          sum_mode);
    }));
    ++launches;
  } else {
    const int64_t C = ws.chunk;
    for (int64_t cb = begin & ~(C - 1); cb < stop; cb += C) {
      if (scaled && ws.exp1_count && !(n_clear > 0 && cb == (begin & ~(C - 1)))) {
        QT_HIP_CHECK(timed(plan, stream, QT_KCLASS_OTHER, -1, 0, 0, [&] {
          return launch_fill_u32(ws.maxbits + ws.exp1_base, ws.exp1_count, 0u, stream);
        }));
        ++launches;
      }
      for (const auto& op : ws.slice_ops) QT_HIP_CHECK(run_op(op, cb));
      f.lg_nsb = ilog2(C);
      f.chunk_base = cb;
      QT_HIP_CHECK(timed(plan, stream, QT_KCLASS_OTHER, -1, 0, 0, [&] {
        return launch_final(f, ws.dfinal, np, (int64_t)np * C, c128, scaled, ws.exps, ws.maxbits, ws.per_slice, stop,
                            stream, sums, sum_mode);
      }));
      ++launches;
    }
  }
  if (!sum_mode || stop <= begin) {
    QT_HIP_CHECK(timed(plan, stream, QT_KCLASS_OTHER, -1, 0, 0,
                       [&] { return launch_slice_sum(ws.per_slice, np << f.n_open, n_range, sums, stream); }));
    ++launches;
  }
  if (ws.trace_on) {
    QT_HIP_CHECK(hipStreamSynchronize(stream));
    int max_levels = 1;
    for (auto& T : ws.segs) max_levels = std::max(max_levels, T.n_levels + 1);
    std::vector<uint64_t> tr((size_t)max_levels * ws.segs.size());
    QT_HIP_CHECK(hipMemcpy(tr.data(), ws.trace_buf, tr.size() * 8, hipMemcpyDeviceToHost));
    int rate_khz = 100000;
    (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, 0);
    for (size_t si = 0; si < ws.segs.size(); ++si) {
      const auto& S = ws.segs[si];
      const uint64_t* t = tr.data() + si * max_levels;
      std::fprintf(stderr, "segment %zu (level %d, %zu steps): total %.1f us\n", si, S.level, S.steps.size(),
                   (double)(t[S.n_levels] - t[0]) * 1e3 / rate_khz);
      for (int L = 0; L < S.n_levels; ++L) {
        int nu = S.level_off[L + 1] - S.level_off[L];
        int maxr = 0, nst = 0;
        for (size_t a = 0; a < S.steps.size(); ++a)
          if (ws.depth[S.steps[a]] == L) {
            maxr = std::max(maxr, plan.steps[S.steps[a]].rank);
            ++nst;
          }
        std::fprintf(stderr, "  level %2d: %6.2f us  steps %2d units %4d max rank %2d\n", L,
                     (double)(t[L + 1] - t[L]) * 1e3 / rate_khz, nst, nu, maxr);
      }
    }
  }
  plan.info.n_launches = launches;
  return QT_OK;
}

qt_status run_plan(qt_plan& plan, int np, const double* gammas, const double* betas, int64_t begin, int64_t end,
                   int64_t stop, hipStream_t stream, double* sums_out = nullptr) {
  QT_TRY(ensure_workspace(plan, np, end - begin));
  return run_plan_ws(plan, *plan.ws, np, gammas, betas, begin, end, stop, stream, sums_out);
}

}  // namespace
}  // namespace qt

namespace qt {
qt_status contract_in_region(qt_plan& plan, char* region, int64_t cap, uint64_t* owner, int np, const double* gammas,
                             const double* betas, int64_t begin, int64_t end, qt_amp* out, double* per_slice_out,
                             hipStream_t stream) {
  if (!plan.ws_static) plan.ws_static = std::make_unique<qt_plan::Workspace>();
  auto& ws = *plan.ws_static;
  const int64_t n_range = end - begin;
  const int64_t rows = (int64_t)np << plan.open_vars.size();
  const bool current = *owner == ws.gen && ws.ext == region && ws.np == np && ws.per_slice_cap >= rows * n_range;
  if (!current) {
    // earlier calls may still read the tables held in the region
    QT_HIP_CHECK(hipDeviceSynchronize());
    const int k = (int)plan.slice_vars.size();
    int64_t chunk = k > 0 ? (1ll << k) : 1;
    if (plan.slice_batch_req > 0)
      while (chunk > 1 && chunk > plan.slice_batch_req) chunk >>= 1;
    int64_t need = 0;
    for (;; chunk >>= 1) {  // sizing passes: the largest slice batch that fits
      ws.release();
      ws.np = 0;
      ws.ext = reinterpret_cast<char*>(256);  // never dereferenced: nothing is written in a sizing pass
      ws.ext_cap = cap;
      ws.counting = true;
      QT_TRY(layout_workspace(plan, ws, np, n_range, chunk));
      need = ws.ext_used;
      if (need <= cap || chunk == 1) break;
    }
    ws.counting = false;
    ws.release();
    ws.np = 0;
    ws.ext = region;
    *owner = 0;
    if (need > cap)
      return fail(QT_EINVAL, "qt_contract_batch_noalloc: the contraction needs " + std::to_string(need) +
                                 " bytes of workspace at one slice per launch; the static scratch holds " +
                                 std::to_string(cap));
    QT_TRY(layout_workspace(plan, ws, np, n_range, chunk));
    *owner = ws.gen;
  }
  QT_TRY(run_plan_ws(plan, ws, np, gammas, betas, begin, end, end, stream));
  if (per_slice_out) {
    const size_t row = (size_t)n_range * 3 * sizeof(double);
    QT_TRY(copy_2d(per_slice_out, row, ws.per_slice, row, row, (size_t)rows, stream));
  }
  const size_t bytes = (size_t)rows * sizeof(qt_amp);
  return copy_2d(out, bytes, ws.sums, bytes, bytes, 1, stream);
}

qt_status run_plan_points(qt_plan& plan, int np, const double* gammas, const double* betas, hipStream_t stream,
                          const double** sums) {
  QT_TRY(run_plan(plan, np, gammas, betas, 0, 1ll << plan.slice_vars.size(), 1ll << plan.slice_vars.size(), stream));
  *sums = plan.ws->sums;
  return QT_OK;
}
}  // namespace qt

namespace qt {
namespace {

// Enqueues one plan's full contraction and its result copies on `stream`
// (all pointers device memory: nothing here waits on the host).
qt_status enqueue_device(qt_plan& plan, int np, const double* gammas, const double* betas, int64_t begin,
                         int64_t end, qt_amp* out, double* per_slice_out, hipStream_t stream) {
  const int64_t n_range = end - begin;
  QT_TRY(run_plan(plan, np, gammas, betas, begin, end, end, stream));
  auto& ws = *plan.ws;
  const size_t rows = (size_t)np << plan.open_vars.size();
  if (per_slice_out) {
    const size_t row = (size_t)n_range * 3 * sizeof(double);
    QT_TRY(copy_2d(per_slice_out, row, ws.per_slice, row, row, rows, stream));
  }
  const size_t bytes = rows * sizeof(qt_amp);
  return copy_2d(out, bytes, ws.sums, bytes, bytes, 1, stream);
}

// Capture on first use (per parameters/results addresses, batch shape and
// workspace generation), then replay.  The workspace is allocated before
// capture, so the graph holds kernels and device-to-device copies only.
qt_status contract_graph(qt_plan& plan, int np, const double* gammas, const double* betas, int64_t begin, int64_t end,
                         qt_amp* out, double* per_slice_out, hipStream_t stream) {
  QT_TRY(ensure_workspace(plan, np, end - begin));
  if (!plan.graphs) plan.graphs = std::make_unique<qt_plan::Graphs>();
  const uint64_t gen = plan.ws->gen;
  qt_plan::Graphs::Entry* hit = nullptr;
  for (auto& e : plan.graphs->entries)
    if (e.np == np && e.begin == begin && e.end == end && e.g == gammas && e.b == betas && e.out == out &&
        e.per_slice == per_slice_out && e.gen == gen)
      hit = &e;
  if (!hit) {
    if (plan.graphs->entries.size() >= 8) plan.graphs->clear();
    hipStream_t cs = nullptr;
    QT_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    const bool prof = plan.prof && plan.prof->enabled;
    if (prof) plan.prof->enabled = false;  // no event nodes in the graph
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    qt_status st = QT_OK;
    if (e == hipSuccess) {
      st = enqueue_device(plan, np, gammas, betas, begin, end, out, per_slice_out, cs);
      e = hipStreamEndCapture(cs, &graph);
    }
    if (prof) plan.prof->enabled = true;
    (void)hipStreamDestroy(cs);
    if (st != QT_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return fail(QT_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return fail(QT_EHIP, std::string("graph instantiation: ") + hipGetErrorString(e));
    }
    plan.graphs->entries.push_back({np, begin, end, gammas, betas, out, per_slice_out, gen, graph, exec});
    hit = &plan.graphs->entries.back();
  }
  QT_HIP_CHECK(hipGraphLaunch(hit->exec, stream));
  return QT_OK;
}

}  // namespace
}  // namespace qt

extern "C" qt_status qt_contract_batch(qt_plan* const* plans, int32_t n_plans, int32_t n_points,
                                       const double* gammas, const double* betas, int64_t slice_begin,
                                       int64_t slice_end, qt_amp* out, double* per_slice_out, void* hip_stream) {
  try {
    if (!plans || n_plans <= 0 || n_points <= 0 || !out) return fail(QT_EINVAL, "qt_contract_batch: bad arguments");
    const int p = plans[0] ? plans[0]->net.p : 0;
    if (p > 0 && (!gammas || !betas)) return fail(QT_EINVAL, "qt_contract_batch: null parameters");
    const int n_open = plans[0] ? (int)plans[0]->open_vars.size() : 0;
    for (int i = 0; i < n_plans; ++i) {
      if (!plans[i]) return fail(QT_EINVAL, "qt_contract_batch: null plan");
      if (plans[i]->net.p != p) return fail(QT_EINVAL, "qt_contract_batch: plans differ in p");
      if ((int)plans[i]->open_vars.size() != n_open)
        return fail(QT_EINVAL, "qt_contract_batch: plans differ in their number of open variables");
      const int64_t ns = 1ll << plans[i]->slice_vars.size();
      if (slice_begin < 0 || slice_end > ns || slice_begin >= slice_end)
        return fail(QT_EINVAL, "qt_contract_batch: slice range outside [0, n_slices)");
    }
    if (((slice_end - slice_begin) * n_points << n_open) > (1ll << 28))
      return fail(QT_EINVAL, "qt_contract_batch: slice range too long for one call");
    const int64_t rows = (int64_t)n_points << n_open;  // results per plan
    hipStream_t stream = (hipStream_t)hip_stream;
    int64_t stop = slice_end;
    bool injected = false;
    if (const char* e = std::getenv("QT_FAULT_AFTER_SLICE")) {
      const int64_t j = std::atoll(e);
      if (j >= slice_begin && j < slice_end) {
        stop = j;
        injected = true;
      }
    }
    const int64_t n_range = slice_end - slice_begin;
    // QT_PLAN_GRAPH: replay an instantiated capture of the whole sequence
    // (device-resident parameters and results only)
    if (n_plans == 1 && (plans[0]->flags & QT_PLAN_GRAPH) && !injected &&
        (p == 0 || (is_device_ptr(gammas) && is_device_ptr(betas))) && is_device_ptr(out) &&
        (!per_slice_out || is_device_ptr(per_slice_out)))
      return contract_graph(*plans[0], n_points, gammas, betas, slice_begin, slice_end, out, per_slice_out, stream);
    // results in device memory are written by the sum launch itself
    const bool dev_out = !injected && is_device_ptr(out);
    for (int i = 0; i < n_plans; ++i) {
      qt_plan& plan = *plans[i];
      double* const direct = dev_out ? reinterpret_cast<double*>(out + (size_t)i * rows) : nullptr;
      if (stop > slice_begin)
        QT_TRY(run_plan(plan, n_points, gammas, betas, slice_begin, slice_end, stop, stream, direct));
      else QT_TRY(ensure_workspace(plan, n_points, n_range));
      auto& ws = *plan.ws;
      if (per_slice_out && stop > slice_begin) {
        const size_t row = (size_t)n_range * 3 * sizeof(double);
        const size_t width = (size_t)(stop - slice_begin) * 3 * sizeof(double);
        QT_TRY(copy_2d(per_slice_out + (size_t)i * rows * n_range * 3, row, ws.per_slice, row, width, rows, stream));
      }
      if (!injected && !(dev_out && stop > slice_begin)) {
        const size_t bytes = (size_t)rows * sizeof(qt_amp);
        QT_TRY(copy_2d(out + (size_t)i * rows, bytes, ws.sums, bytes, bytes, 1, stream));
      }
    }
    if (injected) return fail(QT_EFAULT_INJECTED, "qt_contract_batch: QT_FAULT_AFTER_SLICE fired");
    return QT_OK;
  } catch (const std::exception& ex) {
    return fail(QT_ENOMEM, std::string("qt_contract_batch: ") + ex.what());
  }
}

extern "C" qt_status qt_contract_amplitude(qt_plan* plan, const double* gammas, const double* betas, qt_amp* out,
                                           void* hip_stream) {
  if (!plan) return fail(QT_EINVAL, "qt_contract_amplitude: null plan");
  const int64_t ns = 1ll << plan->slice_vars.size();
  return qt_contract_batch(&plan, 1, 1, gammas, betas, 0, ns, out, nullptr, hip_stream);
}

extern "C" void qt_free_plan(qt_plan* plan) {
  if (!plan) return;
  energy_forget(plan->serial);
  delete plan;
}

extern "C" qt_status qt_plan_set_tuning(qt_plan* plan, const qt_tuning* t) {
  if (!plan || !t) return fail(QT_EINVAL, "qt_plan_set_tuning: null argument");
  auto waves_ok = [](int32_t w) { return w == 0 || (w >= 1 && w <= kXMaxThreads / 64); };
  if (!waves_ok(t->lds_waves) || !waves_ok(t->multi_waves) || !waves_ok(t->grad_waves))
    return fail(QT_EINVAL, "qt_plan_set_tuning: wavefronts per workgroup must be 0 or 1..16");
  if (t->lds_max_rank != 0 && (t->lds_max_rank < 6 || t->lds_max_rank > 16))
    return fail(QT_EINVAL, "qt_plan_set_tuning: lds_max_rank must be 0 or 6..16");
  auto pow2_upto = [](int32_t v, int32_t hi) { return v == 0 || (v >= 1 && v <= hi && (v & (v - 1)) == 0); };
  if (!pow2_upto(t->step_tiles, 16)) return fail(QT_EINVAL, "qt_plan_set_tuning: step_tiles must be 0, 1, 2, 4, 8 or 16");
  if (!pow2_upto(t->gemm_tiles, 64)) return fail(QT_EINVAL, "qt_plan_set_tuning: gemm_tiles must be 0 or a power of two up to 64");
  for (int32_t cap : {t->multi_lds_cap, t->grad_lds_cap})
    if (cap != 0 && (cap < 4096 || cap > 160 * 1024))
      return fail(QT_EINVAL, "qt_plan_set_tuning: multi_lds_cap and grad_lds_cap must be 0 or 4096..163840");
  const bool reschedule = t->lds_waves != plan->tuning.lds_waves || t->lds_max_rank != plan->tuning.lds_max_rank;
  const bool relaunch = t->step_tiles != plan->tuning.step_tiles || t->gemm_tiles != plan->tuning.gemm_tiles;
  plan->tuning = *t;
  if ((reschedule || relaunch) && plan->graphs) plan->graphs->clear();
  if (reschedule) {
    plan->ws.reset();
  }
  return QT_OK;
}

extern "C" qt_status qt_plan_get_tuning(const qt_plan* plan, qt_tuning* out) {
  if (!plan || !out) return fail(QT_EINVAL, "qt_plan_get_tuning: null argument");
  *out = plan->tuning;
  return QT_OK;
}

extern "C" qt_status qt_plan_describe(const qt_plan* plan, char* buf, int64_t cap, int64_t* needed) {
  try {
    if (!plan || !needed) return fail(QT_EINVAL, "qt_plan_describe: null argument");
    qt_plan::Workspace ws;
    const int elt = plan->precision == QT_C128 ? 16 : 8;
    QT_TRY(plan_schedule(const_cast<qt_plan&>(*plan), ws, elt));
    std::string j = "{\"element_bytes\":" + std::to_string(elt) + ",\"n_open\":" +
                    std::to_string(plan->open_vars.size()) + ",\"n_groups\":" + std::to_string(plan->n_groups) +
                    ",\"segments\":[";
    for (size_t si = 0; si < ws.segs.size(); ++si) {
      const auto& S = ws.segs[si];
      int staged = 0, internal = 0;
      for (size_t t = 0; t < plan->tensors.size(); ++t) {
        if (ws.staged_in[t] == (int)si) ++staged;
        else if (ws.lds_off[t] >= 0 && ws.staged_in[t] < 0 && plan->tensors[t].producer >= 0 &&
                 ws.seg_of[plan->tensors[t].producer] == (int)si)
          ++internal;
      }
      const size_t smem = lds_exec_smem_bytes(S.n_slots, S.lds_elems, elt == 16);
      j += std::string(si ? "," : "") + "{\"level\":" + std::to_string(S.level) + ",\"steps\":" +
           std::to_string(S.steps.size()) + ",\"first_step\":" + std::to_string(S.steps.front()) +
           ",\"levels\":" + std::to_string(S.n_levels) + ",\"lds_bytes\":" + std::to_string(smem) +
           ",\"slots\":" + std::to_string(S.n_slots) + ",\"internal\":" + std::to_string(internal) +
           ",\"staged\":" + std::to_string(staged) + ",\"step_list\":[";
      // per step, in plan order: [dependency level, rank, summed, per-input [rank within a slice, has_v, leaf]]
      for (size_t a = 0; a < S.steps.size(); ++a) {
        const SymStep& st = plan->steps[S.steps[a]];
        j += std::string(a ? "," : "") + "[" + std::to_string(ws.depth[S.steps[a]]) + "," +
             std::to_string(st.rank) + "," + std::to_string(st.sum) + ",[";
        for (size_t q = 0; q < st.ins.size(); ++q) {
          const SymTensor& T = plan->tensors[st.ins[q].tensor];
          j += std::string(q ? "," : "") + "[" + std::to_string(T.rank - __builtin_popcount(st.ins[q].smask)) +
               "," + std::to_string(st.ins[q].has_v) + "," + std::to_string(T.leaf >= 0 ? 1 : 0) + "]";
        }
        j += "]]";
      }
      j += "]}";
    }
    j += "],\"stream_steps\":[";
    bool first = true;
    for (auto* ops : {&ws.prefix_ops, &ws.slice_ops})
      for (const auto& op : *ops)
        if (op.seg < 0) {
          const SymStep& st = plan->steps[op.step];
          j += std::string(first ? "" : ",") + "{\"step\":" + std::to_string(op.step) + ",\"rank\":" +
               std::to_string(st.rank) + ",\"inputs\":" + std::to_string(st.ins.size()) + ",\"level\":" +
               std::to_string(st.level) + ",\"bytes\":" + std::to_string(st.bytes_c64) + ",\"in_ranks\":[" +
               [&] {
                 // per input: its rank within one slice, and whether it holds the summed variable
                 std::string r, h;
                 for (size_t q = 0; q < st.ins.size(); ++q) {
                   const int rk = plan->tensors[st.ins[q].tensor].rank - __builtin_popcount(st.ins[q].smask);
                   r += (q ? "," : "") + std::to_string(rk);
                   h += (q ? "," : "") + std::to_string(st.ins[q].has_v);
                 }
                 return r + "],\"in_has_v\":[" + h;
               }() + "]" +
               (st.gemm ? ",\"gemm\":{\"k_bits\":" + std::to_string(st.kvars.size()) + ",\"flops\":" +
                              std::to_string(st.flops) + ",\"tile\":" + [&] {
                                int32_t tb, tm, tn, tk, mode;
                                choose_gemm_tile(*plan, st, tb, tm, tn, tk, mode);
                                return "[" + std::to_string(tb) + "," + std::to_string(tm) + "," +
                                       std::to_string(tn) + "," + std::to_string(tk) + "],\"mode\":\"" +
                                       (mode ? "bf16x3_3m" : (tk == 64 ? "fp32_3m" : "fp32_4m")) + "\"";
                              }() + ",\"layouts\":" + [&] {
                                // per operand, from bit 0 up: the counter each storage bit belongs to
                                const auto& va = plan->tensors[st.ins[0].tensor].vars;
                                const auto& vb = plan->tensors[st.ins[1].tensor].vars;
                                auto has = [](const std::vector<int32_t>& v, int x) {
                                  return std::find(v.begin(), v.end(), x) != v.end();
                                };
                                auto code = [&](int x) {
                                  if (has(st.kvars, x)) return 'k';
                                  const bool ia = has(va, x), ib = has(vb, x);
                                  return ia && ib ? 'b' : (ia ? 'm' : (ib ? 'n' : 's'));
                                };
                                std::string r = "[\"";
                                for (int x : va) r += code(x);
                                r += "\",\"";
                                for (int x : vb) r += code(x);
                                r += "\",\"";
                                for (int x : plan->tensors[st.out].vars) r += code(x);
                                return r + "\"]";
                              }() + "}"
                        : std::string()) +
               "}";
          first = false;
        }
    j += "],\"arena0_units\":" + std::to_string(ws.arena0_units) + ",\"arena1_units\":" +
         std::to_string(ws.arena1_units) + "}";
    *needed = (int64_t)j.size() + 1;
    if (!buf || cap < *needed) return fail(QT_EINVAL, "qt_plan_describe: buffer too small");
    std::memcpy(buf, j.c_str(), j.size() + 1);
    return QT_OK;
  } catch (const std::exception& ex) {
    return fail(QT_ENOMEM, std::string("qt_plan_describe: ") + ex.what());
  }
}

extern "C" qt_status qt_profile_enable(qt_plan* plan, int32_t enable) {
  if (!plan) return fail(QT_EINVAL, "qt_profile_enable: null plan");
  if (!plan->prof) plan->prof = std::make_unique<qt_plan::Profile>();
  plan->prof->enabled = enable != 0;
  return QT_OK;
}

extern "C" qt_status qt_profile_read(qt_plan* plan, qt_kernel_stats* out, int32_t reset) {
  if (!plan || !out) return fail(QT_EINVAL, "qt_profile_read: null argument");
  if (!plan->prof) plan->prof = std::make_unique<qt_plan::Profile>();
  QT_HIP_CHECK(plan->prof->drain());
  for (int i = 0; i < QT_KCLASS_COUNT; ++i) out[i] = plan->prof->acc[i];
  if (reset) {
    for (auto& a : plan->prof->acc) a = qt_kernel_stats{};
    plan->prof->ops.clear();
  }
  return QT_OK;
}

extern "C" qt_status qt_profile_read_ops(qt_plan* plan, qt_op_stats* out, int32_t cap, int32_t* n_ops,
                                         int32_t reset) {
  if (!plan || !n_ops || (cap > 0 && !out)) return fail(QT_EINVAL, "qt_profile_read_ops: null argument");
  if (!plan->prof) plan->prof = std::make_unique<qt_plan::Profile>();
  QT_HIP_CHECK(plan->prof->drain());
  const auto& ops = plan->prof->ops;
  *n_ops = (int32_t)ops.size();
  for (int32_t i = 0; i < cap && i < (int32_t)ops.size(); ++i) out[i] = ops[i];
  if (reset) {
    for (auto& a : plan->prof->acc) a = qt_kernel_stats{};
    plan->prof->ops.clear();
  }
  return QT_OK;
}


