// Internal declarations of the MI355X contractor: network storage, the
// compiled plan, and the step descriptors the kernels consume.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/qtensor_hip.h"
#include "../../include/qtensor_planner.h"

namespace qt {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
qt_status fail(qt_status code, const std::string& msg);
#define QT_TRY(expr)            \
  do {                          \
    qt_status _s = (expr);      \
    if (_s != QT_OK) return _s; \
  } while (0)
#define QT_HIP_CHECK(expr)                                                           \
  do {                                                                               \
    hipError_t _e = (expr);                                                          \
    if (_e != hipSuccess)                                                            \
      return ::qt::fail(QT_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// --------------------------------------------------------------- network
struct Leaf {
  int32_t kind = 0;
  int32_t layer = 0;
  std::vector<int32_t> vars;   // internal (dense) variable ids, as given
  std::vector<double> dense;   // DENSE: 2^rank (re, im), vars[0] most significant
};

}  // namespace qt

struct qt_network {
  int32_t n_vars_ext = 0;         // external id space
  int32_t p = 0;
  std::vector<int32_t> ext_of;    // internal id -> external id
  std::vector<int32_t> int_of;    // external id -> internal id (-1: unused)
  std::vector<qt::Leaf> leaves;
  int32_t n_vars() const { return (int32_t)ext_of.size(); }
};

namespace qt {

// ------------------------------------------------------- device descriptors
// Limits of one bucket-step launch.  A bucket with more inputs is split into
// product steps on the host.
constexpr int kMaxIn = 8;
constexpr int kMaxRuns = 16;  // a 31-bit mask has at most 16 runs
constexpr int kMaxRank = 31;
constexpr int kMaxOpen = 20;  // open output variables of a plan

// One input of a bucket step.  Element index of the value for output
// element x of batch item (pt, sb) with slice id sid:
//   pt*pt_stride + sb*sb_stride + (pext(sid, smask) << slow)
//     + (pext(x, mask) << has_v) + v
// where pext(x, mask) is evaluated from its runs of contiguous bits.
struct DevIn {
  const void* ptr;
  int64_t pt_stride;
  int64_t sb_stride;
  uint32_t smask;
  int32_t slow;
  int32_t has_v;
  int32_t nruns;
  uint8_t run_lo[kMaxRuns];
  uint8_t run_len[kMaxRuns];
  uint8_t run_dst[kMaxRuns];
  // power-of-two scaling (C64_SCALED): exponent / max slots of this tensor
  // instance = exp_base + pt*exp_pt + sb*exp_sb; exp_base < 0 for unscaled
  // leaves.
  int32_t exp_base;
  int32_t exp_pt;
  int32_t exp_sb;
  // Streaming tiles of 1024 outputs (x = tile << 10 | e << 8 | lane): the
  // index splits as pext(tile << 10) + pext(e << 8) + pext(lane); the tile
  // part has its own runs (over the tile index), the e part is tabulated.
  int32_t t_nruns;
  uint8_t t_lo[kMaxRuns];
  uint8_t t_len[kMaxRuns];
  uint8_t t_dst[kMaxRuns];
  uint32_t ep[4];
  // Elements of the tensor's block per batch item when it is small enough
  // (at most x_small_cap(inputs of the step)) for the streaming kernel to
  // stage it in LDS; else 0.
  int32_t small_n;
  int32_t pad;
};
// Staging capacity per input, by the count of inputs the kernel indexes
// (inputs read by no output bit are not staged), as measured on the
// 210-qubit plan: 1024 elements let its three-operand step (a merged
// factor and a rank-10 input beside a large one) read both small inputs from
// LDS; larger static LDS for two operands cost occupancy on its two-operand
// steps.
__host__ __device__ constexpr int x_small_cap(int n_in) {
  return n_in <= 2 ? 512 : (n_in == 3 ? 1024 : (n_in == 4 ? 128 : (n_in == 5 ? 512 : 64)));
}

struct DevStep {
  void* out;
  int64_t chunk_base;    // global slice id of batch item sb = 0
  int32_t r;             // output rank
  int32_t lg_nsb;        // log2(slice batch items of the output level)
  int32_t lg_items;      // log2(number of (pt, sb) items)
  int32_t lg_tiles;      // BIG mode: log2(tiles per item)
  int32_t sum;           // 1: sum over the lowest bit of the has_v inputs; 0: product only
  int32_t n_in;
  int32_t out_exp_base;  // -1: unscaled output
  int32_t out_exp_pt;
  int32_t out_exp_sb;
  int32_t lg_tpb;        // BIG mode: log2(consecutive tiles of one item per workgroup)
  int32_t n_uni;         // BIG mode: the last n_uni inputs are read by no output bit (set at launch)
  int32_t pad;
  DevIn in[kMaxIn];
};

// ------------------------------------------------- LDS executor descriptors
// Operand of a step run by the LDS executor; always in LDS (gate table,
// staged input or internal tensor).  Element index for output x:
//   lds_off + (pext(sid, smask) << slow) + (pext(x, mask) << has_v) + v
// with pext(x) split as pext(unit base) + ep[e] + pext(lane) for
// x = unit base + 64 e + lane.
constexpr int kXRuns = 8;   // executor steps have outputs of rank <= 16
struct XOp {  // 32-bit fields only: they are read with scalar loads
  uint32_t lds_off;
  uint32_t smask;   // slice-id bits (gate operands on slice variables)
  int32_t slow;
  int32_t has_v;
  int32_t slot;     // LDS scale slot, -1: unscaled
  uint32_t lane_runs;  // the runs over lane bits 0..5 (at most 3), packed: see x_lane_runs
  uint32_t ep[4];   // pext(64 e) << has_v for the unit's elements e
  uint8_t run_lo[kXRuns];
  uint8_t run_len[kXRuns];
  uint8_t run_dst[kXRuns];
};

static_assert(kXRuns % 4 == 0 && offsetof(XOp, run_lo) % 4 == 0 && sizeof(XOp) % 4 == 0, "word-aligned run tables");

// The part of an operand's runs that a lane index (bits 0..5) reaches, as
// one word: run i (i < 3) has source bit, length and destination bit (plus
// `shift`, the operand's has_v) in bits 9i..9i+8 (3 bits each), and the
// run count in bits 27..28.
inline uint32_t x_lane_runs(const uint8_t* lo, const uint8_t* len, const uint8_t* dst, int n, int shift) {
  uint32_t w = 0, k = 0;
  for (int i = 0; i < n && lo[i] < 6; ++i) {
    const uint32_t l = lo[i], m = len[i] < 6 - lo[i] ? len[i] : 6 - lo[i];
    w |= (l | m << 3 | ((uint32_t)dst[i] + (uint32_t)shift) << 6) << (9 * k);
    ++k;
  }
  return w | k << 27;
}

// Output of an executor step: LDS (ptr null) or global memory.
struct XOut {
  void* ptr;
  int64_t pt_stride;
  int64_t sb_stride;
  uint32_t lds_off;
  int32_t slot_kind;  // 0: unscaled; 1: LDS slot; 2: global slot
  int32_t slot;
  int32_t exp_pt;
  int32_t exp_sb;
  int32_t pairs;  // LDS executor: every operand holds v at an even base (see XStep)
};

// A step of the LDS executors.  n_in is the exact operand count; in[] is
// padded with identity operands up to 2, 4 or 8.  chunk: the unit's chunk
// where each unit has its own copy (the chunk's part of every operand index
// then folded into lds_off).  out.pairs = 1 when every operand holds the
// summed variable (as bit 0) at an even LDS base, so that the v = 0 and
// v = 1 elements are one aligned pair.
struct XStep {
  XOut out;
  int32_t r;
  int32_t sum;
  int32_t n_in;
  int32_t chunk;
  XOp in[kMaxIn];
};
static_assert(sizeof(XStep) % 64 == 0, "step descriptors are whole 64-byte lines");

// Work unit of the executor: steps of rank >= kXBigRank are cut into units
// of kXEpu * 64 outputs (kXEpu per lane), smaller steps into 64-output units
// (complex128 uses kXEpu / 2 per lane; steps with more than 4 inputs use
// half as many again).  Steps are padded to 2, 4 or 8 inputs.
constexpr int kXBigRank = 8;
constexpr int kXEpu = 4;
constexpr int kXMaxThreads = 1024;
inline int x_nin_class(int n_in) { return n_in <= 2 ? 2 : (n_in <= 4 ? 4 : 8); }
inline int x_epu(int rank, int n_in, int elt) {
  if (rank < kXBigRank) return 1;
  int epu = elt == 8 ? kXEpu : kXEpu / 2;
  if (x_nin_class(n_in) == 8) epu = epu > 1 ? epu / 2 : 1;
  return epu;
}
inline int64_t x_unit_elems(int rank, int n_in, int elt) { return 64 * x_epu(rank, n_in, elt); }

// Global tensor copied into LDS at the start of an executor launch (the
// block of one batch item: 2^rank elements, or the slice-selected block of a
// prefix tensor).
struct XCopy {
  const void* ptr;
  int64_t pt_stride;
  int64_t sb_stride;
  uint32_t smask;
  int32_t slow;
  uint32_t lds_off;
  uint32_t n;
  int32_t gslot;  // global scale slot base (-1: unscaled)
  int32_t exp_pt;
  int32_t exp_sb;
  int32_t lslot;  // LDS scale slot
};

// LDS element area of an executor workgroup: element 0-1 the identity
// operand (1 + 0i), then the gate table of the workgroup's point, then
// staged and internal tensors.  Gate table (element offsets): |+> (1, 1) at
// 2, <0| at 4, <1| at 6, the edge observable at 8, and for layer k (0-based)
// ZZ, ZZ^dagger, RX, RX^dagger at 12 + 16k + {0, 4, 8, 12} (10 + 16p entries).
constexpr int kXGate = 2;
__host__ __device__ inline int x_gate_elems(int p) { return 10 + 16 * p; }
__host__ __device__ inline int x_tensor_base(int p) { return (kXGate + x_gate_elems(p) + 1) & ~1; }
inline int x_gate_off(int kind, int layer) {
  switch (kind) {
    case QT_T_VEC_PLUS: return kXGate + 0;
    case QT_T_BRA_BIT: return kXGate + (layer ? 4 : 2);
    case QT_T_OBS_CUT: return kXGate + 6;
    case QT_T_ZZ: return kXGate + 10 + 16 * (layer - 1);
    case QT_T_ZZ_DAG: return kXGate + 14 + 16 * (layer - 1);
    case QT_T_RX: return kXGate + 18 + 16 * (layer - 1);
    case QT_T_RX_DAG: return kXGate + 22 + 16 * (layer - 1);
    default: return -1;
  }
}

// One launch of the executor: every workgroup runs the same level schedule
// for its batch item (pt, sb).  Work unit u (levels in order) is described
// by steps[u], a copy of its step's descriptor whose pad field holds the
// unit's chunk, so a wavefront reaches its descriptor without first reading
// a unit table.
struct XLaunch {
  const XStep* steps;      // per unit
  const uint2* units;      // unused by the executor (kept for the host)
  const int32_t* level_off;  // n_levels + 1 offsets into units
  const XCopy* copies;     // inputs staged into LDS at the start
  const double* gam;       // point q's gammas at gam + q * pstride, its betas at bet + q * pstride
  const double* bet;
  int32_t pstride;
  int32_t n_levels;
  int32_t lg_nsb;
  int64_t chunk_base;
  int32_t n_slots;         // LDS scale slots
  int32_t lds_elems;       // LDS element area, elements
  int32_t n_copies;
  int32_t p;
  uint64_t* trace;         // optional: workgroup 0 stores wall_clock64() after each level
};

// Multi-program launch (per-edge lightcone networks): item i runs program
// item_prog[i / n_points] at point i % n_points; every tensor of a program
// lives in LDS and its scalar result is formed in an FP64 epilogue.
struct XFinal {
  uint32_t lds_off;
  int32_t slot;
};
struct XProg {
  int32_t steps_off;   // first XStep of the program
  int32_t units_off;   // first unit (units name steps relative to steps_off)
  int32_t levels_off;  // first of its n_levels + 1 level offsets (relative to units_off)
  int32_t n_levels;
  int32_t n_slots;
  int32_t finals_off;  // gradient programs: n_finals values, then their n_finals adjoints
  int32_t n_finals;
  int32_t revs_off;    // first XRev (gradient programs; units name them relative to it)
  int32_t recs_off;    // first of 2p + 1 offsets of its gradient records, grouped by parameter
  int32_t n_recs;
  double log2_const;   // exponent of the |+> normalisations
  // A program too large for the launch's LDS runs from global scratch in
  // the same launch: its element area (area_elems), scale slots and
  // gradient records for point pt start at byte scratch_off + pt *
  // scratch_stride of XMulti::scratch.  -1: LDS.
  int64_t scratch_off;
  int64_t scratch_stride;
  int32_t area_elems;
  // Forward programs in LDS run n_pts points per workgroup: point q's
  // tensors at element q * pt_stride, its scale slots at q * slot_stride.
  int32_t n_pts;
  int32_t pt_stride;
  int32_t slot_stride;
  int32_t rec_stride;  // gradient programs: gradient records per point
  int32_t pad;
};

// Reverse (adjoint) operation of the gradient executor.  For one input T_j
// of a bucket step with output R (Algorithm 1 run backwards), over the
// step's index space z (the output bits, and the summed variable as bit 0):
//   Tbar_j[y] = sum_c Rbar[.] * prod_{i != j} T_i[.]
// where y runs over the bits of T_j and c over the remaining bits of z.
// Operand o is read at lds_off + map_y(y) + map_c(c), each map a list of
// bit runs (source bit, length, destination bit); padding operands read the
// identity element.  For a gate input the result is not stored: it is
// contracted with the gate's derivative by its parameter and kept as one
// FP64 gradient record.
struct XROp {
  uint32_t lds_off;
  int32_t slot;  // scale slot, -1: unscaled
  uint8_t y_lo[kXRuns], y_len[kXRuns], y_dst[kXRuns];
  uint8_t c_lo[kXRuns], c_len[kXRuns], c_dst[kXRuns];
  // The same maps per lane bit b of a unit (linear over disjoint bits):
  // lw[b] = the operand offset of lane bit b (a y bit, or for a small
  // adjoint above its ry bits a bit of the complement group g);
  // iw[b] = that of bit b of the iteration index of the first 64
  // iterations (complement c = g + G i).
  uint32_t lw[6], iw[6];
};
// the executors read these byte tables as 32-bit words
static_assert(kXRuns % 4 == 0 && offsetof(XROp, y_lo) % 4 == 0 && sizeof(XROp) % 4 == 0, "word-aligned run tables");
struct XRev {
  uint32_t out_off;   // LDS element offset of Tbar_j
  int32_t out_slot;   // its scale slot (-1: unscaled)
  int32_t ry;         // bits of y (rank of T_j)
  int32_t nc;         // bits of c
  int32_t n_ops;      // operands (2..8): R-bar, then the step's other inputs
  int32_t gate;       // -1: tensor adjoint; 0..3: derivative of ZZ, ZZ^dagger, RX, RX^dagger
  int32_t param;      // gate parameter: layer k's gamma at k, its beta at p + k
  int32_t rec;        // gradient record of a gate input
  XROp op[kMaxIn];
};
// Unit kinds of the gradient executor (top bits of a unit's first word).
constexpr uint32_t kXUnitRev = 1u << 30;    // reverse operation
constexpr uint32_t kXUnitFinal = 2u << 30;  // adjoints of the closing scalars
constexpr uint32_t kXUnitIndex = (1u << 30) - 1u;

struct XMulti {
  const XProg* progs;
  const XStep* steps;
  const uint2* units;
  const int32_t* level_off;
  const XFinal* finals;
  const int32_t* item_prog;
  const double* gam;       // point q's gammas at gam + q * pstride, its betas at bet + q * pstride
  const double* bet;
  int32_t pstride;
  int32_t pad;
  double* out;             // [points][programs][3]: re, im, log2 scale
  const XRev* revs;        // gradient executor only
  const int32_t* rec_off;
  double* gout;            // [points][programs][2p]: per-edge derivatives
  int32_t n_points;
  int32_t n_progs;
  int32_t p;
  int32_t lds_elems;       // max over the programs run from LDS
  int32_t n_slots;         // max over the programs run from LDS
  int32_t n_recs;          // max over the programs run from LDS
  char* scratch;           // areas of the programs run from global scratch
  const int2* items;       // multi-program executor: (program, first point) per workgroup
};

// Fused GEMM bucket: C[b, m, n] = sum_k A[b, m, k] B[b, n, k] over complex
// values, for every batch item (point, slice).  The counters b, m, n, k run
// over their variables in key order, and every tensor stores its variables
// in key order, so a counter's value enters a tensor's element index as a
// monotone bit deposit into the storage bits of its variables (a mask);
// a prefix tensor adds its slice-selected block.
constexpr int kGBits = 16;
constexpr int kGemmMaxRank = 28;  // per-item operand and output ranks: byte offsets below 2^31  // element-number bits of an operand stage or an output tile
struct DevGemm {
  const void* a;
  const void* b;
  void* c;
  int64_t a_pt, a_sb, b_pt, b_sb, c_pt, c_sb;  // element strides per point and per slice item
  uint32_t a_smask, b_smask;
  int32_t a_slow, b_slow;
  int64_t chunk_base;
  int32_t lg_nsb;
  int32_t n_items;
  int32_t nb, nm, nn, nk;  // counter bits
  int32_t a_exp_base, a_exp_pt, a_exp_sb;  // -1 base: unscaled (a leaf)
  int32_t b_exp_base, b_exp_pt, b_exp_sb;
  int32_t c_exp_base, c_exp_pt, c_exp_sb;
  int32_t tb, tm, tn;      // tile bits of the b, m, n counters (chosen on the host)
  int32_t tk;              // K stage depth (8, 16 or 64; 32 in mode 1)
  int32_t mode;            // 0: FP32 products (3M at depth 64, else 4M); 1: split-BF16 products (3M), QT_C64_SCALED_MFMA_BF16X3
  int32_t tiles;           // output tiles per workgroup (0: the default for the depth)
  // storage bits of each counter in each tensor
  uint32_t a_bm, a_mm, a_km, b_bm, b_nm, b_km, c_bm, c_mm, c_nm;
  // the same without the bits a tile or a stage covers (masked increments)
  uint32_t a_kh, b_kh, b_nh, c_nh;
  // Elements of one K stage's A and B blocks and of one C tile are numbered
  // with the block's bits in storage order; bit j of an element number adds
  // *w[j] to its storage offset and *l[j] to its LDS offset.
  uint32_t aw[kGBits], al[kGBits], bw[kGBits], bl[kGBits], cw[kGBits], cl[kGBits];
};

// Leaf (gate) tensor materialisation record.
struct DevLeaf {
  int32_t kind;
  int32_t layer;
  int32_t rank;
  int32_t off;        // element offset inside one point's leaf block
  int32_t dense_off;  // DENSE: offset (in complex values) into the dense table
  int32_t pad;
};

// Per-slice value of a scalar factor list (final combination).
struct DevFinal {
  int32_t n_factors;
  int32_t lg_nsb;
  int32_t n_open;        // open output bits j: factor f is read at pext(j, its runs), see k_final
  int32_t pad;
  int64_t chunk_base;
  int64_t slice_begin;   // per-slice output index = sid - slice_begin
  int64_t n_range;       // number of slices in the output range (row length)
  double log2_const;     // constant exponent (|+> factors)
};

// ---------------------------------------------------------------- plan
struct SymIn {
  int32_t tensor;
  int32_t has_v;
  uint32_t mask;   // over output bits
  uint32_t smask;  // over slice-id bits
  int32_t slow;
};

struct SymStep {
  int32_t out;          // tensor id
  int32_t level;        // 0 prefix, 1 per slice
  int32_t rank;
  int32_t sum;
  int32_t var;          // eliminated variable (internal id), -1 for product steps
  int32_t nbr;          // neighbour count of the eliminated variable (its width)
  int32_t gemm = 0;     // fused GEMM bucket: ins = {A, B}, summed over kvars
  std::vector<int32_t> kvars;  // GEMM: summed variables, by key (the bucket variable first)
  std::vector<SymIn> ins;
  double bytes_c64;     // algorithmic bytes per item at 8 B per element
  double flops;         // real flops per item
};

struct SymTensor {
  std::vector<int32_t> vars;  // internal ids sorted by key (lowest bit first), incl. slice vars
  int32_t level = 0;
  int32_t leaf = -1;          // leaf index, or -1 for intermediates
  int32_t producer = -1;      // step id
  int32_t consumer = -1;      // step id, or -2 for final scalar factors
  int32_t rank = 0;           // stored rank (= vars.size())
  int32_t exp_slot = -1;      // scalar slot base for exponents
};

int env_int(const char* name, int dflt);
// True for device (or managed) memory of the HIP runtime.
bool is_device_ptr(const void* p);
// Copy between library buffers and caller memory (a 2-D block of `height`
// rows of `width` bytes).  Device to device runs asynchronously on the
// stream; whenever host memory is involved the stream is drained first and
// the copy blocks, so host data is in place (or consumed) on return:
// asynchronous copies to pageable host memory are not ordered by a later
// stream synchronisation.
qt_status copy_2d(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width, size_t height,
                  hipStream_t stream);
// Writes [np][2p] (gammas of a point, then its betas) to device memory `dev`
// from caller arrays [np][p] in host or device memory.
qt_status upload_params_to(double* dev, int np, int p, const double* gammas, const double* betas,
                           hipStream_t stream);
// A tunable: the plan's value when set, else the environment, else dflt.
int tuned(int32_t value, const char* env, int dflt);
void energy_forget(uint64_t serial);  // drops cached energy jobs that use the plan
// Full contraction of a plan at np points through the general schedule;
// *sums receives the device address of its [np][3] (re, im, log2) results.
qt_status run_plan_points(qt_plan& plan, int np, const double* gammas, const double* betas, hipStream_t stream,
                          const double** sums);
bool make_runs(uint32_t mask, int max_runs, uint8_t* lo, uint8_t* len, uint8_t* dst, int32_t& nruns);
// The contraction of qt_contract_batch for one plan with its whole device
// workspace inside `region` (`cap` bytes; no allocation).  *owner names the
// layout the region holds; when it is not this plan's current one, the
// workspace is laid out afresh (the largest slice batch that fits) and its
// tables uploaded, after the device has drained, and *owner is updated.
qt_status contract_in_region(qt_plan& plan, char* region, int64_t cap, uint64_t* owner, int np, const double* gammas,
                             const double* betas, int64_t begin, int64_t end, qt_amp* out, double* per_slice_out,
                             hipStream_t stream);

// Buffers live over closed time intervals, packed first-fit, largest first.
struct Interval {
  int32_t t;
  int64_t size;
  int32_t start, end;
};
int64_t place_intervals(std::vector<Interval>& iv, std::vector<int64_t>& off_out);

}  // namespace qt

struct qt_plan {
  qt_network net;
  int32_t precision = 0;
  int32_t n_order = 0;
  std::vector<int32_t> order;       // internal ids
  int32_t slice_step = 0;           // s
  std::vector<int32_t> slice_vars;  // internal ids, first = most significant
  int32_t n_groups = 0;             // slice groups as given (all fixed at the last group's step)
  std::vector<int32_t> open_vars;   // open output variables, first = most significant output bit
  std::vector<int32_t> key;         // per internal var
  std::vector<qt::SymTensor> tensors;
  std::vector<qt::SymStep> steps;
  std::vector<int32_t> finals;      // tensor ids of scalar factors
  int32_t n_prefix_steps = 0;
  int32_t width = 0, prefix_width = 0, slice_width = 0;
  double prefix_bytes = 0, slice_bytes = 0, prefix_flops = 0, slice_flops = 0;
  double log2_const = 0;            // -1/2 per |+> leaf
  int32_t leaf_block = 0;           // elements of one point's leaves
  std::vector<qt::DevLeaf> dev_leaves;
  std::vector<double> dense_table;  // interleaved, permuted to key order
  int32_t n_exp0 = 0, n_exp1 = 0;   // exponent slots per point / per (point x item)
  int64_t slice_batch_req = 0;
  int32_t flags = 0;
  qt_tuning tuning{};   // execution tunables, 0 = default
  uint64_t serial = 0;  // unique per plan, never reused (cache keys)
  qt_plan_info info{};
  // HIP-event profiling of launches (qt_profile_enable / qt_profile_read)
  struct Profile;
  std::unique_ptr<Profile> prof;
  struct Workspace;
  std::unique_ptr<Workspace> ws;
  std::unique_ptr<Workspace> ws_static;  // laid out in a caller-provided region (qt_contract_batch_noalloc)
  // QT_PLAN_GRAPH: instantiated launch sequences, by call signature
  struct Graphs;
  std::unique_ptr<Graphs> graphs;
  qt_plan();
  ~qt_plan();
};

namespace qt {

// kernels.hip
// gammas/betas: the points' parameters in device memory ([points][p] each),
// which the launch also lays out in `params` ([points][2p]); null: `params`
// already holds them.  clear[0, n_clear): words set to zero by the same
// launch.
hipError_t launch_leaves(const DevLeaf* leaves, int n_leaves, int leaf_block, const double* dense,
                         double* params, const double* gammas, const double* betas, int p, int n_points,
                         void* out, bool c128, hipStream_t stream, uint32_t* clear = nullptr,
                         int64_t n_clear = 0);
// Launches one bucket step; returns the kernel class used (QT_KCLASS_*)
// through *kclass.
hipError_t launch_step(const DevStep& s, bool c128, bool scaled, int* exps, uint32_t* maxbits,
                       int64_t n_elems, hipStream_t stream, int* n_launches, int* kclass);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t value, hipStream_t stream);
// gemm.hip: one fused GEMM bucket for all batch items (complex64, MFMA).
hipError_t launch_gemm(const DevGemm& g, bool scaled, int* exps, uint32_t* maxbits, hipStream_t stream);
// sum_mode 1 (a range of one slice) or 2 (one point, no open output, the
// whole range in this launch's single workgroup of 256): also the range's
// sums into `sums`, as launch_slice_sum would form them.
hipError_t launch_final(const DevFinal& f, const DevIn* factors, int n_points, int64_t n_items,
                        bool c128, bool scaled, const int* exps, const uint32_t* maxbits,
                        double* per_slice, int64_t slice_end, hipStream_t stream, double* sums = nullptr,
                        int sum_mode = 0);
hipError_t launch_lds_exec(const XLaunch& x, int64_t n_items, int waves, bool c128, bool scaled, int* exps,
                           uint32_t* maxbits, hipStream_t stream);
hipError_t launch_lds_multi(const XMulti& m, int n_items, size_t smem, int waves, bool c128, bool scaled,
                            hipStream_t stream);
// The gradient executor runs in complex128 (unscaled) for every precision.
hipError_t launch_lds_grad(const XMulti& m, int n_items, size_t smem, int waves, hipStream_t stream);
size_t lds_grad_smem_bytes(int n_slots, int n_recs, int lds_elems, bool c128);
// Bytes of global scratch per point of a program run from it.
int64_t multi_scratch_bytes(int n_slots, int n_recs, int area_elems, bool c128);
// out[r][q] = sum_i in[(r * n + i) * nq + q] in FP64, in order of i.
// With `weights` ([n], device), entry i counts weights[i] times.
hipError_t launch_rows_sum(const double* in, int rows, int n, int nq, double* out, hipStream_t stream,
                           const double* weights = nullptr);
hipError_t launch_amp_to_real(const double* amp, int64_t n, double* out, hipStream_t stream);
size_t lds_exec_smem_bytes(int n_slots, int lds_elems, bool c128);
hipError_t launch_slice_sum(const double* per_slice, int n_points, int64_t n_range, double* out,
                            hipStream_t stream, const double* weights = nullptr);

}  // namespace qt
