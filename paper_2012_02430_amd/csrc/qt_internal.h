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
  int32_t pad;
};

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
  int32_t pad;
  DevIn in[kMaxIn];
};

// ------------------------------------------------- LDS executor descriptors
// Operand (or output) of a step run by the LDS executor: in LDS when ptr is
// null (element offset lds_off inside the workgroup's tensor area), else in
// global memory at ptr + pt*pt_stride + sb*sb_stride + (pext(sid, smask) << slow).
constexpr int kXRuns = 8;   // executor steps have outputs of rank <= 16
// Work unit of the executor: steps of rank >= kXBigRank are cut into units
// of kXEpu * 64 outputs (kXEpu per lane), smaller steps into 64-output units.
// (complex128 uses kXEpu / 2 per lane and units of half the size).
constexpr int kXBigRank = 8;
constexpr int kXEpu = 4;
constexpr int kXMaxThreads = 512;
inline int64_t x_unit_elems(int rank, int elt) { return rank >= kXBigRank ? 64 * (elt == 8 ? kXEpu : kXEpu / 2) : 64; }
struct XIn {
  const void* ptr;
  int64_t pt_stride;
  int64_t sb_stride;
  uint32_t lds_off;
  uint32_t smask;
  int32_t slow;
  int32_t has_v;
  int32_t nruns;
  int32_t slot_kind;  // 0: unscaled; 1: LDS slot; 2: global slot
  int32_t slot;       // LDS slot index, or global slot base
  int32_t exp_pt;
  int32_t exp_sb;
  int32_t pad;
  uint8_t run_lo[kXRuns];
  uint8_t run_len[kXRuns];
  uint8_t run_dst[kXRuns];
};

struct XStep {
  XIn out;   // output location and scale slot (runs unused)
  int32_t r;
  int32_t sum;
  int32_t n_in;
  int32_t pad;
  XIn in[kMaxIn];
};

// One launch of the executor: every workgroup runs the same level schedule
// for its batch item (pt, sb).
struct XLaunch {
  const XStep* steps;
  const uint2* units;      // (step, 64-element chunk) work units, level by level
  const int32_t* level_off;  // n_levels + 1 offsets into units
  int32_t n_levels;
  int32_t lg_nsb;
  int64_t chunk_base;
  int32_t n_slots;         // LDS scale slots
  int32_t lds_elems;       // tensor area, elements
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
  qt_plan_info info{};
  // HIP-event profiling of launches (qt_profile_enable / qt_profile_read)
  struct Profile;
  std::unique_ptr<Profile> prof;
  struct Workspace;
  std::unique_ptr<Workspace> ws;
  qt_plan();
  ~qt_plan();
};

namespace qt {

// kernels.hip
hipError_t launch_leaves(const DevLeaf* leaves, int n_leaves, int leaf_block, const double* dense,
                         const double* params, int p, int n_points, void* out, bool c128,
                         hipStream_t stream);
// Launches one bucket step; returns the kernel class used (QT_KCLASS_*)
// through *kclass.
hipError_t launch_step(const DevStep& s, bool c128, bool scaled, int* exps, uint32_t* maxbits,
                       int64_t n_elems, hipStream_t stream, int* n_launches, int* kclass);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t value, hipStream_t stream);
hipError_t launch_final(const DevFinal& f, const DevIn* factors, int n_points, int64_t n_items,
                        bool c128, bool scaled, const int* exps, const uint32_t* maxbits,
                        double* per_slice, int64_t slice_end, hipStream_t stream);
hipError_t launch_lds_exec(const XLaunch& x, int64_t n_items, int waves, bool c128, bool scaled, int* exps,
                           uint32_t* maxbits, hipStream_t stream);
size_t lds_exec_smem_bytes(int n_slots, int lds_elems, bool c128);
hipError_t launch_slice_sum(const double* per_slice, int n_points, int64_t n_range, double* out,
                            hipStream_t stream);

}  // namespace qt
