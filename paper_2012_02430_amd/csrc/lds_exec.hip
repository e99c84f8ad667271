// LDS executor: one workgroup per batch item (point, slice) runs a segment
// of bucket steps whose tensors are small enough to live in its LDS.
//
// At the start the workgroup materialises its point's gate table and copies
// the segment's external inputs (results of earlier launches) into LDS; from
// then on every operand is read from LDS.  The steps are grouped into
// dependency levels (a step's level is one more than the deepest step of
// the segment that produced one of its inputs) and all steps of a level run
// concurrently: the level's work is cut into units of 64 x EPU outputs of
// one step, handed round-robin to the wavefronts, with one barrier between
// levels.  A unit is uniform over its wavefront, so its descriptor is read
// with scalar loads.  Each output element computes, like the streaming
// kernels,
//   out[x] = prod_{j} T_j[x, v=0] + prod_{j} T_j[x, v=1]
// (an input without the summed variable contributes the same value to both
// products), and is written to LDS or, when it leaves the segment, to
// global memory.
#include <hip/hip_runtime.h>

#include "qt_internal.h"

namespace qt {
namespace {

// Complex product with its fused multiply-adds written out, so that every
// executor variant (per point or point-batched, LDS or global scratch)
// rounds it the same way whatever the compiler would contract.
__device__ __forceinline__ float2 xmul(float2 a, float2 b) {
  return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 xmul(double2 a, double2 b) {
  return make_double2(__builtin_fma(a.x, b.x, -(a.y * b.y)), __builtin_fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 xadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 xadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 xscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 xscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

template <typename E> struct XReal;
template <> struct XReal<float2> { using R = float; };
template <> struct XReal<double2> { using R = double; };

template <typename E> struct XRaw;
template <> struct alignas(8) XRaw<float2> { float x, y; };
template <> struct alignas(16) XRaw<double2> { double x, y; };
// Global pointers typed in the global address space so that they are never
// merged with LDS pointers into generic (flat) accesses.
template <typename E>
using gconst_t = const __attribute__((address_space(1))) XRaw<E>*;
template <typename E>
using gmut_t = __attribute__((address_space(1))) XRaw<E>*;

template <int N>
__device__ __forceinline__ uint32_t xpext_all(uint32_t x, const uint8_t (&lo)[N], const uint8_t (&len)[N],
                                              const uint8_t (&dst)[N]) {
  // The byte tables are read as 32-bit words (each table is 4-byte aligned
  // and a multiple of 4 long): a byte-indexed read of a wavefront-uniform
  // table becomes a chain of vector byte loads, a word read at a constant
  // offset a scalar load.  Runs are packed from index 0; a word of four
  // empty runs ends the list, and an empty run inside a word contributes 0.
  static_assert(N % 4 == 0, "run tables are read as words");
  const uint32_t* const wl = reinterpret_cast<const uint32_t*>(lo);
  const uint32_t* const wn = reinterpret_cast<const uint32_t*>(len);
  const uint32_t* const wd = reinterpret_cast<const uint32_t*>(dst);
  uint32_t r = 0;
#pragma unroll
  for (int w = 0; w < N / 4; ++w) {
    const uint32_t nw = wn[w];
    if (nw == 0) break;
    const uint32_t lw = wl[w], dw = wd[w];
#pragma unroll
    for (int b = 0; b < 32; b += 8) {
      const uint32_t n = (nw >> b) & 0xffu;
      r |= ((x >> ((lw >> b) & 0xffu)) & ((1u << n) - 1u)) << ((dw >> b) & 0xffu);
    }
  }
  return r;
}

// pext of a lane index through the operand's lane runs (packed by the host:
// run i has source bit, length and destination bit in bits 9i..9i+8, the
// count in bits 27..28).
__device__ __forceinline__ uint32_t xpext_lane_word(uint32_t lane, uint32_t w) {
  const uint32_t k = w >> 27;
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if ((uint32_t)i >= k) break;
    const uint32_t f = w >> (9 * i);
    r |= ((lane >> (f & 7u)) & ((1u << ((f >> 3) & 7u)) - 1u)) << ((f >> 6) & 7u);
  }
  return r;
}

// pext of x through the runs held in words w (lo[0..1], len[2..3],
// dst[4..5]; kXRuns = 8), up to the first empty run.
__device__ __forceinline__ uint32_t xpext_words(uint32_t x, const uint32_t (&w)[6]) {
  static_assert(kXRuns == 8, "two words per table");
  uint32_t r = 0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int b = 0; b < 32; b += 8) {
      const uint32_t n = (w[2 + h] >> b) & 0xffu;
      if (n == 0) return r;
      r |= ((x >> ((w[h] >> b) & 0xffu)) & ((1u << n) - 1u)) << ((w[4 + h] >> b) & 0xffu);
    }
  }
  return r;
}

__device__ __forceinline__ uint32_t xpext_bits(uint64_t x, uint32_t m) {
  uint32_t r = 0;
  int o = 0;
  while (m) {
    const int b = __ffs(m) - 1;
    r |= (uint32_t)((x >> b) & 1u) << o;
    ++o;
    m &= m - 1;
  }
  return r;
}

// Max over the wavefront of non-negative values given as their float bits
// (their integer max): DPP steps inside each row of 16 lanes (swap of
// neighbours, of pairs, mirror of each half row, mirror of the row), then
// the four row maxima through readlane.  Exact; no LDS round trips.
__device__ __forceinline__ uint32_t xwave_max(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));  // row_mirror
  const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0), b = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
  const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 32), d = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
  return max(max(a, b), max(c, d));
}

// Power of two that brings max|x| into [0.5, 1), clamped so that 2^-shift is
// a normal float.
__device__ __forceinline__ int xshift(uint32_t maxbits) {
  // ilogb + 1 from the biased exponent field; a subnormal max (field 0)
  // lands on the lower clamp, as ilogb would, and an infinite one on the
  // upper
  if (maxbits == 0) return 0;
  const int s = (int)((maxbits >> 23) & 0xffu) - 126;
  return s > 127 ? 127 : s;
}
__device__ __forceinline__ float xpow2neg(int sh) { return __int_as_float((127 - sh) << 23); }

// Holds a wavefront-uniform value in a scalar register from this point on:
// the scalar loads it comes from complete here and are not scheduled among
// later LDS accesses.
__device__ __forceinline__ uint32_t xpin(uint32_t v) {
  asm volatile("" : "+s"(v));
  return v;
}
__device__ __forceinline__ int xpin(int v) {
  asm volatile("" : "+s"(v));
  return v;
}
__device__ __forceinline__ uint64_t xpin(uint64_t v) {
  asm volatile("" : "+s"(v));
  return v;
}
__device__ __forceinline__ int64_t xpin(int64_t v) {
  asm volatile("" : "+s"(v));
  return v;
}

// The output part of a step descriptor and its rank and sum flag, as the
// unit uses them (loaded with the operand fields, pinned with them).
struct XOutRegs {
  uint64_t ptr;
  int64_t pt_stride, sb_stride;
  uint32_t lds_off;
  int slot_kind, slot, exp_pt, exp_sb, r, sum;
  __device__ __forceinline__ void load(const XStep& st) {
    ptr = reinterpret_cast<uint64_t>(st.out.ptr);
    pt_stride = st.out.pt_stride;
    sb_stride = st.out.sb_stride;
    lds_off = st.out.lds_off;
    slot_kind = st.out.slot_kind;
    slot = st.out.slot;
    exp_pt = st.out.exp_pt;
    exp_sb = st.out.exp_sb;
    r = st.r;
    sum = st.sum;
  }
  __device__ __forceinline__ void pin() {
    ptr = xpin(ptr);
    pt_stride = xpin(pt_stride);
    sb_stride = xpin(sb_stride);
    lds_off = xpin(lds_off);
    slot_kind = xpin(slot_kind);
    slot = xpin(slot);
    exp_pt = xpin(exp_pt);
    exp_sb = xpin(exp_sb);
    r = xpin(r);
    sum = xpin(sum);
  }
};

struct XCtx {
  uint32_t pt, sb;
  uint64_t sid;
  uint32_t lane;
};

// The operands of a unit's outputs: element e of operand j at LDS index
// base + lp + ep (lp and ep shifted by has_v), and its v = 1 partner.
template <typename E, int NIN, int EPU>
__device__ __forceinline__ void x_load_ops(const E* __restrict__ lds, const uint32_t (&base)[NIN],
                                           const uint32_t (&lp)[NIN], const uint32_t (&ep)[NIN][EPU],
                                           const uint32_t (&hv)[NIN], E (&a0)[EPU][NIN], E (&a1)[EPU][NIN]) {
#pragma unroll
  for (int e = 0; e < EPU; ++e) {
#pragma unroll
    for (int j = 0; j < NIN; ++j) {
      const uint32_t i = base[j] + lp[j] + ep[j][e];
      a0[e][j] = lds[i];
      a1[e][j] = lds[i + hv[j]];
    }
  }
}

// The two elements of an operand at v = 0 and v = 1: adjacent (v is the
// lowest bit of every operand that holds it) and, at an even index, one
// aligned access.
template <typename E>
struct alignas(2 * sizeof(E)) XPair {
  E a, b;
};

// x_load_ops for a step whose every operand holds v at an even base (the
// host checks both): each pair in one read, which also spreads the lanes of
// a wavefront over all LDS banks where two reads at a stride of two
// elements would conflict.
template <typename E, int NIN, int EPU>
__device__ __forceinline__ void x_load_pairs(const E* __restrict__ lds, const uint32_t (&base)[NIN],
                                             const uint32_t (&lp)[NIN], const uint32_t (&ep)[NIN][EPU],
                                             E (&a0)[EPU][NIN], E (&a1)[EPU][NIN]) {
#pragma unroll
  for (int e = 0; e < EPU; ++e) {
#pragma unroll
    for (int j = 0; j < NIN; ++j) {
      const XPair<E> q = *reinterpret_cast<const XPair<E>*>(lds + base[j] + lp[j] + ep[j][e]);
      a0[e][j] = q.a;
      a1[e][j] = q.b;
    }
  }
}

// PRE: read the unit's descriptor words in one batch held in scalar
// registers, then its scale slots and operands (a few round trips per unit
// instead of one per field), else read each field where it is used (kernels
// short of registers).  FOLDED: the descriptor is the unit's own copy, with
// the chunk's part of each operand index already in lds_off.  PAIRS: the
// step is flagged out.pairs (every operand holds v at an even base), and
// each (v = 0, v = 1) pair is one aligned read.
template <typename E, bool SCALED, int NIN, int EPU, bool PRE = true, bool FOLDED = false, bool PAIRS = false>
__device__ __forceinline__ void x_unit(const XStep& st, uint32_t chunk, const XCtx& c, E* __restrict__ lds,
                                       uint32_t* __restrict__ smax, int* __restrict__ sexp, int* __restrict__ gexps,
                                       uint32_t* __restrict__ gmax) {
  using R = typename XReal<E>::R;
  const uint32_t cx = chunk * EPU * 64u;
  uint32_t base[NIN], lp[NIN];
  R sc[NIN];
  int eacc = 0;
  uint32_t hvv[NIN], epv[NIN][EPU];
  int slotv[NIN];  // scale slot per operand, -1: unscaled (its scale stays 1 and is not applied)
  XOutRegs ov;
  E a0[EPU][NIN], a1[EPU][NIN];
  if constexpr (PRE) {
    // Setup in phases so that each phase's loads issue together: every
    // descriptor word the unit uses (one batch of scalar loads, held in
    // scalar registers: a wait on a scalar load also drains the LDS accesses
    // in flight, so none may fall between the operand loads), then the
    // scale slots (read even for an unscaled operand, at slot 0, and
    // ignored), then the index maps.
    uint32_t smk[NIN];
    int slw[NIN], slot[NIN];
#pragma unroll
    for (int j = 0; j < NIN; ++j) {
      base[j] = st.in[j].lds_off;
      smk[j] = st.in[j].smask;
      slw[j] = st.in[j].slow;
      slot[j] = st.in[j].slot;
      hvv[j] = (uint32_t)st.in[j].has_v;
#pragma unroll
      for (int e = 0; e < EPU; ++e) epv[j][e] = st.in[j].ep[e];
    }
    ov.load(st);
    uint32_t lw[NIN];
#pragma unroll
    for (int j = 0; j < NIN; ++j) lw[j] = st.in[j].lane_runs;
    if constexpr (!FOLDED) {
      if (chunk != 0) {
        uint32_t rw[NIN][6];
#pragma unroll
        for (int j = 0; j < NIN; ++j) {
          const uint32_t* const w = reinterpret_cast<const uint32_t*>(st.in[j].run_lo);
#pragma unroll
          for (int q = 0; q < 6; ++q) rw[j][q] = w[q];
        }
#pragma unroll
        for (int j = 0; j < NIN; ++j) lw[j] = xpin(lw[j]);
#pragma unroll
        for (int j = 0; j < NIN; ++j) base[j] += xpext_words(cx, rw[j]) << hvv[j];
      }
    }
#pragma unroll
    for (int j = 0; j < NIN; ++j) {
      base[j] = xpin(base[j]);
      smk[j] = xpin(smk[j]);
      slw[j] = xpin(slw[j]);
      slot[j] = xpin(slot[j]);
      hvv[j] = xpin(hvv[j]);
      lw[j] = xpin(lw[j]);
#pragma unroll
      for (int e = 0; e < EPU; ++e) epv[j][e] = xpin(epv[j][e]);
    }
    ov.pin();
    uint32_t mbits[NIN];
    int mexp[NIN];
    if (SCALED) {
#pragma unroll
      for (int j = 0; j < NIN; ++j) {
        const int q = slot[j] >= 0 ? slot[j] : 0;
        mbits[j] = smax[q];
        mexp[j] = sexp[q];
      }
    }
#pragma unroll
    for (int j = 0; j < NIN; ++j) slotv[j] = slot[j];
    // the lane part from the packed lane runs (the chunk part, unless
    // folded into lds_off, was added to base above: past the first chunk,
    // whose part is zero, from the run tables as words, 6 per operand: lo,
    // len, dst for runs 0-3 and 4-7)
#pragma unroll
    for (int j = 0; j < NIN; ++j) lp[j] = xpext_lane_word(c.lane, lw[j]);
#pragma unroll
    for (int j = 0; j < NIN; ++j)
      if (smk[j]) base[j] += xpext_bits(c.sid, smk[j]) << slw[j];
    // the operand loads issue before the scale slots are waited for; the
    // slots (the same in every lane) are then decoded on the scalar unit
    if constexpr (PAIRS) x_load_pairs<E, NIN, EPU>(lds, base, lp, epv, a0, a1);
    else x_load_ops<E, NIN, EPU>(lds, base, lp, epv, hvv, a0, a1);
#pragma unroll
    for (int j = 0; j < NIN; ++j) {
      sc[j] = (R)1;
      if (SCALED && slot[j] >= 0) {
        const int sh = xshift((uint32_t)__builtin_amdgcn_readfirstlane((int)mbits[j]));
        sc[j] = (R)xpow2neg(sh);
        eacc += __builtin_amdgcn_readfirstlane(mexp[j]) + sh;
      }
    }
  } else {
    ov.load(st);
#pragma unroll
    for (int j = 0; j < NIN; ++j) {
      const XOp& in = st.in[j];
      hvv[j] = (uint32_t)in.has_v;
#pragma unroll
      for (int e = 0; e < EPU; ++e) epv[j][e] = in.ep[e];
      base[j] = in.lds_off + (xpext_bits(c.sid, in.smask) << in.slow);
      lp[j] = xpext_lane_word(c.lane, in.lane_runs);
      if (chunk != 0) lp[j] += xpext_all(cx, in.run_lo, in.run_len, in.run_dst) << in.has_v;
      slotv[j] = in.slot;
      sc[j] = (R)1;
      if (SCALED && in.slot >= 0) {
        const int sh = xshift(smax[in.slot]);
        sc[j] = (R)xpow2neg(sh);
        eacc += sexp[in.slot] + sh;
      }
    }
    x_load_ops<E, NIN, EPU>(lds, base, lp, epv, hvv, a0, a1);
  }
  const uint32_t n = 1u << ov.r;
  float m = 0.f;
  E res[EPU];
  // the product over operands in their order, each scaled operand times
  // its power of two first (an unscaled one is used as loaded)
  E t0[EPU], t1[EPU];
#pragma unroll
  for (int j = 0; j < NIN; ++j) {
    if (SCALED && slotv[j] >= 0) {
#pragma unroll
      for (int e = 0; e < EPU; ++e) {
        a0[e][j] = xscale(a0[e][j], sc[j]);
        a1[e][j] = xscale(a1[e][j], sc[j]);
      }
    }
#pragma unroll
    for (int e = 0; e < EPU; ++e) {
      t0[e] = j == 0 ? a0[e][0] : xmul(t0[e], a0[e][j]);
      t1[e] = j == 0 ? a1[e][0] : xmul(t1[e], a1[e][j]);
    }
  }
#pragma unroll
  for (int e = 0; e < EPU; ++e) {
    res[e] = ov.sum ? xadd(t0[e], t1[e]) : t0[e];
    const uint32_t x = cx + e * 64u + c.lane;
    if (SCALED && x < n) m = fmaxf(m, fmaxf(fabsf((float)res[e].x), fabsf((float)res[e].y)));
  }
  if (ov.ptr == 0) {
#pragma unroll
    for (int e = 0; e < EPU; ++e) {
      const uint32_t x = cx + e * 64u + c.lane;
      if (x < n) lds[ov.lds_off + x] = res[e];
    }
  } else {
    gmut_t<E> g = (gmut_t<E>)(reinterpret_cast<E*>(ov.ptr) + (int64_t)c.pt * ov.pt_stride +
                              (int64_t)c.sb * ov.sb_stride);
#pragma unroll
    for (int e = 0; e < EPU; ++e) {
      const uint32_t x = cx + e * 64u + c.lane;
      if (x < n) {
        g[x].x = res[e].x;
        g[x].y = res[e].y;
      }
    }
  }
  if (SCALED && ov.slot_kind != 0) {
    const uint32_t mw = xwave_max(__float_as_uint(m));
    if (c.lane == 0) {
      if (ov.slot_kind == 1) {
        atomicMax(smax + ov.slot, mw);
        if (chunk == 0) sexp[ov.slot] = eacc;
      } else {
        const int g = ov.slot + (int)c.pt * ov.exp_pt + (int)c.sb * ov.exp_sb;
        atomicMax(gmax + g, mw);
        if (chunk == 0) gexps[g] = eacc;
      }
    }
  }
}

// Gate table entry t of the workgroup's point (layout: x_gate_off), FP64
// trigonometry rounded to the element type (Section III-A conventions).
template <typename E>
__device__ __forceinline__ E x_gate2(int t, const double* gam, const double* bet) {
  using R = typename XReal<E>::R;
  E v;
  double re = 0.0, im = 0.0;
  if (t < 10) {
    const int a = t >> 1, i = t & 1;  // |+>, <0|, <1|, observable (two pairs)
    if (a == 0) re = 1.0;
    else if (a == 1) re = i == 0 ? 1.0 : 0.0;
    else if (a == 2) re = i == 0 ? 0.0 : 1.0;
    else if (a == 3) re = i == 0 ? 0.0 : 1.0;
    else re = i == 0 ? 1.0 : 0.0;
  } else {
    const int u = t - 10, k = u >> 4, g = (u >> 2) & 3, i = u & 3;
    double sn, cs;
    const bool diag = i == 0 || i == 3;
    if (g < 2) {
      sincos(gam[k], &sn, &cs);
      re = diag ? 1.0 : cs;
      im = diag ? 0.0 : (g == 0 ? -sn : sn);
    } else {
      sincos(bet[k], &sn, &cs);
      re = diag ? cs : 0.0;
      im = diag ? 0.0 : (g == 2 ? -sn : sn);
    }
  }
  v.x = (R)re;
  v.y = (R)im;
  return v;
}
template <typename E>
__device__ __forceinline__ E x_gate(int t, const double* prm, int p) {
  return x_gate2<E>(t, prm, prm + p);
}

// The step, unit, level and copy tables are separate read-only, non-aliasing
// arguments so that their (wavefront-uniform) reads become scalar loads.
template <typename E, bool SCALED>
__global__ __launch_bounds__(kXMaxThreads) void k_lds_exec(const XLaunch X, const XStep* __restrict__ steps,
                                                           const uint2* __restrict__ units,
                                                           const int32_t* __restrict__ level_off,
                                                           const XCopy* __restrict__ copies,
                                                           int* __restrict__ gexps, uint32_t* __restrict__ gmax,
                                                           uint64_t* __restrict__ trace) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int slots16 = (X.n_slots + 3) & ~3;
  uint32_t* smax = reinterpret_cast<uint32_t*>(smem);
  int* sexp = reinterpret_cast<int*>(smem + 4 * slots16);
  E* lds = reinterpret_cast<E*>(smem + 8 * slots16);

  XCtx c;
  const uint32_t item = blockIdx.x;
  c.sb = item & ((1u << X.lg_nsb) - 1u);
  c.pt = item >> X.lg_nsb;
  c.sid = (uint64_t)X.chunk_base + c.sb;
  const int tid = threadIdx.x;
  c.lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nw = blockDim.x >> 6;

  for (int i = tid; i < X.n_slots; i += blockDim.x) {
    smax[i] = 0u;
    sexp[i] = 0;
  }
  if (tid < 2) {
    lds[tid].x = 1;
    lds[tid].y = 0;
  }
  for (int t = tid; t < x_gate_elems(X.p); t += blockDim.x)
    lds[kXGate + t] = x_gate2<E>(t, X.gam + (int64_t)c.pt * X.pstride, X.bet + (int64_t)c.pt * X.pstride);
  // stage the segment's external inputs (with their scale slots)
  for (int e = wave; e < X.n_copies; e += nw) {
    const XCopy& cp = copies[e];
    gconst_t<E> src = (gconst_t<E>)(reinterpret_cast<const E*>(cp.ptr) + (int64_t)c.pt * cp.pt_stride +
                                     (int64_t)c.sb * cp.sb_stride + ((int64_t)xpext_bits(c.sid, cp.smask) << cp.slow));
    for (uint32_t i0 = 0; i0 < cp.n; i0 += 256) {
      E v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t i = i0 + q * 64 + c.lane;
        if (i < cp.n) {
          v[q].x = src[i].x;
          v[q].y = src[i].y;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t i = i0 + q * 64 + c.lane;
        if (i < cp.n) lds[cp.lds_off + i] = v[q];
      }
    }
    if (SCALED && c.lane == 0 && cp.gslot >= 0) {
      const int g = cp.gslot + (int)c.pt * cp.exp_pt + (int)c.sb * cp.exp_sb;
      smax[cp.lslot] = gmax[g];
      sexp[cp.lslot] = gexps[g];
    }
  }
  __syncthreads();

  constexpr int kBig = sizeof(E) == 8 ? kXEpu : kXEpu / 2;
  const bool tracing = trace != nullptr && blockIdx.x == 0 && tid == 0;
  if (tracing) trace[0] = wall_clock64();
  for (int L = 0; L < X.n_levels; ++L) {
    const int u_beg = level_off[L];
    const int u_end = level_off[L + 1];
    for (int u = u_beg + wave; u < u_end; u += nw) {
      const XStep& st = steps[u];
      const uint32_t chunk = (uint32_t)st.chunk;
      const bool big = st.r >= kXBigRank;
      constexpr int kHalf = kBig > 1 ? kBig / 2 : 1;
      if (st.out.pairs != 0 && st.n_in <= 5) {
        // exact operand counts, pairs read as one access
        switch (st.n_in) {
          case 1:
          case 2:
            if (big) x_unit<E, SCALED, 2, kBig, true, true, true>(st, chunk, c, lds, smax, sexp, gexps, gmax);
            else x_unit<E, SCALED, 2, 1, true, true, true>(st, chunk, c, lds, smax, sexp, gexps, gmax);
            break;
          case 3:
            if (big) x_unit<E, SCALED, 3, kBig, true, true, true>(st, chunk, c, lds, smax, sexp, gexps, gmax);
            else x_unit<E, SCALED, 3, 1, true, true, true>(st, chunk, c, lds, smax, sexp, gexps, gmax);
            break;
          case 4:
            if (big) x_unit<E, SCALED, 4, kBig, true, true, true>(st, chunk, c, lds, smax, sexp, gexps, gmax);
            else x_unit<E, SCALED, 4, 1, true, true, true>(st, chunk, c, lds, smax, sexp, gexps, gmax);
            break;
          default:
            if (big) x_unit<E, SCALED, 5, kHalf, true, true, true>(st, chunk, c, lds, smax, sexp, gexps, gmax);
            else x_unit<E, SCALED, 5, 1, true, true, true>(st, chunk, c, lds, smax, sexp, gexps, gmax);
            break;
        }
      } else if (st.n_in <= 2) {
        if (big) x_unit<E, SCALED, 2, kBig, true, true>(st, chunk, c, lds, smax, sexp, gexps, gmax);
        else x_unit<E, SCALED, 2, 1, true, true>(st, chunk, c, lds, smax, sexp, gexps, gmax);
      } else if (st.n_in <= 4) {
        if (big) x_unit<E, SCALED, 4, kBig, true, true>(st, chunk, c, lds, smax, sexp, gexps, gmax);
        else x_unit<E, SCALED, 4, 1, true, true>(st, chunk, c, lds, smax, sexp, gexps, gmax);
      } else {
        if (big) x_unit<E, SCALED, 8, (kBig > 1 ? kBig / 2 : 1), true, true>(st, chunk, c, lds, smax, sexp, gexps, gmax);
        else x_unit<E, SCALED, 8, 1, true, true>(st, chunk, c, lds, smax, sexp, gexps, gmax);
      }
    }
    // Wavefronts without a unit in this level touch the next level's unit
    // descriptors (one word per 64-byte line) while the others work, so the
    // next level starts on scalar-cache hits.  Only idle wavefronts wait on
    // these loads; the busy ones never issue them.
    const int n_busy = u_end - u_beg < nw ? u_end - u_beg : nw;
    if (wave >= n_busy && L + 1 < X.n_levels) {
      // the next level's descriptors are consecutive: its lines go round
      // the idle wavefronts, four loads in flight per wavefront (indices
      // clamped to the last line rather than branched on)
      const int nb = level_off[L + 1];
      const int ne = level_off[L + 2] < nb + nw ? level_off[L + 2] : nb + nw;
      constexpr int kLines = (int)(sizeof(XStep) / 64);
      const int idle = nw - n_busy, nl = (ne - nb) * kLines;
      const uint32_t* d = reinterpret_cast<const uint32_t*>(steps + nb);
      for (int k = wave - n_busy; k < nl; k += 4 * idle) {
        const uint32_t w0 = d[16 * k];
        const uint32_t w1 = d[16 * min(k + idle, nl - 1)];
        const uint32_t w2 = d[16 * min(k + 2 * idle, nl - 1)];
        const uint32_t w3 = d[16 * min(k + 3 * idle, nl - 1)];
        asm volatile("" : : "s"(w0), "s"(w1), "s"(w2), "s"(w3));  // keeps the loads; emits nothing
      }
    }
    __syncthreads();
    if (tracing) trace[L + 1] = wall_clock64();
  }
}

}  // namespace

size_t lds_exec_smem_bytes(int n_slots, int lds_elems, bool c128) {
  const size_t slots16 = (size_t)((n_slots + 3) & ~3);
  return 8 * slots16 + (size_t)lds_elems * (c128 ? 16 : 8);
}

hipError_t launch_lds_exec(const XLaunch& x, int64_t n_items, int waves, bool c128, bool scaled, int* exps,
                           uint32_t* maxbits, hipStream_t stream) {
  if (n_items == 0 || x.n_levels == 0) return hipSuccess;
  const size_t smem = lds_exec_smem_bytes(x.n_slots, x.lds_elems, c128);
  const dim3 grid((unsigned)n_items), block((unsigned)(64 * waves));
  const void* fn = c128 ? reinterpret_cast<const void*>(&k_lds_exec<double2, false>)
                        : (scaled ? reinterpret_cast<const void*>(&k_lds_exec<float2, true>)
                                  : reinterpret_cast<const void*>(&k_lds_exec<float2, false>));
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  if (c128)
    hipLaunchKernelGGL((k_lds_exec<double2, false>), grid, block, smem, stream, x, x.steps, x.units, x.level_off,
                       x.copies, exps, maxbits, x.trace);
  else if (scaled)
    hipLaunchKernelGGL((k_lds_exec<float2, true>), grid, block, smem, stream, x, x.steps, x.units, x.level_off,
                       x.copies, exps, maxbits, x.trace);
  else
    hipLaunchKernelGGL((k_lds_exec<float2, false>), grid, block, smem, stream, x, x.steps, x.units, x.level_off,
                       x.copies, exps, maxbits, x.trace);
  return hipGetLastError();
}

}  // namespace qt

namespace qt {
namespace {

// Synchronisation between levels.  The barrier's workgroup-scope release
// and acquire order global as well as LDS accesses, and the wavefronts of a
// workgroup run on one compute unit and share its vector L1, so an item in
// global scratch needs no device-scope fence (whose L2 write-back would be
// paid at every level).
template <bool GLOBAL>
__device__ __forceinline__ void x_level_sync() {
  __syncthreads();
}

// Byte layout of a program's global scratch per point: element area, then
// the scale slots (max bits, then exponents), then the gradient records.
struct XArea {
  int64_t elem_bytes, slot_bytes, rec_bytes;
};
__host__ __device__ inline XArea x_area(int n_slots, int n_recs, int area_elems, int elt) {
  XArea a;
  a.elem_bytes = ((int64_t)area_elems * elt + 15) & ~(int64_t)15;
  a.slot_bytes = 4 * (int64_t)((n_slots + 3) & ~3);
  a.rec_bytes = 8 * (int64_t)((n_recs + 1) & ~1);
  return a;
}

// One (program, point) item of the multi-program executor: the point's gate
// table, the program's levels, then its value in an FP64 epilogue (the
// product of the closing scalars with the accumulated exponent).  `area`
// is the item's element area (LDS, or global scratch with GLOBAL).
template <typename E, bool SCALED, bool GLOBAL>
__device__ __forceinline__ void x_multi_item(const XMulti& M, const XProg& P, int prog_id,
                                             const XStep* __restrict__ psteps, const uint2* __restrict__ punits,
                                             const int32_t* __restrict__ plev, const XFinal* __restrict__ finals,
                                             const XCtx& c, int tid, int wave, int nw, E* area, uint32_t* smax,
                                             int* sexp) {
  for (int i = tid; i < P.n_slots; i += blockDim.x) {
    smax[i] = 0u;
    sexp[i] = 0;
  }
  if (tid < 2) {
    area[tid].x = 1;
    area[tid].y = 0;
  }
  for (int t = tid; t < x_gate_elems(M.p); t += blockDim.x)
    area[kXGate + t] = x_gate2<E>(t, M.gam + (int64_t)c.pt * M.pstride, M.bet + (int64_t)c.pt * M.pstride);
  x_level_sync<GLOBAL>();
  constexpr int kBig = sizeof(E) == 8 ? kXEpu : kXEpu / 2;
  for (int L = 0; L < P.n_levels; ++L) {
    const int u_end = plev[L + 1];
    for (int u = plev[L] + wave; u < u_end; u += nw) {
      const uint2 un = punits[u];
      const XStep& st = psteps[un.x];
      const bool big = st.r >= kXBigRank;
      if (st.n_in <= 2) {
        if (big) x_unit<E, SCALED, 2, kBig>(st, un.y, c, area, smax, sexp, nullptr, nullptr);
        else x_unit<E, SCALED, 2, 1>(st, un.y, c, area, smax, sexp, nullptr, nullptr);
      } else if (st.n_in <= 4) {
        if (big) x_unit<E, SCALED, 4, kBig>(st, un.y, c, area, smax, sexp, nullptr, nullptr);
        else x_unit<E, SCALED, 4, 1>(st, un.y, c, area, smax, sexp, nullptr, nullptr);
      } else {
        if (big) x_unit<E, SCALED, 8, (kBig > 1 ? kBig / 2 : 1)>(st, un.y, c, area, smax, sexp, nullptr, nullptr);
        else x_unit<E, SCALED, 8, 1>(st, un.y, c, area, smax, sexp, nullptr, nullptr);
      }
    }
    x_level_sync<GLOBAL>();
  }
  if (tid == 0) {
    double re = 1.0, im = 0.0, ex = P.log2_const;
    for (int f = 0; f < P.n_finals; ++f) {
      const XFinal& F = finals[P.finals_off + f];
      const E a = area[F.lds_off];
      const double ar = (double)a.x, ai = (double)a.y;
      if (SCALED && F.slot >= 0) ex += sexp[F.slot];
      const double nr = re * ar - im * ai;
      im = re * ai + im * ar;
      re = nr;
    }
    double* o = M.out + 3 * ((int64_t)c.pt * M.n_progs + prog_id);
    o[0] = re;
    o[1] = im;
    o[2] = ex;
  }
}

// Max of non-negative values (float bits) over each aligned group of 2^lg
// lanes (lg <= 5): DPP steps inside rows of 16 lanes (swap of neighbours, of
// pairs, mirror of each half row, mirror of the row), then one lane
// exchange across the two rows of a 32-lane group.  Every lane of a group
// ends with the group's max.
__device__ __forceinline__ uint32_t xseg_max(uint32_t v, int lg) {
  if (lg >= 1) v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
  if (lg >= 2) v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
  if (lg >= 3) v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
  if (lg >= 4) v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
  if (lg >= 5) v = max(v, (uint32_t)__shfl_xor((int)v, 16));
  return v;
}

// A unit of a point-batched lightcone program.  The workgroup holds the
// tensors of `npts` points of one program, point q's area at element q *
// stride and its scale slots at q * S.  A step with fewer than 64 outputs
// is packed: its unit covers 64 / 2^r points, lane = (point, output); a
// larger step's unit covers 64 x EPU outputs of one point (uy = point x
// chunks + chunk), as in the per-point executor.  Operands and the output
// are in LDS; the output's scale slot belongs to the step alone, so a
// packed unit stores its point's max and exponent directly.
template <typename E, bool SCALED, int NIN, int EPU>
__device__ __forceinline__ void x_unit_pts(const XStep& st, uint32_t uy, uint32_t lane, uint32_t npts, uint32_t stride,
                                           uint32_t S, E* __restrict__ lds, uint32_t* __restrict__ smax,
                                           int* __restrict__ sexp) {
  using R = typename XReal<E>::R;
  // every descriptor word first, in one batch of scalar loads held in
  // scalar registers (a wait on a scalar load drains the LDS accesses in
  // flight, so none may fall between the operand loads)
  uint32_t base[NIN], lw[NIN], hvv[NIN], epv[NIN][EPU];
  int slot[NIN];
#pragma unroll
  for (int j = 0; j < NIN; ++j) {
    base[j] = st.in[j].lds_off;
    slot[j] = st.in[j].slot;
    lw[j] = st.in[j].lane_runs;
    hvv[j] = (uint32_t)st.in[j].has_v;
#pragma unroll
    for (int e = 0; e < EPU; ++e) epv[j][e] = st.in[j].ep[e];
  }
  const int r = xpin(st.r);
  const int sum = xpin(st.sum);
  const uint32_t o_off = xpin(st.out.lds_off);
  const int o_slot = xpin(st.out.slot);
#pragma unroll
  for (int j = 0; j < NIN; ++j) {
    base[j] = xpin(base[j]);
    slot[j] = xpin(slot[j]);
    lw[j] = xpin(lw[j]);
    hvv[j] = xpin(hvv[j]);
#pragma unroll
    for (int e = 0; e < EPU; ++e) epv[j][e] = xpin(epv[j][e]);
  }
  const uint32_t n = 1u << r;
  const bool packed = r < 6;
  uint32_t q, xl, chunk = 0;
  if (packed) {
    q = (uy << (6 - r)) + (lane >> r);
    xl = lane & (n - 1u);
  } else {
    constexpr int lg_epu = EPU == 4 ? 2 : (EPU == 2 ? 1 : 0);
    const int lgc = r - 6 - lg_epu;
    chunk = uy & ((1u << lgc) - 1u);
    q = uy >> lgc;
    xl = lane;
  }
  const bool valid = q < npts;
  const uint32_t qq = valid ? q : 0u;
  const uint32_t qoff = qq * stride, soff = qq * S;
  const uint32_t cx = chunk * EPU * 64u;
  uint32_t lp[NIN];
  R sc[NIN];
  int eacc = 0;
#pragma unroll
  for (int j = 0; j < NIN; ++j) base[j] += qoff;
  uint32_t mbits[NIN];
  int mexp[NIN];
  if (SCALED) {
#pragma unroll
    for (int j = 0; j < NIN; ++j) {
      const uint32_t s = soff + (uint32_t)(slot[j] >= 0 ? slot[j] : 0);
      mbits[j] = smax[s];
      mexp[j] = sexp[s];
    }
  }
#pragma unroll
  for (int j = 0; j < NIN; ++j) lp[j] = xpext_lane_word(xl, lw[j]);
  if (chunk != 0) {
    // past the first chunk (wavefront-uniform): the run tables as words
    uint32_t rw[NIN][6];
#pragma unroll
    for (int j = 0; j < NIN; ++j) {
      const uint32_t* const w = reinterpret_cast<const uint32_t*>(st.in[j].run_lo);
#pragma unroll
      for (int k = 0; k < 6; ++k) rw[j][k] = w[k];
    }
#pragma unroll
    for (int j = 0; j < NIN; ++j) lp[j] += xpext_words(cx, rw[j]) << hvv[j];
  }
  E a0[EPU][NIN], a1[EPU][NIN];
  x_load_ops<E, NIN, EPU>(lds, base, lp, epv, hvv, a0, a1);
#pragma unroll
  for (int j = 0; j < NIN; ++j) {
    sc[j] = (R)1;
    if (SCALED && slot[j] >= 0) {
      const int sh = xshift(mbits[j]);
      sc[j] = (R)xpow2neg(sh);
      eacc += mexp[j] + sh;
    }
  }
  float m = 0.f;
  // the product over operands in their order, each scaled operand times its
  // power of two first (an unscaled one is used as loaded)
  E t0[EPU], t1[EPU];
#pragma unroll
  for (int j = 0; j < NIN; ++j) {
    if (SCALED && slot[j] >= 0) {
#pragma unroll
      for (int e = 0; e < EPU; ++e) {
        a0[e][j] = xscale(a0[e][j], sc[j]);
        a1[e][j] = xscale(a1[e][j], sc[j]);
      }
    }
#pragma unroll
    for (int e = 0; e < EPU; ++e) {
      t0[e] = j == 0 ? a0[e][0] : xmul(t0[e], a0[e][j]);
      t1[e] = j == 0 ? a1[e][0] : xmul(t1[e], a1[e][j]);
    }
  }
#pragma unroll
  for (int e = 0; e < EPU; ++e) {
    const E res = sum ? xadd(t0[e], t1[e]) : t0[e];
    const uint32_t x = cx + e * 64u + xl;
    if (valid && x < n) {
      lds[qoff + o_off + x] = res;
      if (SCALED) m = fmaxf(m, fmaxf(fabsf((float)res.x), fabsf((float)res.y)));
    }
  }
  if (SCALED) {
    if (packed) {
      const uint32_t mw = xseg_max(__float_as_uint(m), r);
      if (valid && xl == 0u) {
        smax[soff + o_slot] = mw;
        sexp[soff + o_slot] = eacc;
      }
    } else {
      const uint32_t mw = xwave_max(__float_as_uint(m));
      if (lane == 0u && valid) {
        atomicMax(smax + soff + o_slot, mw);
        if (chunk == 0) sexp[soff + o_slot] = eacc;
      }
    }
  }
}

// x_unit_pts on the step's exact input count (no identity operands read or
// multiplied); outputs per lane as the host's units assume: kBig for big
// steps of up to four inputs, half that above four, one for small steps.
template <typename E, bool SCALED, int kBig>
__device__ __forceinline__ void x_unit_pts_any(const XStep& st, uint32_t uy, uint32_t lane, uint32_t npts,
                                               uint32_t stride, uint32_t S, E* __restrict__ lds,
                                               uint32_t* __restrict__ smax, int* __restrict__ sexp) {
  constexpr int kHalf = kBig > 1 ? kBig / 2 : 1;
  const bool big = st.r >= kXBigRank;
  switch (st.n_in) {
    case 1:
    case 2:
      if (big) x_unit_pts<E, SCALED, 2, kBig>(st, uy, lane, npts, stride, S, lds, smax, sexp);
      else x_unit_pts<E, SCALED, 2, 1>(st, uy, lane, npts, stride, S, lds, smax, sexp);
      break;
    case 3:
      if (big) x_unit_pts<E, SCALED, 3, kBig>(st, uy, lane, npts, stride, S, lds, smax, sexp);
      else x_unit_pts<E, SCALED, 3, 1>(st, uy, lane, npts, stride, S, lds, smax, sexp);
      break;
    case 4:
      if (big) x_unit_pts<E, SCALED, 4, kBig>(st, uy, lane, npts, stride, S, lds, smax, sexp);
      else x_unit_pts<E, SCALED, 4, 1>(st, uy, lane, npts, stride, S, lds, smax, sexp);
      break;
    case 5:
      if (big) x_unit_pts<E, SCALED, 5, kHalf>(st, uy, lane, npts, stride, S, lds, smax, sexp);
      else x_unit_pts<E, SCALED, 5, 1>(st, uy, lane, npts, stride, S, lds, smax, sexp);
      break;
    default:
      if (big) x_unit_pts<E, SCALED, 8, kHalf>(st, uy, lane, npts, stride, S, lds, smax, sexp);
      else x_unit_pts<E, SCALED, 8, 1>(st, uy, lane, npts, stride, S, lds, smax, sexp);
      break;
  }
}

// One point-batched item of the multi-program executor: up to P.n_pts
// points (from pt0) of one program in the workgroup's LDS.
template <typename E, bool SCALED>
__device__ __forceinline__ void x_multi_pts(const XMulti& M, const XProg& P, int prog_id, uint32_t pt0,
                                            const XStep* __restrict__ psteps, const uint2* __restrict__ punits,
                                            const int32_t* __restrict__ plev, const XFinal* __restrict__ finals,
                                            int tid, int wave, int nw, unsigned char* smem) {
  const uint32_t np = (uint32_t)P.n_pts;
  const uint32_t npts = min(np, (uint32_t)M.n_points - pt0);
  const uint32_t S = (uint32_t)P.slot_stride, stride = (uint32_t)P.pt_stride;
  uint32_t* smax = reinterpret_cast<uint32_t*>(smem);
  int* sexp = reinterpret_cast<int*>(smem + 4 * np * S);
  E* lds = reinterpret_cast<E*>(smem + 8 * np * S);
  for (uint32_t i = tid; i < np * S; i += blockDim.x) {
    smax[i] = 0u;
    sexp[i] = 0;
  }
  const uint32_t ge = (uint32_t)x_gate_elems(M.p);
  for (uint32_t i = tid; i < np * (ge + kXGate); i += blockDim.x) {
    const uint32_t q = i / (ge + kXGate), t = i - q * (ge + kXGate);
    E v;
    if (t < (uint32_t)kXGate) {
      v.x = 1;
      v.y = 0;
    } else {
      const uint32_t pq = pt0 + min(q, npts - 1u);
      v = x_gate2<E>((int)(t - kXGate), M.gam + (int64_t)pq * M.pstride, M.bet + (int64_t)pq * M.pstride);
    }
    lds[q * stride + t] = v;
  }
  __syncthreads();
  constexpr int kBig = sizeof(E) == 8 ? kXEpu : kXEpu / 2;
  const uint32_t lane = tid & 63;
  for (int L = 0; L < P.n_levels; ++L) {
    const int u_end = plev[L + 1];
    for (int u = plev[L] + wave; u < u_end; u += nw) {
      const uint2 un = punits[u];
      const XStep& st = psteps[un.x];
      x_unit_pts_any<E, SCALED, kBig>(st, un.y, lane, npts, stride, S, lds, smax, sexp);
    }
    __syncthreads();
  }
  for (uint32_t q = tid; q < npts; q += blockDim.x) {
    double re = 1.0, im = 0.0, ex = P.log2_const;
    for (int f = 0; f < P.n_finals; ++f) {
      const XFinal& F = finals[P.finals_off + f];
      const E a = lds[q * stride + F.lds_off];
      const double ar = (double)a.x, ai = (double)a.y;
      if (SCALED && F.slot >= 0) ex += sexp[q * S + F.slot];
      const double nr = re * ar - im * ai;
      im = re * ai + im * ar;
      re = nr;
    }
    double* o = M.out + 3 * ((int64_t)(pt0 + q) * M.n_progs + prog_id);
    o[0] = re;
    o[1] = im;
    o[2] = ex;
  }
}

// Multi-program executor: one workgroup per item runs a whole network (a
// per-edge lightcone) -- every edge and point of an energy evaluation in one
// launch.  An item is a group of points of one program whose tensors, for
// all of them, fit the launch's LDS: the points share the descriptor loads
// and the barriers of the level chain, and the small steps fill the lanes
// with several points.  A program too large for that runs one point per
// item from its own global scratch area.
template <typename E, bool SCALED>
__global__ __launch_bounds__(kXMaxThreads) void k_lds_multi(const XMulti M, const XProg* __restrict__ progs,
                                                            const XStep* __restrict__ steps,
                                                            const uint2* __restrict__ units,
                                                            const int32_t* __restrict__ level_off,
                                                            const XFinal* __restrict__ finals,
                                                            const int2* __restrict__ items) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int2 it = items[blockIdx.x];
  const int prog_id = it.x;
  const XProg& P = progs[prog_id];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nw = blockDim.x >> 6;
  const XStep* psteps = steps + P.steps_off;
  const uint2* punits = units + P.units_off;
  const int32_t* plev = level_off + P.levels_off;
  if (P.scratch_off >= 0) {
    XCtx c;
    c.pt = (uint32_t)it.y;
    c.sb = 0;
    c.sid = 0;
    c.lane = tid & 63;
    const XArea a = x_area(P.n_slots, 0, P.area_elems, (int)sizeof(E));
    char* base = M.scratch + P.scratch_off + (int64_t)c.pt * P.scratch_stride;
    x_multi_item<E, SCALED, true>(M, P, prog_id, psteps, punits, plev, finals, c, tid, wave, nw,
                                  reinterpret_cast<E*>(base), reinterpret_cast<uint32_t*>(base + a.elem_bytes),
                                  reinterpret_cast<int*>(base + a.elem_bytes + a.slot_bytes));
  } else {
    x_multi_pts<E, SCALED>(M, P, prog_id, (uint32_t)it.y, psteps, punits, plev, finals, tid, wave, nw, smem);
  }
}

__global__ void k_amp_to_real(const double* __restrict__ amp, int64_t n, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double e = amp[3 * i + 2];
    const double fl = floor(e);
    out[i] = ldexp(amp[3 * i] * exp2(e - fl), (int)fl);
  }
}

}  // namespace

hipError_t launch_lds_multi(const XMulti& m, int n_items, size_t smem, int waves, bool c128, bool scaled,
                            hipStream_t stream) {
  if (n_items == 0) return hipSuccess;
  const dim3 grid((unsigned)n_items), block((unsigned)(64 * waves));
  const void* fn = c128 ? reinterpret_cast<const void*>(&k_lds_multi<double2, false>)
                        : (scaled ? reinterpret_cast<const void*>(&k_lds_multi<float2, true>)
                                  : reinterpret_cast<const void*>(&k_lds_multi<float2, false>));
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  if (c128)
    hipLaunchKernelGGL((k_lds_multi<double2, false>), grid, block, smem, stream, m, m.progs, m.steps, m.units,
                       m.level_off, m.finals, m.items);
  else if (scaled)
    hipLaunchKernelGGL((k_lds_multi<float2, true>), grid, block, smem, stream, m, m.progs, m.steps, m.units,
                       m.level_off, m.finals, m.items);
  else
    hipLaunchKernelGGL((k_lds_multi<float2, false>), grid, block, smem, stream, m, m.progs, m.steps, m.units,
                       m.level_off, m.finals, m.items);
  return hipGetLastError();
}

hipError_t launch_amp_to_real(const double* amp, int64_t n, double* out, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_amp_to_real, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, amp, n, out);
  return hipGetLastError();
}

}  // namespace qt

namespace qt {
namespace {

// Derivative of entry y (row-major over the gate's two bits) of a
// parametrised gate by its parameter, from the gate's own table block gt:
// ZZ(t) has 1 on the diagonal and e^{-it} off it, so its derivative is 0 and
// -i times the entry; ZZ^dagger (e^{+it}) gives +i times the entry.  RX(t)
// has cos t on the diagonal and -i sin t off it: the diagonal derivative
// -sin t is the imaginary part of an off-diagonal entry, the off-diagonal
// one -i cos t is -i times a diagonal entry (RX^dagger: signs flipped).
template <typename E>
__device__ __forceinline__ double2 x_dgate(int kind, uint32_t y, const E* gt) {
  const bool diag = y == 0 || y == 3;
  const double dr = (double)gt[0].x, di = (double)gt[0].y;  // diagonal entry
  const double or_ = (double)gt[1].x, oi = (double)gt[1].y; // off-diagonal entry
  switch (kind) {
    case 0: return diag ? make_double2(0.0, 0.0) : make_double2(oi, -or_);
    case 1: return diag ? make_double2(0.0, 0.0) : make_double2(-oi, or_);
    case 2: return diag ? make_double2(oi, 0.0) : make_double2(di, -dr);
    default: return diag ? make_double2(-oi, 0.0) : make_double2(-di, dr);
  }
}

// One wavefront runs one unit of a reverse operation: 64 outputs y of a
// large adjoint, or all 2^ry outputs of a small one with the complement
// counter c split over G = 64 / 2^ry lane groups (lane group g takes
// c = g + G i) and the groups summed by a fixed butterfly.  The bit maps are
// linear over disjoint bits, so an operand's index is base + map_c(g) +
// map_c(G i): a per-lane constant plus a wavefront-uniform term.  The
// uniform terms of 64 iterations are computed at once, one iteration per
// lane, and each iteration reads its own with one lane read per operand.
template <typename E, bool SCALED, int NOPS>
__device__ __forceinline__ void x_runit(const XRev& rv, uint32_t chunk, uint32_t lane, E* __restrict__ lds,
                                        uint32_t* __restrict__ smax, int* __restrict__ sexp,
                                        double* __restrict__ gacc) {
  using R = typename XReal<E>::R;
  const int ry = rv.ry;
  const bool wide = ry >= 6;
  const uint32_t y = wide ? chunk * 64u + lane : (lane & ((1u << ry) - 1u));
  const uint32_t g = wide ? 0u : (lane >> ry);
  const uint32_t G = wide ? 1u : (64u >> ry);
  const uint32_t C = 1u << rv.nc;
  uint32_t base[NOPS];
  R sc[NOPS];
  int eacc = 0;
#pragma unroll
  for (int o = 0; o < NOPS; ++o) {
    const XROp& op = rv.op[o];
    base[o] = op.lds_off + xpext_all(y, op.y_lo, op.y_len, op.y_dst) + xpext_all(g, op.c_lo, op.c_len, op.c_dst);
    sc[o] = (R)1;
    if (SCALED && op.slot >= 0) {
      const int sh = xshift(smax[op.slot]);
      sc[o] = (R)xpow2neg(sh);
      eacc += sexp[op.slot] + sh;
    }
  }
  // Four iterations in flight (their operand reads issue together), each
  // into its own partial sum; the partial sums are added in a fixed order.
  constexpr int kU = 4;
  E part[kU];
#pragma unroll
  for (int k = 0; k < kU; ++k) {
    part[k].x = 0;
    part[k].y = 0;
  }
  const bool live = g < C;  // lane groups beyond a short complement add nothing
  const uint32_t n_it = C > G ? C / G : 1u;
  for (uint32_t ib = 0; ib < n_it; ib += 64) {
    uint32_t cm[NOPS];
    const uint32_t ci = (ib + lane) * G;
#pragma unroll
    for (int o = 0; o < NOPS; ++o) cm[o] = xpext_all(ci, rv.op[o].c_lo, rv.op[o].c_len, rv.op[o].c_dst);
    const uint32_t nb = n_it - ib < 64u ? n_it - ib : 64u;
    uint32_t t = 0;
    for (; t + kU <= nb; t += kU) {
      E v[kU];
#pragma unroll
      for (int k = 0; k < kU; ++k) {
        v[k] = lds[base[0] + (uint32_t)__builtin_amdgcn_readlane((int)cm[0], (int)(t + k))];
        if (SCALED) v[k] = xscale(v[k], sc[0]);
      }
#pragma unroll
      for (int o = 1; o < NOPS; ++o) {
        E x[kU];
#pragma unroll
        for (int k = 0; k < kU; ++k) x[k] = lds[base[o] + (uint32_t)__builtin_amdgcn_readlane((int)cm[o], (int)(t + k))];
#pragma unroll
        for (int k = 0; k < kU; ++k) {
          if (SCALED) x[k] = xscale(x[k], sc[o]);
          v[k] = xmul(v[k], x[k]);
        }
      }
      if (live) {
#pragma unroll
        for (int k = 0; k < kU; ++k) part[k] = xadd(part[k], v[k]);
      }
    }
    for (; t < nb; ++t) {
      E v = lds[base[0] + (uint32_t)__builtin_amdgcn_readlane((int)cm[0], (int)t)];
      if (SCALED) v = xscale(v, sc[0]);
#pragma unroll
      for (int o = 1; o < NOPS; ++o) {
        E x = lds[base[o] + (uint32_t)__builtin_amdgcn_readlane((int)cm[o], (int)t)];
        if (SCALED) x = xscale(x, sc[o]);
        v = xmul(v, x);
      }
      if (live) part[0] = xadd(part[0], v);
    }
  }
  E acc = xadd(xadd(part[0], part[1]), xadd(part[2], part[3]));
  if (!wide) {
    for (uint32_t off = 1u << ry; off < 64u; off <<= 1) {
      acc.x += __shfl_xor(acc.x, (int)off);
      acc.y += __shfl_xor(acc.y, (int)off);
    }
  }
  if (rv.gate >= 0) {
    double v = 0.0;
    if (g == 0) {
      const double2 d = x_dgate(rv.gate, y, lds + rv.out_off);
      v = (double)acc.x * d.x - (double)acc.y * d.y;
    }
    for (uint32_t off = 1; off < (1u << ry); off <<= 1) v += __shfl_xor(v, (int)off);
    if (lane == 0) gacc[rv.rec] = SCALED ? ldexp(v, eacc) : v;
    return;
  }
  if (g == 0) lds[rv.out_off + y] = acc;
  if (SCALED) {
    const float m = g == 0 ? fmaxf(fabsf((float)acc.x), fabsf((float)acc.y)) : 0.f;
    const uint32_t mw = xwave_max(__float_as_uint(m));
    if (lane == 0) {
      atomicMax(smax + rv.out_slot, mw);
      if (chunk == 0) sexp[rv.out_slot] = eacc;
    }
  }
}

// x_runit for every point of a point-batched item (unscaled elements):
// the unit's maps are decoded once, then each point's reduction runs in
// turn on its own tensors (element offset q * stride) and records (q * R).
template <typename E, int NOPS>
__device__ __forceinline__ void x_runit_pts(const XRev& rv, uint32_t chunk, uint32_t lane, uint32_t npts,
                                            uint32_t stride, uint32_t R, E* __restrict__ lds,
                                            double* __restrict__ gacc) {
  const int ry = rv.ry;
  const bool wide = ry >= 6;
  const uint32_t y = wide ? chunk * 64u + lane : (lane & ((1u << ry) - 1u));
  const uint32_t g = wide ? 0u : (lane >> ry);
  const uint32_t G = wide ? 1u : (64u >> ry);
  const uint32_t C = 1u << rv.nc;
  // operand offsets from the per-lane-bit weights (the run tables only for
  // a wide adjoint's chunk part and the iteration blocks past the first)
  uint32_t base[NOPS], cml[NOPS];
#pragma unroll
  for (int o = 0; o < NOPS; ++o) {
    const XROp& op = rv.op[o];
    uint32_t lw[6], iw[6];
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      lw[b] = op.lw[b];
      iw[b] = op.iw[b];
    }
    uint32_t bo = op.lds_off, co = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      const bool on = (lane >> b) & 1u;
      bo += on ? lw[b] : 0u;
      co += on ? iw[b] : 0u;
    }
    if (wide && chunk != 0) bo += xpext_all(chunk * 64u, op.y_lo, op.y_len, op.y_dst);
    base[o] = bo;
    cml[o] = co;
  }
  const bool live = g < C;
  const uint32_t n_it = C > G ? C / G : 1u;
  const bool one_block = n_it <= 64u;
  uint32_t cm[NOPS];
#pragma unroll
  for (int o = 0; o < NOPS; ++o) cm[o] = cml[o];
  constexpr int kU = 4;
  for (uint32_t q = 0; q < npts; ++q) {
    const uint32_t qo = q * stride;
    E part[kU];
#pragma unroll
    for (int k = 0; k < kU; ++k) {
      part[k].x = 0;
      part[k].y = 0;
    }
    for (uint32_t ib = 0; ib < n_it; ib += 64) {
      if (!one_block) {
#pragma unroll
        for (int o = 0; o < NOPS; ++o)
          cm[o] = cml[o] + (ib ? xpext_all(ib * G, rv.op[o].c_lo, rv.op[o].c_len, rv.op[o].c_dst) : 0u);
      }
      const uint32_t nb = n_it - ib < 64u ? n_it - ib : 64u;
      uint32_t t = 0;
      for (; t + kU <= nb; t += kU) {
        E v[kU];
#pragma unroll
        for (int k = 0; k < kU; ++k)
          v[k] = lds[qo + base[0] + (uint32_t)__builtin_amdgcn_readlane((int)cm[0], (int)(t + k))];
#pragma unroll
        for (int o = 1; o < NOPS; ++o) {
          E x[kU];
#pragma unroll
          for (int k = 0; k < kU; ++k)
            x[k] = lds[qo + base[o] + (uint32_t)__builtin_amdgcn_readlane((int)cm[o], (int)(t + k))];
#pragma unroll
          for (int k = 0; k < kU; ++k) v[k] = xmul(v[k], x[k]);
        }
        if (live) {
#pragma unroll
          for (int k = 0; k < kU; ++k) part[k] = xadd(part[k], v[k]);
        }
      }
      for (; t < nb; ++t) {
        E v = lds[qo + base[0] + (uint32_t)__builtin_amdgcn_readlane((int)cm[0], (int)t)];
#pragma unroll
        for (int o = 1; o < NOPS; ++o) v = xmul(v, lds[qo + base[o] + (uint32_t)__builtin_amdgcn_readlane((int)cm[o], (int)t)]);
        if (live) part[0] = xadd(part[0], v);
      }
    }
    E acc = xadd(xadd(part[0], part[1]), xadd(part[2], part[3]));
    if (!wide) {
      for (uint32_t off = 1u << ry; off < 64u; off <<= 1) {
        acc.x += __shfl_xor(acc.x, (int)off);
        acc.y += __shfl_xor(acc.y, (int)off);
      }
    }
    if (rv.gate >= 0) {
      double v = 0.0;
      if (g == 0) {
        const double2 d = x_dgate(rv.gate, y, lds + qo + rv.out_off);
        v = (double)acc.x * d.x - (double)acc.y * d.y;
      }
      for (uint32_t off = 1; off < (1u << ry); off <<= 1) v += __shfl_xor(v, (int)off);
      if (lane == 0) gacc[q * R + rv.rec] = v;
    } else if (g == 0) {
      lds[qo + rv.out_off + y] = acc;
    }
  }
}

// Adjoints of a program's closing scalars: the item's value is
// 2^log2_const times their product, so the adjoint of scalar f is
// 2^log2_const times the product of the others (FP64, renormalised).
template <typename E, bool SCALED>
__device__ void x_final_adjoints(const XProg& P, const XFinal* __restrict__ fin, const E* lds, uint32_t* smax,
                                 int* sexp, E* ldsw) {
  const int nf = P.n_finals;
  for (int f = 0; f < nf; ++f) {
    double re = 1.0, im = 0.0;
    int e = 0;
    for (int h = 0; h < nf; ++h) {
      if (h == f) continue;
      const E a = lds[fin[h].lds_off];
      const double ar = (double)a.x, ai = (double)a.y;
      const double nr = re * ar - im * ai;
      im = re * ai + im * ar;
      re = nr;
      if (SCALED && fin[h].slot >= 0) e += sexp[fin[h].slot];
    }
    const XFinal& B = fin[nf + f];
    if (SCALED) {
      const double fl = floor(P.log2_const);
      const double s = exp2(P.log2_const - fl);
      re *= s;
      im *= s;
      e += (int)fl;
      const double m = fmax(fabs(re), fabs(im));
      if (m > 0.0) {
        const int k = ilogb(m) + 1;
        re = ldexp(re, -k);
        im = ldexp(im, -k);
        e += k;
      }
      E v;
      v.x = (typename XReal<E>::R)re;
      v.y = (typename XReal<E>::R)im;
      ldsw[B.lds_off] = v;
      smax[B.slot] = __float_as_uint(fmaxf(fabsf((float)re), fabsf((float)im)));
      sexp[B.slot] = e;
    } else {
      const double s = exp2(P.log2_const);
      E v;
      v.x = (typename XReal<E>::R)(re * s);
      v.y = (typename XReal<E>::R)(im * s);
      ldsw[B.lds_off] = v;
    }
  }
}

// One unit of the gradient schedule: a forward or recomputation step, a
// reverse operation, or the adjoints of the closing scalars.
template <typename E, bool SCALED>
__device__ __forceinline__ void x_grad_unit(const uint2 un, const XStep* __restrict__ psteps,
                                            const XRev* __restrict__ prevs, const XProg& P,
                                            const XFinal* __restrict__ pfin, const XCtx& c, E* __restrict__ lds,
                                            uint32_t* __restrict__ smax, int* __restrict__ sexp,
                                            double* __restrict__ gacc, const double* prm) {
  constexpr int kBig = sizeof(E) == 8 ? kXEpu : kXEpu / 2;
  const uint32_t kind = un.x & ~kXUnitIndex;
  const uint32_t idx = un.x & kXUnitIndex;
  if (kind == 0) {
    const XStep& st = psteps[idx];
    const bool big = st.r >= kXBigRank;
    if (st.n_in <= 2) {
      if (big) x_unit<E, SCALED, 2, kBig, false>(st, un.y, c, lds, smax, sexp, nullptr, nullptr);
      else x_unit<E, SCALED, 2, 1, false>(st, un.y, c, lds, smax, sexp, nullptr, nullptr);
    } else if (st.n_in <= 4) {
      if (big) x_unit<E, SCALED, 4, kBig, false>(st, un.y, c, lds, smax, sexp, nullptr, nullptr);
      else x_unit<E, SCALED, 4, 1, false>(st, un.y, c, lds, smax, sexp, nullptr, nullptr);
    } else {
      if (big) x_unit<E, SCALED, 8, (kBig > 1 ? kBig / 2 : 1), false>(st, un.y, c, lds, smax, sexp, nullptr, nullptr);
      else x_unit<E, SCALED, 8, 1, false>(st, un.y, c, lds, smax, sexp, nullptr, nullptr);
    }
  } else if (kind == kXUnitRev) {
    const XRev& rv = prevs[idx];
    switch (rv.n_ops) {
      case 1:
      case 2: x_runit<E, SCALED, 2>(rv, un.y, c.lane, lds, smax, sexp, gacc); break;
      case 3: x_runit<E, SCALED, 3>(rv, un.y, c.lane, lds, smax, sexp, gacc); break;
      case 4: x_runit<E, SCALED, 4>(rv, un.y, c.lane, lds, smax, sexp, gacc); break;
      case 5: x_runit<E, SCALED, 5>(rv, un.y, c.lane, lds, smax, sexp, gacc); break;
      case 6: x_runit<E, SCALED, 6>(rv, un.y, c.lane, lds, smax, sexp, gacc); break;
      default: x_runit<E, SCALED, 8>(rv, un.y, c.lane, lds, smax, sexp, gacc); break;
    }
  } else if (c.lane == 0) {
    x_final_adjoints<E, SCALED>(P, pfin, lds, smax, sexp, lds);
  }
}

// Item value (thread 0: product of the closing scalars, FP64, with the
// accumulated exponent) and its 2p derivatives (threads 1..2p: each the sum
// of its parameter's gradient records in record order).
template <typename E, bool SCALED>
__device__ __forceinline__ void x_grad_epilogue(const XMulti& M, const XProg& P, int prog_id,
                                                const XFinal* __restrict__ pfin, const int32_t* __restrict__ rec_off,
                                                uint32_t pt, int tid, const E* lds, const int* sexp,
                                                const double* gacc) {
  if (tid == 0) {
    double re = 1.0, im = 0.0, ex = P.log2_const;
    for (int f = 0; f < P.n_finals; ++f) {
      const XFinal& F = pfin[f];
      const E a = lds[F.lds_off];
      const double ar = (double)a.x, ai = (double)a.y;
      if (SCALED && F.slot >= 0) ex += sexp[F.slot];
      const double nr = re * ar - im * ai;
      im = re * ai + im * ar;
      re = nr;
    }
    double* o = M.out + 3 * ((int64_t)pt * M.n_progs + prog_id);
    o[0] = re;
    o[1] = im;
    o[2] = ex;
  } else if (tid <= 2 * M.p) {
    const int q = tid - 1;
    const int32_t* ro = rec_off + P.recs_off;
    double s = 0.0;
    for (int r = ro[q]; r < ro[q + 1]; ++r) s += gacc[r];
    M.gout[((int64_t)pt * M.n_progs + prog_id) * 2 * M.p + q] = s;
  }
}

// Gradient executor: one workgroup per (program, point) item runs the
// program's forward steps, the adjoints of its closing scalars, its
// recomputation steps and its reverse operations, all from one level
// schedule, then forms the item's value (as the multi-program executor) and
// its derivatives by the 2p parameters, each the FP64 sum of the parameter's
// gradient records in record order.  Items too large for the launch's LDS
// run the same schedule from their global scratch area.
template <typename E, bool SCALED, bool GLOBAL>
__device__ __forceinline__ void x_grad_item(const XMulti& M, const XProg& P, int prog_id,
                                            const XStep* __restrict__ psteps, const XRev* __restrict__ prevs,
                                            const uint2* __restrict__ punits, const int32_t* __restrict__ plev,
                                            const XFinal* __restrict__ pfin, const int32_t* __restrict__ rec_off,
                                            const XCtx& c, int tid, int wave, int nw, E* area, uint32_t* smax,
                                            int* sexp, double* gacc) {
  const double* prm = M.gam + (int64_t)c.pt * M.pstride;
  const double* prb = M.bet + (int64_t)c.pt * M.pstride;
  for (int i = tid; i < P.n_slots; i += blockDim.x) {
    smax[i] = 0u;
    sexp[i] = 0;
  }
  if (tid < 2) {
    area[tid].x = 1;
    area[tid].y = 0;
  }
  for (int t = tid; t < x_gate_elems(M.p); t += blockDim.x) area[kXGate + t] = x_gate2<E>(t, prm, prb);
  x_level_sync<GLOBAL>();
  for (int L = 0; L < P.n_levels; ++L) {
    const int u_end = plev[L + 1];
    for (int u = plev[L] + wave; u < u_end; u += nw)
      x_grad_unit<E, SCALED>(punits[u], psteps, prevs, P, pfin, c, area, smax, sexp, gacc, prm);
    x_level_sync<GLOBAL>();
  }
  x_grad_epilogue<E, SCALED>(M, P, prog_id, pfin, rec_off, c.pt, tid, area, sexp, gacc);
}

// One point-batched item of the gradient executor: up to P.n_pts points
// (from pt0) of one program in the workgroup's LDS, point q's tensors at
// element q * pt_stride, its scale slots at q * slot_stride and its
// gradient records at q * rec_stride.  Forward and recomputation steps run
// as point-batched units; a reverse operation's unit names its point; the
// adjoints of the closing scalars take one lane per point.
template <typename E, bool SCALED>
__device__ __forceinline__ void x_grad_pts(const XMulti& M, const XProg& P, int prog_id, uint32_t pt0,
                                           const XStep* __restrict__ psteps, const XRev* __restrict__ prevs,
                                           const uint2* __restrict__ punits, const int32_t* __restrict__ plev,
                                           const XFinal* __restrict__ pfin, const int32_t* __restrict__ rec_off,
                                           int tid, int wave, int nw, unsigned char* smem) {
  const uint32_t np = (uint32_t)P.n_pts;
  const uint32_t npts = min(np, (uint32_t)M.n_points - pt0);
  const uint32_t S = (uint32_t)P.slot_stride, R = (uint32_t)P.rec_stride, stride = (uint32_t)P.pt_stride;
  uint32_t* smax = reinterpret_cast<uint32_t*>(smem);
  int* sexp = reinterpret_cast<int*>(smem + 4 * np * S);
  double* gacc = reinterpret_cast<double*>(smem + 8 * np * S);
  E* lds = reinterpret_cast<E*>(smem + 8 * np * S + 8 * np * R);
  for (uint32_t i = tid; i < np * S; i += blockDim.x) {
    smax[i] = 0u;
    sexp[i] = 0;
  }
  const uint32_t ge = (uint32_t)x_gate_elems(M.p);
  for (uint32_t i = tid; i < np * (ge + kXGate); i += blockDim.x) {
    const uint32_t q = i / (ge + kXGate), t = i - q * (ge + kXGate);
    E v;
    if (t < (uint32_t)kXGate) {
      v.x = 1;
      v.y = 0;
    } else {
      const uint32_t pq = pt0 + min(q, npts - 1u);
      v = x_gate2<E>((int)(t - kXGate), M.gam + (int64_t)pq * M.pstride, M.bet + (int64_t)pq * M.pstride);
    }
    lds[q * stride + t] = v;
  }
  __syncthreads();
  constexpr int kBig = sizeof(E) == 8 ? kXEpu : kXEpu / 2;
  const uint32_t lane = tid & 63;
  for (int L = 0; L < P.n_levels; ++L) {
    const int u_end = plev[L + 1];
    for (int u = plev[L] + wave; u < u_end; u += nw) {
      const uint2 un = punits[u];
      const uint32_t kind = un.x & ~kXUnitIndex, idx = un.x & kXUnitIndex;
      if (kind == 0) {
        const XStep& st = psteps[idx];
        x_unit_pts_any<E, SCALED, kBig>(st, un.y, lane, npts, stride, S, lds, smax, sexp);
      } else if (kind == kXUnitRev) {
        static_assert(!SCALED, "the gradient pass runs on unscaled elements");
        const XRev& rv = prevs[idx];
        switch (rv.n_ops) {  // exact operand counts: no identity operands read or multiplied
          case 1:
          case 2: x_runit_pts<E, 2>(rv, un.y, lane, npts, stride, R, lds, gacc); break;
          case 3: x_runit_pts<E, 3>(rv, un.y, lane, npts, stride, R, lds, gacc); break;
          case 4: x_runit_pts<E, 4>(rv, un.y, lane, npts, stride, R, lds, gacc); break;
          case 5: x_runit_pts<E, 5>(rv, un.y, lane, npts, stride, R, lds, gacc); break;
          case 6: x_runit_pts<E, 6>(rv, un.y, lane, npts, stride, R, lds, gacc); break;
          default: x_runit_pts<E, 8>(rv, un.y, lane, npts, stride, R, lds, gacc); break;
        }
      } else if (lane < npts) {
        E* lq = lds + lane * stride;
        x_final_adjoints<E, SCALED>(P, pfin, lq, smax + lane * S, sexp + lane * S, lq);
      }
    }
    __syncthreads();
  }
  const uint32_t per = 2u * (uint32_t)M.p + 1u;
  const int32_t* ro = rec_off + P.recs_off;
  for (uint32_t i = tid; i < npts * per; i += blockDim.x) {
    const uint32_t q = i / per, k = i - q * per;
    const uint32_t pt = pt0 + q;
    if (k == 0) {
      double re = 1.0, im = 0.0, ex = P.log2_const;
      for (int f = 0; f < P.n_finals; ++f) {
        const XFinal& F = pfin[f];
        const E a = lds[q * stride + F.lds_off];
        const double ar = (double)a.x, ai = (double)a.y;
        if (SCALED && F.slot >= 0) ex += sexp[q * S + F.slot];
        const double nr = re * ar - im * ai;
        im = re * ai + im * ar;
        re = nr;
      }
      double* o = M.out + 3 * ((int64_t)pt * M.n_progs + prog_id);
      o[0] = re;
      o[1] = im;
      o[2] = ex;
    } else {
      double s = 0.0;
      for (int r = ro[k - 1]; r < ro[k]; ++r) s += gacc[q * R + r];
      M.gout[((int64_t)pt * M.n_progs + prog_id) * 2 * M.p + (k - 1)] = s;
    }
  }
}

template <typename E, bool SCALED>
__global__ __launch_bounds__(kXMaxThreads) void k_lds_grad(
    const XMulti M, const XProg* __restrict__ progs, const XStep* __restrict__ steps, const XRev* __restrict__ revs,
    const uint2* __restrict__ units, const int32_t* __restrict__ level_off, const XFinal* __restrict__ finals,
    const int2* __restrict__ items, const int32_t* __restrict__ rec_off) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int2 it = items[blockIdx.x];
  const int prog_id = it.x;
  const XProg& P = progs[prog_id];
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nw = blockDim.x >> 6;
  const XStep* psteps = steps + P.steps_off;
  const XRev* prevs = revs + P.revs_off;
  const uint2* punits = units + P.units_off;
  const int32_t* plev = level_off + P.levels_off;
  const XFinal* pfin = finals + P.finals_off;
  if (P.scratch_off >= 0) {
    XCtx c;
    c.pt = (uint32_t)it.y;
    c.sb = 0;
    c.sid = 0;
    c.lane = tid & 63;
    const XArea a = x_area(P.n_slots, P.n_recs, P.area_elems, (int)sizeof(E));
    char* base = M.scratch + P.scratch_off + (int64_t)c.pt * P.scratch_stride;
    x_grad_item<E, SCALED, true>(M, P, prog_id, psteps, prevs, punits, plev, pfin, rec_off, c, tid, wave, nw,
                                 reinterpret_cast<E*>(base), reinterpret_cast<uint32_t*>(base + a.elem_bytes),
                                 reinterpret_cast<int*>(base + a.elem_bytes + a.slot_bytes),
                                 reinterpret_cast<double*>(base + a.elem_bytes + 2 * a.slot_bytes));
  } else {
    x_grad_pts<E, SCALED>(M, P, prog_id, (uint32_t)it.y, psteps, prevs, punits, plev, pfin, rec_off, tid, wave, nw,
                          smem);
  }
}

// One workgroup per output (r, q): lane-strided partial sums in index order
// (entry i times w[i] when weights are given), then a fixed tree, so the
// result does not depend on timing.
__global__ __launch_bounds__(256) void k_rows_sum(const double* __restrict__ in, int n, int nq,
                                                  const double* __restrict__ w, double* __restrict__ out) {
  __shared__ double part[256];
  const int r = blockIdx.x / nq, q = blockIdx.x % nq;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += in[((int64_t)r * n + i) * nq + q] * (w ? w[i] : 1.0);
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = part[0];
}

}  // namespace

size_t lds_grad_smem_bytes(int n_slots, int n_recs, int lds_elems, bool c128) {
  const size_t slots16 = (size_t)((n_slots + 3) & ~3);
  const size_t recs2 = (size_t)((n_recs + 1) & ~1);
  return 8 * slots16 + 8 * recs2 + (size_t)lds_elems * (c128 ? 16 : 8);
}

hipError_t launch_lds_grad(const XMulti& m, int n_items, size_t smem, int waves, hipStream_t stream) {
  if (n_items == 0) return hipSuccess;
  const dim3 grid((unsigned)n_items), block((unsigned)(64 * waves));
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lds_grad<double2, false>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_lds_grad<double2, false>), grid, block, smem, stream, m, m.progs, m.steps, m.revs, m.units,
                     m.level_off, m.finals, m.items, m.rec_off);
  return hipGetLastError();
}

int64_t multi_scratch_bytes(int n_slots, int n_recs, int area_elems, bool c128) {
  const XArea a = x_area(n_slots, n_recs, area_elems, c128 ? 16 : 8);
  return (a.elem_bytes + 2 * a.slot_bytes + a.rec_bytes + 255) & ~(int64_t)255;
}

hipError_t launch_rows_sum(const double* in, int rows, int n, int nq, double* out, hipStream_t stream,
                           const double* weights) {
  if (rows == 0 || nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rows_sum, dim3((unsigned)(rows * nq)), dim3(256), 0, stream, in, n, nq, weights, out);
  return hipGetLastError();
}

}  // namespace qt
