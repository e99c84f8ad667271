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

__device__ __forceinline__ float2 xmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 xmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
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
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) r |= ((x >> lo[i]) & ((1u << len[i]) - 1u)) << dst[i];
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

// Power of two that brings max|x| into [0.5, 1), clamped so that 2^-shift is
// a normal float.
__device__ __forceinline__ int xshift(uint32_t maxbits) {
  if (maxbits == 0) return 0;
  const int s = ilogbf(__uint_as_float(maxbits)) + 1;
  return s < -126 ? -126 : (s > 127 ? 127 : s);
}
__device__ __forceinline__ float xpow2neg(int sh) { return __int_as_float((127 - sh) << 23); }

struct XCtx {
  uint32_t pt, sb;
  uint64_t sid;
  uint32_t lane;
};

template <typename E, bool SCALED, int NIN, int EPU>
__device__ __forceinline__ void x_unit(const XStep& st, uint32_t chunk, const XCtx& c, E* __restrict__ lds,
                                       uint32_t* __restrict__ smax, int* __restrict__ sexp, int* __restrict__ gexps,
                                       uint32_t* __restrict__ gmax) {
  using R = typename XReal<E>::R;
  const uint32_t cx = chunk * EPU * 64u;
  uint32_t base[NIN], lp[NIN];
  R sc[NIN];
  int eacc = 0;
#pragma unroll
  for (int j = 0; j < NIN; ++j) {
    const XOp& in = st.in[j];
    base[j] = in.lds_off + (xpext_bits(c.sid, in.smask) << in.slow);
    const uint32_t pc = xpext_all(cx, in.run_lo, in.run_len, in.run_dst);
    lp[j] = xpext_all(c.lane, in.run_lo, in.run_len, in.run_dst) + pc;
    sc[j] = (R)1;
    if (SCALED && in.slot >= 0) {
      const int sh = xshift(smax[in.slot]);
      sc[j] = (R)xpow2neg(sh);
      eacc += sexp[in.slot] + sh;
    }
  }
  E a0[EPU][NIN], a1[EPU][NIN];
#pragma unroll
  for (int e = 0; e < EPU; ++e) {
#pragma unroll
    for (int j = 0; j < NIN; ++j) {
      const uint32_t hv = (uint32_t)st.in[j].has_v;
      const uint32_t i = base[j] + ((lp[j] + st.in[j].ep[e]) << hv);
      a0[e][j] = lds[i];
      a1[e][j] = lds[i + hv];
    }
  }
  const XOut& o = st.out;
  const uint32_t n = 1u << st.r;
  float m = 0.f;
  E res[EPU];
#pragma unroll
  for (int e = 0; e < EPU; ++e) {
    E t0 = a0[e][0], t1 = a1[e][0];
    if (SCALED) {
      t0 = xscale(t0, sc[0]);
      t1 = xscale(t1, sc[0]);
    }
#pragma unroll
    for (int j = 1; j < NIN; ++j) {
      E x0 = a0[e][j], x1 = a1[e][j];
      if (SCALED) {
        x0 = xscale(x0, sc[j]);
        x1 = xscale(x1, sc[j]);
      }
      t0 = xmul(t0, x0);
      t1 = xmul(t1, x1);
    }
    res[e] = st.sum ? xadd(t0, t1) : t0;
    const uint32_t x = cx + e * 64u + c.lane;
    if (SCALED && x < n) m = fmaxf(m, fmaxf(fabsf((float)res[e].x), fabsf((float)res[e].y)));
  }
  if (o.ptr == nullptr) {
#pragma unroll
    for (int e = 0; e < EPU; ++e) {
      const uint32_t x = cx + e * 64u + c.lane;
      if (x < n) lds[o.lds_off + x] = res[e];
    }
  } else {
    gmut_t<E> g = (gmut_t<E>)(reinterpret_cast<E*>(o.ptr) + (int64_t)c.pt * o.pt_stride + (int64_t)c.sb * o.sb_stride);
#pragma unroll
    for (int e = 0; e < EPU; ++e) {
      const uint32_t x = cx + e * 64u + c.lane;
      if (x < n) {
        g[x].x = res[e].x;
        g[x].y = res[e].y;
      }
    }
  }
  if (SCALED) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) m = fmaxf(m, __shfl_xor(m, off));
    if (c.lane == 0) {
      if (o.slot_kind == 1) {
        atomicMax(smax + o.slot, __float_as_uint(m));
        if (chunk == 0) sexp[o.slot] = eacc;
      } else if (o.slot_kind == 2) {
        const int g = o.slot + (int)c.pt * o.exp_pt + (int)c.sb * o.exp_sb;
        atomicMax(gmax + g, __float_as_uint(m));
        if (chunk == 0) gexps[g] = eacc;
      }
    }
  }
}

// Gate table entry t of the workgroup's point (layout: x_gate_off), FP64
// trigonometry rounded to the element type (Section III-A conventions).
template <typename E>
__device__ __forceinline__ E x_gate(int t, const double* prm, int p) {
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
      sincos(prm[k], &sn, &cs);
      re = diag ? 1.0 : cs;
      im = diag ? 0.0 : (g == 0 ? -sn : sn);
    } else {
      sincos(prm[p + k], &sn, &cs);
      re = diag ? cs : 0.0;
      im = diag ? 0.0 : (g == 2 ? -sn : sn);
    }
  }
  v.x = (R)re;
  v.y = (R)im;
  return v;
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
  if (tid < x_gate_elems(X.p)) lds[kXGate + tid] = x_gate<E>(tid, X.params + (int64_t)c.pt * 2 * X.p, X.p);
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
    const int u_end = level_off[L + 1];
    for (int u = level_off[L] + wave; u < u_end; u += nw) {
      const uint2 un = units[u];
      const XStep& st = steps[un.x];
      const bool big = st.r >= kXBigRank;
      if (st.n_in <= 2) {
        if (big) x_unit<E, SCALED, 2, kBig>(st, un.y, c, lds, smax, sexp, gexps, gmax);
        else x_unit<E, SCALED, 2, 1>(st, un.y, c, lds, smax, sexp, gexps, gmax);
      } else if (st.n_in <= 4) {
        if (big) x_unit<E, SCALED, 4, kBig>(st, un.y, c, lds, smax, sexp, gexps, gmax);
        else x_unit<E, SCALED, 4, 1>(st, un.y, c, lds, smax, sexp, gexps, gmax);
      } else {
        if (big) x_unit<E, SCALED, 8, (kBig > 1 ? kBig / 2 : 1)>(st, un.y, c, lds, smax, sexp, gexps, gmax);
        else x_unit<E, SCALED, 8, 1>(st, un.y, c, lds, smax, sexp, gexps, gmax);
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

// Multi-program executor: one workgroup per (program, point) item runs a
// whole network (a per-edge lightcone) in LDS, then forms its scalar
// result: the product of the network's closing scalars in FP64 with the
// accumulated power-of-two exponent.
template <typename E, bool SCALED>
__global__ __launch_bounds__(kXMaxThreads) void k_lds_multi(const XMulti M, const XProg* __restrict__ progs,
                                                            const XStep* __restrict__ steps,
                                                            const uint2* __restrict__ units,
                                                            const int32_t* __restrict__ level_off,
                                                            const XFinal* __restrict__ finals,
                                                            const int32_t* __restrict__ item_prog) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int slots16 = (M.n_slots + 3) & ~3;
  uint32_t* smax = reinterpret_cast<uint32_t*>(smem);
  int* sexp = reinterpret_cast<int*>(smem + 4 * slots16);
  E* lds = reinterpret_cast<E*>(smem + 8 * slots16);

  const uint32_t item = blockIdx.x;
  const int prog_id = item_prog[item / (uint32_t)M.n_points];
  const XProg& P = progs[prog_id];
  XCtx c;
  c.pt = item % (uint32_t)M.n_points;
  c.sb = 0;
  c.sid = 0;
  const int tid = threadIdx.x;
  c.lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nw = blockDim.x >> 6;

  for (int i = tid; i < P.n_slots; i += blockDim.x) {
    smax[i] = 0u;
    sexp[i] = 0;
  }
  if (tid < 2) {
    lds[tid].x = 1;
    lds[tid].y = 0;
  }
  if (tid < x_gate_elems(M.p)) lds[kXGate + tid] = x_gate<E>(tid, M.params + (int64_t)c.pt * 2 * M.p, M.p);
  __syncthreads();

  constexpr int kBig = sizeof(E) == 8 ? kXEpu : kXEpu / 2;
  const XStep* psteps = steps + P.steps_off;
  const uint2* punits = units + P.units_off;
  const int32_t* plev = level_off + P.levels_off;
  for (int L = 0; L < P.n_levels; ++L) {
    const int u_end = plev[L + 1];
    for (int u = plev[L] + wave; u < u_end; u += nw) {
      const uint2 un = punits[u];
      const XStep& st = psteps[un.x];
      const bool big = st.r >= kXBigRank;
      if (st.n_in <= 2) {
        if (big) x_unit<E, SCALED, 2, kBig>(st, un.y, c, lds, smax, sexp, nullptr, nullptr);
        else x_unit<E, SCALED, 2, 1>(st, un.y, c, lds, smax, sexp, nullptr, nullptr);
      } else if (st.n_in <= 4) {
        if (big) x_unit<E, SCALED, 4, kBig>(st, un.y, c, lds, smax, sexp, nullptr, nullptr);
        else x_unit<E, SCALED, 4, 1>(st, un.y, c, lds, smax, sexp, nullptr, nullptr);
      } else {
        if (big) x_unit<E, SCALED, 8, (kBig > 1 ? kBig / 2 : 1)>(st, un.y, c, lds, smax, sexp, nullptr, nullptr);
        else x_unit<E, SCALED, 8, 1>(st, un.y, c, lds, smax, sexp, nullptr, nullptr);
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    double re = 1.0, im = 0.0, ex = P.log2_const;
    for (int f = 0; f < P.n_finals; ++f) {
      const XFinal& F = finals[P.finals_off + f];
      const E a = lds[F.lds_off];
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

__global__ void k_amp_to_real(const double* __restrict__ amp, int64_t n, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double e = amp[3 * i + 2];
    const double fl = floor(e);
    out[i] = ldexp(amp[3 * i] * exp2(e - fl), (int)fl);
  }
}

}  // namespace

hipError_t launch_lds_multi(const XMulti& m, int n_item_progs, int waves, bool c128, bool scaled, hipStream_t stream) {
  const int64_t n_items = (int64_t)n_item_progs * m.n_points;
  if (n_items == 0) return hipSuccess;
  const size_t smem = lds_exec_smem_bytes(m.n_slots, m.lds_elems, c128);
  const dim3 grid((unsigned)n_items), block((unsigned)(64 * waves));
  const void* fn = c128 ? reinterpret_cast<const void*>(&k_lds_multi<double2, false>)
                        : (scaled ? reinterpret_cast<const void*>(&k_lds_multi<float2, true>)
                                  : reinterpret_cast<const void*>(&k_lds_multi<float2, false>));
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  if (c128)
    hipLaunchKernelGGL((k_lds_multi<double2, false>), grid, block, smem, stream, m, m.progs, m.steps, m.units,
                       m.level_off, m.finals, m.item_prog);
  else if (scaled)
    hipLaunchKernelGGL((k_lds_multi<float2, true>), grid, block, smem, stream, m, m.progs, m.steps, m.units,
                       m.level_off, m.finals, m.item_prog);
  else
    hipLaunchKernelGGL((k_lds_multi<float2, false>), grid, block, smem, stream, m, m.progs, m.steps, m.units,
                       m.level_off, m.finals, m.item_prog);
  return hipGetLastError();
}

hipError_t launch_amp_to_real(const double* amp, int64_t n, double* out, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_amp_to_real, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, amp, n, out);
  return hipGetLastError();
}

}  // namespace qt
