// LDS executor: one workgroup per batch item runs a segment of bucket steps
// whose tensors are small enough to live in the workgroup's LDS.
//
// The steps of a segment are grouped into dependency levels (a step's level
// is one more than the deepest step of the segment that produced one of its
// inputs), and all steps of a level run concurrently: the level's work is
// cut into 64-element units of one step each, handed round-robin to the
// workgroup's wavefronts, with a single barrier between levels.  A unit is
// uniform over its wavefront, so its descriptors are read with scalar loads.
// Each element computes, like the streaming kernels,
//   out[x] = prod_{j without v} T_j[x] * sum_{v} prod_{j with v} T_j[x, v],
// reading operands from LDS or global memory (results of earlier launches,
// gate tensors) and writing the output to LDS or global memory.
#include <hip/hip_runtime.h>

#include <type_traits>

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
template <typename E> __device__ __forceinline__ E xone();
template <> __device__ __forceinline__ float2 xone<float2>() { return make_float2(1.f, 0.f); }
template <> __device__ __forceinline__ double2 xone<double2>() { return make_double2(1.0, 0.0); }

__device__ __forceinline__ uint32_t xpext_runs(uint32_t x, const XIn& in) {
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < kXRuns; ++i)
    if (i < in.nruns) r |= ((x >> in.run_lo[i]) & ((1u << in.run_len[i]) - 1u)) << in.run_dst[i];
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

__device__ __forceinline__ int xshift(uint32_t maxbits) {
  if (maxbits == 0) return 0;
  return ilogbf(__uint_as_float(maxbits)) + 1;
}

template <typename E> struct XReal;
template <> struct XReal<float2> { using R = float; };
template <> struct XReal<double2> { using R = double; };

struct XCtx {
  uint32_t pt, sb;
  uint64_t sid;
  uint32_t lane;
};

// One work unit: EPU x 64 consecutive outputs of one step.  Every load of
// the unit is issued before any arithmetic; inputs without the summed
// variable are read twice at the same index (no branch between the two
// products).
template <typename E, bool SCALED, int NIN, int EPU>
__device__ __forceinline__ void x_unit(const XStep& st, uint32_t chunk, const XCtx& c, E* __restrict__ lds,
                                       uint32_t* __restrict__ smax, int* __restrict__ sexp, int* __restrict__ gexps,
                                       uint32_t* __restrict__ gmax) {
  using R = typename XReal<E>::R;
  const E* src[NIN];
  R sc[NIN];
  int eacc = 0;
#pragma unroll
  for (int j = 0; j < NIN; ++j) {
    const XIn& in = st.in[j];
    if (in.ptr == nullptr)
      src[j] = lds + in.lds_off;
    else
      src[j] = reinterpret_cast<const E*>(in.ptr) + (int64_t)c.pt * in.pt_stride + (int64_t)c.sb * in.sb_stride +
               ((int64_t)xpext_bits(c.sid, in.smask) << in.slow);
    sc[j] = (R)1;
    if (SCALED && in.slot_kind != 0) {
      int sh, ex;
      if (in.slot_kind == 1) {
        sh = xshift(smax[in.slot]);
        ex = sexp[in.slot];
      } else {
        const int g = in.slot + (int)c.pt * in.exp_pt + (int)c.sb * in.exp_sb;
        sh = xshift(gmax[g]);
        ex = gexps[g];
      }
      sc[j] = (R)ldexp(1.0, -sh);
      eacc += ex + sh;
    }
  }
  const uint32_t n = 1u << st.r;
  E a0[EPU][NIN], a1[EPU][NIN];
#pragma unroll
  for (int e = 0; e < EPU; ++e) {
    uint32_t x = (chunk * EPU + e) * 64u + c.lane;
    x = x < n ? x : 0u;
#pragma unroll
    for (int j = 0; j < NIN; ++j) {
      const int hv = st.in[j].has_v;
      const uint32_t idx = xpext_runs(x, st.in[j]) << hv;
      a0[e][j] = src[j][idx];
      a1[e][j] = src[j][idx + hv];
    }
  }
  const XIn& o = st.out;
  E* dst = o.ptr == nullptr
               ? lds + o.lds_off
               : reinterpret_cast<E*>(const_cast<void*>(o.ptr)) + (int64_t)c.pt * o.pt_stride + (int64_t)c.sb * o.sb_stride;
  float m = 0.f;
#pragma unroll
  for (int e = 0; e < EPU; ++e) {
    const uint32_t x = (chunk * EPU + e) * 64u + c.lane;
    E t0 = xscale(a0[e][0], sc[0]), t1 = xscale(a1[e][0], sc[0]);
#pragma unroll
    for (int j = 1; j < NIN; ++j) {
      t0 = xmul(t0, xscale(a0[e][j], sc[j]));
      t1 = xmul(t1, xscale(a1[e][j], sc[j]));
    }
    const E res = st.sum ? xadd(t0, t1) : t0;
    if (x < n) {
      dst[x] = res;
      if (SCALED) m = fmaxf(m, fmaxf(fabsf((float)res.x), fabsf((float)res.y)));
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

template <typename E, bool SCALED, int EPU>
__device__ __forceinline__ void x_dispatch(const XStep& st, uint32_t chunk, const XCtx& c, E* lds, uint32_t* smax,
                                           int* sexp, int* gexps, uint32_t* gmax) {
  switch (st.n_in) {
    case 1: x_unit<E, SCALED, 1, EPU>(st, chunk, c, lds, smax, sexp, gexps, gmax); break;
    case 2: x_unit<E, SCALED, 2, EPU>(st, chunk, c, lds, smax, sexp, gexps, gmax); break;
    case 3: x_unit<E, SCALED, 3, EPU>(st, chunk, c, lds, smax, sexp, gexps, gmax); break;
    case 4: x_unit<E, SCALED, 4, EPU>(st, chunk, c, lds, smax, sexp, gexps, gmax); break;
    case 5: x_unit<E, SCALED, 5, EPU>(st, chunk, c, lds, smax, sexp, gexps, gmax); break;
    case 6: x_unit<E, SCALED, 6, EPU>(st, chunk, c, lds, smax, sexp, gexps, gmax); break;
    case 7: x_unit<E, SCALED, 7, EPU>(st, chunk, c, lds, smax, sexp, gexps, gmax); break;
    default: x_unit<E, SCALED, 8, EPU>(st, chunk, c, lds, smax, sexp, gexps, gmax); break;
  }
}

template <typename E, bool SCALED>
__global__ __launch_bounds__(kXMaxThreads) void k_lds_exec(const XLaunch X, int* __restrict__ gexps, uint32_t* __restrict__ gmax) {
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
  __syncthreads();

  for (int L = 0; L < X.n_levels; ++L) {
    const int u_end = X.level_off[L + 1];
    for (int u = X.level_off[L] + wave; u < u_end; u += nw) {
      const uint2 un = X.units[u];
      const XStep& st = X.steps[un.x];
      if (st.r >= kXBigRank)
        x_dispatch<E, SCALED, (sizeof(E) == 8 ? kXEpu : kXEpu / 2)>(st, un.y, c, lds, smax, sexp, gexps, gmax);
      else
        x_dispatch<E, SCALED, 1>(st, un.y, c, lds, smax, sexp, gexps, gmax);
    }
    __syncthreads();
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
  hipError_t e;
  if (c128) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lds_exec<double2, false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_lds_exec<double2, false>), grid, block, smem, stream, x, exps, maxbits);
  } else if (scaled) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lds_exec<float2, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_lds_exec<float2, true>), grid, block, smem, stream, x, exps, maxbits);
  } else {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lds_exec<float2, false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_lds_exec<float2, false>), grid, block, smem, stream, x, exps, maxbits);
  }
  return hipGetLastError();
}

}  // namespace qt
