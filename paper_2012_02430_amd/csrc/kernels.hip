// Bucket-elimination kernels for gfx950 (CDNA4, 64-wide wavefronts).
//
// A bucket step (Algorithm 1, inner loop and the sum over v) computes
//   out[x] = prod_{j without v} T_j[x]  *  sum_{v=0,1} prod_{j with v} T_j[x, v]
// for every output index x of every batch item (point, slice).  Every tensor
// stores its variables ordered by one global key in which the eliminated
// variable of a bucket is the lowest bit of every tensor of that bucket, so
// the two v-values of an input are adjacent (one 16-byte load for complex64)
// and every input's index is a monotone bit-extraction (pext) of the output
// index: contiguous runs of output bits map to contiguous runs of input bits.
// Slice variables carry the highest keys, so fixing them selects a
// contiguous block (the paper's "first t indices" blocks, Section VI-B).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "qt_internal.h"

namespace qt {
namespace {

constexpr int kWG = 256;
constexpr int kEPT = 4;                 // elements per thread, BIG mode
constexpr int kLgTile = 10;             // log2(kWG * kEPT)
constexpr int kMaxLgTpb = 4;            // BIG mode: at most 16 tiles per workgroup

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// Raw buffer over the 4 GiB window at p: loads and stores then take a
// 32-bit per-lane byte offset (a tile's offsets are small; the tile's base
// is uniform) instead of a 64-bit address per lane.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)0xffffffff, 0x00020000);
}
typedef unsigned u2v __attribute__((ext_vector_type(2)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

template <typename E> struct Cx;
template <> struct Cx<float2> {
  using R = float;
  __device__ static float2 one() { return make_float2(1.f, 0.f); }
  __device__ static float2 from(double re, double im) { return make_float2((float)re, (float)im); }
  __device__ static void load_pair(const void* p, int64_t idx, float2& a0, float2& a1) {
    const float4 v = *(reinterpret_cast<const float4*>(reinterpret_cast<const float2*>(p) + idx));
    a0 = make_float2(v.x, v.y);
    a1 = make_float2(v.z, v.w);
  }
  __device__ static float2 bload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const u2v v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
  }
  __device__ static void bload_pair(__amdgpu_buffer_rsrc_t r, uint32_t off, float2& a0, float2& a1) {
    const u4v v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    a0 = make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
    a1 = make_float2(__uint_as_float(v.z), __uint_as_float(v.w));
  }
  __device__ static void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, float2 a) {
    u2v v;
    v.x = __float_as_uint(a.x);
    v.y = __float_as_uint(a.y);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, 0);
  }
};
template <> struct Cx<double2> {
  using R = double;
  __device__ static double2 one() { return make_double2(1.0, 0.0); }
  __device__ static double2 from(double re, double im) { return make_double2(re, im); }
  __device__ static void load_pair(const void* p, int64_t idx, double2& a0, double2& a1) {
    const double2* q = reinterpret_cast<const double2*>(p) + idx;
    a0 = q[0];
    a1 = q[1];
  }
  __device__ static double2 bload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  }
  __device__ static void bload_pair(__amdgpu_buffer_rsrc_t r, uint32_t off, double2& a0, double2& a1) {
    a0 = bload(r, off);
    a1 = bload(r, off + 16u);
  }
  __device__ static void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, double2 a) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4v, a), r, off, 0, 0);
  }
};

__device__ __forceinline__ uint32_t pext_runs(uint32_t x, const DevIn& in) {
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < kMaxRuns; ++i)
    if (i < in.nruns) r |= ((x >> in.run_lo[i]) & ((1u << in.run_len[i]) - 1u)) << in.run_dst[i];
  return r;
}

__device__ __forceinline__ uint32_t pext_tile(uint32_t tile, const DevIn& in) {
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < kMaxRuns; ++i)
    if (i < in.t_nruns) r |= ((tile >> in.t_lo[i]) & ((1u << in.t_len[i]) - 1u)) << in.t_dst[i];
  return r;
}

__device__ __forceinline__ uint32_t pext_bits(uint64_t x, uint32_t m) {
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

// Exponent of the power of two that brings max|x| into [0.5, 1).
__device__ __forceinline__ int scale_shift(uint32_t maxbits) {
  if (maxbits == 0) return 0;
  return ilogbf(__uint_as_float(maxbits)) + 1;
}

__device__ __forceinline__ float wave_max(float m) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) m = fmaxf(m, __shfl_xor(m, o));
  return m;
}

template <typename E>
__device__ __forceinline__ float abs_max(E v) {
  return (float)fmax(fabs((double)v.x), fabs((double)v.y));
}
__device__ __forceinline__ float abs_max(float2 v) { return fmaxf(fabsf(v.x), fabsf(v.y)); }

// BIG mode: each workgroup covers 2^lg_tpb consecutive tiles of kWG*kEPT
// outputs of one batch item, so every per-item quantity (input bases, scale
// factors) is uniform and found once, and the part of each input index that
// depends on the tile is computed on the scalar unit.  All loads of a
// thread for a tile (kEPT elements x NIN inputs x the two values of v) are
// issued before any arithmetic.  An input without the summed variable is
// read twice at the same index, so the two products t0 (v = 0) and t1
// (v = 1) need no branch.  The output max of the workgroup's tiles is
// posted once.
template <typename E, bool SCALED, int NIN>
__global__ __launch_bounds__(kWG) void k_step_big(const DevStep s, int* __restrict__ exps,
                                                  uint32_t* __restrict__ maxbits) {
  using R = typename Cx<E>::R;
  const int lg_groups = s.lg_tiles - s.lg_tpb;  // tile groups per item
  const uint32_t item = blockIdx.x >> lg_groups;
  const uint32_t tile0 = (blockIdx.x & ((1u << lg_groups) - 1u)) << s.lg_tpb;
  const uint32_t sb = item & ((1u << s.lg_nsb) - 1u);
  const uint32_t pt = item >> s.lg_nsb;
  const uint64_t sid = (uint64_t)s.chunk_base + sb;
  const uint32_t tid = threadIdx.x;

  // The group's tiles differ in their low lg_tpb bits only, and pext is
  // linear over disjoint bits: an input's tile part is that of the first
  // tile plus one weight per set low bit (a few scalar adds per tile, and no
  // run tables live across the tile loop).
  // Small inputs (gates and small factors, at most x_small_cap(NIN)
  // elements per item) are staged in LDS once and read from there: their
  // loads would otherwise cost vector memory instructions on the same path
  // as the large operands' for a few cached bytes.
  __shared__ E sm[NIN][x_small_cap(NIN)];
  const E* src[NIN];
  uint32_t lanep[NIN], tw[NIN][kMaxLgTpb], tbase[NIN];
  R scale[NIN];
  int eacc = 0;
  bool any_small = false;
#pragma unroll
  for (int j = 0; j < NIN; ++j) {
    const DevIn& in = s.in[j];
    const E* blk = reinterpret_cast<const E*>(in.ptr) + (int64_t)pt * in.pt_stride + (int64_t)sb * in.sb_stride +
                   ((int64_t)pext_bits(sid, in.smask) << in.slow);
    tbase[j] = pext_tile(tile0, in) << in.has_v;
    src[j] = blk + tbase[j];
    if (in.small_n) {
      any_small = true;
      for (int i = (int)tid; i < in.small_n; i += kWG) sm[j][i] = blk[i];
    }
#pragma unroll
    for (int b = 0; b < kMaxLgTpb; ++b) tw[j][b] = b < s.lg_tpb ? pext_tile(1u << b, in) << in.has_v : 0u;
    lanep[j] = pext_runs(tid, in);
    scale[j] = (R)1;
    if (SCALED && in.exp_base >= 0) {
      const int slot = in.exp_base + (int)pt * in.exp_pt + (int)sb * in.exp_sb;
      const int sh = scale_shift(maxbits[slot]);
      scale[j] = (R)ldexp(1.0, -sh);
      eacc += exps[slot] + sh;
    }
  }
  // Inputs that no output bit indexes (the last s.n_uni: gates and factors
  // on v and slice variables alone) hold the same two values for every
  // output of the item: their product is formed once, here, and multiplies
  // the product of the others.
  E g0 = Cx<E>::one(), g1 = Cx<E>::one();
  const int nu = s.n_uni;
#pragma unroll
  for (int q = 0; q < kMaxIn - NIN; ++q) {
    if (q >= nu) break;
    const DevIn& in = s.in[NIN + q];
    const E* blk = reinterpret_cast<const E*>(in.ptr) + (int64_t)pt * in.pt_stride + (int64_t)sb * in.sb_stride +
                   ((int64_t)pext_bits(sid, in.smask) << in.slow);
    E u0 = blk[0], u1 = blk[in.has_v];
    if (SCALED && in.exp_base >= 0) {
      const int slot = in.exp_base + (int)pt * in.exp_pt + (int)sb * in.exp_sb;
      const int sh = scale_shift(maxbits[slot]);
      const R f = (R)ldexp(1.0, -sh);
      u0 = cscale(u0, f);
      u1 = cscale(u1, f);
      eacc += exps[slot] + sh;
    }
    g0 = q == 0 ? u0 : cmul(g0, u0);
    g1 = q == 0 ? u1 : cmul(g1, u1);
  }
  if (any_small) __syncthreads();
  E* const out = reinterpret_cast<E*>(s.out) + ((int64_t)item << s.r);
  float mx = 0.f;
  const uint32_t n_here = 1u << s.lg_tpb;
  for (uint32_t t = 0; t < n_here; ++t) {
    const uint32_t tile = tile0 + t;
    __amdgpu_buffer_rsrc_t rs[NIN];
    uint32_t tpart[NIN];
#pragma unroll
    for (int j = 0; j < NIN; ++j) {
      uint32_t part = 0;
#pragma unroll
      for (int b = 0; b < kMaxLgTpb; ++b) part += (t >> b) & 1u ? tw[j][b] : 0u;
      rs[j] = rsrc_of(src[j] + part);
      tpart[j] = tbase[j] + part;
    }
    E a0[kEPT][NIN], a1[kEPT][NIN];
#pragma unroll
    for (int e = 0; e < kEPT; ++e) {
#pragma unroll
      for (int j = 0; j < NIN; ++j) {
        const int hv = s.in[j].has_v;
        const uint32_t li = (s.in[j].ep[e] + lanep[j]) << hv;
        if (s.in[j].small_n) {
          a0[e][j] = sm[j][tpart[j] + li];
          a1[e][j] = sm[j][tpart[j] + li + (uint32_t)hv];
        } else if (hv) {
          Cx<E>::bload_pair(rs[j], li * (uint32_t)sizeof(E), a0[e][j], a1[e][j]);
        } else {
          a0[e][j] = Cx<E>::bload(rs[j], li * (uint32_t)sizeof(E));
          a1[e][j] = a0[e][j];
        }
      }
    }
    const __amdgpu_buffer_rsrc_t ro = rsrc_of(out + ((int64_t)tile << kLgTile));
    // product over the inputs in their order (a scaled input times its power
    // of two first; an unscaled one as loaded), then the uniform factor
    E t0[kEPT], t1[kEPT];
#pragma unroll
    for (int j = 0; j < NIN; ++j) {
      if (SCALED && s.in[j].exp_base >= 0) {
#pragma unroll
        for (int e = 0; e < kEPT; ++e) {
          a0[e][j] = cscale(a0[e][j], scale[j]);
          a1[e][j] = cscale(a1[e][j], scale[j]);
        }
      }
#pragma unroll
      for (int e = 0; e < kEPT; ++e) {
        t0[e] = j == 0 ? a0[e][0] : cmul(t0[e], a0[e][j]);
        t1[e] = j == 0 ? a1[e][0] : cmul(t1[e], a1[e][j]);
      }
    }
    if (nu) {
#pragma unroll
      for (int e = 0; e < kEPT; ++e) {
        t0[e] = cmul(t0[e], g0);
        t1[e] = cmul(t1[e], g1);
      }
    }
#pragma unroll
    for (int e = 0; e < kEPT; ++e) {
      const E res = s.sum ? cadd(t0[e], t1[e]) : t0[e];
      Cx<E>::bstore(ro, (((uint32_t)e << 8) | tid) * (uint32_t)sizeof(E), res);
      if (SCALED) mx = fmaxf(mx, abs_max(res));
    }
  }
  if (SCALED) {
    __shared__ float red[kWG / 64];
    mx = wave_max(mx);
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    __syncthreads();
    if (tid == 0) {
      float m = red[0];
#pragma unroll
      for (int w = 1; w < kWG / 64; ++w) m = fmaxf(m, red[w]);
      const int slot = s.out_exp_base + (int)pt * s.out_exp_pt + (int)sb * s.out_exp_sb;
      atomicMax(maxbits + slot, __float_as_uint(m));
      if (tile0 == 0) exps[slot] = eacc;
    }
  }
}

// SMALL mode: one output element per thread over the flattened
// (point, slice item, x) space; outputs smaller than a tile.
template <typename E, bool SCALED, int NIN>
__global__ __launch_bounds__(kWG) void k_step_small(const DevStep s, int* __restrict__ exps,
                                                    uint32_t* __restrict__ maxbits, int64_t n_elems) {
  using R = typename Cx<E>::R;
  const int64_t g0 = (int64_t)blockIdx.x * kWG + threadIdx.x;
  const bool valid = g0 < n_elems;
  const int64_t g = valid ? g0 : 0;
  const uint32_t x = (uint32_t)(g & ((1ll << s.r) - 1));
  const uint32_t item = (uint32_t)(g >> s.r);
  const uint32_t sb = item & ((1u << s.lg_nsb) - 1u);
  const uint32_t pt = item >> s.lg_nsb;
  const uint64_t sid = (uint64_t)s.chunk_base + sb;
  E a0[NIN], a1[NIN];
  R scale[NIN];
  int eacc = 0;
#pragma unroll
  for (int j = 0; j < NIN; ++j) {
    const DevIn& in = s.in[j];
    const int hv = in.has_v;
    const E* src = reinterpret_cast<const E*>(in.ptr) + (int64_t)pt * in.pt_stride + (int64_t)sb * in.sb_stride +
                   ((int64_t)pext_bits(sid, in.smask) << in.slow);
    const int64_t idx = (int64_t)pext_runs(x, in) << hv;
    a0[j] = src[idx];
    a1[j] = src[idx + hv];
    scale[j] = (R)1;
    if (SCALED && in.exp_base >= 0) {
      const int slot = in.exp_base + (int)pt * in.exp_pt + (int)sb * in.exp_sb;
      const int sh = scale_shift(maxbits[slot]);
      scale[j] = (R)ldexp(1.0, -sh);
      eacc += exps[slot] + sh;
    }
  }
  E t0 = cscale(a0[0], scale[0]), t1 = cscale(a1[0], scale[0]);
#pragma unroll
  for (int j = 1; j < NIN; ++j) {
    t0 = cmul(t0, cscale(a0[j], scale[j]));
    t1 = cmul(t1, cscale(a1[j], scale[j]));
  }
  const E res = s.sum ? cadd(t0, t1) : t0;
  if (valid) reinterpret_cast<E*>(s.out)[g] = res;
  if (SCALED) {
    float m = valid ? abs_max(res) : 0.f;
    const int seg = s.r < 6 ? s.r : 6;
    for (int o = 1; o < (1 << seg); o <<= 1) m = fmaxf(m, __shfl_xor(m, o));
    const uint32_t lane = threadIdx.x & 63;
    if (valid && (lane & ((1u << seg) - 1u)) == 0) {
      const int slot = s.out_exp_base + (int)pt * s.out_exp_pt + (int)sb * s.out_exp_sb;
      atomicMax(maxbits + slot, __float_as_uint(m));
      if (x == 0) exps[slot] = eacc;
    }
  }
}

// Gate tensors from (gamma, beta), FP64 trigonometry rounded to the element
// type (Section III-A conventions; see qtensor_hip.h for each kind).
template <typename E>
__global__ void k_leaves(const DevLeaf* __restrict__ leaves, int n_leaves, int leaf_block,
                         const double* __restrict__ dense, double* __restrict__ params,
                         const double* __restrict__ gammas, const double* __restrict__ betas, int p,
                         int n_points, E* __restrict__ out, uint32_t* __restrict__ clear, int64_t n_clear) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // scale slots the run starts from zero (its first fill, folded in here)
  for (int64_t i = t; i < n_clear; i += (int64_t)gridDim.x * blockDim.x) clear[i] = 0u;
  // parameters given in device memory ([points][p] each): read from there,
  // and laid out as [points][2p] (gammas, then betas) for the later launches
  if (gammas) {
    const int64_t n2 = (int64_t)n_points * 2 * p;
    for (int64_t i = t; i < n2; i += (int64_t)gridDim.x * blockDim.x) {
      const int64_t q = i / (2 * p), k = i - q * 2 * p;
      params[i] = k < p ? gammas[q * p + k] : betas[q * p + k - p];
    }
  }
  if (t >= (int64_t)n_leaves * n_points) return;
  const int pt = (int)(t / n_leaves);
  const DevLeaf L = leaves[t % n_leaves];
  E* o = out + (int64_t)pt * leaf_block + L.off;
  const double* const gp = gammas ? gammas + (int64_t)pt * p : params + (int64_t)pt * 2 * p;
  const double* const bp = gammas ? betas + (int64_t)pt * p : params + (int64_t)pt * 2 * p + p;
  switch (L.kind) {
    case QT_T_VEC_PLUS:
      o[0] = Cx<E>::from(1.0, 0.0);
      o[1] = Cx<E>::from(1.0, 0.0);
      break;
    case QT_T_BRA_BIT:
      o[0] = Cx<E>::from(L.layer == 0 ? 1.0 : 0.0, 0.0);
      o[1] = Cx<E>::from(L.layer == 0 ? 0.0 : 1.0, 0.0);
      break;
    case QT_T_ZZ:
    case QT_T_ZZ_DAG: {
      double sn, cs;
      sincos(gp[L.layer - 1], &sn, &cs);
      const double im = L.kind == QT_T_ZZ ? -sn : sn;
      o[0] = Cx<E>::from(1.0, 0.0);
      o[1] = Cx<E>::from(cs, im);
      o[2] = Cx<E>::from(cs, im);
      o[3] = Cx<E>::from(1.0, 0.0);
      break;
    }
    case QT_T_RX:
    case QT_T_RX_DAG: {
      double sn, cs;
      sincos(bp[L.layer - 1], &sn, &cs);
      const double im = L.kind == QT_T_RX ? -sn : sn;
      o[0] = Cx<E>::from(cs, 0.0);
      o[1] = Cx<E>::from(0.0, im);
      o[2] = Cx<E>::from(0.0, im);
      o[3] = Cx<E>::from(cs, 0.0);
      break;
    }
    case QT_T_OBS_CUT:
      o[0] = Cx<E>::from(0.0, 0.0);
      o[1] = Cx<E>::from(1.0, 0.0);
      o[2] = Cx<E>::from(1.0, 0.0);
      o[3] = Cx<E>::from(0.0, 0.0);
      break;
    default: {  // DENSE, already permuted to storage order on the host
      const int n = 1 << L.rank;
      for (int i = 0; i < n; ++i) o[i] = Cx<E>::from(dense[2 * (L.dense_off + i)], dense[2 * (L.dense_off + i) + 1]);
    }
  }
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Sum over a range of slices of one result row (a workgroup of 256
// threads): the largest exponent of the nonzero values, then each value
// rescaled to it, weighted, in a fixed order of partial sums.
__device__ __forceinline__ void x_slice_sum_block(const double* __restrict__ ps, int64_t n_range,
                                                  const double* __restrict__ w, double* __restrict__ out,
                                                  double* sre, double* sim) {
  const int tid = threadIdx.x;
  double emax = -INFINITY;
  for (int64_t i = tid; i < n_range; i += 256)
    if (ps[3 * i] != 0.0 || ps[3 * i + 1] != 0.0) emax = fmax(emax, ps[3 * i + 2]);
  sre[tid] = emax;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) sre[tid] = fmax(sre[tid], sre[tid + o]);
    __syncthreads();
  }
  emax = sre[0];
  __syncthreads();
  double re = 0.0, im = 0.0;
  if (emax != -INFINITY) {
    for (int64_t i = tid; i < n_range; i += 256) {
      const double d = ps[3 * i + 2] - emax;
      if (ps[3 * i] != 0.0 || ps[3 * i + 1] != 0.0) {
        const double f = exp2(d - (int)d) * (w ? w[i] : 1.0);
        re += ldexp(ps[3 * i], (int)d) * f;
        im += ldexp(ps[3 * i + 1], (int)d) * f;
      }
    }
  }
  sre[tid] = re;
  sim[tid] = im;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      sre[tid] += sre[tid + o];
      sim[tid] += sim[tid + o];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = sre[0];
    out[1] = sim[0];
    out[2] = emax == -INFINITY ? 0.0 : emax;
  }
}

// Per-slice value: product of the plan's closing factors (results of
// buckets that closed to a scalar, Algorithm 1 "result <- result * R"), with
// its exponent, in FP64.  With open output variables the closing factors
// are tensors over subsets of them, and thread (item, j) forms output
// element j (the open variables' values): the product of every factor at
// the bits of j it holds (its runs over j), i.e. their outer product.
template <typename E, bool SCALED>
__device__ __forceinline__ void x_final_value(const DevFinal& f, const DevIn* __restrict__ fac,
                                              const int* __restrict__ exps, const uint32_t* __restrict__ maxbits,
                                              double* __restrict__ per_slice, double* __restrict__ sums,
                                              int sum_mode, uint32_t oj, uint32_t sb, uint32_t pt, uint64_t sid) {
  double re = 1.0, im = 0.0, ex = f.log2_const;
  for (int j = 0; j < f.n_factors; ++j) {
    const DevIn in = fac[j];
    const int64_t idx = (int64_t)pt * in.pt_stride + (int64_t)sb * in.sb_stride +
                        ((int64_t)pext_bits(sid, in.smask) << in.slow) + (int64_t)pext_runs(oj, in);
    const E a = reinterpret_cast<const E*>(in.ptr)[idx];
    double ar = (double)a.x, ai = (double)a.y;
    if (SCALED && in.exp_base >= 0) {
      const int slot = in.exp_base + (int)pt * in.exp_pt + (int)sb * in.exp_sb;
      const int sh = scale_shift(maxbits[slot]);
      ar = ldexp(ar, -sh);
      ai = ldexp(ai, -sh);
      ex += exps[slot] + sh;
    }
    const double nr = re * ar - im * ai;
    im = re * ai + im * ar;
    re = nr;
  }
  double* o = per_slice + 3 * ((((int64_t)pt << f.n_open) + oj) * f.n_range + (int64_t)(sid - f.slice_begin));
  o[0] = re;
  o[1] = im;
  o[2] = ex;
  if (sum_mode == 1) {
    // a range of one slice: its sum, as k_slice_sum forms it (a zero value
    // reported with exponent 0)
    const bool nz = re != 0.0 || im != 0.0;
    double* s = sums + 3 * (((int64_t)pt << f.n_open) + oj);
    s[0] = nz ? 0.0 + re : 0.0;
    s[1] = nz ? 0.0 + im : 0.0;
    s[2] = nz ? ex : 0.0;
  }
}

template <typename E, bool SCALED>
__global__ void k_final(const DevFinal f, const DevIn* __restrict__ fac, int n_points, int64_t n_items,
                        const int* __restrict__ exps, const uint32_t* __restrict__ maxbits,
                        double* __restrict__ per_slice, int64_t slice_end, double* __restrict__ sums,
                        int sum_mode) {
  const int64_t tj = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t oj = (uint32_t)(tj & ((1ll << f.n_open) - 1));  // open output index
  const int64_t t = tj >> f.n_open;
  const uint32_t sb = (uint32_t)(t & ((1ll << f.lg_nsb) - 1));
  const uint32_t pt = (uint32_t)(t >> f.lg_nsb);
  const uint64_t sid = (uint64_t)f.chunk_base + sb;
  if (tj < (n_items << f.n_open) && (int64_t)sid >= f.slice_begin && (int64_t)sid < slice_end)
    x_final_value<E, SCALED>(f, fac, exps, maxbits, per_slice, sums, sum_mode, oj, sb, pt, sid);
  if (sum_mode == 2) {
    // the whole range in this one workgroup (one point, no open output):
    // its sum, as k_slice_sum forms it
    __shared__ double sre[256], sim[256];
    __syncthreads();
    x_slice_sum_block(per_slice, f.n_range, nullptr, sums, sre, sim);
  }
}

// Deterministic FP64 sum over slices (Algorithm 1's final reduction): common
// exponent = max over non-zero slices, thread t adds slices t, t+256, ... in
// order, then a fixed-shape tree over the 256 partial sums.  With weights w
// (non-negative), slice i enters w[i] times (the same sum over edges whose
// lightcones are deduplicated: each class once, times its size).
__global__ __launch_bounds__(256) void k_slice_sum(const double* __restrict__ per_slice, int64_t n_range,
                                                   const double* __restrict__ w, double* __restrict__ out) {
  __shared__ double sre[256], sim[256];
  const int pt = blockIdx.x;
  x_slice_sum_block(per_slice + 3 * (int64_t)pt * n_range, n_range, w, out + 3 * pt, sre, sim);
}

}  // namespace

hipError_t launch_leaves(const DevLeaf* leaves, int n_leaves, int leaf_block, const double* dense,
                         double* params, const double* gammas, const double* betas, int p, int n_points,
                         void* out, bool c128, hipStream_t stream, uint32_t* clear, int64_t n_clear) {
  int64_t n = std::max<int64_t>((int64_t)n_leaves * n_points, gammas ? (int64_t)n_points * 2 * p : 0);
  n = std::max<int64_t>(n, std::min<int64_t>(n_clear, (int64_t)1 << 20));  // the clear strides over the grid
  if (n == 0) return hipSuccess;
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (c128)
    hipLaunchKernelGGL(k_leaves<double2>, grid, block, 0, stream, leaves, n_leaves, leaf_block, dense, params,
                       gammas, betas, p, n_points, reinterpret_cast<double2*>(out), clear, n_clear);
  else
    hipLaunchKernelGGL(k_leaves<float2>, grid, block, 0, stream, leaves, n_leaves, leaf_block, dense, params,
                       gammas, betas, p, n_points, reinterpret_cast<float2*>(out), clear, n_clear);
  return hipGetLastError();
}

namespace {

template <typename E, bool SCALED, int NIN>
void launch_step_t(const DevStep& s, int* exps, uint32_t* maxbits, int64_t n_elems, hipStream_t stream) {
  if (s.r >= kLgTile) {
    DevStep t = s;
    t.lg_tiles = s.r - kLgTile;
    // a few tiles per workgroup: the per-item setup and the output max are
    // paid once per group of tiles
    t.lg_tpb = std::min(std::min(t.lg_tiles, kMaxLgTpb), std::max(0, s.lg_tpb));
    hipLaunchKernelGGL((k_step_big<E, SCALED, NIN>), dim3((unsigned)(n_elems >> (kLgTile + t.lg_tpb))), dim3(kWG), 0,
                       stream, t, exps, maxbits);
  } else {
    hipLaunchKernelGGL((k_step_small<E, SCALED, NIN>), dim3((unsigned)((n_elems + kWG - 1) / kWG)), dim3(kWG), 0,
                       stream, s, exps, maxbits, n_elems);
  }
}

template <typename E, bool SCALED>
void launch_step_n(const DevStep& s0, int* exps, uint32_t* maxbits, int64_t n_elems, hipStream_t stream) {
  DevStep s = s0;
  int nin = s.n_in;
  if (s.r >= kLgTile) {
    // inputs that no output bit indexes go last; the big kernel multiplies
    // their product in once per item (and stages only the others)
    DevIn tmp[kMaxIn];
    int k = 0;
    for (int j = 0; j < s.n_in; ++j)
      if (s.in[j].nruns != 0) tmp[k++] = s.in[j];
    const int nn = k;
    for (int j = 0; j < s.n_in; ++j)
      if (s.in[j].nruns == 0) tmp[k++] = s.in[j];
    if (nn > 0 && nn < s.n_in) {
      for (int j = 0; j < s.n_in; ++j) s.in[j] = tmp[j];
      for (int j = 0; j < nn; ++j)
        if (s.in[j].small_n > x_small_cap(nn)) s.in[j].small_n = 0;
      s.n_uni = s.n_in - nn;
      nin = nn;
    }
  }
  switch (nin) {
    case 1: launch_step_t<E, SCALED, 1>(s, exps, maxbits, n_elems, stream); break;
    case 2: launch_step_t<E, SCALED, 2>(s, exps, maxbits, n_elems, stream); break;
    case 3: launch_step_t<E, SCALED, 3>(s, exps, maxbits, n_elems, stream); break;
    case 4: launch_step_t<E, SCALED, 4>(s, exps, maxbits, n_elems, stream); break;
    case 5: launch_step_t<E, SCALED, 5>(s, exps, maxbits, n_elems, stream); break;
    case 6: launch_step_t<E, SCALED, 6>(s, exps, maxbits, n_elems, stream); break;
    case 7: launch_step_t<E, SCALED, 7>(s, exps, maxbits, n_elems, stream); break;
    default: launch_step_t<E, SCALED, 8>(s, exps, maxbits, n_elems, stream); break;
  }
}

}  // namespace

hipError_t launch_step(const DevStep& s, bool c128, bool scaled, int* exps, uint32_t* maxbits, int64_t n_elems,
                       hipStream_t stream, int* n_launches, int* kclass) {
  if (n_elems == 0) return hipSuccess;
  if (s.n_in < 1 || s.n_in > kMaxIn) return hipErrorInvalidValue;
  if (n_launches) ++*n_launches;
  if (kclass) *kclass = s.r >= kLgTile ? QT_KCLASS_STEP_STREAM : QT_KCLASS_STEP_SMALL;
  if (c128)
    launch_step_n<double2, false>(s, exps, maxbits, n_elems, stream);
  else if (scaled)
    launch_step_n<float2, true>(s, exps, maxbits, n_elems, stream);
  else
    launch_step_n<float2, false>(s, exps, maxbits, n_elems, stream);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t value, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, n, value);
  return hipGetLastError();
}

hipError_t launch_final(const DevFinal& f, const DevIn* factors, int n_points, int64_t n_items, bool c128,
                        bool scaled, const int* exps, const uint32_t* maxbits, double* per_slice,
                        int64_t slice_end, hipStream_t stream, double* sums, int sum_mode) {
  const int64_t n = n_items << f.n_open;
  // sums: 1, a range of one slice; 2, the whole range in one workgroup (one
  // point, no open output)
  if (sum_mode < 0 || sum_mode > 2 || (sum_mode && !sums) || (sum_mode == 1 && f.n_range != 1) ||
      (sum_mode == 2 && (n_points != 1 || f.n_open != 0 || n > 256)))
    return hipErrorInvalidValue;
  if (n > 0x7fffffffll * 256) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (c128)
    hipLaunchKernelGGL((k_final<double2, false>), grid, block, 0, stream, f, factors, n_points, n_items, exps,
                       maxbits, per_slice, slice_end, sums, sum_mode);
  else if (scaled)
    hipLaunchKernelGGL((k_final<float2, true>), grid, block, 0, stream, f, factors, n_points, n_items, exps,
                       maxbits, per_slice, slice_end, sums, sum_mode);
  else
    hipLaunchKernelGGL((k_final<float2, false>), grid, block, 0, stream, f, factors, n_points, n_items, exps,
                       maxbits, per_slice, slice_end, sums, sum_mode);
  return hipGetLastError();
}

hipError_t launch_slice_sum(const double* per_slice, int n_points, int64_t n_range, double* out,
                            hipStream_t stream, const double* weights) {
  hipLaunchKernelGGL(k_slice_sum, dim3(n_points), dim3(256), 0, stream, per_slice, n_range, weights, out);
  return hipGetLastError();
}

}  // namespace qt
