// Fused GEMM bucket on the matrix cores: for every batch item (point,
// slice) and batch index b,
//   C[b, m, n] = sum_k A[b, m, k] * B[b, n, k]        (complex64)
// with the power-of-two scaling of the other bucket steps (each operand
// block is multiplied by 2^-shift of its measured max on load, the output
// exponent is the sum of the operands' exponents and shifts, and the
// output max is collected for the next consumer).
//
// A workgroup (4 wavefronts) computes one TM x TN tile of C for one (item,
// b).  Per K stage it gathers a TM x TK block of A and a TN x TK block of B
// through their bit maps into LDS, split into real and imaginary planes;
// each wavefront owns a 16 x 16 sub-tile and accumulates it in FP32 with
// v_mfma_f32_16x16x4_f32: per 4-deep slice of K, four products form
//   Re += Ar Br - Ai Bi,   Im += Ar Bi + Ai Br.
// Operand lane layout of that instruction (16 x 4 A, 4 x 16 B, 16 x 16 D):
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16], and holds
// D[4 (l / 16) + r][l % 16] in accumulator register r.
// Each K stage is accumulated from zero and added to the running total with
// Kahan compensation, so the rounding error grows with the stage depth (16)
// plus a constant rather than with K (up to 2^20 here).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "qt_internal.h"

namespace qt {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kGThreads = 256;
constexpr int kTK = 16;

__device__ __forceinline__ uint32_t gmap(const GMap& g, uint32_t x) {
  uint32_t r = 0;
  for (int i = 0; i < g.n; ++i) r |= ((x >> g.lo[i]) & ((1u << g.len[i]) - 1u)) << g.dst[i];
  return r;
}

__device__ __forceinline__ uint32_t gpext(uint64_t x, uint32_t m) {
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

__device__ __forceinline__ int gshift(uint32_t maxbits) {
  if (maxbits == 0) return 0;
  const int s = ilogbf(__uint_as_float(maxbits)) + 1;
  return s < -126 ? -126 : (s > 127 ? 127 : s);
}

template <int TM, int TN>
__global__ __launch_bounds__(kGThreads) void k_gemm(const DevGemm g, int* __restrict__ exps,
                                                    uint32_t* __restrict__ maxbits, uint32_t tiles_per_block,
                                                    uint64_t n_tiles) {
  constexpr int kLgM = TM == 32 ? 5 : 4, kLgN = TN == 32 ? 5 : 4;
  constexpr int kTileBits = kLgM + kLgN;
  __shared__ float sAr[TM][kTK + 1], sAi[TM][kTK + 1], sBr[TN][kTK + 1], sBi[TN][kTK + 1];
  __shared__ float sCr[TM * (TN + 1)], sCi[TM * (TN + 1)];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;

  // Output order: the tile's bits sorted by their position in C, so that
  // consecutive threads write consecutive addresses where C's low bits are
  // tile bits.  Bit j of a write index t carries C offset cw[j] and LDS
  // offset lw[j] (all wavefront-uniform).
  uint32_t cw[kTileBits], lw[kTileBits];
  {
    uint32_t pos[kTileBits];
#pragma unroll
    for (int i = 0; i < kTileBits; ++i) {
      const bool isn = i >= kLgM;
      const int bit = isn ? i - kLgM : i;
      cw[i] = isn ? gmap(g.c_n, 1u << bit) : gmap(g.c_m, 1u << bit);
      lw[i] = isn ? (1u << bit) : (1u << bit) * (TN + 1);
      pos[i] = cw[i];
    }
    for (int i = 1; i < kTileBits; ++i)  // insertion sort by C offset (tiny, uniform)
      for (int j = i; j > 0 && pos[j - 1] > pos[j]; --j) {
        uint32_t t = pos[j]; pos[j] = pos[j - 1]; pos[j - 1] = t;
        t = cw[j]; cw[j] = cw[j - 1]; cw[j - 1] = t;
        t = lw[j]; lw[j] = lw[j - 1]; lw[j - 1] = t;
      }
  }

  const uint32_t n_nt = (1u << g.nn) / TN, n_mt = (1u << g.nm) / TM;
  const uint32_t K = 1u << g.nk;
  const int tk = K < (uint32_t)kTK ? (int)K : kTK;  // K >= 8
  constexpr int kALoads = (TM * kTK + kGThreads - 1) / kGThreads, kBLoads = (TN * kTK + kGThreads - 1) / kGThreads;
  constexpr int kSubN = TN / 16;
  constexpr int kSubs = (TM / 16) * kSubN;
  const int wm = wave / kSubN, wn = wave % kSubN;
  const int li = lane & 15, lk = lane >> 4;

  for (uint32_t it = 0; it < tiles_per_block; ++it) {
    const uint64_t tile_id = (uint64_t)blockIdx.x * tiles_per_block + it;
    if (tile_id >= n_tiles) break;
    // tile -> (n tile, m tile, batch index, item), n tile fastest
    uint64_t bid = tile_id;
    const uint32_t nt = (uint32_t)(bid % n_nt);
    bid /= n_nt;
    const uint32_t mt = (uint32_t)(bid % n_mt);
    bid /= n_mt;
    const uint32_t bb = (uint32_t)(bid & ((1ull << g.nb) - 1ull));
    const uint32_t item = (uint32_t)(bid >> g.nb);
    const uint32_t sb = item & ((1u << g.lg_nsb) - 1u);
    const uint32_t pt = item >> g.lg_nsb;
    const uint64_t sid = (uint64_t)g.chunk_base + sb;

    const float2* A = reinterpret_cast<const float2*>(g.a) + (int64_t)pt * g.a_pt + (int64_t)sb * g.a_sb +
                      ((int64_t)gpext(sid, g.a_smask) << g.a_slow) + gmap(g.a_b, bb);
    const float2* B = reinterpret_cast<const float2*>(g.b) + (int64_t)pt * g.b_pt + (int64_t)sb * g.b_sb +
                      ((int64_t)gpext(sid, g.b_smask) << g.b_slow) + gmap(g.b_b, bb);
    float2* C = reinterpret_cast<float2*>(g.c) + (int64_t)pt * g.c_pt + (int64_t)sb * g.c_sb + gmap(g.c_b, bb) +
                gmap(g.c_m, mt * TM) + gmap(g.c_n, nt * TN);

    float sa = 1.f, sbs = 1.f;
    int eacc = 0;
    if (g.a_exp_base >= 0) {
      const int slot = g.a_exp_base + (int)pt * g.a_exp_pt + (int)sb * g.a_exp_sb;
      const int sh = gshift(maxbits[slot]);
      sa = __int_as_float((127 - sh) << 23);
      eacc += exps[slot] + sh;
    }
    if (g.b_exp_base >= 0) {
      const int slot = g.b_exp_base + (int)pt * g.b_exp_pt + (int)sb * g.b_exp_sb;
      const int sh = gshift(maxbits[slot]);
      sbs = __int_as_float((127 - sh) << 23);
      eacc += exps[slot] + sh;
    }

    // per-thread load coordinates (fixed over the K loop); the k part of an
    // index splits as map(k0) + map(ki) because k0 is a multiple of tk
    uint32_t a_off[kALoads], a_ki[kALoads], b_off[kBLoads], b_ki[kBLoads];
    int a_mi[kALoads], b_ni[kBLoads];
#pragma unroll
    for (int q = 0; q < kALoads; ++q) {
      const int e = tid + q * kGThreads;
      a_mi[q] = e / tk;
      a_ki[q] = (uint32_t)(e % tk);
      a_off[q] = gmap(g.a_m, mt * TM + (uint32_t)a_mi[q]) + gmap(g.a_k, a_ki[q]);
    }
#pragma unroll
    for (int q = 0; q < kBLoads; ++q) {
      const int e = tid + q * kGThreads;
      b_ni[q] = e / tk;
      b_ki[q] = (uint32_t)(e % tk);
      b_off[q] = gmap(g.b_n, nt * TN + (uint32_t)b_ni[q]) + gmap(g.b_k, b_ki[q]);
    }

    v4f totR = {0.f, 0.f, 0.f, 0.f}, totI = {0.f, 0.f, 0.f, 0.f};  // running sums
    v4f cmpR = {0.f, 0.f, 0.f, 0.f}, cmpI = {0.f, 0.f, 0.f, 0.f};  // their compensations
    float2 va[kALoads], vb[kBLoads];
    auto fetch = [&](uint32_t k0) {
      const uint32_t ka = gmap(g.a_k, k0), kb = gmap(g.b_k, k0);
#pragma unroll
      for (int q = 0; q < kALoads; ++q)
        if (a_mi[q] < TM) va[q] = A[a_off[q] + ka];
#pragma unroll
      for (int q = 0; q < kBLoads; ++q)
        if (b_ni[q] < TN) vb[q] = B[b_off[q] + kb];
    };
    fetch(0);
    for (uint32_t k0 = 0; k0 < K; k0 += (uint32_t)tk) {
#pragma unroll
      for (int q = 0; q < kALoads; ++q)
        if (a_mi[q] < TM) {
          sAr[a_mi[q]][a_ki[q]] = va[q].x * sa;
          sAi[a_mi[q]][a_ki[q]] = va[q].y * sa;
        }
#pragma unroll
      for (int q = 0; q < kBLoads; ++q)
        if (b_ni[q] < TN) {
          sBr[b_ni[q]][b_ki[q]] = vb[q].x * sbs;
          sBi[b_ni[q]][b_ki[q]] = vb[q].y * sbs;
        }
      __syncthreads();
      if (k0 + (uint32_t)tk < K) fetch(k0 + (uint32_t)tk);  // next stage in flight during the products
      if (wave < kSubs) {
        v4f accR = {0.f, 0.f, 0.f, 0.f}, accI = {0.f, 0.f, 0.f, 0.f};
        for (int kk = 0; kk < tk; kk += 4) {
          const float ar = sAr[wm * 16 + li][kk + lk], ai = sAi[wm * 16 + li][kk + lk];
          const float br = sBr[wn * 16 + li][kk + lk], bi = sBi[wn * 16 + li][kk + lk];
          accR = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, accR, 0, 0, 0);
          accR = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, bi, accR, 0, 0, 0);
          accI = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bi, accI, 0, 0, 0);
          accI = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br, accI, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float yr = accR[r] - cmpR[r], tr = totR[r] + yr;
          cmpR[r] = (tr - totR[r]) - yr;
          totR[r] = tr;
          const float yi = accI[r] - cmpI[r], ti = totI[r] + yi;
          cmpI[r] = (ti - totI[r]) - yi;
          totI[r] = ti;
        }
      }
      __syncthreads();
    }

    // stage the tile in LDS, then write it in C order
    if (wave < kSubs) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = (wm * 16 + 4 * lk + r) * (TN + 1) + wn * 16 + li;
        sCr[o] = totR[r];
        sCi[o] = totI[r];
      }
    }
    __syncthreads();
    float m = 0.f;
#pragma unroll
    for (int q = 0; q < (TM * TN) / kGThreads; ++q) {
      const uint32_t t = (uint32_t)(tid + q * kGThreads);
      uint32_t co = 0, lo = 0;
#pragma unroll
      for (int j = 0; j < kTileBits; ++j)
        if ((t >> j) & 1u) {
          co += cw[j];
          lo += lw[j];
        }
      float2 v;
      v.x = sCr[lo];
      v.y = sCi[lo];
      C[co] = v;
      m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
    if (g.c_exp_base >= 0) {
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) m = fmaxf(m, __shfl_xor(m, off));
      const int slot = g.c_exp_base + (int)pt * g.c_exp_pt + (int)sb * g.c_exp_sb;
      if (lane == 0) atomicMax(maxbits + slot, __float_as_uint(m));
      if (tid == 0 && bb == 0 && mt == 0 && nt == 0) exps[slot] = eacc;
    }
    __syncthreads();  // sC is rewritten by the next tile
  }
}

template <int TM, int TN>
hipError_t go(const DevGemm& g, int* exps, uint32_t* maxbits, hipStream_t stream) {
  const uint64_t n_tiles = ((uint64_t)g.n_items << g.nb) * ((1ull << g.nm) / TM) * ((1ull << g.nn) / TN);
  if (n_tiles == 0) return hipSuccess;
  // short-K products get several tiles per workgroup (their setup is a
  // large part of a tile's work); keep >= 16K workgroups in flight
  const uint32_t tpb = g.nk <= 5 ? (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(8, n_tiles / 16384)) : 1u;
  const uint64_t grid = (n_tiles + tpb - 1) / tpb;
  if (grid > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_gemm<TM, TN>), dim3((unsigned)grid), dim3(kGThreads), 0, stream, g, exps, maxbits, tpb,
                     n_tiles);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm(const DevGemm& g, bool scaled, int* exps, uint32_t* maxbits, hipStream_t stream) {
  if (!scaled || g.nm < 4 || g.nn < 4 || g.nk < 3) return hipErrorInvalidValue;
  const bool m32 = g.nm >= 5, n32 = g.nn >= 5;
  if (m32 && n32) return go<32, 32>(g, exps, maxbits, stream);
  if (m32) return go<32, 16>(g, exps, maxbits, stream);
  if (n32) return go<16, 32>(g, exps, maxbits, stream);
  return go<16, 16>(g, exps, maxbits, stream);
}

}  // namespace qt
