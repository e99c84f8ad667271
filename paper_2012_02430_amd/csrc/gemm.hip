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

// Unrolled with an early exit: every table read has a constant offset, so
// the tables stay scalar kernel-argument loads (a loop-indexed read of the
// by-value argument became dependent vector loads).
__device__ __forceinline__ uint32_t gmap(const GMap& g, uint32_t x) {
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < kGRuns; ++i) {
    if (i >= g.n) break;
    r |= ((x >> g.lo[i]) & ((1u << g.len[i]) - 1u)) << g.dst[i];
  }
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

// Tile: NB = 2^TB batch indices x TM = 2^LM rows x TN = 2^LN columns, the
// low bits of the b, m and n counters.  The host picks (TB, LM, LN) so that
// the tile's bits are C's lowest storage bits where it can, which makes the
// tile's output one contiguous block.  Wavefront w owns the 16 x 16
// sub-tile (batch, m block, n block) number w.
template <int TB, int LM, int LN>
__global__ __launch_bounds__(kGThreads) void k_gemm(const DevGemm g, int* __restrict__ exps,
                                                    uint32_t* __restrict__ maxbits, uint32_t tiles_per_block,
                                                    uint64_t n_tiles) {
  constexpr int NB = 1 << TB, TM = 1 << LM, TN = 1 << LN;
  constexpr int kARows = NB * TM, kBRows = NB * TN;
  constexpr int kTileBits = TB + LM + LN;
  constexpr int kTileElems = NB * TM * TN;
  constexpr int kSubM = TM / 16, kSubN = TN / 16;
  constexpr int kSubs = NB * kSubM * kSubN;
  static_assert(kSubs <= kGThreads / 64, "one 16 x 16 sub-tile per wavefront");
  __shared__ float sAr[kARows][kTK + 1], sAi[kARows][kTK + 1], sBr[kBRows][kTK + 1], sBi[kBRows][kTK + 1];
  __shared__ float sCr[NB * TM * (TN + 1)], sCi[NB * TM * (TN + 1)];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;

  // Output order: the tile's bits sorted by their position in C; bit j of a
  // write index t carries C offset cw[j] and staging offset lw[j].
  uint32_t cw[kTileBits], lw[kTileBits];
  {
    uint32_t pos[kTileBits];
#pragma unroll
    for (int i = 0; i < kTileBits; ++i) {
      if (i < TB) {
        cw[i] = gmap(g.c_b, 1u << i);
        lw[i] = (1u << i) * TM * (TN + 1);
      } else if (i < TB + LM) {
        cw[i] = gmap(g.c_m, 1u << (i - TB));
        lw[i] = (1u << (i - TB)) * (TN + 1);
      } else {
        cw[i] = gmap(g.c_n, 1u << (i - TB - LM));
        lw[i] = 1u << (i - TB - LM);
      }
      pos[i] = cw[i];
    }
    for (int i = 1; i < kTileBits; ++i)  // insertion sort by C offset (tiny, uniform)
      for (int j = i; j > 0 && pos[j - 1] > pos[j]; --j) {
        uint32_t t = pos[j]; pos[j] = pos[j - 1]; pos[j - 1] = t;
        t = cw[j]; cw[j] = cw[j - 1]; cw[j - 1] = t;
        t = lw[j]; lw[j] = lw[j - 1]; lw[j - 1] = t;
      }
  }

  const uint32_t n_nt = (1u << g.nn) / TN, n_mt = (1u << g.nm) / TM, n_bt = (1u << g.nb) / NB;
  const uint32_t K = 1u << g.nk;
  const int tk = K < (uint32_t)kTK ? (int)K : kTK;  // K >= 8
  constexpr int kALoads = (kARows * kTK + kGThreads - 1) / kGThreads;
  constexpr int kBLoads = (kBRows * kTK + kGThreads - 1) / kGThreads;
  constexpr int kCWrites = (kTileElems + kGThreads - 1) / kGThreads;
  const int wb = wave / (kSubM * kSubN), wm = (wave / kSubN) % kSubM, wn = wave % kSubN;
  const int li = lane & 15, lk = lane >> 4;

  // Per-thread parts of every index, the same for all tiles: maps are
  // linear over disjoint bits, so an element's offset is its in-tile part
  // plus the tile's base (uniform).  Row r of the A block is (batch r / TM,
  // m r % TM), k part ki.  A thread's elements are numbered with the block's
  // bits sorted by their storage position, so consecutive lanes load
  // consecutive addresses wherever the layout allows.
  uint32_t a_loc[kALoads], a_ki[kALoads], b_loc[kBLoads], b_ki[kBLoads], c_loc[kCWrites], s_loc[kCWrites];
  int a_r[kALoads], b_r[kBLoads];
  const int lg_tk = tk == 16 ? 4 : 3;
  auto number = [&](const GMap& mb, const GMap& mx, const GMap& mk, int lx, int nq, int rows, uint32_t* loc,
                    uint32_t* kis, int* rs) {
    // block bits: batch (TB), m or n (lx), k (lg_tk), each with its storage offset, row and k weights
    constexpr int kMaxBits = 2 + 5 + 4;
    uint32_t off[kMaxBits], rw[kMaxBits], kw[kMaxBits];
    const int nbits = TB + lx + lg_tk;
    for (int i = 0; i < nbits; ++i) {
      if (i < TB) {
        off[i] = gmap(mb, 1u << i);
        rw[i] = (1u << i) << lx;
        kw[i] = 0;
      } else if (i < TB + lx) {
        off[i] = gmap(mx, 1u << (i - TB));
        rw[i] = 1u << (i - TB);
        kw[i] = 0;
      } else {
        off[i] = gmap(mk, 1u << (i - TB - lx));
        rw[i] = 0;
        kw[i] = 1u << (i - TB - lx);
      }
    }
    for (int i = 1; i < nbits; ++i)  // by storage offset
      for (int j = i; j > 0 && off[j - 1] > off[j]; --j) {
        uint32_t t = off[j]; off[j] = off[j - 1]; off[j - 1] = t;
        t = rw[j]; rw[j] = rw[j - 1]; rw[j - 1] = t;
        t = kw[j]; kw[j] = kw[j - 1]; kw[j - 1] = t;
      }
    for (int q = 0; q < nq; ++q) {
      const uint32_t e = (uint32_t)(tid + q * kGThreads);
      uint32_t o = 0, r = 0, k = 0;
      for (int j = 0; j < nbits; ++j)
        if ((e >> j) & 1u) {
          o += off[j];
          r += rw[j];
          k += kw[j];
        }
      loc[q] = o;
      rs[q] = e < (uint32_t)(rows * tk) ? (int)r : rows;  // rows: no element
      kis[q] = k;
    }
  };
  number(g.a_b, g.a_m, g.a_k, LM, kALoads, kARows, a_loc, a_ki, a_r);
  number(g.b_b, g.b_n, g.b_k, LN, kBLoads, kBRows, b_loc, b_ki, b_r);
#pragma unroll
  for (int q = 0; q < kCWrites; ++q) {
    const uint32_t t = (uint32_t)(tid + q * kGThreads);
    uint32_t co = 0, lo = 0;
#pragma unroll
    for (int j = 0; j < kTileBits; ++j)
      if ((t >> j) & 1u) {
        co += cw[j];
        lo += lw[j];
      }
    c_loc[q] = co;
    s_loc[q] = lo;
  }

  // A workgroup takes a contiguous range of tiles, n tile fastest.  The
  // counter maps are monotone bit deposits, so stepping the n tile advances
  // the n parts of the B and C offsets by one masked increment each
  // ((x | ~M) + 1) & M; the rest is recomputed when the n tile wraps.
  const uint32_t mak = gmap(g.a_k, (K - 1u) & ~(uint32_t)(tk - 1));  // k bits above a stage
  const uint32_t mbk = gmap(g.b_k, (K - 1u) & ~(uint32_t)(tk - 1));
  const uint32_t mbn = gmap(g.b_n, ((1u << g.nn) - 1u) & ~(uint32_t)(TN - 1));
  const uint32_t mcn = gmap(g.c_n, ((1u << g.nn) - 1u) & ~(uint32_t)(TN - 1));
  const uint64_t first = (uint64_t)blockIdx.x * tiles_per_block;
  uint32_t nt = 0, mt = 0, bt = 0, item = 0, sb = 0, pt = 0;
  uint32_t bn = 0, cn = 0;
  float sa = 1.f, sbs = 1.f;
  int eacc = 0;
  const float2* A = nullptr;
  const float2* Bb = nullptr;
  float2* Cb = nullptr;
  for (uint32_t it = 0; it < tiles_per_block; ++it) {
    const uint64_t tile_id = first + it;
    if (tile_id >= n_tiles) break;
    if (it == 0 || nt + 1 == n_nt) {
      // tile -> (n tile, m tile, batch tile, item)
      uint64_t bid = tile_id;
      nt = (uint32_t)(bid % n_nt);
      bid /= n_nt;
      mt = (uint32_t)(bid % n_mt);
      bid /= n_mt;
      bt = (uint32_t)(bid % n_bt);
      item = (uint32_t)(bid / n_bt);
      sb = item & ((1u << g.lg_nsb) - 1u);
      pt = item >> g.lg_nsb;
      const uint64_t sid = (uint64_t)g.chunk_base + sb;
      const uint32_t b0 = bt * NB;
      A = reinterpret_cast<const float2*>(g.a) + (int64_t)pt * g.a_pt + (int64_t)sb * g.a_sb +
          ((int64_t)gpext(sid, g.a_smask) << g.a_slow) + gmap(g.a_b, b0) + gmap(g.a_m, mt * TM);
      Bb = reinterpret_cast<const float2*>(g.b) + (int64_t)pt * g.b_pt + (int64_t)sb * g.b_sb +
           ((int64_t)gpext(sid, g.b_smask) << g.b_slow) + gmap(g.b_b, b0);
      Cb = reinterpret_cast<float2*>(g.c) + (int64_t)pt * g.c_pt + (int64_t)sb * g.c_sb + gmap(g.c_b, b0) +
           gmap(g.c_m, mt * TM);
      bn = gmap(g.b_n, nt * TN);
      cn = gmap(g.c_n, nt * TN);
      // operand scales of the item
      sa = 1.f;
      sbs = 1.f;
      eacc = 0;
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
    } else {
      ++nt;
      bn = ((bn | ~mbn) + 1u) & mbn;
      cn = ((cn | ~mcn) + 1u) & mcn;
    }
    const float2* B = Bb + bn;
    float2* C = Cb + cn;

    v4f totR = {0.f, 0.f, 0.f, 0.f}, totI = {0.f, 0.f, 0.f, 0.f};  // running sums
    v4f cmpR = {0.f, 0.f, 0.f, 0.f}, cmpI = {0.f, 0.f, 0.f, 0.f};  // their compensations
    float2 va[kALoads], vb[kBLoads];
    // k part of the stage base: stepping k0 by tk is a masked increment of
    // its storage offset
    uint32_t ka = 0, kb = 0;
    auto fetch = [&]() {
#pragma unroll
      for (int q = 0; q < kALoads; ++q)
        if (a_r[q] < kARows) va[q] = A[a_loc[q] + ka];
#pragma unroll
      for (int q = 0; q < kBLoads; ++q)
        if (b_r[q] < kBRows) vb[q] = B[b_loc[q] + kb];
    };
    fetch();
    for (uint32_t k0 = 0; k0 < K; k0 += (uint32_t)tk) {
#pragma unroll
      for (int q = 0; q < kALoads; ++q)
        if (a_r[q] < kARows) {
          sAr[a_r[q]][a_ki[q]] = va[q].x * sa;
          sAi[a_r[q]][a_ki[q]] = va[q].y * sa;
        }
#pragma unroll
      for (int q = 0; q < kBLoads; ++q)
        if (b_r[q] < kBRows) {
          sBr[b_r[q]][b_ki[q]] = vb[q].x * sbs;
          sBi[b_r[q]][b_ki[q]] = vb[q].y * sbs;
        }
      __syncthreads();
      if (k0 + (uint32_t)tk < K) {  // next stage in flight during the products
        ka = ((ka | ~mak) + 1u) & mak;
        kb = ((kb | ~mbk) + 1u) & mbk;
        fetch();
      }
      if (wave < kSubs) {
        const int ra = wb * TM + wm * 16 + li, rbw = wb * TN + wn * 16 + li;
        v4f accR = {0.f, 0.f, 0.f, 0.f}, accI = {0.f, 0.f, 0.f, 0.f};
        for (int kk = 0; kk < tk; kk += 4) {
          const float ar = sAr[ra][kk + lk], ai = sAi[ra][kk + lk];
          const float br = sBr[rbw][kk + lk], bi = sBi[rbw][kk + lk];
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
        const int o = (wb * TM + wm * 16 + 4 * lk + r) * (TN + 1) + wn * 16 + li;
        sCr[o] = totR[r];
        sCi[o] = totI[r];
      }
    }
    __syncthreads();
    float m = 0.f;
#pragma unroll
    for (int q = 0; q < kCWrites; ++q) {
      if (tid + q * kGThreads < kTileElems) {
        float2 v;
        v.x = sCr[s_loc[q]];
        v.y = sCi[s_loc[q]];
        C[c_loc[q]] = v;
        m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
      }
    }
    if (g.c_exp_base >= 0) {
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) m = fmaxf(m, __shfl_xor(m, off));
      const int slot = g.c_exp_base + (int)pt * g.c_exp_pt + (int)sb * g.c_exp_sb;
      if (lane == 0) atomicMax(maxbits + slot, __float_as_uint(m));
      if (tid == 0 && bt == 0 && mt == 0 && nt == 0) exps[slot] = eacc;
    }
    __syncthreads();  // sC is rewritten by the next tile
  }
}

template <int TB, int LM, int LN>
hipError_t go(const DevGemm& g, int* exps, uint32_t* maxbits, hipStream_t stream) {
  const uint64_t n_tiles = ((uint64_t)g.n_items << (g.nb - TB)) << ((g.nm - LM) + (g.nn - LN));
  if (n_tiles == 0) return hipSuccess;
  // short-K products get several tiles per workgroup (their setup is a
  // large part of a tile's work); keep >= 16K workgroups in flight
  // short-K products: about 4K workgroups over contiguous tile ranges, so
  // the per-thread setup is paid once per workgroup; long-K products have
  // enough work per tile: one tile per workgroup keeps the CUs full
  const uint32_t tpb = g.nk <= 5 ? (uint32_t)std::max<uint64_t>(1, (n_tiles + 4095) / 4096) : 1u;
  const uint64_t grid = (n_tiles + tpb - 1) / tpb;
  if (grid > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_gemm<TB, LM, LN>), dim3((unsigned)grid), dim3(kGThreads), 0, stream, g, exps, maxbits, tpb,
                     n_tiles);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm(const DevGemm& g, bool scaled, int* exps, uint32_t* maxbits, hipStream_t stream) {
  if (!scaled || g.nm < 4 || g.nn < 4 || g.nk < 3 || g.tb > g.nb || g.tm > g.nm || g.tn > g.nn)
    return hipErrorInvalidValue;
  switch (g.tb * 100 + g.tm * 10 + g.tn) {
    case 55: return go<0, 5, 5>(g, exps, maxbits, stream);
    case 154: return go<1, 5, 4>(g, exps, maxbits, stream);
    case 145: return go<1, 4, 5>(g, exps, maxbits, stream);
    case 244: return go<2, 4, 4>(g, exps, maxbits, stream);
    case 54: return go<0, 5, 4>(g, exps, maxbits, stream);
    case 45: return go<0, 4, 5>(g, exps, maxbits, stream);
    case 144: return go<1, 4, 4>(g, exps, maxbits, stream);
    case 44: return go<0, 4, 4>(g, exps, maxbits, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace qt
