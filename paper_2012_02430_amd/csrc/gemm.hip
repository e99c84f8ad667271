// Fused GEMM bucket on the matrix cores: for every batch item (point,
// slice) and batch index b,
//   C[b, m, n] = sum_k A[b, m, k] * B[b, n, k]        (complex64)
// with the power-of-two scaling of the other bucket steps (each operand
// block is multiplied by 2^-shift of its measured max on load, the output
// exponent is the sum of the operands' exponents and shifts, and the
// output max is collected for the next consumer).
//
// A workgroup (4 wavefronts) computes NB x TM x TN tiles of C (NB batch
// indices of one item) over a contiguous range of tiles.  Per K stage it
// gathers an (NB TM) x TK block of A and an (NB TN) x TK block of B into LDS,
// split into real and imaginary planes; the next stage (of the same tile or
// of the next one) is loaded into registers while the matrix cores work on
// the current one.  Each wavefront owns a 16 x 16 sub-tile and accumulates
// it in FP32 with v_mfma_f32_16x16x4_f32: per 4-deep slice of K, four
// products form
//   Re += Ar Br - Ai Bi,   Im += Ar Bi + Ai Br.
// Operand lane layout of that instruction (16 x 4 A, 4 x 16 B, 16 x 16 D):
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16], and holds
// D[4 (l / 16) + r][l % 16] in accumulator register r.
// Each K stage is accumulated from zero and added to the running total with
// Kahan compensation, so the rounding error grows with the stage depth (16
// or 64) plus a constant rather than with K (up to 2^20 here).
//
// Split-BF16 mode (QT_C64_SCALED_MFMA_BF16X3, MODE 1, 32-deep stages): each
// scaled operand value x is split into three BF16 parts x = h + m + l + r
// with h = bf16(x), m = bf16(x - h), l = bf16(x - h - m) (|r| <= 2^-24 |x|
// roughly), and a real product x y is formed from the six part products
// whose order is at least 2^-16 (hh, hm, mh, hl, lh, mm) on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation, which keeps about the
// accuracy of an FP32 product.  The complex product takes three real
// products (3M): T1 = Ar Br, T2 = Ai Bi, T3 = (Ar + Ai)(Br + Bi), then
// Re = T1 - T2 and Im = T3 - T1 - T2 per stage.  The MFMA lane layout
// (lane l holds A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16],
// j = 0..7) matches the FP32 one above with eight K values per lane.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "qt_internal.h"

namespace qt {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef unsigned v2u __attribute__((ext_vector_type(2)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// x = h + m + l (+ a remainder below 2^-24 |x|), each part BF16 (rounded to
// nearest), stored as three 16-bit words.
__device__ __forceinline__ void split3(float x, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)x;
  const float r1 = x - (float)h;
  m = (__bf16)r1;
  l = (__bf16)(r1 - (float)m);
}

// Raw buffer over the 4 GiB window at p (offsets are checked against it).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)0xffffffff, 0x00020000);
}

constexpr int kGThreads = 256;

// x deposited into the set bits of m, low to high (uniform values: scalar work)
__device__ __forceinline__ uint32_t dep(uint32_t x, uint32_t m) {
  uint32_t r = 0;
  for (; m; m &= m - 1u, x >>= 1)
    if (x & 1u) r |= m & (0u - m);
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

// Offset of element number e of a numbered block: the weights of its set
// bits.  Bits 0..7 come from the thread index (per lane); the bits above
// from the unrolled element slot q (uniform).
__device__ __forceinline__ uint32_t lane_part(const uint32_t* w, int tid) {
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += (tid >> j) & 1 ? w[j] : 0u;
  return s;
}
__device__ __forceinline__ uint32_t slot_part(const uint32_t* w, int q) {
  uint32_t s = 0;
#pragma unroll
  for (int j = 8; j < kGBits; ++j)
    if (((q << 8) >> j) & 1) s += w[j];
  return s;
}

// s_waitcnt on the vector memory counter alone (at most N operations in
// flight; the LDS and export counters at their maxima)
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 16, "");
  __builtin_amdgcn_s_waitcnt(0x0F70 | N);
}

// Tile: NB = 2^TB batch indices x TM = 2^LM rows x TN = 2^LN columns, the
// low bits of the b, m and n counters.  TK is the depth of a K stage (a
// compile-time constant: the guards of the stage loads fold away, and the
// compiler counts the loads and stores in flight exactly, so a tile's stage
// does not wait for the previous tile's output stores).  Wavefront w owns
// the 16 x 16 sub-tile (batch, m block, n block) number w.
//
// Tiles are numbered n fastest, then m, then the batch tile, then the item.
// A workgroup takes `tiles_per_block` consecutive tiles, a power of two that
// divides the tiles of one (item, batch tile), so its range stays inside
// one: the item's scales and bases are found once, and a step to the next
// tile advances the n (or, when n wraps, the m) parts of the offsets by one
// masked increment ((x | ~M) + 1) & M.
template <int TB, int LM, int LN, int TK, int MODE>
__global__ __launch_bounds__(kGThreads) void k_gemm(const DevGemm g, int* __restrict__ exps,
                                                    uint32_t* __restrict__ maxbits, uint32_t tiles_per_block,
                                                    uint64_t n_tiles) {
  constexpr int NB = 1 << TB, TM = 1 << LM, TN = 1 << LN;
  constexpr int kARows = NB * TM, kBRows = NB * TN;
  constexpr int kTileElems = NB * TM * TN;
  constexpr int kSubM = TM / 16, kSubN = TN / 16;
  constexpr int kSubs = NB * kSubM * kSubN;
  static_assert(kSubs <= kGThreads / 64, "one 16 x 16 sub-tile per wavefront");
  static_assert(MODE == 0 || TK == 32, "split-BF16 stages are 32 deep");
  // operand row pitch (in elements of the plane): FP32 planes: the products
  // read row li (0..15) at depth lk (0..3) per lane, and 16 + 1 and 64 + 4
  // put those 64 reads in distinct banks; BF16 planes: each lane reads 16
  // bytes (eight K values), rows 80 bytes apart
  constexpr int kP = MODE == 1 ? TK + 8 : (TK == 64 ? 68 : 17);
  // stage elements per operand: a multiple of the block size, or (8-deep
  // stages of the smallest tiles) less than it
  constexpr uint32_t a_elems = kARows * TK, b_elems = kBRows * TK;
  constexpr int kALoads = (a_elems + kGThreads - 1) / kGThreads, kBLoads = (b_elems + kGThreads - 1) / kGThreads;
  constexpr int kCWrites = kTileElems / kGThreads;
  static_assert((a_elems < kGThreads || a_elems % kGThreads == 0) && (b_elems < kGThreads || b_elems % kGThreads == 0) &&
                    kTileElems % kGThreads == 0,
                "");
  // FP32: real and imaginary planes of A and B; BF16: nine planes each
  // (parts h, m, l of Re, Im and Re + Im), two bytes per element
  constexpr int kOpFloats = MODE == 1 ? 9 * (kARows + kBRows) * kP / 2 : 2 * (kARows + kBRows) * kP;
  constexpr int kCFloats = 2 * kARows * (TN + 1);
  // operand planes and the output staging share the LDS: the staging is
  // written only after the last stage's products
  __shared__ __align__(16) float smem[kOpFloats > kCFloats ? kOpFloats : kCFloats];
  float* const sAr = smem;
  float* const sAi = sAr + kARows * kP;
  float* const sBr = sAi + kARows * kP;
  float* const sBi = sBr + kBRows * kP;
  __bf16* const hA = reinterpret_cast<__bf16*>(smem);   // plane 3 c + part of A: hA + (3 c + part) kARows kP
  __bf16* const hB = hA + 9 * kARows * kP;
  float* const sCr = smem;
  float* const sCi = smem + kARows * (TN + 1);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;

  // Workgroups are dealt to the XCDs round robin; give each XCD a
  // contiguous share of the tile ranges so that neighbouring tiles (which
  // share operand blocks) meet in the same L2.
  uint32_t blk = blockIdx.x;
  {
    const uint32_t nbk = gridDim.x, q = nbk / 8u, r = nbk % 8u, x = blk % 8u, i = blk / 8u;
    blk = (x < r ? x * (q + 1u) : r * (q + 1u) + (x - r) * q) + i;
  }
  const uint64_t first = (uint64_t)blk * tiles_per_block;
  if (first >= n_tiles) return;
  const uint32_t n_here = (uint32_t)(n_tiles - first < tiles_per_block ? n_tiles - first : tiles_per_block);

  const uint32_t lg_nt = (uint32_t)(g.nn - LN), lg_mt = (uint32_t)(g.nm - LM), lg_bt = (uint32_t)(g.nb - TB);
  const uint32_t n_nt = 1u << lg_nt;
  const uint32_t n_stages = (1u << g.nk) / (uint32_t)TK;
  const bool a_lane = a_elems >= kGThreads || (uint32_t)tid < a_elems;
  const bool b_lane = b_elems >= kGThreads || (uint32_t)tid < b_elems;
  const int wb = wave / (kSubM * kSubN), wm = (wave / kSubN) % kSubM, wn = wave % kSubN;
  const int li = lane & 15, lk = lane >> 4;

  // Per-lane parts of the numbered offsets, in bytes; a slot's uniform part
  // goes into the (scalar) base address.
  const uint32_t a_vo = lane_part(g.aw, tid) * 8u, b_vo = lane_part(g.bw, tid) * 8u, c_vo = lane_part(g.cw, tid) * 8u;
  const uint32_t a_lo = lane_part(g.al, tid) * 4u, b_lo = lane_part(g.bl, tid) * 4u, c_lo = lane_part(g.cl, tid) * 4u;

  // the range's (item, batch tile) and its first (m, n) tile
  uint32_t nt = (uint32_t)first & (n_nt - 1u);
  uint64_t bid = first >> lg_nt;
  const uint32_t mt = (uint32_t)bid & ((1u << lg_mt) - 1u);
  bid >>= lg_mt;
  const uint32_t bt = (uint32_t)bid & ((1u << lg_bt) - 1u);
  const uint32_t item = (uint32_t)(bid >> lg_bt);
  const uint32_t sb = item & ((1u << g.lg_nsb) - 1u);
  const uint32_t pt = item >> g.lg_nsb;
  const uint64_t sid = (uint64_t)g.chunk_base + sb;
  const float2* const A0 = reinterpret_cast<const float2*>(g.a) + (int64_t)pt * g.a_pt + (int64_t)sb * g.a_sb +
                           ((int64_t)gpext(sid, g.a_smask) << g.a_slow) + dep(bt * NB, g.a_bm);
  const float2* const B0 = reinterpret_cast<const float2*>(g.b) + (int64_t)pt * g.b_pt + (int64_t)sb * g.b_sb +
                           ((int64_t)gpext(sid, g.b_smask) << g.b_slow) + dep(bt * NB, g.b_bm);
  float2* const C0 = reinterpret_cast<float2*>(g.c) + (int64_t)pt * g.c_pt + (int64_t)sb * g.c_sb + dep(bt * NB, g.c_bm);
  uint32_t am = dep(mt * TM, g.a_mm), cm = dep(mt * TM, g.c_mm);
  uint32_t bn = dep(nt * TN, g.b_nm), cn = dep(nt * TN, g.c_nm);
  const uint32_t a_mh = g.a_mm & ~dep(TM - 1u, g.a_mm), c_mh = g.c_mm & ~dep(TM - 1u, g.c_mm);
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
  const int c_slot = g.c_exp_base >= 0 ? g.c_exp_base + (int)pt * g.c_exp_pt + (int)sb * g.c_exp_sb : -1;
  // the item's first tile is the first of its range
  if (c_slot >= 0 && tid == 0 && bt == 0 && mt == 0 && nt == 0) exps[c_slot] = eacc;

  // Buffer accesses: the per-lane byte offset in a VGPR, the slot's and the
  // tile's uniform part as the scalar offset (operand ranks are at most 28,
  // so both stay below 2^31 bytes).
  const __amdgpu_buffer_rsrc_t rA = make_rsrc(A0), rB = make_rsrc(B0), rC = make_rsrc(C0);
  v2f va[kALoads], vb[kBLoads];
  auto fetch = [&](uint32_t ao, uint32_t bo) {
#pragma unroll
    for (int q = 0; q < kALoads; ++q)
      if ((uint32_t)(q * kGThreads) < a_elems && a_lane)
        va[q] = __builtin_bit_cast(v2f, __builtin_amdgcn_raw_buffer_load_b64(rA, a_vo, (ao + slot_part(g.aw, q)) * 8u, 0));
#pragma unroll
    for (int q = 0; q < kBLoads; ++q)
      if ((uint32_t)(q * kGThreads) < b_elems && b_lane)
        vb[q] = __builtin_bit_cast(v2f, __builtin_amdgcn_raw_buffer_load_b64(rB, b_vo, (bo + slot_part(g.bw, q)) * 8u, 0));
  };
  // LDS element (plane p) at byte offset o
  auto lds = [&](float* plane, uint32_t o) -> float& { return *reinterpret_cast<float*>(reinterpret_cast<char*>(plane) + o); };

  uint32_t ka = 0, kb = 0;  // k parts of the stage in registers
  fetch(am, bn);
  // The loads and stores in flight share one counter, which the compiler
  // counts per path: with the first stage's loads complete on entry and the
  // prefetched stage's loads complete at the end of each tile (only that
  // tile's output stores may still be in flight), both ways into the loop
  // agree, and the first stage write of a tile does not wait for the previous
  // tile's stores to leave.
  wait_vm<0>();
  float mrun = 0.f;  // output max over the range
  for (uint32_t it = 0; it < n_here; ++it) {
    v4f totR, totI;                                                 // running sums
    v4f cmpR = {0.f, 0.f, 0.f, 0.f}, cmpI = {0.f, 0.f, 0.f, 0.f};  // their compensations
    // the next tile's m and n parts
    uint32_t am2 = am, cm2 = cm, bn2 = bn, cn2 = cn;
    if (nt + 1u < n_nt) {
      bn2 = ((bn | ~g.b_nh) + 1u) & g.b_nh;
      cn2 = ((cn | ~g.c_nh) + 1u) & g.c_nh;
    } else {
      bn2 = cn2 = 0;
      am2 = ((am | ~a_mh) + 1u) & a_mh;
      cm2 = ((cm | ~c_mh) + 1u) & c_mh;
    }
    for (uint32_t s = 0; s < n_stages; ++s) {
      if constexpr (MODE == 0) {
#pragma unroll
        for (int q = 0; q < kALoads; ++q)
          if ((uint32_t)(q * kGThreads) < a_elems && a_lane) {
            const uint32_t o = a_lo + slot_part(g.al, q) * 4u;
            lds(sAr, o) = va[q].x * sa;
            lds(sAi, o) = va[q].y * sa;
          }
#pragma unroll
        for (int q = 0; q < kBLoads; ++q)
          if ((uint32_t)(q * kGThreads) < b_elems && b_lane) {
            const uint32_t o = b_lo + slot_part(g.bl, q) * 4u;
            lds(sBr, o) = vb[q].x * sbs;
            lds(sBi, o) = vb[q].y * sbs;
          }
      } else {
        // element offsets in the planes (a_lo, b_lo count 4 bytes per element)
#pragma unroll
        for (int q = 0; q < kALoads; ++q)
          if ((uint32_t)(q * kGThreads) < a_elems && a_lane) {
            const uint32_t o = (a_lo >> 2) + slot_part(g.al, q);
            const float re = va[q].x * sa, im = va[q].y * sa;
            split3(re, hA[o], hA[o + kARows * kP], hA[o + 2 * kARows * kP]);
            split3(im, hA[o + 3 * kARows * kP], hA[o + 4 * kARows * kP], hA[o + 5 * kARows * kP]);
            split3(re + im, hA[o + 6 * kARows * kP], hA[o + 7 * kARows * kP], hA[o + 8 * kARows * kP]);
          }
#pragma unroll
        for (int q = 0; q < kBLoads; ++q)
          if ((uint32_t)(q * kGThreads) < b_elems && b_lane) {
            const uint32_t o = (b_lo >> 2) + slot_part(g.bl, q);
            const float re = vb[q].x * sbs, im = vb[q].y * sbs;
            split3(re, hB[o], hB[o + kBRows * kP], hB[o + 2 * kBRows * kP]);
            split3(im, hB[o + 3 * kBRows * kP], hB[o + 4 * kBRows * kP], hB[o + 5 * kBRows * kP]);
            split3(re + im, hB[o + 6 * kBRows * kP], hB[o + 7 * kBRows * kP], hB[o + 8 * kBRows * kP]);
          }
      }
      __syncthreads();
      // the next stage, of this tile or of the next one, in flight during the products
      // (one call site: the stage registers have one definition in the loop,
      // which the compiler neither copies nor waits for before the products)
      {
        const bool more = s + 1u < n_stages;
        ka = more ? ((ka | ~g.a_kh) + 1u) & g.a_kh : 0u;
        kb = more ? ((kb | ~g.b_kh) + 1u) & g.b_kh : 0u;
        if (more || it + 1u < n_here) fetch((more ? am : am2) + ka, (more ? bn : bn2) + kb);
      }
      if (wave < kSubs) {
        v4f accR = {0.f, 0.f, 0.f, 0.f}, accI = {0.f, 0.f, 0.f, 0.f};
        if constexpr (MODE == 0) {
          const float* ar_p = sAr + (wb * TM + wm * 16 + li) * kP + lk;
          const float* ai_p = sAi + (wb * TM + wm * 16 + li) * kP + lk;
          const float* br_p = sBr + (wb * TN + wn * 16 + li) * kP + lk;
          const float* bi_p = sBi + (wb * TN + wn * 16 + li) * kP + lk;
          if constexpr (TK == 64) {
            // long sums (MFMA-bound): three products per 4-deep slice (3M),
            // T1 = Ar Br, T2 = Ai Bi, T3 = (Ar + Ai)(Br + Bi).  The sum over
            // the stage only needs A and B to pair the same K in each lane,
            // so lane (li, lk) takes K = 16 lk + j in instruction j: sixteen
            // contiguous values per row, read 16 bytes at a time (the row
            // pitch of 68 floats keeps 8 consecutive lanes in distinct banks)
            const float* ar16 = ar_p - lk + 16 * lk;
            const float* ai16 = ai_p - lk + 16 * lk;
            const float* br16 = br_p - lk + 16 * lk;
            const float* bi16 = bi_p - lk + 16 * lk;
            v4f t1 = {0.f, 0.f, 0.f, 0.f}, t2 = t1, t3 = t1;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const v4f ar = *reinterpret_cast<const v4f*>(ar16 + 4 * c);
              const v4f ai = *reinterpret_cast<const v4f*>(ai16 + 4 * c);
              const v4f br = *reinterpret_cast<const v4f*>(br16 + 4 * c);
              const v4f bi = *reinterpret_cast<const v4f*>(bi16 + 4 * c);
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                t1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[j], br[j], t1, 0, 0, 0);
                t2 = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[j], bi[j], t2, 0, 0, 0);
                t3 = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[j] + ai[j], br[j] + bi[j], t3, 0, 0, 0);
              }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              accR[r] = t1[r] - t2[r];
              accI[r] = t3[r] - t1[r] - t2[r];
            }
          } else {
            for (int kk = 0; kk < TK; kk += 4) {
              const float ar = ar_p[kk], ai = ai_p[kk], br = br_p[kk], bi = bi_p[kk];
              accR = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, accR, 0, 0, 0);
              accR = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, bi, accR, 0, 0, 0);
              accI = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bi, accI, 0, 0, 0);
              accI = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br, accI, 0, 0, 0);
            }
          }
        } else {
          // lane (li, lk) reads K values 8 lk .. 8 lk + 7 of its row
          const __bf16* a_row = hA + (wb * TM + wm * 16 + li) * kP + 8 * lk;
          const __bf16* b_row = hB + (wb * TN + wn * 16 + li) * kP + 8 * lk;
          v4f t[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {  // Re, Im, Re + Im
            const v8bf ah = *reinterpret_cast<const v8bf*>(a_row + (3 * c) * kARows * kP);
            const v8bf am = *reinterpret_cast<const v8bf*>(a_row + (3 * c + 1) * kARows * kP);
            const v8bf al = *reinterpret_cast<const v8bf*>(a_row + (3 * c + 2) * kARows * kP);
            const v8bf bh = *reinterpret_cast<const v8bf*>(b_row + (3 * c) * kBRows * kP);
            const v8bf bm = *reinterpret_cast<const v8bf*>(b_row + (3 * c + 1) * kBRows * kP);
            const v8bf bl = *reinterpret_cast<const v8bf*>(b_row + (3 * c + 2) * kBRows * kP);
            v4f x = {0.f, 0.f, 0.f, 0.f};
            // smallest terms first
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, x, 0, 0, 0);
            x = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, x, 0, 0, 0);
            t[c] = x;
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            accR[r] = t[0][r] - t[1][r];
            accI[r] = t[2][r] - t[0][r] - t[1][r];
          }
        }
        if (s == 0) {
          totR = accR;
          totI = accI;
        } else {
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
      }
      __syncthreads();
    }

    // stage the tile in LDS (over the operand planes), then write it in C order
    if (wave < kSubs) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = (wb * TM + wm * 16 + 4 * lk + r) * (TN + 1) + wn * 16 + li;
        sCr[o] = totR[r];
        sCi[o] = totI[r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kCWrites; ++q) {
      const uint32_t o = c_lo + slot_part(g.cl, q) * 4u;
      v2f v;
      v.x = lds(sCr, o);
      v.y = lds(sCi, o);
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, v), rC, c_vo, (cm + cn + slot_part(g.cw, q)) * 8u, 0);
      mrun = fmaxf(mrun, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
    wait_vm<kCWrites>();  // the stage loads issued before these stores
    __syncthreads();  // the staging is overwritten by the next tile's first stage
    nt = nt + 1u < n_nt ? nt + 1u : 0u;
    am = am2;
    cm = cm2;
    bn = bn2;
    cn = cn2;
  }
  if (c_slot >= 0) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) mrun = fmaxf(mrun, __shfl_xor(mrun, off));
    if (lane == 0) atomicMax(maxbits + c_slot, __float_as_uint(mrun));
  }
}

template <int TB, int LM, int LN, int TK, int MODE>
hipError_t go(const DevGemm& g, int* exps, uint32_t* maxbits, hipStream_t stream) {
  const uint64_t n_tiles = ((uint64_t)g.n_items << (g.nb - TB)) << ((g.nm - LM) + (g.nn - LN));
  if (n_tiles == 0) return hipSuccess;
  // Short tile ranges: the workgroups resident on one XCD then cover a
  // window of neighbouring tiles whose operand blocks they share in its L2
  // (a long range per workgroup streams its own B block, which the L2 does
  // not hold for all of them).  A short-K tile is little work, so a few
  // tiles per workgroup pay its setup once; a long-K tile takes one.  The
  // range is a power of two that divides the tiles of one (item, batch tile).
  const int want = std::max(1, g.tiles > 0 ? g.tiles : env_int("QT_GEMM_TILES", g.nk <= 5 ? 16 : 1));
  const int lg_block = (g.nm - LM) + (g.nn - LN);
  int lg = 0;
  while (lg < lg_block && (2 << lg) <= want) ++lg;
  const uint32_t tpb = 1u << lg;
  const uint64_t grid = (n_tiles + tpb - 1) / tpb;
  if (grid > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_gemm<TB, LM, LN, TK, MODE>), dim3((unsigned)grid), dim3(kGThreads), 0, stream, g, exps,
                     maxbits, tpb, n_tiles);
  return hipGetLastError();
}

template <int TK, int MODE>
hipError_t go_shape(const DevGemm& g, int* exps, uint32_t* maxbits, hipStream_t stream) {
  switch (g.tb * 100 + g.tm * 10 + g.tn) {
    case 55: return go<0, 5, 5, TK, MODE>(g, exps, maxbits, stream);
    case 154: return go<1, 5, 4, TK, MODE>(g, exps, maxbits, stream);
    case 145: return go<1, 4, 5, TK, MODE>(g, exps, maxbits, stream);
    case 244: return go<2, 4, 4, TK, MODE>(g, exps, maxbits, stream);
    case 54: return go<0, 5, 4, TK, MODE>(g, exps, maxbits, stream);
    case 45: return go<0, 4, 5, TK, MODE>(g, exps, maxbits, stream);
    case 144: return go<1, 4, 4, TK, MODE>(g, exps, maxbits, stream);
    case 44: return go<0, 4, 4, TK, MODE>(g, exps, maxbits, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_gemm(const DevGemm& g, bool scaled, int* exps, uint32_t* maxbits, hipStream_t stream) {
  if (!scaled || g.nm < 4 || g.nn < 4 || g.nk < 3 || g.tb > g.nb || g.tm > g.nm || g.tn > g.nn)
    return hipErrorInvalidValue;
  // stage depth: 64 needs K >= 64; 16 (or 8 for K = 8) otherwise; the
  // split-BF16 products take 32-deep stages (K >= 32)
  if (g.mode == 1) return g.tk == 32 && g.nk >= 5 ? go_shape<32, 1>(g, exps, maxbits, stream) : hipErrorInvalidValue;
  if (g.tk == 64 && g.nk >= 6) return go_shape<64, 0>(g, exps, maxbits, stream);
  if (g.tk == 16 && g.nk >= 4) return go_shape<16, 0>(g, exps, maxbits, stream);
  if (g.tk == 8 && g.nk == 3) return go_shape<8, 0>(g, exps, maxbits, stream);
  return hipErrorInvalidValue;
}

}  // namespace qt
