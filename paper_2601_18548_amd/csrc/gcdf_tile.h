// Tile engine of the fused batched neural-GCDF query for gfx950 (MI355X):
// device code shared by the query, sphere-query and serving kernels.
//
// One workgroup (8 waves, two per SIMD, in the BF16 modes; 4 in FP32) owns a
// tile of 64 queries: 64 points of one knot (dense all-pairs mode) or 64
// entries of a pair list.  For the
// tile it runs the whole query without touching HBM in between:
//   base-frame transform -> input layer (FP32, VALU) -> hidden layers on
//   matrix cores -> output dot -> reverse sweep on matrix cores (transposed
//   weights) -> input-layer gradient (FP32) -> chain rule to (x, y, yaw, arm)
//   -> stores of d / J -> per-knot minimum (64-bit ordered-key atomic min).
// (Steps of the query: Sec. III-B base-frame transform and chain rule,
// Sec. III-C network on [p', a], Sec. IV-A constraint over all knot/point
// pairs, Sec. IV-A knot-major stacking.)
//
// Work split inside the tile: every hidden layer is C[W x 64] = M[W x W] B[W x 64]
// with M = W_l (forward) or W_l^T (reverse) and B = the previous layer's
// activations (forward) or back-propagated gradients (reverse).  With n waves,
// wave w owns output rows [w*W/n, (w+1)*W/n) for all 64 queries; B lives in LDS
// (written by the epilogue of the previous layer, read by every wave); the A fragments
// stream from global memory (L2-resident, pre-packed so each 32x16 fragment is
// one contiguous 1 KiB block: one dwordx4 per lane).  Each weight byte fetched
// is used for 64 queries.
//
// Precision modes:
//   FP32   : v_mfma_f32_32x32x2_f32, activations FP32 in LDS.
//   BF16   : v_mfma_f32_32x32x16_bf16, activations rounded to BF16, FP32 accumulate.
//   BF16X2 : as BF16 but each activation is split x = hi + lo (both BF16) and both
//            halves are multiplied (2 MFMAs per fragment pair); hidden weights must
//            lie on the BF16 grid to be exact.
//   BF16X2F16 : forward layers as BF16X2; the reverse sweep multiplies FP16
//            back-propagated values by the FP16 copy of the transposed BF16 weights
//            (v_mfma_f32_32x32x16_f16, one MFMA per fragment pair), the values
//            scaled by 2^6 to keep them in FP16's normal range.
// The SiLU derivative needed by the reverse sweep is kept in FP32 registers for
// layers 2 and 3 and recomputed for layer 1 from the input layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "gcdf_internal.h"

namespace gcdf {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(2 * sizeof(float)))) float f32x2;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(4 * sizeof(_Float16)))) _Float16 f16x4;

constexpr float kLog2e = 1.4426950408889634f;

// SiLU and its derivative from one exp and one reciprocal.
__device__ __forceinline__ void silu_fwd(float z, float& h, float& dh) {
  float t = __builtin_amdgcn_exp2f(-z * kLog2e);
  float sg = __builtin_amdgcn_rcpf(1.0f + t);
  h = z * sg;
  dh = sg + h * (1.0f - sg);  // s (1 + z (1 - s))
}
__device__ __forceinline__ float silu_only(float z) {
  float t = __builtin_amdgcn_exp2f(-z * kLog2e);
  return z * __builtin_amdgcn_rcpf(1.0f + t);
}
__device__ __forceinline__ float silu_prime_only(float z) {
  float t = __builtin_amdgcn_exp2f(-z * kLog2e);
  float sg = __builtin_amdgcn_rcpf(1.0f + t);
  return sg + z * sg * (1.0f - sg);
}

// The reverse sweep's SiLU' values are parked in accumulation registers
// (AGPRs), which the matrix cores do not need because accumulators are kept in
// ordinary VGPRs; vector ALU instructions cannot read AGPRs, so values move with
// v_accvgpr_write / v_accvgpr_read.
__device__ __forceinline__ float park(float x) {
  float a;
  asm("v_accvgpr_write_b32 %0, %1" : "=a"(a) : "v"(x));
  return a;
}
// `after` is an extra input that orders the read after the value it is used
// with (the layer's finished accumulator); otherwise the compiler hoists the
// read above the K loop and keeps every unparked value live through it.
__device__ __forceinline__ float unpark(float a, float after) {
  float x;
  asm("v_accvgpr_read_b32 %0, %1 ; %2" : "=v"(x) : "a"(a), "v"(after));
  return x;
}

// Input-layer pre-activation, in one fixed order shared by every path:
// c = b1 + sum_a W1[r][3+a] arm[a] (the knot's arm term), then
// z1 = c + W1[r][0] p'x + W1[r][1] p'y + W1[r][2] p'z.
__device__ __forceinline__ float arm_term(float b1, float w3, float w4, float w5, float w6, float w7, float w8,
                                          const float* arm) {
  float c = b1;
  c += w3 * arm[0];
  c += w4 * arm[1];
  c += w5 * arm[2];
  c += w6 * arm[3];
  c += w7 * arm[4];
  c += w8 * arm[5];
  return c;
}
__device__ __forceinline__ float input_preact(float c, float w0, float w1, float w2, const float* x) {
  return c + w0 * x[0] + w1 * x[1] + w2 * x[2];
}
// Sphere obstacles (network input [p', r, a]): the radius term comes last,
// z1 = c + W1[r][0] p'x + W1[r][1] p'y + W1[r][2] p'z + W1[r][radius] r, with r
// at position kXinRadius of the per-query record.
constexpr int kXinRadius = 12;
constexpr int kXinTarget = 13;  // training with the fused loss: the sample's target distance
template <bool SPH>
__device__ __forceinline__ float input_preact_t(float c, float w0, float w1, float w2, float wr, const float* x) {
  if constexpr (SPH) return input_preact(c, w0, w1, w2, x) + wr * x[kXinRadius];
  return input_preact(c, w0, w1, w2, x);
}

// Waves per workgroup: 8 (two per SIMD) for width 512 on BF16 matrix cores, where
// the per-wave registers of four waves (accumulators, parked SiLU' values, the
// weight prefetch) would fill the register file and leave nothing to hide the
// weight stream's L2 latency; 4 otherwise.
template <int W, int MODE>
constexpr int waves_for() {
  return MODE != kFP32 ? 8 : 4;
}

// Arithmetic of one K loop and of the LDS stores that feed it.  Every mode
// uses its own throughout, except kBF16X2F16: BF16X2 forward, and kF16 (single
// FP16 products; an arithmetic kind, never a context mode) in the reverse sweep.
constexpr int kF16 = 4;
template <int MODE>
constexpr int fwd_arith() {
  return MODE == kBF16X2F16 ? kBF16X2 : MODE;
}
template <int MODE>
constexpr int rev_arith() {
  return MODE == kBF16X2F16 ? kF16 : MODE;
}
// Scale of the reverse sweep's seed (kBF16X2F16): back-propagated values between
// ~1e-6 and ~1e3 stay normal FP16 numbers; the input-layer gradient is
// multiplied back by its inverse.  Powers of two, so both steps are exact.
template <int MODE>
constexpr float rev_scale() {
  return MODE == kBF16X2F16 ? 64.0f : 1.0f;
}

// The split modes order each K step's elements as the accumulators hold them (see
// the activation tile below), so no lanes are exchanged before the LDS stores.
template <int MODE>
constexpr bool lane_k_order() {
  return MODE == kBF16X2 || MODE == kBF16X2F16;
}

template <int W, int MODE>
struct Geo {
  static constexpr int NW = waves_for<W, MODE>();    // waves per workgroup
  static constexpr int THREADS = 64 * NW;
  static constexpr int MT = W / (32 * NW);           // 32-row M tiles per wave
  // The packed matrices and row vectors are laid out for 4 row groups of PMT M
  // tiles each (pack_matrix, lane_major_pos); with 8 waves, waves 2p and 2p+1
  // split row group p, SUB waves per group.
  static constexpr int PMT = W / (32 * kWaves);
  static constexpr int SUB = NW / kWaves;
  // the per-query reduction buffer shares the activation tile when 8 waves would
  // not leave room for it (the tile is idle by then)
  static constexpr bool RED_IN_ACT = NW > kWaves;
  static constexpr int NKB = W / 16;                 // 16-deep K blocks (bf16)
  // bytes of the activation tile per K step (16 rows in the BF16 modes, 8 in FP32);
  // BF16X2 keeps a step's hi and lo halves next to each other, lo at LO_OFF
  static constexpr int STEP_BYTES = fwd_arith<MODE>() == kBF16X2 ? 4096 : 2048;
  static constexpr int LO_OFF = 2048;
  static constexpr int NK8 = W / 8;                  // 8-deep K groups (fp32: 4 MFMAs of K=2)
  static constexpr int ACT_BYTES = W * kTileQ * 4;   // fp32, or bf16 hi + bf16 lo
  static constexpr int XIN_FLOATS = 17;              // per query: p'(3), cos, sin, arm(6), seed, radius, target, pad; odd stride: lanes reading one field of 32 queries hit 32 different banks
  static constexpr int RED_VALS = 10;                // d + 9 input-gradient components
  static constexpr int RED_BYTES = NW * RED_VALS * kTileQ * 4;
  static constexpr int LDS_BYTES = ACT_BYTES + kTileQ * XIN_FLOATS * 4 + W * 4 + (RED_IN_ACT ? 0 : RED_BYTES) + 4 * W * 4;
  static_assert(!RED_IN_ACT || RED_BYTES <= ACT_BYTES, "reduction buffer must fit the activation tile");
  static_assert(MT >= 1 && PMT == SUB * MT, "row groups must split evenly");
};

// ----------------------------------------------------------------------------
// Activation tile in LDS (64 query columns).
//  bf16 modes: K step s (rows 16s .. 16s+15) occupies STEP_BYTES at s*STEP_BYTES:
//    its hi half, then (BF16X2) its lo half at +LO_OFF, so one base register with
//    small immediate offsets reaches both.  A half holds 16-byte groups (kh, n) at
//    byte kh*1024 + n*16.  Pure BF16: group (kh, n) holds rows 16s + 8kh + j at
//    position j.  The split modes (lane_k_order) hold rows 16s + 8(j/4) + 4kh + j%4
//    at position j instead, which is the set of rows lane (n, kh) has in its
//    accumulators, so their epilogues store without exchanging lanes; the packed
//    weights order their K elements the same way (the sum over K is unchanged).
//    The B fragment of step s, column block nt is the 2 KiB half, lane (n0, kh)
//    reading the 16 bytes at kh*1024 + nt*512 + n0*16: every lane reads its own
//    consecutive 16 bytes (no bank conflicts).
//  fp32 mode : element (k, n) at (((k/8)*64 + n)*2 + k%2)*4 + (k%8)/2 floats; the
//    B fragment of step s, block nt starts at s*2048 + nt*1024, lane (n0, kh) at
//    +n0*32 + kh*16.
//
// Every address below is a per-lane base (computed once) plus a compile-time
// constant, so the constants fold into the instructions' offset fields instead
// of occupying registers.
// ----------------------------------------------------------------------------
template <int W, int MODE>
struct Lane {
  static constexpr int MT = Geo<W, MODE>::MT;
  int lane, wave, h, n0, kh, rbase;
  char* act_w;        // write base, hi plane (or the fp32 tile)
  char* act_w_lo;     // write base, lo plane
  const char* act_r;  // read base
  __device__ __forceinline__ Lane(char* act, int tid) {
    lane = tid & 63;
    wave = tid >> 6;
    h = lane >> 5;
    kh = h;
    n0 = lane & 31;
    rbase = 32 * MT * wave;
    if constexpr (MODE == kFP32) {
      act_w = act + 4 * (((rbase >> 3) * kTileQ + n0) * 8 + 2 * h);
      act_r = act + n0 * 32 + kh * 16;
    } else {
      act_w = act + (rbase >> 4) * Geo<W, MODE>::STEP_BYTES + h * 1024 + n0 * 16;
      act_r = act + kh * 1024 + n0 * 16;
    }
    act_w_lo = act_w + Geo<W, MODE>::LO_OFF;
  }
};

// Write rows R0..R0+3 (R0 = rbase + 32 i + 8 g + 4 h) of column n = 32 nt + n0 (fp32).
template <int W, int MODE, int I, int G, int NT>
__device__ __forceinline__ void act_store4_fp32(const Lane<W, MODE>& L, const float v[4]) {
  constexpr int off = (4 * I + G) * 2048 + NT * 1024;
  *reinterpret_cast<f32x2*>(L.act_w + off) = f32x2{v[0], v[2]};       // rows R0, R0+2 (k%2 = 0)
  *reinterpret_cast<f32x2*>(L.act_w + off + 16) = f32x2{v[1], v[3]};  // rows R0+1, R0+3 (k%2 = 1)
}

// Pack four floats into two dwords of bf16 (FP16 for kF16), round to nearest even.
template <int AM>
__device__ __forceinline__ void pack4(const float v[4], uint32_t& d0, uint32_t& d1) {
  f32x2 d;
  if constexpr (AM == kF16) {
    f16x4 h4;
#pragma unroll
    for (int r = 0; r < 4; ++r) h4[r] = (_Float16)v[r];
    d = __builtin_bit_cast(f32x2, h4);
  } else {
    bf16x4 h4;
#pragma unroll
    for (int r = 0; r < 4; ++r) h4[r] = (__bf16)v[r];
    d = __builtin_bit_cast(f32x2, h4);
  }
  d0 = __float_as_uint(d[0]);
  d1 = __float_as_uint(d[1]);
}

// bf16 modes: write rows of the group pair g = 2 GP, 2 GP + 1 (v[0..3] for g = 2 GP,
// v[4..7] for g = 2 GP + 1) of column n = 32 nt + n0.  Lane (n0, h) holds k%8 in
// [4h, 4h+4) of both 8-groups kh = 0 (g even) and kh = 1 (g odd).  SWAP (pure
// BF16): one swap across the lane halves gives lane (n0, kh) the whole 8-group kh,
// written as 16 bytes; otherwise (lane_k_order) the lane writes its own 8 values.
// act_pack8 forms the 16-byte words (w[0..3] for the hi plane, w[4..7] for the lo
// plane) and act_write8 stores them, so a caller can do the arithmetic before a
// barrier and the stores after it.  AM: the arithmetic (fwd_arith / rev_arith).
template <int AM, bool SWAP>
__device__ __forceinline__ void act_pack8(const float v[8], uint32_t (&w)[8]) {
  auto put = [&](const uint32_t e0, const uint32_t e1, const uint32_t o0, const uint32_t o1, uint32_t* out) {
    if constexpr (!SWAP) {
      out[0] = e0;
      out[1] = e1;
      out[2] = o0;
      out[3] = o1;
      return;
    }
    // e: g even (kh 0), o: g odd (kh 1).  Lanes 32..63 of the first operand trade
    // with lanes 0..31 of the second: afterwards lane (n0, kh) has k%8 in [0, 4)
    // in the first and [4, 8) in the second
    const auto s0 = __builtin_amdgcn_permlane32_swap(e0, o0, false, false);
    const auto s1 = __builtin_amdgcn_permlane32_swap(e1, o1, false, false);
    out[0] = s0[0];
    out[1] = s1[0];
    out[2] = s0[1];
    out[3] = s1[1];
  };
  uint32_t d[4];  // bf16 pairs (v0 v1), (v2 v3), (v4 v5), (v6 v7)
  pack4<AM>(v, d[0], d[1]);
  pack4<AM>(v + 4, d[2], d[3]);
  if constexpr (AM == kBF16X2) {
    // lo = v - hi, with hi read back from the packed pairs (the same rounding);
    // formed before the swaps, which overwrite their operands
    float lo[8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      lo[2 * k] = v[2 * k] - __uint_as_float(d[k] << 16);
      lo[2 * k + 1] = v[2 * k + 1] - __uint_as_float(d[k] & 0xffff0000u);
    }
    uint32_t l[4];
    pack4<AM>(lo, l[0], l[1]);
    pack4<AM>(lo + 4, l[2], l[3]);
    put(l[0], l[1], l[2], l[3], w + 4);
  }
  put(d[0], d[1], d[2], d[3], w);
}

template <int W, int MODE, int I, int GP, int NT, int AM = fwd_arith<MODE>()>
__device__ __forceinline__ void act_write8(const Lane<W, MODE>& L, const uint32_t (&w)[8]) {
  constexpr int off = (2 * I + GP) * Geo<W, MODE>::STEP_BYTES + NT * 512;
  typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;
  *reinterpret_cast<u32x4*>(L.act_w + off) = u32x4{w[0], w[1], w[2], w[3]};
  if constexpr (AM == kBF16X2) *reinterpret_cast<u32x4*>(L.act_w_lo + off) = u32x4{w[4], w[5], w[6], w[7]};
}

template <int W, int MODE, int I, int GP, int NT, int AM = fwd_arith<MODE>()>
__device__ __forceinline__ void act_store8(const Lane<W, MODE>& L, const float v[8]) {
  uint32_t w[8];
  act_pack8<AM, !lane_k_order<MODE>()>(v, w);
  act_write8<W, MODE, I, GP, NT, AM>(L, w);
}

// Either layout: rows of groups g = 2 GP, 2 GP + 1 (see act_store8).
template <int W, int MODE, int I, int GP, int NT, int AM = fwd_arith<MODE>()>
__device__ __forceinline__ void act_store_pair(const Lane<W, MODE>& L, const float v[8]) {
  if constexpr (MODE == kFP32) {
    act_store4_fp32<W, MODE, I, 2 * GP, NT>(L, v);
    act_store4_fp32<W, MODE, I, 2 * GP + 1, NT>(L, v + 4);
  } else {
    act_store8<W, MODE, I, GP, NT, AM>(L, v);
  }
}

// Compile-time loop helper: f(integral_constant<0>), ..., f(integral_constant<N-1>).
template <int N, int B = 0, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < N) {
    f(std::integral_constant<int, B>{});
    static_for<N, B + 1>(f);
  }
}

// ----------------------------------------------------------------------------
// acc[i][nt] += M[rows of wave, :] x act[:, 32nt .. 32nt+31]
// A fragments come through a buffer descriptor (uniform, SGPRs) of the matrix's
// packed stream, laid out for 4 row groups of PMT M tiles: fragment (kstep, j) of
// row group p at byte p*stream_bytes + ((kstep*PMT + j)*64 + lane)*16.  A wave
// that is share s of group p reads j = s*MT + i, so one 32-bit VGPR offset
// (voff = p*stream_bytes + s*MT*1024 + lane*16) serves every matrix and step; the
// step goes in the scalar offset and i*1024 in the instruction's immediate.
// Software pipeline: A is loaded two K steps ahead, B (LDS) one step ahead.
// AM is the K loop's arithmetic (fwd_arith / rev_arith of the tile's mode).
// ----------------------------------------------------------------------------
template <int AM>
struct BFrag {
  bf16x8 h[2], l[2];
  f32x4 f[2];
};

template <int W, int MODE, int AM>
__device__ __forceinline__ void load_b(BFrag<AM>& b, const char* br) {
  if constexpr (AM == kFP32) {
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) b.f[nt] = *reinterpret_cast<const f32x4*>(br + nt * 1024);
  } else {
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      b.h[nt] = *reinterpret_cast<const bf16x8*>(br + nt * 512);
      if constexpr (AM == kBF16X2) b.l[nt] = *reinterpret_cast<const bf16x8*>(br + Geo<W, MODE>::LO_OFF + nt * 512);
    }
  }
}

template <int W, int MODE>
__device__ __forceinline__ void load_a(f32x4 (&af)[(Geo<W, MODE>::MT)], __amdgpu_buffer_rsrc_t rs, int voff, int step) {
  const int soff = step * Geo<W, MODE>::PMT * 1024;
#pragma unroll
  for (int i = 0; i < Geo<W, MODE>::MT; ++i)
    af[i] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff + i * 1024, soff, 0));
}

// One K step: for each M tile i, its MFMAs (hi then lo halves alternating over
// the two column blocks, so accumulations into one tile are two MFMAs apart),
// then at once the reload of a[i] for step `next` -- the fragment's registers
// are free as soon as its last MFMA has issued.  The scheduling barriers keep
// the compiler from sinking the loads to the end of the loop body.  ZC: the
// accumulators start at zero, so the first product of each tile reads a zero C
// operand instead of registers cleared beforehand.
template <int W, int MODE, int AM, bool ZC = false>
__device__ __forceinline__ void mma_step_reload(f32x16 (&acc)[(Geo<W, MODE>::MT)][2], f32x4 (&af)[(Geo<W, MODE>::MT)],
                                                const BFrag<AM>& b, __amdgpu_buffer_rsrc_t rs, int voff,
                                                int next) {
  constexpr int MT = Geo<W, MODE>::MT;
  const int soff = next * Geo<W, MODE>::PMT * 1024;
  const f32x16 zero = {};
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    if constexpr (AM == kFP32) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
          acc[i][nt] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i][q], b.f[nt][q], (ZC && q == 0) ? zero : acc[i][nt],
                                                            0, 0, 0);
    } else if constexpr (AM == kF16) {
      const f16x8 a8 = __builtin_bit_cast(f16x8, af[i]);
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
        acc[i][nt] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a8, __builtin_bit_cast(f16x8, b.h[nt]),
                                                            ZC ? zero : acc[i][nt], 0, 0, 0);
    } else {
      const bf16x8 a8 = __builtin_bit_cast(bf16x8, af[i]);
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
        acc[i][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a8, b.h[nt], ZC ? zero : acc[i][nt], 0, 0, 0);
      if constexpr (AM == kBF16X2) {
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
          acc[i][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a8, b.l[nt], acc[i][nt], 0, 0, 0);
      }
    }
    af[i] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff + i * 1024, soff, 0));
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int W, int MODE>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t stream_rsrc(const void* base) {
  constexpr int bytes = W * W * (MODE == kFP32 ? 4 : 2);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}

// The A fragments of a layer's first two K steps, loaded ahead of the layer.
// Training loads them before the previous layer's dump: the vector-memory counter
// completes in order, so a wait for fragments issued after the dump's stores
// would also wait for those stores.
template <int W, int MODE>
struct APre {
  f32x4 a0[Geo<W, MODE>::MT], a1[Geo<W, MODE>::MT];
};
template <int W, int MODE>
__device__ __forceinline__ void preload_a(APre<W, MODE>& p, __amdgpu_buffer_rsrc_t rs, int voff) {
  load_a<W, MODE>(p.a0, rs, voff, 0);
  load_a<W, MODE>(p.a1, rs, voff, 1);
}

// ZERO: acc starts at zero (its contents on entry are not read).  a0, a1: the A
// fragments of steps 0 and 1, already requested (preload_a).
template <int W, int MODE, int AM, bool ZERO = false>
__device__ __forceinline__ void layer_gemm_pre(f32x16 (&acc)[(Geo<W, MODE>::MT)][2], __amdgpu_buffer_rsrc_t rs,
                                               int voff, const char* br, f32x4 (&a0)[(Geo<W, MODE>::MT)],
                                               f32x4 (&a1)[(Geo<W, MODE>::MT)]) {
  constexpr int NS = (MODE == kFP32) ? Geo<W, MODE>::NK8 : Geo<W, MODE>::NKB;  // even, >= 16
  constexpr int SB = Geo<W, MODE>::STEP_BYTES;
  BFrag<AM> b0, b1;
  load_b<W, MODE, AM>(b0, br);
  int s = 0;
  if constexpr (ZERO) {  // steps 0 and 1, the first writing acc from a zero C operand
    load_b<W, MODE, AM>(b1, br + SB);
    __builtin_amdgcn_sched_barrier(0);
    mma_step_reload<W, MODE, AM, true>(acc, a0, b0, rs, voff, 2);
    load_b<W, MODE, AM>(b0, br + 2 * SB);
    __builtin_amdgcn_sched_barrier(0);
    mma_step_reload<W, MODE, AM>(acc, a1, b1, rs, voff, 3);
    br += 2 * SB;
    s = 2;
  }
#pragma unroll 1
  for (; s < NS; s += 2) {
    load_b<W, MODE, AM>(b1, br + SB);  // B of step s+1, one step ahead
    __builtin_amdgcn_sched_barrier(0);
    mma_step_reload<W, MODE, AM>(acc, a0, b0, rs, voff, s + 2 < NS ? s + 2 : NS - 1);
    load_b<W, MODE, AM>(b0, s + 2 < NS ? br + 2 * SB : br);  // B of step s+2
    __builtin_amdgcn_sched_barrier(0);
    mma_step_reload<W, MODE, AM>(acc, a1, b1, rs, voff, s + 3 < NS ? s + 3 : NS - 1);
    br += 2 * SB;
  }
}

template <int W, int MODE, int AM, bool ZERO = false>
__device__ __forceinline__ void layer_gemm(f32x16 (&acc)[(Geo<W, MODE>::MT)][2], __amdgpu_buffer_rsrc_t rs, int voff,
                                           const char* br) {
  APre<W, MODE> p;
  preload_a<W, MODE>(p, rs, voff);
  layer_gemm_pre<W, MODE, AM, ZERO>(acc, rs, voff, br, p.a0, p.a1);
}

// The reverse layers' accumulators start at zero: in single FP16 the first
// products read a zero C operand (no clearing moves); the split forms clear the
// registers first (the peeled first steps cost them spilled registers at W=512).
template <int MODE>
constexpr bool rev_zero_c() {
  return rev_arith<MODE>() == kF16;
}
template <int W, int MODE>
__device__ __forceinline__ void zero_acc(f32x16 (&acc)[(Geo<W, MODE>::MT)][2]) {
#pragma unroll
  for (int i = 0; i < Geo<W, MODE>::MT; ++i)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[i][nt][j] = 0.f;
}

__device__ __forceinline__ uint32_t ordered_bits(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// ----------------------------------------------------------------------------
// Training: copy the LDS activation tile (hi plane for the BF16 modes) to HBM in
// the blocked feature-major layout: element (f, i) of a [W x batch] array sits at
// ((i / S) * W + f) * S + i % S with S = 16 bytes of samples (8 BF16 or 4 FP32),
// so the 16-byte fragments of consecutive features are adjacent.  Zeros for the
// ragged tail of the tile.  All threads take part.  (The stores go through the
// caches on purpose: the weight-gradient kernels that follow read the dumps back,
// largely from the last-level cache; non-temporal stores made the backward pass
// half again as slow.)
// BF16: the tile is transposed into `stage` (32 KiB of LDS, the idle half of a
// pure-BF16 tile) and then copied out, so that a wave's store instruction writes
// 1 KiB of consecutive pieces instead of 16 bytes into each of 64 cache lines.
// Piece P (16 bytes: 8 samples of one feature) sits at slot P ^ ((P >> 4) & 7),
// which spreads the 16 pieces written by 16 consecutive lanes over 16 different
// bank groups, and those read by 16 consecutive lanes too.
// BF16, with sums: the copy also adds, over the tile's samples i, to LDS rows
// (per feature f) sum_i x[f][i] w_i (w_i = seed_i, or 1) in a fixed order
// (samples within a piece, pieces in order, then the two lanes sharing a
// feature), and optionally sum_i x[f][i] v_c(i) for the nine network inputs v_c
// on the matrix cores (the pieces are the A fragments of a 32 x 32 x 16 product
// over samples; v is split into BF16 hi + lo).  In the copy, wave w owns features
// 32w .. 32w + 31, its lane halves taking alternate 8-sample blocks.  store
// false: the sums only, nothing written to HBM.
// ----------------------------------------------------------------------------
struct DumpSums {
  float* row;          // [W]: sum_i x[f][i] w_i
  const float* seed;   // w_i = seed[i * XIN_FLOATS] (the records' seed slot), or NULL: w_i = 1
  float* in_rows;      // [9][W]: sum_i x[f][i] v_c(i), or NULL
  const __bf16* vt;    // the tile's inputs v_c(i) as BF16 hi [9][64], then lo [9][64]
};

template <int W, int MODE>
__device__ __forceinline__ void dump_tile(const char* act, char* stage, void* dst, int64_t ldb, int64_t q0,
                                          int nvalid, const DumpSums* sums = nullptr, bool store = true) {
  (void)ldb;
  for (int f = threadIdx.x; f < W && MODE == kFP32; f += Geo<W, MODE>::THREADS) {
    const float* a = reinterpret_cast<const float*>(act);
#pragma unroll 4
    for (int n = 0; n < kTileQ; n += 4) {
      f32x4 v;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int nn = n + u;
        v[u] = nn < nvalid ? a[(((f >> 3) * kTileQ + nn) * 2 + (f & 1)) * 4 + ((f & 7) >> 1)] : 0.f;
      }
      float* o = static_cast<float*>(dst) + (((q0 + n) >> 2) * W + f) * 4;
      *reinterpret_cast<f32x4*>(o) = v;
    }
  }
  if constexpr (MODE != kFP32) {
    // The hi plane holds, for each group of 8 features and each query n, the 8
    // features' values as one 16-byte word.  A thread reads the 8x8 block of 8
    // consecutive queries, transposes it in registers and stages the 8 features'
    // 16-byte pieces of that query block; then every thread copies pieces out.
    static_assert(MODE == kBF16 && W * kTileQ * 2 <= Geo<W, MODE>::ACT_BYTES / 2, "staging needs a pure-BF16 tile");
    typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;
    const char* a = act;
    constexpr int NG = W / 8;  // feature groups
    constexpr int NP = W * (kTileQ / 8);  // pieces: (query block nb, feature f) at nb W + f
    // Each wave stages exactly the pieces it copies out below (features 32 w ..
    // 32 w + 31: feature groups 4 w .. 4 w + 3, every query block), so the copy
    // needs no workgroup barrier: one wave's LDS operations complete in order.
    static_assert(Geo<W, MODE>::NW * 4 == NG, "each wave stages four feature groups");
    if ((threadIdx.x & 63) < 32) {
      const int g8 = 4 * (threadIdx.x >> 6) + (threadIdx.x & 3), nb = (threadIdx.x & 31) >> 2;
      const int gbyte = (g8 >> 1) * Geo<W, MODE>::STEP_BYTES + (g8 & 1) * 1024;  // 16-feature step, 8-feature half
      u32x4 m[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int n = nb * 8 + j;
        m[j] = n < nvalid ? *reinterpret_cast<const u32x4*>(a + gbyte + n * 16) : u32x4{0u, 0u, 0u, 0u};
      }
#pragma unroll
      for (int fl = 0; fl < 8; ++fl) {  // feature 8 g8 + fl: halves of word fl/2 of every m[j]
        u32x4 row;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const uint32_t x0 = m[2 * jj][fl >> 1], x1 = m[2 * jj + 1][fl >> 1];
          row[jj] = (fl & 1) ? ((x0 >> 16) | (x1 & 0xffff0000u)) : ((x0 & 0xffffu) | (x1 << 16));
        }
        const int P = nb * W + 8 * g8 + fl;
        *reinterpret_cast<u32x4*>(stage + (P ^ ((P >> 4) & 7)) * 16) = row;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // the tile's pieces are consecutive in the dump: piece P at element ((q0 / 8) W + P) 8
    constexpr int T = Geo<W, MODE>::THREADS;
    static_assert(T % W == 0, "a thread's pieces share one feature");
    constexpr int XF = Geo<W, MODE>::XIN_FLOATS;
    static_assert(T / 64 == W / 32 && NP == T * 4, "the copy: one 32-feature block per wave, 4 rounds");
    const int lane = threadIdx.x & 63, half = lane >> 5;
    const int f = 32 * (threadIdx.x >> 6) + (lane & 31);
    __bf16* o = static_cast<__bf16*>(dst) + (q0 >> 3) * W * 8;
    float part = 0.f;
    f32x16 dacc;
#pragma unroll
    for (int j = 0; j < 16; ++j) dacc[j] = 0.f;
    const int c = lane & 31;  // input column of the v fragments
#pragma unroll
    for (int st = 0; st < kTileQ / 16; ++st) {  // 16 samples per round: blocks 2 st (lanes < 32), 2 st + 1
      const int nb = 2 * st + half;
      const int P = nb * W + f;
      const u32x4 v = *reinterpret_cast<const u32x4*>(stage + (P ^ ((P >> 4) & 7)) * 16);
      if (store) *reinterpret_cast<u32x4*>(o + P * 8) = v;
      if (sums) {
        const int n0 = nb * 8;  // word w: samples n0 + 2w (low half), n0 + 2w + 1
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const uint32_t word = v[e >> 1];
          const float x = __uint_as_float((e & 1) ? (word & 0xffff0000u) : (word << 16));
          part += sums->seed ? x * sums->seed[(n0 + e) * XF] : x;
        }
        if (sums->in_rows) {
          // A: 8 samples of feature f (lane = (f % 32, half)); B: v_c of the same 8
          // samples (lane = (c, half)), hi then lo
          const bf16x8 a = __builtin_bit_cast(bf16x8, v);
          bf16x8 bh, bl;
          if (c < 9) {
            bh = *reinterpret_cast<const bf16x8*>(sums->vt + c * kTileQ + n0);
            bl = *reinterpret_cast<const bf16x8*>(sums->vt + (9 + c) * kTileQ + n0);
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) bh[e] = bl[e] = (__bf16)0.f;
          }
          dacc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bh, dacc, 0, 0, 0);
          dacc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bl, dacc, 0, 0, 0);
        }
      }
    }
    if (sums) {
      part += __shfl_xor(part, 32);
      if (half == 0) sums->row[f] += part;
      if (sums->in_rows && c < 9) {
        // C layout: lane (c, half) holds rows 8 (j/4) + 4 half + j%4 of the wave's 32 features
        float* r = sums->in_rows + c * W + 32 * (threadIdx.x >> 6);
#pragma unroll
        for (int j = 0; j < 16; ++j) r[8 * (j >> 2) + 4 * half + (j & 3)] += dacc[j];
      }
    }
  }
}

// ----------------------------------------------------------------------------
// Layer bodies (compile-time layer index so every register array is static).
// Element j of acc[i][nt] is row R = rbase + 32 i + 8 (j/4) + 4 (lane/32) + j%4
// of the layer output and query column n = 32 nt + lane%32.
// ----------------------------------------------------------------------------
// Row-indexed vectors (b1..b4, w_out, the input-layer rows and the per-knot
// arm term) are stored in lane-major order: the 16*MT rows one lane touches,
// R = rbase + 32 i + 8 g + 4 h + r, sit at position
// ((p*2 + h)*PMT + s*MT + i)*16 + 4 g + r for a wave that is share s of row
// group p (with 4 waves, p = wave, s = 0, PMT = MT), so each lane addresses them
// from one base with small constant offsets.
template <int W, int MODE>
struct Bases {
  const float* bh;    // LDS copy of b2, b3, b4 (lane-major), at this lane's block
  const float* w5;    // LDS copy of w_out (lane-major), at this lane's block
  const float* w1;    // input layer rows (lane-major, 12 floats per row), at this lane's block
  const float* w1a;   // input layer row rbase + lane%32 (its A fragment row in M tile 0; tile i at +16 i rows)
  const float* crow;  // per-knot input-layer constant (LDS, lane-major), at this lane's block
  const float* xin;   // xin + n0 * XIN_FLOATS
  int voff;           // lane offset inside a matrix's fragment stream (see load_a)
};

// Dump of the current LDS tile for training (no-op when not training).
struct TileDump {
  const char* act;  // the LDS activation tile
  char* stage;      // BF16: LDS staging of a dump (the tile's idle half)
  void* H;
  void* G;
  int64_t ldb, q0;
  int nvalid;
  size_t layer_elems;  // W * ldb
  size_t elem_bytes;
  // fused MSE loss (Job::target): per-wave output partial sums, the per-query
  // records (slot 11 takes the seed), and the loss terms
  float* dred;
  float* xin;
  const float* target;
  float* seed_out;
  float* sq_out;
  float* d_out;  // the distances, when asked for
  float mse_scale, inv_b;
  float b5;  // the output bias
  // per-workgroup sums over its samples (LDS, [kTrainSumRows][width]; NULL when
  // these gradients are reduced from the dumps instead): rows 0..3 the bias
  // gradients sum_i g_l (l = 1..4), row 4 dL/dw_out = sum_i seed_i h4_i, rows
  // 5..13 dW1[:, c] = sum_i g1_i v_c(i), row 14 (first entry) db_out = sum_i seed_i,
  // row 15 (first entry) the fused loss sum_i (d_i - target_i)^2 / B
  float* bsum;
  __bf16* vt;  // with bsum: the tile's network inputs, transposed, BF16 hi [9][64] then lo
  float* sp1;  // BF16: SiLU'(z1) of the input layer kept in LDS for the reverse sweep (see train_sp1)
  int width;
  __device__ __forceinline__ float* row(int r) const { return bsum ? bsum + r * width : nullptr; }
  __device__ __forceinline__ void* h(int l) const { return static_cast<char*>(H) + l * layer_elems * elem_bytes; }
  __device__ __forceinline__ void* g(int l) const { return static_cast<char*>(G) + l * layer_elems * elem_bytes; }
};

// Whether a hidden-layer epilogue keeps its packed results in registers across
// the barrier (two waves per SIMD).  At width 512 the last forward layer, which
// also carries the output-layer sums, would spill, so it stores after the barrier
// as before; so does training's last forward layer, which stores h4 first.
template <int W, int MODE, bool TRAIN>
constexpr bool defer_stores(bool last_forward) {
  return Geo<W, MODE>::SUB > 1 && (!last_forward || (Geo<W, MODE>::MT == 1 && !TRAIN));
}

// The packed words of elements 8 GP .. 8 GP + 7 of an accumulator go back into
// those elements (consumed in order, so no extra registers), and are written out
// after the barrier.
template <int MODE, int AM, int GP>
__device__ __forceinline__ void park_packed(const float v[8], f32x16& a) {
  uint32_t w[8];
  act_pack8<AM, !lane_k_order<MODE>()>(v, w);
  constexpr int NWORDS = AM == kBF16X2 ? 8 : 4;  // hi and lo words, or hi only
#pragma unroll
  for (int k = 0; k < NWORDS; ++k) a[8 * GP + k] = __uint_as_float(w[k]);
}

template <int W, int MODE, int AM>
__device__ __forceinline__ void write_packed(const Lane<W, MODE>& ln, const f32x16 (&acc)[(Geo<W, MODE>::MT)][2]) {
  static_for<Geo<W, MODE>::MT>([&](auto I) {
    static_for<2>([&](auto GP) {
      static_for<2>([&](auto NT) {
        uint32_t w[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) w[k] = __float_as_uint(acc[I][NT][8 * GP + k]);
        act_write8<W, MODE, I, GP, NT, AM>(ln, w);
      });
    });
  });
}

template <int W, int MODE, int L, bool TRAIN>
__device__ __forceinline__ void fwd_hidden(const DevNet& net, const Lane<W, MODE>& ln, const Bases<W, MODE>& b,
                                           float (&sp)[2][(Geo<W, MODE>::MT)][2][16], float (&dpart)[2], int want_grad,
                                           const TileDump& td, APre<W, MODE>& ap) {
  constexpr int MT = Geo<W, MODE>::MT;
  f32x16 acc[MT][2];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const f32x4 b4 = *reinterpret_cast<const f32x4*>(b.bh + L * W + 16 * i + 4 * g);
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][nt][4 * g + r] = b4[r];
    }
  if constexpr (TRAIN)
    layer_gemm_pre<W, MODE, fwd_arith<MODE>()>(acc, stream_rsrc<W, MODE>(net.fwd[L]), b.voff, ln.act_r, ap.a0, ap.a1);
  else
    layer_gemm<W, MODE, fwd_arith<MODE>()>(acc, stream_rsrc<W, MODE>(net.fwd[L]), b.voff, ln.act_r);
  // arithmetic of what this layer stores: the next layer's activations, or g4
  // for the reverse sweep
  constexpr int SA = L == 2 ? rev_arith<MODE>() : fwd_arith<MODE>();
  // With two waves per SIMD the epilogue arithmetic runs before the barrier (the
  // results wait in registers), overlapping the K loops of waves still running;
  // only the stores into the tile they read wait for it.
  constexpr bool DEFER = defer_stores<W, MODE, TRAIN>(L == 2);
  if constexpr (!DEFER) __syncthreads();
  if constexpr (TRAIN && L == 2) {
    // training: the layer-4 activations h4 go through LDS first (for dL/dw_out),
    // and the output-layer partial sums are taken here, so that a fused loss can
    // finish d before the reverse sweep
    static_for<MT>([&](auto I) {
      static_for<2>([&](auto GP) {
        const f32x4 w5r[2] = {*reinterpret_cast<const f32x4*>(b.w5 + 16 * I + 8 * GP),
                              *reinterpret_cast<const f32x4*>(b.w5 + 16 * I + 8 * GP + 4)};
        static_for<2>([&](auto NT) {
          float v[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            // SiLU' replaces z4 in the accumulator, for g4 below
            float dv;
            silu_fwd(acc[I][NT][8 * GP + q], v[q], dv);
            acc[I][NT][8 * GP + q] = dv;
            dpart[NT] += w5r[q >> 2][q & 3] * v[q];
          }
          act_store_pair<W, MODE, I, GP, NT>(ln, v);
        });
      });
    });
    if (td.target) {
      // d over the rows: lane halves, then waves in order, as at the end of the tile
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const float dp = dpart[nt] + __shfl_xor(dpart[nt], 32);
        if (ln.h == 0) td.dred[ln.wave * kTileQ + 32 * nt + ln.n0] = dp;
      }
    }
    __syncthreads();
    if (threadIdx.x < kTileQ && (td.target || td.bsum)) {  // wave 0, one lane per query
      const int n = threadIdx.x;
      float* seedp = td.xin + n * Geo<W, MODE>::XIN_FLOATS + 11;
      float sq = 0.f;
      if (td.target) {
        float sum = td.dred[n];
#pragma unroll
        for (int w = 1; w < Geo<W, MODE>::NW; ++w) sum += td.dred[w * kTileQ + n];
        const float dv = sum + td.b5;
        const bool valid = n < td.nvalid;
        const int64_t q = td.q0 + n;
        const float r = valid ? dv - td.xin[n * Geo<W, MODE>::XIN_FLOATS + kXinTarget] : 0.f;
        const float seed = td.mse_scale * r;  // dL/dd for L = mean (d - target)^2
        sq = td.inv_b * (r * r);
        *seedp = seed;
        if (valid && td.d_out) td.d_out[q] = dv;
        if (valid && td.seed_out) {  // for the reductions from the dumps (FP32)
          td.seed_out[q] = seed;
          td.sq_out[q] = sq;
        }
      }
      if (td.bsum) {
        // db_out = sum_i seed_i and the loss, over the tile (fixed butterfly), then
        // over this workgroup's tiles in order
        float sd = *seedp;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
          sd += __shfl_xor(sd, off);
          sq += __shfl_xor(sq, off);
        }
        if (n == 0) {
          td.row(14)[0] += sd;
          td.row(15)[0] += sq;
        }
      }
    }
    // h4 is needed only for dL/dw_out = sum_i seed_i h4_i: summed here when the
    // tile engine keeps the bias sums, else written out (after a barrier: wave 0
    // wrote the seeds the copy reads)
    __syncthreads();
    const DumpSums sm{td.row(4), td.xin + 11, nullptr, td.vt};
    dump_tile<W, MODE>(td.act, td.stage, td.h(3), td.ldb, td.q0, td.nvalid, td.bsum ? &sm : nullptr, !td.bsum);
    __syncthreads();  // h4 fully read before g4 overwrites the tile; seeds written
  }
  static_for<MT>([&](auto I) {
    static_for<2>([&](auto GP) {
      f32x4 w5r[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
      if constexpr (L == 2) {
        w5r[0] = *reinterpret_cast<const f32x4*>(b.w5 + 16 * I + 8 * GP);
        w5r[1] = *reinterpret_cast<const f32x4*>(b.w5 + 16 * I + 8 * GP + 4);
      }
      static_for<2>([&](auto NT) {
        const float seed = b.xin[NT * 32 * Geo<W, MODE>::XIN_FLOATS + 11] * rev_scale<MODE>();
        float v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int j = 8 * GP + q;  // accumulator element: g = 2 GP + q/4, r = q%4
          float hv, dv;
          if constexpr (TRAIN && L == 2) dv = acc[I][NT][j];  // SiLU'(z4), kept above
          else silu_fwd(acc[I][NT][j], hv, dv);
          if constexpr (L < 2) {
            sp[L][I][NT][j] = park(dv);
            v[q] = hv;
          } else {
            if constexpr (!TRAIN) dpart[NT] += w5r[q >> 2][q & 3] * hv;  // (training: summed above)
            v[q] = seed * (w5r[q >> 2][q & 3] * dv);  // g4 = seed * w5 * SiLU'(z4)
          }
        }
        if (L < 2 || want_grad) {
          if constexpr (DEFER) park_packed<MODE, SA, GP>(v, acc[I][NT]);
          else act_store_pair<W, MODE, I, GP, NT, SA>(ln, v);
        }
      });
      __builtin_amdgcn_sched_barrier(0);
    });
  });
  if constexpr (L == 2) {
    // Materialise the output-layer partial sums here; left alone, the compiler
    // sinks them to their use after the reverse sweep and keeps every h4 and
    // w_out value live through it.
    asm volatile("" : "+v"(dpart[0]), "+v"(dpart[1]));
  }
  if constexpr (DEFER) {
    __syncthreads();  // every wave has finished reading the tile
    if (L < 2 || want_grad) write_packed<W, MODE, SA>(ln, acc);
  }
  __syncthreads();
  // training: h2, h3 (layers 2, 3) or g4 (layer 4) to HBM; the tile is next
  // overwritten only after the following K loop and its barrier
  if constexpr (TRAIN) {  // h2, h3, or g4 (with db4 = sum_i g4_i)
    preload_a<W, MODE>(ap, stream_rsrc<W, MODE>(L < 2 ? net.fwd[L + 1] : net.bwd[2]), b.voff);  // the next layer's
    const DumpSums sm{td.row(3), nullptr, nullptr, td.vt};
    dump_tile<W, MODE>(td.act, td.stage, L < 2 ? td.h(L + 1) : td.g(3), td.ldb, td.q0, td.nvalid,
                       (L == 2 && td.bsum) ? &sm : nullptr);
  }
}

template <int W, int MODE, int L, bool TRAIN>
__device__ __forceinline__ void bwd_hidden(const DevNet& net, const Lane<W, MODE>& ln, const Bases<W, MODE>& b,
                                           const float (&sp)[2][(Geo<W, MODE>::MT)][2][16], const TileDump& td,
                                           APre<W, MODE>& ap) {
  constexpr int MT = Geo<W, MODE>::MT;
  f32x16 acc[MT][2];
  constexpr int RA = rev_arith<MODE>();
  // Single FP16 products use only the hi halves of the tile, so the two reverse
  // layers alternate halves: g4 (hi) -> g3 (lo) -> g2 (hi).  Nobody reads the half
  // a layer writes, so its stores need no barrier before them.
  constexpr bool PP = RA == kF16 && !TRAIN;
  const char* br = (PP && L == 1) ? ln.act_r + Geo<W, MODE>::LO_OFF : ln.act_r;
  if constexpr (!rev_zero_c<MODE>()) zero_acc<W, MODE>(acc);
  if constexpr (TRAIN)
    layer_gemm_pre<W, MODE, RA, rev_zero_c<MODE>()>(acc, stream_rsrc<W, MODE>(net.bwd[L]), b.voff, br, ap.a0, ap.a1);
  else
    layer_gemm<W, MODE, RA, rev_zero_c<MODE>()>(acc, stream_rsrc<W, MODE>(net.bwd[L]), b.voff, br);
  constexpr bool DEFER = !PP && defer_stores<W, MODE, TRAIN>(false);  // as in fwd_hidden
  if constexpr (!DEFER && !PP) __syncthreads();
  static_for<MT>([&](auto I) {
    static_for<2>([&](auto GP) {
      static_for<2>([&](auto NT) {
        float v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int j = 8 * GP + q;
          v[q] = acc[I][NT][j] * unpark(sp[L - 1][I][NT][j], acc[I][NT][j]);
        }
        if constexpr (PP) {
          uint32_t w[8];
          act_pack8<RA, !lane_k_order<MODE>()>(v, w);
          typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;
          constexpr int off = (2 * I + GP) * Geo<W, MODE>::STEP_BYTES + NT * 512;
          *reinterpret_cast<u32x4*>((L == 2 ? ln.act_w_lo : ln.act_w) + off) = u32x4{w[0], w[1], w[2], w[3]};
        } else if constexpr (DEFER) {
          park_packed<MODE, RA, GP>(v, acc[I][NT]);
        } else {
          act_store_pair<W, MODE, I, GP, NT, RA>(ln, v);
        }
      });
      __builtin_amdgcn_sched_barrier(0);
    });
  });
  if constexpr (DEFER) {
    __syncthreads();  // every wave has finished reading the tile
    write_packed<W, MODE, RA>(ln, acc);
  }
  __syncthreads();
  if constexpr (TRAIN) {  // g3 or g2, with their bias sums
    preload_a<W, MODE>(ap, stream_rsrc<W, MODE>(net.bwd[L - 1]), b.voff);  // the next layer's
    const DumpSums sm{td.row(L), nullptr, nullptr, td.vt};
    dump_tile<W, MODE>(td.act, td.stage, td.g(L), td.ldb, td.q0, td.nvalid, td.bsum ? &sm : nullptr);
  }
}

// Pure-BF16 pair-list tiles of width 256 (point obstacles; the training
// configuration) take the input layer's pre-activations from the matrix cores:
// z1 = b1 + W1 v over the 9 inputs, K
// padded to 16 (p' at k = 0..2, the arm joints at 3..8), as the split products
// W1h vh + W1h vl + W1l vh accumulated in FP32 (h: the BF16 rounding, l: the BF16
// rounding of the rest; the terms left out are below 2^-16 |W1| |v|).  The
// prologue stages the tile's inputs as B fragments at `vb` (query n at byte 64 n:
// 16 BF16 hi, then 16 lo).  The forward and the reverse sweep's recomputation
// both call this for M tile I, so they see the same z1.
template <int W, int MODE>
constexpr bool mma_input(bool pairs, bool sph) {
  return W == 256 && MODE == kBF16 && pairs && !sph;  // (at width 512 the recomputation would spill)
}
constexpr int kVbBytes = 64;  // per query: B fragments of the inputs, hi then lo

template <int W, int MODE, int I>
__device__ __forceinline__ void input_gemm(const Lane<W, MODE>& ln, const Bases<W, MODE>& b, const char* vb,
                                           f32x16 (&z)[2]) {
  bf16x8 bh[2], bl[2];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const char* p = vb + (32 * nt + ln.n0) * kVbBytes + ln.kh * 16;
    bh[nt] = *reinterpret_cast<const bf16x8*>(p);
    bl[nt] = *reinterpret_cast<const bf16x8*>(p + 32);
  }
  // A: row m = lane%32 of the tile, inputs 8 kh .. 8 kh + 7
  const float* w = b.w1a + I * 16 * 12;
  const f32x4 wa = *reinterpret_cast<const f32x4*>(w);
  const f32x4 wb = *reinterpret_cast<const f32x4*>(w + 4);
  const f32x2 wc = *reinterpret_cast<const f32x2*>(w + 8);
  const float lo8[8] = {wa[0], wa[1], wa[2], wb[0], wb[1], wb[2], wb[3], wc[0]};  // k = 0..7 (slot 3 is b1)
  bf16x8 ah, al;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float a = ln.kh ? (e == 0 ? wc[1] : 0.f) : lo8[e];  // k = 8: the last arm joint
    const __bf16 hi = (__bf16)a;
    ah[e] = hi;
    al[e] = (__bf16)(a - (float)hi);
  }
  // b1 of the accumulator layout's rows (lane-major block of this lane)
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float bias = b.w1[(16 * I + 4 * g + r) * 12 + 3];
      z[0][4 * g + r] = bias;
      z[1][4 * g + r] = bias;
    }
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    z[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[nt], z[nt], 0, 0, 0);
    z[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[nt], z[nt], 0, 0, 0);
    z[nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[nt], z[nt], 0, 0, 0);
  }
}

// Last reverse layer: g1 = (W2^T g2) * SiLU'(z1) with z1 recomputed, then the
// input-layer gradient e = W1^T g1 accumulated per lane in FP32.
template <int W, int MODE, bool PAIRS, bool TRAIN, bool SPH, class F>
__device__ __forceinline__ void bwd_input(const DevNet& net, const Lane<W, MODE>& ln, const Bases<W, MODE>& b,
                                          float (&epart)[2][9], const TileDump& td, const char* vb,
                                          APre<W, MODE>& ap, F&& before_copy) {
  constexpr int MT = Geo<W, MODE>::MT;
  constexpr int XF = Geo<W, MODE>::XIN_FLOATS;
  f32x16 acc[MT][2];
  if constexpr (!rev_zero_c<MODE>()) zero_acc<W, MODE>(acc);
  if constexpr (TRAIN)
    layer_gemm_pre<W, MODE, rev_arith<MODE>(), rev_zero_c<MODE>()>(acc, stream_rsrc<W, MODE>(net.bwd[0]), b.voff,
                                                                   ln.act_r, ap.a0, ap.a1);
  else
    layer_gemm<W, MODE, rev_arith<MODE>(), rev_zero_c<MODE>()>(acc, stream_rsrc<W, MODE>(net.bwd[0]), b.voff,
                                                               ln.act_r);
  float g1keep[TRAIN ? MT : 1][2][16];
  constexpr bool KEPT = TRAIN && MODE == kBF16;  // SiLU'(z1) kept by the input layer
  if constexpr (KEPT) {
    constexpr int T = Geo<W, MODE>::THREADS;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const f32x4 sv = *reinterpret_cast<const f32x4*>(td.sp1 + (((i * 2 + nt) * 4 + g) * T + threadIdx.x) * 4);
#pragma unroll
          for (int r = 0; r < 4; ++r) g1keep[i][nt][4 * g + r] = acc[i][nt][4 * g + r] * sv[r];
        }
  }
  constexpr bool MMA = !KEPT && mma_input<W, MODE>(PAIRS, SPH);  // z1 from the matrix cores again
  if constexpr (MMA) {
    static_for<MT>([&](auto I) {
      f32x16 z[2];
      input_gemm<W, MODE, I>(ln, b, vb, z);
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float* w = b.w1 + (16 * I + 4 * g + r) * 12;
          const f32x4 wa = *reinterpret_cast<const f32x4*>(w);
          const f32x4 wb = *reinterpret_cast<const f32x4*>(w + 4);
          const f32x2 wc = *reinterpret_cast<const f32x2*>(w + 8);
#pragma unroll
          for (int nt = 0; nt < 2; ++nt) {
            const float g1 = acc[I][nt][4 * g + r] * silu_prime_only(z[nt][4 * g + r]);
            if constexpr (TRAIN) {
              g1keep[I][nt][4 * g + r] = g1;
            } else {
              epart[nt][0] += wa[0] * g1;
              epart[nt][1] += wa[1] * g1;
              epart[nt][2] += wa[2] * g1;
              epart[nt][3] += wb[0] * g1;
              epart[nt][4] += wb[1] * g1;
              epart[nt][5] += wb[2] * g1;
              epart[nt][6] += wb[3] * g1;
              epart[nt][7] += wc[0] * g1;
              epart[nt][8] += wc[1] * g1;
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
    });
  }
#pragma unroll
  for (int i = 0; i < ((KEPT || MMA) ? 0 : MT); ++i)
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float* w = b.w1 + (16 * i + 4 * g + r) * 12;
        const f32x4 wa = *reinterpret_cast<const f32x4*>(w);
        const f32x4 wb = *reinterpret_cast<const f32x4*>(w + 4);
        f32x4 wc;  // slots 8, 9 (arm), 10 (radius weight), 11
        if constexpr (SPH) {
          wc = *reinterpret_cast<const f32x4*>(w + 8);
        } else {
          const f32x2 w2 = *reinterpret_cast<const f32x2*>(w + 8);
          wc = f32x4{w2[0], w2[1], 0.f, 0.f};
        }
        const float cr = PAIRS ? wa[3] : b.crow[16 * i + 4 * g + r];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
          const float* x = b.xin + nt * 32 * XF;
          const float c = PAIRS ? arm_term(wa[3], wb[0], wb[1], wb[2], wb[3], wc[0], wc[1], x + 5) : cr;
          const float z = input_preact_t<SPH>(c, wa[0], wa[1], wa[2], wc[2], x);
          const float g1 = acc[i][nt][4 * g + r] * silu_prime_only(z);
          if constexpr (TRAIN) {
            g1keep[i][nt][4 * g + r] = g1;  // training needs g1, not J
          } else {
            epart[nt][0] += wa[0] * g1;
            epart[nt][1] += wa[1] * g1;
            epart[nt][2] += wa[2] * g1;
            epart[nt][3] += wb[0] * g1;
            epart[nt][4] += wb[1] * g1;
            epart[nt][5] += wb[2] * g1;
            epart[nt][6] += wb[3] * g1;
            epart[nt][7] += wc[0] * g1;
            epart[nt][8] += wc[1] * g1;
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
  if constexpr (TRAIN) {
    // training: g1 through LDS to HBM (every wave has finished reading g2)
    __syncthreads();
    static_for<MT>([&](auto I) {
      static_for<2>([&](auto GP) {
        static_for<2>([&](auto NT) {
          float v[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) v[q] = g1keep[I][NT][8 * GP + q];
          act_store_pair<W, MODE, I, GP, NT>(ln, v);
        });
      });
    });
    __syncthreads();
    before_copy();
    // g1 is needed only for db1 and dW1 = sum_i g1_i v_i^T: summed here when the
    // tile engine keeps the sums, else written out
    const DumpSums sm{td.row(0), nullptr, td.row(5), td.vt};
    dump_tile<W, MODE>(td.act, td.stage, td.g(0), td.ldb, td.q0, td.nvalid, td.bsum ? &sm : nullptr, !td.bsum);
  }
}

// Input layer (FP32): z1 = W1 [p'; a] + b1, h1 = SiLU(z1) -> LDS.  KEEP: SiLU'(z1)
// also goes to sp1 (train_sp1's layout) for the reverse sweep.
template <int W, int MODE, bool PAIRS, bool SPH, bool KEEP = false>
__device__ __forceinline__ void fwd_input(const Lane<W, MODE>& ln, const Bases<W, MODE>& b, const char* vb,
                                          float* sp1 = nullptr) {
  constexpr int MT = Geo<W, MODE>::MT;
  constexpr int XF = Geo<W, MODE>::XIN_FLOATS;
  if constexpr (mma_input<W, MODE>(PAIRS, SPH)) {
    static_for<MT>([&](auto I) {
      f32x16 z[2];
      input_gemm<W, MODE, I>(ln, b, vb, z);
      static_for<2>([&](auto GP) {
        static_for<2>([&](auto NT) {
          float v[8], dv[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            if constexpr (KEEP) silu_fwd(z[NT][8 * GP + q], v[q], dv[q]);
            else v[q] = silu_only(z[NT][8 * GP + q]);
          }
          act_store_pair<W, MODE, I, GP, NT>(ln, v);
          if constexpr (KEEP) {
            constexpr int T = Geo<W, MODE>::THREADS;
            constexpr int k = ((I * 2 + NT) * 16 + 8 * GP) / 4;  // first of the two 16-byte groups
#pragma unroll
            for (int h = 0; h < 2; ++h)
              *reinterpret_cast<f32x4*>(sp1 + ((k + h) * T + threadIdx.x) * 4) =
                  f32x4{dv[4 * h], dv[4 * h + 1], dv[4 * h + 2], dv[4 * h + 3]};
          }
        });
        __builtin_amdgcn_sched_barrier(0);
      });
    });
    return;
  }
  static_for<MT>([&](auto I) {
    static_for<2>([&](auto GP) {
      f32x4 wa[8], wb[8];
      f32x2 wc[8];
      float cr[8], wr[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float* w = b.w1 + (16 * I + 8 * GP + q) * 12;
        wa[q] = *reinterpret_cast<const f32x4*>(w);
        wr[q] = SPH ? w[10] : 0.f;
        if constexpr (PAIRS) {
          wb[q] = *reinterpret_cast<const f32x4*>(w + 4);
          wc[q] = *reinterpret_cast<const f32x2*>(w + 8);
        } else {
          cr[q] = b.crow[16 * I + 8 * GP + q];
        }
      }
      static_for<2>([&](auto NT) {
        const float* x = b.xin + NT * 32 * XF;
        float v[8], dv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          float c = PAIRS ? 0.f : cr[q];
          if constexpr (PAIRS) c = arm_term(wa[q][3], wb[q][0], wb[q][1], wb[q][2], wb[q][3], wc[q][0], wc[q][1], x + 5);
          const float z = input_preact_t<SPH>(c, wa[q][0], wa[q][1], wa[q][2], wr[q], x);
          if constexpr (KEEP) silu_fwd(z, v[q], dv[q]);
          else v[q] = silu_only(z);
        }
        act_store_pair<W, MODE, I, GP, NT>(ln, v);
        if constexpr (KEEP) {
          constexpr int T = Geo<W, MODE>::THREADS;
          constexpr int k = ((I * 2 + NT) * 16 + 8 * GP) / 4;  // first of the two 16-byte groups
#pragma unroll
          for (int h = 0; h < 2; ++h)
            *reinterpret_cast<f32x4*>(sp1 + ((k + h) * T + threadIdx.x) * 4) =
                f32x4{dv[4 * h], dv[4 * h + 1], dv[4 * h + 2], dv[4 * h + 3]};
        }
      });
      __builtin_amdgcn_sched_barrier(0);
    });
  });
}

// ----------------------------------------------------------------------------
// Per-workgroup state and the body that processes one tile.
// ----------------------------------------------------------------------------
template <int W, int MODE>
struct TileCtx {
  char* act;
  float* xin;   // [64][16]
  float* crow;  // [W]
  float* red;   // [waves][10][64]
  uint32_t* ovf;  // LDS word: a tile of this workgroup overflowed FP16 (see report_overflow)
  float b5;       // the output bias, read once (every tile's final sum adds it)
  // BF16 training, wave 0: the next tile's inputs (knot, point, target) of this
  // lane's query, fetched during the tile before (see process_tile)
  float nx[13];
  bool nx_ok;
  Lane<W, MODE> ln;
  Bases<W, MODE> b;
  __device__ __forceinline__ TileCtx(char* lds, uint32_t* ovf_word, const DevNet& net, int tid)
      : act(lds), ovf(ovf_word), b5(*net.b5p), nx_ok(false), ln(lds, tid) {
    if (tid == 0) *ovf = 0u;  // ordered before any tile's use by the tile's first barrier
    using G = Geo<W, MODE>;
    constexpr int MT = G::MT;
    xin = reinterpret_cast<float*>(lds + G::ACT_BYTES);
    crow = xin + kTileQ * G::XIN_FLOATS;
    float* after = crow + W;
    if constexpr (G::RED_IN_ACT) {
      red = reinterpret_cast<float*>(lds);
    } else {
      red = after;
      after += G::RED_BYTES / 4;
    }
    float* vec = after;  // [4][W]: b2, b3, b4, w_out
    for (int i = tid; i < 4 * W; i += G::THREADS) vec[i] = i < 3 * W ? net.bh[i] : net.w5[i - 3 * W];
    // bytes of one row group's fragment stream (1 KiB per fragment, PMT per K step)
    const size_t stream_bytes = (size_t)(MODE == kFP32 ? G::NK8 : G::NKB) * G::PMT * 1024;
    const int pw = ln.wave / G::SUB, sub = ln.wave % G::SUB;  // row group, and this wave's share of it
    // this lane's block of lane-major rows (see lane_major_pos: 16 PMT per (group, h))
    const int lblk = ((pw * 2 + ln.h) * G::PMT + sub * MT) * 16;
    b.bh = vec + lblk;
    b.w5 = vec + 3 * W + lblk;
    b.w1 = net.w1p + lblk * 12;
    {  // row m = lane%32 of M tile 0 is lane-major row ((pw 2 + h_m) PMT + sub MT) 16 + 4 g_m + r_m
      const int m = ln.n0;
      b.w1a = net.w1p + ((((pw * 2 + ((m >> 2) & 1)) * G::PMT + sub * MT) * 16) + 4 * (m >> 3) + (m & 3)) * 12;
    }
    b.crow = crow + lblk;
    b.xin = xin + ln.n0 * G::XIN_FLOATS;
    b.voff = (int)(pw * stream_bytes) + sub * MT * 1024 + ln.lane * 16;
    // Two waves per SIMD: the first four waves take the matrix cores first, so
    // they reach each layer's epilogue (vector ALU) early and run it while the
    // other four are still in their K loops.
    if constexpr (G::SUB > 1) {
      if (ln.wave < kWaves) __builtin_amdgcn_s_setprio(1);
    }
  }
};

// LDS that training adds after the query's own: the fused loss's per-wave
// partial sums ([waves][64]) and, for pure BF16, the per-workgroup sums of
// TileDump::bsum ([kTrainSumRows][W]) and the tile's transposed inputs
// (TileDump::vt).
template <int W, int MODE>
constexpr int train_extra_lds() {
  return Geo<W, MODE>::NW * kTileQ * 4 +
         (MODE == kBF16 ? kTrainSumRows * W * 4 + 2 * 9 * kTileQ * 2 + W * kTileQ * 4 : 0);
}
template <int W, int MODE>
__device__ __forceinline__ float* train_bsum(char* lds) {
  if constexpr (MODE == kBF16) return reinterpret_cast<float*>(lds + Geo<W, MODE>::LDS_BYTES + Geo<W, MODE>::NW * kTileQ * 4);
  return nullptr;
}
template <int W, int MODE>
__device__ __forceinline__ __bf16* train_vt(char* lds) {
  if constexpr (MODE == kBF16) return reinterpret_cast<__bf16*>(train_bsum<W, MODE>(lds) + kTrainSumRows * W);
  return nullptr;
}
// BF16 training: SiLU'(z1) of the tile (W x 64 floats), written by the input layer
// and read back by the last reverse layer, each thread its own values (16-byte
// group k of thread t at float (k THREADS + t) 4), so no barrier orders them.
template <int W, int MODE>
__device__ __forceinline__ float* train_sp1(char* lds) {
  if constexpr (MODE == kBF16) return reinterpret_cast<float*>(train_vt<W, MODE>(lds) + 2 * 9 * kTileQ);
  return nullptr;
}

// One tile: 64 points of knot kk starting at point q0 (dense), or pair-list
// entries q0 .. q0+63 (pairs).  Every thread of the workgroup calls it; it ends
// with a barrier, so consecutive calls can reuse the shared memory.  SPH: the
// obstacles are spheres (x, y, z, r) and the network input is [p', r, a].
template <int W, int MODE, bool PAIRS, bool TRAIN = false, bool GATHER = false, bool SPH = false>
__device__ __forceinline__ void process_tile(const DevNet& net, const Job& job, int want_grad, int64_t kk,
                                             int64_t q0, TileCtx<W, MODE>& tc) {
  using G = Geo<W, MODE>;
  constexpr int MT = G::MT;
  constexpr int XF = G::XIN_FLOATS;
  const int tid = threadIdx.x;
  float* xin = tc.xin;
  float* crow = tc.crow;
  float* red = tc.red;
  const Lane<W, MODE>& ln = tc.ln;
  const Bases<W, MODE>& b = tc.b;
  const int64_t qlimit = PAIRS ? job.npairs : (GATHER ? job.row_off[kk + 1] : job.Np);

  // BF16 training: sample i = knot i, point i; the inputs of a workgroup's next tile
  // are fetched before this tile's last copy (no vector-memory wait comes between
  // them and the barrier that ends the tile) and read from registers by its prologue
  constexpr bool PREFETCH = TRAIN && PAIRS && MODE == kBF16 && !SPH;
  const bool fetched = PREFETCH && tc.nx_ok;
  auto fetch_next = [&]() {
    if constexpr (PREFETCH) {
      const int64_t qn = q0 + (int64_t)gridDim.x * kTileQ;
      tc.nx_ok = qn < qlimit && !job.csr_off && !job.kidx && !job.pidx && !job.pidx32;
      if (tid < kTileQ && tc.nx_ok) {
        const int64_t q = qn + tid;
        const int64_t qc = q < qlimit ? q : qlimit - 1;
        const float* kn = job.knots + qc * kInDim;
#pragma unroll
        for (int c = 0; c < kInDim; ++c) tc.nx[c] = kn[c];
        const float* pt = job.points + qc * 3;
#pragma unroll
        for (int c = 0; c < 3; ++c) tc.nx[kInDim + c] = pt[c];
        tc.nx[12] = (!job.seed && job.target && q < qlimit) ? job.target[qc] : 0.f;
      }
    }
  };

  // ---- prologue: base-frame points (+ per-knot arm term of the input layer) ----
  if (tid < kTileQ) {
    const int64_t q = q0 + tid;
    const int64_t qc = q < qlimit ? q : qlimit - 1;   // clamp the ragged tail (never stored)
    int64_t ki = 0, pi = 0;
    if constexpr (PAIRS) {
      if (job.csr_off) {
        // knot of row qc: the last i < csr_n with csr_off[i] <= qc (empty partitions skipped)
        int64_t lo = 0, hi = job.csr_n - 1;
        while (lo < hi) {
          const int64_t mid = (lo + hi + 1) >> 1;
          if (job.csr_off[mid] <= qc) lo = mid; else hi = mid - 1;
        }
        ki = lo;
        pi = job.csr_idx[qc];
      } else {
        ki = job.kidx ? job.kidx[qc] : qc;
        pi = job.pidx32 ? (int64_t)job.pidx32[qc] : (job.pidx ? job.pidx[qc] : qc);
      }
    } else {
      ki = kk;
      pi = GATHER ? (int64_t)job.pgather[qc] : qc;
    }
    float kn[kInDim], pxyz[4];
    if (fetched) {
#pragma unroll
      for (int c = 0; c < kInDim; ++c) kn[c] = tc.nx[c];
#pragma unroll
      for (int c = 0; c < 3; ++c) pxyz[c] = tc.nx[kInDim + c];
      pxyz[3] = 0.f;
    } else {
      if constexpr (PAIRS) {
        const float* knp = job.knots + ki * kInDim;
#pragma unroll
        for (int c = 0; c < kInDim; ++c) kn[c] = knp[c];
      } else {
        // one knot per tile: scalar loads (the knots are read-only during the launch)
        const __attribute__((address_space(4))) float* knp =
            (const __attribute__((address_space(4))) float*)(job.knots + ki * kInDim);
#pragma unroll
        for (int c = 0; c < kInDim; ++c) kn[c] = knp[c];
      }
      if ((PAIRS || GATHER) && (uint64_t)pi >= (uint64_t)job.Np) {
        pxyz[0] = pxyz[1] = pxyz[2] = pxyz[3] = __builtin_nanf("");  // bad point index: NaN results
      } else {
        const float* pt = job.points + pi * (SPH ? 4 : 3);
        pxyz[0] = pt[0];
        pxyz[1] = pt[1];
        pxyz[2] = pt[2];
        pxyz[3] = SPH ? pt[3] : 0.f;
      }
    }
    float sn, cs;
    sincosf(kn[2], &sn, &cs);
    const float ux = pxyz[0] - kn[0], uy = pxyz[1] - kn[1];
    // the record's address is formed here, once per tile: hoisted out of the tile
    // loop, its pieces were kept in spill slots and reloaded one by one
    int tq = tid;
    asm volatile("" : "+v"(tq));
    float* x = xin + tq * XF;
    x[0] = cs * ux + sn * uy;
    x[1] = -sn * ux + cs * uy;
    x[2] = pxyz[2];
    x[3] = cs;
    x[4] = sn;
#pragma unroll
    for (int c = 0; c < 6; ++c) x[5 + c] = kn[3 + c];
    // reverse-sweep seed: dL/dd for training, else 1 (multiplying by 1 is exact;
    // the constant is formed here, a copy kept from before the tile loop was spilled)
    float one = 1.f;
    asm volatile("" : "+v"(one));
    x[11] = job.seed ? (q < qlimit ? job.seed[qc] : 0.f) : one;
    // the fused loss's target, fetched with the inputs rather than after the forward
    if constexpr (TRAIN)
      x[kXinTarget] = fetched ? tc.nx[12] : (!job.seed && job.target && q < qlimit) ? job.target[qc] : 0.f;
    if constexpr (TRAIN && MODE == kBF16) {
      // the network inputs transposed and split into BF16 hi + lo, for dW1 on the
      // matrix cores (the ragged tail's inputs meet zero gradients)
      __bf16* vt = train_vt<W, MODE>(tc.act);
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        const float v = x[c < 3 ? c : c + 2];
        const __bf16 hi = (__bf16)v;
        vt[c * kTileQ + tid] = hi;
        vt[(9 + c) * kTileQ + tid] = (__bf16)(v - (float)hi);
      }
    }
    if constexpr (SPH) x[kXinRadius] = pxyz[3];  // the radius passes through the rigid transform
    if constexpr (mma_input<W, MODE>(PAIRS, SPH)) {
      // the inputs as B fragments of the matrix-core input layer (input_gemm), in
      // the idle half of the activation tile
      const float v[16] = {x[0], x[1], x[2], x[5], x[6], x[7], x[8], x[9], x[10], 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      bf16x8 vh[2], vl[2];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const __bf16 hi = (__bf16)v[k];
        vh[k >> 3][k & 7] = hi;
        vl[k >> 3][k & 7] = (__bf16)(v[k] - (float)hi);
      }
      char* o = tc.act + G::ACT_BYTES / 2 + tid * kVbBytes;
      *reinterpret_cast<bf16x8*>(o) = vh[0];
      *reinterpret_cast<bf16x8*>(o + 16) = vh[1];
      *reinterpret_cast<bf16x8*>(o + 32) = vl[0];
      *reinterpret_cast<bf16x8*>(o + 48) = vl[1];
    }
    if constexpr (PAIRS) {
      if (job.dumpV) {
        const bool ok = q < qlimit;
#pragma unroll
        for (int c = 0; c < 3; ++c) job.dumpV[c * job.ldb + q] = ok ? x[c] : 0.f;
#pragma unroll
        for (int c = 0; c < 6; ++c) job.dumpV[(3 + c) * job.ldb + q] = ok ? x[5 + c] : 0.f;
      }
    }
  }
  if constexpr (!PAIRS) {
    // the knot's arm joints, by scalar loads as above
    const __attribute__((address_space(4))) float* ka =
        (const __attribute__((address_space(4))) float*)(job.knots + kk * kInDim + 3);
    float arm[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) arm[c] = ka[c];
    int r0 = tid;  // (opaque, so the addresses below are formed here, per tile, not kept spilled)
    asm volatile("" : "+v"(r0));
    for (int r = r0; r < W; r += G::THREADS) {  // r: lane-major position
      const float* w = net.w1p + r * 12;
      crow[r] = arm_term(w[3], w[4], w[5], w[6], w[7], w[8], w[9], arm);
    }
  }
  __syncthreads();

  TileDump td{};
  if constexpr (TRAIN) {
    td.act = tc.act;
    td.H = job.dumpH;
    td.G = job.dumpG;
    td.ldb = job.ldb;
    td.q0 = q0;
    td.nvalid = (int)(qlimit - q0 < kTileQ ? qlimit - q0 : kTileQ);
    td.layer_elems = (size_t)W * job.ldb;
    td.elem_bytes = MODE == kFP32 ? 4 : 2;
    // LDS beyond the query's own: the fused loss's partial sums ([waves][64]); the
    // idle half of a pure-BF16 tile stages the dumps
    td.stage = tc.act + G::ACT_BYTES / 2;
    td.dred = reinterpret_cast<float*>(tc.act + G::LDS_BYTES);
    td.bsum = train_bsum<W, MODE>(tc.act);
    td.vt = train_vt<W, MODE>(tc.act);
    td.sp1 = train_sp1<W, MODE>(tc.act);
    td.width = W;
    td.xin = xin;
    td.target = job.seed ? nullptr : job.target;
    td.seed_out = job.seed_out;
    td.sq_out = job.sq_out;
    td.d_out = job.seed ? nullptr : job.d;
    td.mse_scale = job.mse_scale;
    td.b5 = tc.b5;
    td.inv_b = job.inv_b;
  }
  fwd_input<W, MODE, PAIRS, SPH, TRAIN && MODE == kBF16>(ln, b, tc.act + G::ACT_BYTES / 2, td.sp1);
  __syncthreads();
  APre<W, MODE> ap;  // training: each layer's first weight fragments, requested before the dump ahead of it
  if constexpr (TRAIN) {
    preload_a<W, MODE>(ap, stream_rsrc<W, MODE>(net.fwd[0]), b.voff);
    dump_tile<W, MODE>(td.act, td.stage, td.h(0), td.ldb, td.q0, td.nvalid);  // h1
  }

  // ---- hidden layers 2..4 (forward), keeping SiLU' of layers 2 and 3 ----
  float sp[2][MT][2][16];
  float dpart[2] = {0.f, 0.f};
  fwd_hidden<W, MODE, 0, TRAIN>(net, ln, b, sp, dpart, want_grad, td, ap);
  fwd_hidden<W, MODE, 1, TRAIN>(net, ln, b, sp, dpart, want_grad, td, ap);
  fwd_hidden<W, MODE, 2, TRAIN>(net, ln, b, sp, dpart, want_grad, td, ap);

  // ---- reverse sweep: W4^T, W3^T (into LDS), W2^T (into the input-layer gradient) ----
  float epart[2][9];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt)
#pragma unroll
    for (int c = 0; c < 9; ++c) epart[nt][c] = 0.f;
  if (want_grad) {
    bwd_hidden<W, MODE, 2, TRAIN>(net, ln, b, sp, td, ap);
    bwd_hidden<W, MODE, 1, TRAIN>(net, ln, b, sp, td, ap);
    bwd_input<W, MODE, PAIRS, TRAIN, SPH>(net, ln, b, epart, td, tc.act + G::ACT_BYTES / 2, ap, fetch_next);
    if constexpr (rev_arith<MODE>() == kF16) {
      // a lane whose output partial sum is finite but whose input-gradient partial
      // sums are not: the FP16 reverse sweep overflowed (the forward accumulates in
      // FP32; a non-finite input point makes every partial non-finite).  Noted in
      // LDS, reported to the host once per workgroup when the kernel ends
      // (report_overflow).
      uint32_t bad = 0;
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        float t = 0.f;
#pragma unroll
        for (int c = 0; c < 9; ++c) t += epart[nt][c];
        bad |= (uint32_t)(!__builtin_isfinite(t)) & (uint32_t)__builtin_isfinite(dpart[nt]);
      }
      if (bad) *tc.ovf = 1u;
    }
  }

  // ---- reduce d and e over the rows: lane halves, then waves (fixed order) ----
  // (training needs neither: the fused loss finished d inside the tile)
  if constexpr (!TRAIN) {
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      dpart[nt] += __shfl_xor(dpart[nt], 32);
#pragma unroll
      for (int c = 0; c < 9; ++c) epart[nt][c] += __shfl_xor(epart[nt][c], 32);
    }
    // the reduction buffer may share the activation tile: every wave must have
    // finished reading it
    if constexpr (G::RED_IN_ACT) __syncthreads();
    if (ln.h == 0) {
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) {
        const int n = 32 * nt + ln.n0;
        red[(ln.wave * G::RED_VALS + 0) * kTileQ + n] = dpart[nt];
#pragma unroll
        for (int c = 0; c < 9; ++c) red[(ln.wave * G::RED_VALS + 1 + c) * kTileQ + n] = epart[nt][c];
      }
    }
    __syncthreads();

    // ---- per query: final sums, chain rule, stores, per-knot minimum ----
    if (tid < kTileQ) {
      // recomputed here rather than kept from the prologue (the compiler would
      // otherwise hold q0 + tid through the whole tile, in a spill slot)
      int n = tid;
      asm volatile("" : "+v"(n));
      float vals[G::RED_VALS];
#pragma unroll
      for (int c = 0; c < G::RED_VALS; ++c) {
        float sum = red[(0 * G::RED_VALS + c) * kTileQ + n];
#pragma unroll
        for (int w = 1; w < G::NW; ++w) sum += red[(w * G::RED_VALS + c) * kTileQ + n];
        vals[c] = sum;
      }
      if constexpr (rev_scale<MODE>() != 1.0f) {
#pragma unroll
        for (int c = 1; c < G::RED_VALS; ++c) vals[c] *= 1.0f / rev_scale<MODE>();
      }
      const float dv = vals[0] + tc.b5;
      const int64_t q = q0 + n;
      const bool valid = q < qlimit;
      const int64_t out = (PAIRS || GATHER) ? q : kk * job.Np + q;
      // outputs are streamed with non-temporal stores: written once and never read
      // here, they would otherwise evict the packed weights from L2
      if (valid && job.d) __builtin_nontemporal_store(dv, job.d + out);
      if (!TRAIN && valid && job.J && want_grad) {  // (training computes g1, not J)
        const float* x = xin + n * XF;
        const float cs = x[3], sn = x[4];
        const float* e = vals + 1;
        float* Jo = job.J + out * kInDim;
        __builtin_nontemporal_store(-(cs * e[0] - sn * e[1]), Jo + 0);
        __builtin_nontemporal_store(-(sn * e[0] + cs * e[1]), Jo + 1);
        __builtin_nontemporal_store(e[0] * x[1] - e[1] * x[0], Jo + 2);
#pragma unroll
        for (int c = 3; c < 9; ++c) __builtin_nontemporal_store(e[c], Jo + c);
      }
      if constexpr (!PAIRS) {
        if (job.minkey) {
          unsigned long long key = valid ? (((unsigned long long)ordered_bits(dv) << 32) | (uint32_t)q) : ~0ull;
#pragma unroll
          for (int off = 32; off >= 1; off >>= 1) {
            unsigned long long o = __shfl_xor(key, off);
            key = o < key ? o : key;
          }
          if (n == 0 && key != ~0ull) atomicMin(job.minkey + kk, key);
        }
      }
    }
  }  // !TRAIN
  // The next tile's prologue rewrites xin and crow: every wave has passed the
  // barrier above (crow's last reader), and xin's readers here are wave 0,
  // which also writes it, in program order.
  __syncthreads();
}

// End of a kernel that ran tiles: if any tile of this workgroup flagged an FP16
// overflow, write the context's host-visible flag (all threads call it).
template <int W, int MODE>
__device__ __forceinline__ void report_overflow(const DevNet& net, const TileCtx<W, MODE>& tc) {
  if constexpr (rev_arith<MODE>() == kF16) {
    __syncthreads();
    if (threadIdx.x == 0 && *tc.ovf && net.overflow)
      __hip_atomic_store(net.overflow, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// ----------------------------------------------------------------------------
// One-shot kernel: a persistent grid strides over all tiles of one job.
// ----------------------------------------------------------------------------
template <int W, int MODE, bool PAIRS, int OCC, bool TRAIN = false, bool GATHER = false, bool SPH = false>
__global__ __launch_bounds__((Geo<W, MODE>::THREADS), OCC) void fused_query(const DevNet net, const Job job, int want_grad,
                                                             int64_t ntiles) {
  static_assert(Geo<W, MODE>::LDS_BYTES + (TRAIN ? train_extra_lds<W, MODE>() : 0) + 16 <= 160 * 1024,
                "the workgroup's LDS exceeds the compute unit's 160 KiB");
  __shared__ __attribute__((aligned(16))) char lds[Geo<W, MODE>::LDS_BYTES + (TRAIN ? train_extra_lds<W, MODE>() : 0)];
  __shared__ uint32_t ovf;
  TileCtx<W, MODE> tc(lds, &ovf, net, threadIdx.x);
  float* bsum = TRAIN ? train_bsum<W, MODE>(lds) : nullptr;
  if (bsum) {  // ordered before the first tile's sums by its barriers
    for (int j = threadIdx.x; j < kTrainSumRows * W; j += Geo<W, MODE>::THREADS) bsum[j] = 0.f;
  }
  const int64_t nblk = PAIRS ? 0 : (job.Np + kTileQ - 1) / kTileQ;
  int64_t kk = PAIRS ? 0 : blockIdx.x / nblk;  // dense: the knot of the current tile
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    if constexpr (PAIRS) {
      process_tile<W, MODE, true, TRAIN, false, SPH>(net, job, want_grad, 0, tile * kTileQ, tc);
    } else if constexpr (GATHER) {
      if (tile >= job.tile_off[job.K]) break;  // the grid is sized by an upper bound
      int64_t lo = 0, hi = job.K - 1;            // knot: the last i with tile_off[i] <= tile
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (job.tile_off[mid] <= tile) lo = mid; else hi = mid - 1;
      }
      process_tile<W, MODE, false, false, true, SPH>(net, job, want_grad, lo,
                                                     job.row_off[lo] + (tile - job.tile_off[lo]) * kTileQ, tc);
    } else {
      process_tile<W, MODE, false, false, false, SPH>(net, job, want_grad, kk, (tile - kk * nblk) * kTileQ, tc);
      // the next tile's knot: at most one knot further when a knot has at least as
      // many tiles as the grid has workgroups, with no 64-bit division then
      const int64_t next = tile + gridDim.x;
      if (next < (kk + 2) * nblk) kk += next >= (kk + 1) * nblk ? 1 : 0;
      else kk = next / nblk;
    }
  }
  if (bsum) {  // this workgroup's sums; summed over workgroups in order afterwards
    __syncthreads();
    for (int j = threadIdx.x; j < kTrainSumRows * W; j += Geo<W, MODE>::THREADS)
      job.bias_part[(int64_t)j * gridDim.x + blockIdx.x] = bsum[j];
  }
  report_overflow<W, MODE>(net, tc);
}

// ----------------------------------------------------------------------------
// Host-side launchers of fused_query (grid = min(tiles, CUs)); each source file
// instantiates the obstacle kind (SPH) it serves.
// ----------------------------------------------------------------------------
template <int W, int MODE, bool PAIRS, bool SPH>
static hipError_t launch_t(const DevNet& net, const Job& job, bool want_grad, int num_cu, hipStream_t s) {
  constexpr int OCC = 1;
  const int64_t ntiles = PAIRS ? (job.npairs + kTileQ - 1) / kTileQ
                               : (job.tile_off ? job.ntiles_bound : job.K * ((job.Np + kTileQ - 1) / kTileQ));
  if (ntiles <= 0) return hipSuccess;
  const int grid = fused_grid(ntiles, num_cu);
  if constexpr (PAIRS && W == 256 && (MODE == kFP32 || MODE == kBF16) && !SPH) {  // training: width 256, FP32 or BF16
    if (job.dumpH) {
      // the kernel writes its sums to bias_part, no J, and d only with the fused loss
      if ((MODE == kBF16 && !job.bias_part) || job.J || (job.d && !job.target)) return hipErrorInvalidValue;
      hipLaunchKernelGGL((fused_query<W, MODE, true, OCC, true>), dim3(grid), dim3((Geo<W, MODE>::THREADS)), 0, s, net, job, 1,
                         ntiles);
      return hipGetLastError();
    }
  }
  if (job.dumpH || job.seed) return hipErrorInvalidValue;  // a seed is honoured by the training instantiation only
  if constexpr (!PAIRS) {
    if (job.tile_off) {
      hipLaunchKernelGGL((fused_query<W, MODE, false, OCC, false, true, SPH>), dim3(grid), dim3((Geo<W, MODE>::THREADS)), 0, s, net,
                         job, want_grad ? 1 : 0, ntiles);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((fused_query<W, MODE, PAIRS, OCC, false, false, SPH>), dim3(grid), dim3((Geo<W, MODE>::THREADS)), 0, s, net, job,
                     want_grad ? 1 : 0, ntiles);
  return hipGetLastError();
}

template <int W, int MODE, bool SPH>
static hipError_t launch_m(const DevNet& net, const Job& job, bool pairs, bool want_grad, int num_cu, hipStream_t s) {
  return pairs ? launch_t<W, MODE, true, SPH>(net, job, want_grad, num_cu, s)
               : launch_t<W, MODE, false, SPH>(net, job, want_grad, num_cu, s);
}

template <int W, bool SPH>
static hipError_t launch_w(const DevNet& net, const Job& job, bool pairs, bool want_grad, int num_cu, hipStream_t s) {
  switch (net.mode) {
    case kFP32: return launch_m<W, kFP32, SPH>(net, job, pairs, want_grad, num_cu, s);
    case kBF16: return launch_m<W, kBF16, SPH>(net, job, pairs, want_grad, num_cu, s);
    case kBF16X2F16: return launch_m<W, kBF16X2F16, SPH>(net, job, pairs, want_grad, num_cu, s);
    default: return launch_m<W, kBF16X2, SPH>(net, job, pairs, want_grad, num_cu, s);
  }
}

}  // namespace gcdf
