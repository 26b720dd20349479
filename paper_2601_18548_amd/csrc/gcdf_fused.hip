// Fused batched neural-GCDF query kernel for gfx950 (MI355X).
//
// One workgroup (4 waves, one per SIMD) owns a tile of 64 queries: 64 points
// of one knot (dense all-pairs mode) or 64 entries of a pair list.  For the
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
// activations (forward) or back-propagated gradients (reverse).  Wave w owns
// output rows [w*W/4, (w+1)*W/4) for all 64 queries; B lives in LDS (written by
// the epilogue of the previous layer, read by all four waves); the A fragments
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
// The SiLU derivative needed by the reverse sweep is kept in FP32 registers for
// layers 2 and 3 and recomputed for layer 1 from the input layer.
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

template <int W>
struct Geo {
  static constexpr int MT = W / (32 * kWaves);       // 32-row M tiles per wave
  static constexpr int NKB = W / 16;                 // 16-deep K blocks (bf16)
  static constexpr int NK8 = W / 8;                  // 8-deep K groups (fp32: 4 MFMAs of K=2)
  static constexpr int ACT_BYTES = W * kTileQ * 4;   // fp32, or bf16 hi + bf16 lo
  static constexpr int XIN_FLOATS = 17;              // per query: p'(3), cos, sin, arm(6), seed, pad; odd stride: lanes reading one field of 32 queries hit 32 different banks
  static constexpr int RED_VALS = 10;                // d + 9 input-gradient components
  static constexpr int LDS_BYTES =
      ACT_BYTES + kTileQ * XIN_FLOATS * 4 + W * 4 + kWaves * RED_VALS * kTileQ * 4 + 4 * W * 4;
};

// ----------------------------------------------------------------------------
// Activation tile in LDS (64 query columns).
//  bf16 modes: hi plane then lo plane (W*128 bytes each).  Element (k, n) sits in
//    the 16-byte group (k/16, (k%16)/8, n) at byte ((k/16)*2 + (k%16)/8)*1024 + n*16,
//    position k%8 inside it.  The B fragment of K step s, column block nt is the
//    2 KiB at s*2048, lane (n0, kh) reading the 16 bytes at kh*1024 + nt*512 + n0*16:
//    every lane reads its own consecutive 16 bytes (no bank conflicts).
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
  static constexpr int MT = W / (32 * kWaves);
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
      act_w = act + (rbase >> 4) * 2048 + h * 1024 + n0 * 16;
      act_r = act + kh * 1024 + n0 * 16;
    }
    act_w_lo = act_w + W * kTileQ * 2;
  }
};

// Write rows R0..R0+3 (R0 = rbase + 32 i + 8 g + 4 h) of column n = 32 nt + n0 (fp32).
template <int W, int MODE, int I, int G, int NT>
__device__ __forceinline__ void act_store4_fp32(const Lane<W, MODE>& L, const float v[4]) {
  constexpr int off = (4 * I + G) * 2048 + NT * 1024;
  *reinterpret_cast<f32x2*>(L.act_w + off) = f32x2{v[0], v[2]};       // rows R0, R0+2 (k%2 = 0)
  *reinterpret_cast<f32x2*>(L.act_w + off + 16) = f32x2{v[1], v[3]};  // rows R0+1, R0+3 (k%2 = 1)
}

// Pack four floats into two dwords of bf16 (round to nearest even).
__device__ __forceinline__ void pack4(const float v[4], uint32_t& d0, uint32_t& d1) {
  bf16x4 h4;
#pragma unroll
  for (int r = 0; r < 4; ++r) h4[r] = (__bf16)v[r];
  const f32x2 d = __builtin_bit_cast(f32x2, h4);
  d0 = __float_as_uint(d[0]);
  d1 = __float_as_uint(d[1]);
}

// bf16 modes: write rows of the group pair g = 2 GP, 2 GP + 1 (v[0..3] for g = 2 GP,
// v[4..7] for g = 2 GP + 1) of column n = 32 nt + n0.  Lane (n0, h) holds k%8 in
// [4h, 4h+4) of both 8-groups kh = 0 (g even) and kh = 1 (g odd); one swap across
// the lane halves gives lane (n0, kh) the whole 8-group kh, written as 16 bytes.
template <int W, int MODE, int I, int GP, int NT>
__device__ __forceinline__ void act_store8(const Lane<W, MODE>& L, const float v[8]) {
  constexpr int off = (2 * I + GP) * 2048 + NT * 512;
  auto put = [&](char* base, const float* x) {
    uint32_t e0, e1, o0, o1;  // e: g even (kh 0), o: g odd (kh 1)
    pack4(x, e0, e1);
    pack4(x + 4, o0, o1);
    // lanes 32..63 of the first operand trade with lanes 0..31 of the second:
    // afterwards lane (n0, kh) has k%8 in [0, 4) in the first and [4, 8) in the second
    const auto s0 = __builtin_amdgcn_permlane32_swap(e0, o0, false, false);
    const auto s1 = __builtin_amdgcn_permlane32_swap(e1, o1, false, false);
    typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;
    *reinterpret_cast<u32x4*>(base + off) = u32x4{s0[0], s1[0], s0[1], s1[1]};
  };
  put(L.act_w, v);
  if constexpr (MODE == kBF16X2) {
    float lo[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) lo[r] = v[r] - (float)(__bf16)v[r];
    put(L.act_w_lo, lo);
  }
}

// Either layout: rows of groups g = 2 GP, 2 GP + 1 (see act_store8).
template <int W, int MODE, int I, int GP, int NT>
__device__ __forceinline__ void act_store_pair(const Lane<W, MODE>& L, const float v[8]) {
  if constexpr (MODE == kFP32) {
    act_store4_fp32<W, MODE, I, 2 * GP, NT>(L, v);
    act_store4_fp32<W, MODE, I, 2 * GP + 1, NT>(L, v + 4);
  } else {
    act_store8<W, MODE, I, GP, NT>(L, v);
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
// packed stream: fragment (kstep, i) of this wave at byte
// wave*stream_bytes + ((kstep*MT + i)*64 + lane)*16 -- one 32-bit VGPR offset
// (voff = wave*stream_bytes + lane*16) serves every matrix and step; the step goes
// in the scalar offset and i*1024 in the instruction's immediate.
// Software pipeline: A is loaded two K steps ahead, B (LDS) one step ahead.
// ----------------------------------------------------------------------------
template <int MODE>
struct BFrag {
  bf16x8 h[2], l[2];
  f32x4 f[2];
};

template <int W, int MODE>
__device__ __forceinline__ void load_b(BFrag<MODE>& b, const char* br) {
  if constexpr (MODE == kFP32) {
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) b.f[nt] = *reinterpret_cast<const f32x4*>(br + nt * 1024);
  } else {
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      b.h[nt] = *reinterpret_cast<const bf16x8*>(br + nt * 512);
      if constexpr (MODE == kBF16X2) b.l[nt] = *reinterpret_cast<const bf16x8*>(br + W * kTileQ * 2 + nt * 512);
    }
  }
}

template <int W>
__device__ __forceinline__ void load_a(f32x4 (&af)[Geo<W>::MT], __amdgpu_buffer_rsrc_t rs, int voff, int step) {
  const int soff = step * Geo<W>::MT * 1024;
#pragma unroll
  for (int i = 0; i < Geo<W>::MT; ++i)
    af[i] = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff + i * 1024, soff, 0));
}

// One K step: for each M tile i, its MFMAs (hi then lo halves alternating over
// the two column blocks, so accumulations into one tile are two MFMAs apart),
// then at once the reload of a[i] for step `next` -- the fragment's registers
// are free as soon as its last MFMA has issued.  The scheduling barriers keep
// the compiler from sinking the loads to the end of the loop body.
template <int W, int MODE>
__device__ __forceinline__ void mma_step_reload(f32x16 (&acc)[Geo<W>::MT][2], f32x4 (&af)[Geo<W>::MT],
                                                const BFrag<MODE>& b, __amdgpu_buffer_rsrc_t rs, int voff,
                                                int next) {
  constexpr int MT = Geo<W>::MT;
  const int soff = next * MT * 1024;
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    if constexpr (MODE == kFP32) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
          acc[i][nt] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i][q], b.f[nt][q], acc[i][nt], 0, 0, 0);
    } else {
      const bf16x8 a8 = __builtin_bit_cast(bf16x8, af[i]);
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) acc[i][nt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a8, b.h[nt], acc[i][nt], 0, 0, 0);
      if constexpr (MODE == kBF16X2) {
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

template <int W, int MODE>
__device__ __forceinline__ void layer_gemm(f32x16 (&acc)[Geo<W>::MT][2], __amdgpu_buffer_rsrc_t rs, int voff,
                                           const char* br) {
  constexpr int MT = Geo<W>::MT;
  constexpr int NS = (MODE == kFP32) ? Geo<W>::NK8 : Geo<W>::NKB;  // even
  f32x4 a0[MT], a1[MT];
  BFrag<MODE> b0, b1;
  load_a<W>(a0, rs, voff, 0);
  load_a<W>(a1, rs, voff, 1);
  load_b<W, MODE>(b0, br);
#pragma unroll 1
  for (int s = 0; s < NS; s += 2) {
    load_b<W, MODE>(b1, br + 2048);  // B of step s+1, one step ahead
    __builtin_amdgcn_sched_barrier(0);
    mma_step_reload<W, MODE>(acc, a0, b0, rs, voff, s + 2 < NS ? s + 2 : NS - 1);
    load_b<W, MODE>(b0, s + 2 < NS ? br + 4096 : br);  // B of step s+2
    __builtin_amdgcn_sched_barrier(0);
    mma_step_reload<W, MODE>(acc, a1, b1, rs, voff, s + 3 < NS ? s + 3 : NS - 1);
    br += 4096;
  }
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
// ragged tail of the tile.  All threads take part.
// ----------------------------------------------------------------------------
template <int W, int MODE>
__device__ __forceinline__ void dump_tile(const char* act, void* dst, int64_t ldb, int64_t q0, int nvalid) {
  (void)ldb;
  for (int f = threadIdx.x; f < W && MODE == kFP32; f += kThreads) {
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
    // consecutive queries, transposes it in registers and writes the 8 features'
    // 16-byte pieces of that query block.
    typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;
    const char* a = act;
    constexpr int NG = W / 8;  // feature groups
    for (int t = threadIdx.x; t < NG * (kTileQ / 8); t += kThreads) {
      const int g8 = t % NG, nb = t / NG;
      const int gbyte = ((g8 >> 1) * 2 + (g8 & 1)) * 1024;  // 16-feature block, 8-feature half
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
        __bf16* o = static_cast<__bf16*>(dst) + (((q0 >> 3) + nb) * W + 8 * g8 + fl) * 8;
        *reinterpret_cast<u32x4*>(o) = row;
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
// ((wave*2 + h)*MT + i)*16 + 4 g + r, so each lane addresses them from one base
// with small constant offsets.
template <int W, int MODE>
struct Bases {
  const float* bh;    // LDS copy of b2, b3, b4 (lane-major), at this lane's block
  const float* w5;    // LDS copy of w_out (lane-major), at this lane's block
  const float* w1;    // input layer rows (lane-major, 12 floats per row), at this lane's block
  const float* crow;  // per-knot input-layer constant (LDS, lane-major), at this lane's block
  const float* xin;   // xin + n0 * XIN_FLOATS
  int voff;           // lane offset inside a matrix's fragment stream: wave*stream_bytes + lane*16
};

// Dump of the current LDS tile for training (no-op when not training).
struct TileDump {
  const char* act;  // the LDS activation tile
  void* H;
  void* G;
  int64_t ldb, q0;
  int nvalid;
  size_t layer_elems;  // W * ldb
  size_t elem_bytes;
  __device__ __forceinline__ void* h(int l) const { return static_cast<char*>(H) + l * layer_elems * elem_bytes; }
  __device__ __forceinline__ void* g(int l) const { return static_cast<char*>(G) + l * layer_elems * elem_bytes; }
};

template <int W, int MODE, int L, bool TRAIN>
__device__ __forceinline__ void fwd_hidden(const DevNet& net, const Lane<W, MODE>& ln, const Bases<W, MODE>& b,
                                           float (&sp)[2][Geo<W>::MT][2][16], float (&dpart)[2], int want_grad,
                                           const TileDump& td) {
  constexpr int MT = Geo<W>::MT;
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
  layer_gemm<W, MODE>(acc, stream_rsrc<W, MODE>(net.fwd[L]), b.voff, ln.act_r);
  __syncthreads();
  if constexpr (TRAIN && L == 2) {
    // training: the layer-4 activations h4 go through LDS first (for dL/dw_out)
    static_for<MT>([&](auto I) {
      static_for<2>([&](auto GP) {
        static_for<2>([&](auto NT) {
          float v[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) v[q] = silu_only(acc[I][NT][8 * GP + q]);
          act_store_pair<W, MODE, I, GP, NT>(ln, v);
        });
      });
    });
    __syncthreads();
    dump_tile<W, MODE>(td.act, td.h(3), td.ldb, td.q0, td.nvalid);
    __syncthreads();  // h4 fully read before g4 overwrites the tile
  }
  static_for<MT>([&](auto I) {
    static_for<2>([&](auto GP) {
      f32x4 w5r[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
      if constexpr (L == 2) {
        w5r[0] = *reinterpret_cast<const f32x4*>(b.w5 + 16 * I + 8 * GP);
        w5r[1] = *reinterpret_cast<const f32x4*>(b.w5 + 16 * I + 8 * GP + 4);
      }
      static_for<2>([&](auto NT) {
        const float seed = b.xin[NT * 32 * Geo<W>::XIN_FLOATS + 11];
        float v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int j = 8 * GP + q;  // accumulator element: g = 2 GP + q/4, r = q%4
          float hv, dv;
          silu_fwd(acc[I][NT][j], hv, dv);
          if constexpr (L < 2) {
            sp[L][I][NT][j] = park(dv);
            v[q] = hv;
          } else {
            dpart[NT] += w5r[q >> 2][q & 3] * hv;
            v[q] = seed * (w5r[q >> 2][q & 3] * dv);  // g4 = seed * w5 * SiLU'(z4)
          }
        }
        if (L < 2 || want_grad) act_store_pair<W, MODE, I, GP, NT>(ln, v);
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
  __syncthreads();
  // training: h2, h3 (layers 2, 3) or g4 (layer 4) to HBM; the tile is next
  // overwritten only after the following K loop and its barrier
  if constexpr (TRAIN) dump_tile<W, MODE>(td.act, L < 2 ? td.h(L + 1) : td.g(3), td.ldb, td.q0, td.nvalid);
}

template <int W, int MODE, int L, bool TRAIN>
__device__ __forceinline__ void bwd_hidden(const DevNet& net, const Lane<W, MODE>& ln, const Bases<W, MODE>& b,
                                           const float (&sp)[2][Geo<W>::MT][2][16], const TileDump& td) {
  constexpr int MT = Geo<W>::MT;
  f32x16 acc[MT][2];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[i][nt][j] = 0.f;
  layer_gemm<W, MODE>(acc, stream_rsrc<W, MODE>(net.bwd[L]), b.voff, ln.act_r);
  __syncthreads();
  static_for<MT>([&](auto I) {
    static_for<2>([&](auto GP) {
      static_for<2>([&](auto NT) {
        float v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int j = 8 * GP + q;
          v[q] = acc[I][NT][j] * unpark(sp[L - 1][I][NT][j], acc[I][NT][j]);
        }
        act_store_pair<W, MODE, I, GP, NT>(ln, v);
      });
      __builtin_amdgcn_sched_barrier(0);
    });
  });
  __syncthreads();
  if constexpr (TRAIN) dump_tile<W, MODE>(td.act, td.g(L), td.ldb, td.q0, td.nvalid);  // g3 or g2
}

// Last reverse layer: g1 = (W2^T g2) * SiLU'(z1) with z1 recomputed, then the
// input-layer gradient e = W1^T g1 accumulated per lane in FP32.
template <int W, int MODE, bool PAIRS, bool TRAIN>
__device__ __forceinline__ void bwd_input(const DevNet& net, const Lane<W, MODE>& ln, const Bases<W, MODE>& b,
                                          float (&epart)[2][9], const TileDump& td) {
  constexpr int MT = Geo<W>::MT;
  constexpr int XF = Geo<W>::XIN_FLOATS;
  f32x16 acc[MT][2];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[i][nt][j] = 0.f;
  layer_gemm<W, MODE>(acc, stream_rsrc<W, MODE>(net.bwd[0]), b.voff, ln.act_r);
  float g1keep[TRAIN ? MT : 1][2][16];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float* w = b.w1 + (16 * i + 4 * g + r) * 12;
        const f32x4 wa = *reinterpret_cast<const f32x4*>(w);
        const f32x4 wb = *reinterpret_cast<const f32x4*>(w + 4);
        const f32x2 wc = *reinterpret_cast<const f32x2*>(w + 8);
        const float cr = PAIRS ? wa[3] : b.crow[16 * i + 4 * g + r];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
          const float* x = b.xin + nt * 32 * XF;
          const float c = PAIRS ? arm_term(wa[3], wb[0], wb[1], wb[2], wb[3], wc[0], wc[1], x + 5) : cr;
          const float z = input_preact(c, wa[0], wa[1], wa[2], x);
          const float g1 = acc[i][nt][4 * g + r] * silu_prime_only(z);
          epart[nt][0] += wa[0] * g1;
          epart[nt][1] += wa[1] * g1;
          epart[nt][2] += wa[2] * g1;
          epart[nt][3] += wb[0] * g1;
          epart[nt][4] += wb[1] * g1;
          epart[nt][5] += wb[2] * g1;
          epart[nt][6] += wb[3] * g1;
          epart[nt][7] += wc[0] * g1;
          epart[nt][8] += wc[1] * g1;
          if constexpr (TRAIN) g1keep[i][nt][4 * g + r] = g1;
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
    dump_tile<W, MODE>(td.act, td.g(0), td.ldb, td.q0, td.nvalid);
  }
}

// Input layer (FP32): z1 = W1 [p'; a] + b1, h1 = SiLU(z1) -> LDS.
template <int W, int MODE, bool PAIRS>
__device__ __forceinline__ void fwd_input(const Lane<W, MODE>& ln, const Bases<W, MODE>& b) {
  constexpr int MT = Geo<W>::MT;
  constexpr int XF = Geo<W>::XIN_FLOATS;
  static_for<MT>([&](auto I) {
    static_for<2>([&](auto GP) {
      f32x4 wa[8], wb[8];
      f32x2 wc[8];
      float cr[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float* w = b.w1 + (16 * I + 8 * GP + q) * 12;
        wa[q] = *reinterpret_cast<const f32x4*>(w);
        if constexpr (PAIRS) {
          wb[q] = *reinterpret_cast<const f32x4*>(w + 4);
          wc[q] = *reinterpret_cast<const f32x2*>(w + 8);
        } else {
          cr[q] = b.crow[16 * I + 8 * GP + q];
        }
      }
      static_for<2>([&](auto NT) {
        const float* x = b.xin + NT * 32 * XF;
        float v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          float c = PAIRS ? 0.f : cr[q];
          if constexpr (PAIRS) c = arm_term(wa[q][3], wb[q][0], wb[q][1], wb[q][2], wb[q][3], wc[q][0], wc[q][1], x + 5);
          v[q] = silu_only(input_preact(c, wa[q][0], wa[q][1], wa[q][2], x));
        }
        act_store_pair<W, MODE, I, GP, NT>(ln, v);
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
  float* red;   // [4][10][64]
  Lane<W, MODE> ln;
  Bases<W, MODE> b;
  __device__ __forceinline__ TileCtx(char* lds, const DevNet& net, int tid)
      : act(lds), ln(lds, tid) {
    using G = Geo<W>;
    constexpr int MT = G::MT;
    xin = reinterpret_cast<float*>(lds + G::ACT_BYTES);
    crow = xin + kTileQ * G::XIN_FLOATS;
    red = crow + W;
    float* vec = red + kWaves * G::RED_VALS * kTileQ;  // [4][W]: b2, b3, b4, w_out
    for (int i = tid; i < 4 * W; i += kThreads) vec[i] = i < 3 * W ? net.bh[i] : net.w5[i - 3 * W];
    // bytes of one matrix's fragment stream per wave (1 KiB per fragment)
    const size_t stream_bytes = (size_t)(MODE == kFP32 ? G::NK8 : G::NKB) * MT * 1024;
    const int lblk = (ln.wave * 2 + ln.h) * MT * 16;  // this lane's block of lane-major rows
    b.bh = vec + lblk;
    b.w5 = vec + 3 * W + lblk;
    b.w1 = net.w1p + lblk * 12;
    b.crow = crow + lblk;
    b.xin = xin + ln.n0 * G::XIN_FLOATS;
    b.voff = (int)(ln.wave * stream_bytes) + ln.lane * 16;
  }
};

// One tile: 64 points of knot kk starting at point q0 (dense), or pair-list
// entries q0 .. q0+63 (pairs).  Every thread of the workgroup calls it; it ends
// with a barrier, so consecutive calls can reuse the shared memory.
template <int W, int MODE, bool PAIRS, bool TRAIN = false, bool GATHER = false>
__device__ __forceinline__ void process_tile(const DevNet& net, const Job& job, int want_grad, int64_t kk,
                                             int64_t q0, TileCtx<W, MODE>& tc) {
  using G = Geo<W>;
  constexpr int MT = G::MT;
  constexpr int XF = G::XIN_FLOATS;
  const int tid = threadIdx.x;
  float* xin = tc.xin;
  float* crow = tc.crow;
  float* red = tc.red;
  const Lane<W, MODE>& ln = tc.ln;
  const Bases<W, MODE>& b = tc.b;
  const int64_t qlimit = PAIRS ? job.npairs : (GATHER ? job.row_off[kk + 1] : job.Np);

  // ---- prologue: base-frame points (+ per-knot arm term of the input layer) ----
  if (tid < kTileQ) {
    const int64_t q = q0 + tid;
    const int64_t qc = q < qlimit ? q : qlimit - 1;   // clamp the ragged tail (never stored)
    int64_t ki, pi;
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
        pi = job.pidx ? job.pidx[qc] : qc;
      }
    } else {
      ki = kk;
      pi = GATHER ? (int64_t)job.pgather[qc] : qc;
    }
    const float* kn = job.knots + ki * kInDim;
    float pxyz[3];
    if ((PAIRS || GATHER) && (uint64_t)pi >= (uint64_t)job.Np) {
      pxyz[0] = pxyz[1] = pxyz[2] = __builtin_nanf("");  // bad point index: NaN results
    } else {
      const float* pt = job.points + pi * 3;
      pxyz[0] = pt[0];
      pxyz[1] = pt[1];
      pxyz[2] = pt[2];
    }
    float sn, cs;
    sincosf(kn[2], &sn, &cs);
    const float ux = pxyz[0] - kn[0], uy = pxyz[1] - kn[1];
    float* x = xin + tid * XF;
    x[0] = cs * ux + sn * uy;
    x[1] = -sn * ux + cs * uy;
    x[2] = pxyz[2];
    x[3] = cs;
    x[4] = sn;
#pragma unroll
    for (int c = 0; c < 6; ++c) x[5 + c] = kn[3 + c];
    // reverse-sweep seed: dL/dd for training, else 1 (multiplying by 1 is exact)
    x[11] = job.seed ? (q < qlimit ? job.seed[qc] : 0.f) : 1.f;
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
    const float* kn = job.knots + kk * kInDim;
    for (int r = tid; r < W; r += kThreads) {  // r: lane-major position
      const float* w = net.w1p + r * 12;
      crow[r] = arm_term(w[3], w[4], w[5], w[6], w[7], w[8], w[9], kn + 3);
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
  }
  fwd_input<W, MODE, PAIRS>(ln, b);
  __syncthreads();
  if constexpr (TRAIN) dump_tile<W, MODE>(td.act, td.h(0), td.ldb, td.q0, td.nvalid);  // h1

  // ---- hidden layers 2..4 (forward), keeping SiLU' of layers 2 and 3 ----
  float sp[2][MT][2][16];
  float dpart[2] = {0.f, 0.f};
  fwd_hidden<W, MODE, 0, TRAIN>(net, ln, b, sp, dpart, want_grad, td);
  fwd_hidden<W, MODE, 1, TRAIN>(net, ln, b, sp, dpart, want_grad, td);
  fwd_hidden<W, MODE, 2, TRAIN>(net, ln, b, sp, dpart, want_grad, td);

  // ---- reverse sweep: W4^T, W3^T (into LDS), W2^T (into the input-layer gradient) ----
  float epart[2][9];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt)
#pragma unroll
    for (int c = 0; c < 9; ++c) epart[nt][c] = 0.f;
  if (want_grad) {
    bwd_hidden<W, MODE, 2, TRAIN>(net, ln, b, sp, td);
    bwd_hidden<W, MODE, 1, TRAIN>(net, ln, b, sp, td);
    bwd_input<W, MODE, PAIRS, TRAIN>(net, ln, b, epart, td);
  }

  // ---- reduce d and e over the rows: lane halves, then waves (fixed order) ----
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    dpart[nt] += __shfl_xor(dpart[nt], 32);
#pragma unroll
    for (int c = 0; c < 9; ++c) epart[nt][c] += __shfl_xor(epart[nt][c], 32);
  }
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
    const int n = tid;
    float vals[G::RED_VALS];
#pragma unroll
    for (int c = 0; c < G::RED_VALS; ++c) {
      float sum = red[(0 * G::RED_VALS + c) * kTileQ + n];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) sum += red[(w * G::RED_VALS + c) * kTileQ + n];
      vals[c] = sum;
    }
    const float dv = vals[0] + *net.b5p;
    const int64_t q = q0 + n;
    const bool valid = q < qlimit;
    const int64_t out = (PAIRS || GATHER) ? q : kk * job.Np + q;
    // outputs are streamed with non-temporal stores: written once and never read
    // here, they would otherwise evict the packed weights from L2
    if (valid && job.d) __builtin_nontemporal_store(dv, job.d + out);
    if (valid && job.J && want_grad) {
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
  // The next tile's prologue rewrites xin and crow: every wave has passed the
  // barrier above (crow's last reader), and xin's readers here are wave 0,
  // which also writes it, in program order.
  __syncthreads();
}

// ----------------------------------------------------------------------------
// One-shot kernel: a persistent grid strides over all tiles of one job.
// ----------------------------------------------------------------------------
template <int W, int MODE, bool PAIRS, int OCC, bool TRAIN = false, bool GATHER = false>
__global__ __launch_bounds__(kThreads, OCC) void fused_query(const DevNet net, const Job job, int want_grad,
                                                             int64_t ntiles) {
  __shared__ __attribute__((aligned(16))) char lds[Geo<W>::LDS_BYTES];
  TileCtx<W, MODE> tc(lds, net, threadIdx.x);
  const int64_t nblk = PAIRS ? 0 : (job.Np + kTileQ - 1) / kTileQ;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    if constexpr (PAIRS) {
      process_tile<W, MODE, true, TRAIN>(net, job, want_grad, 0, tile * kTileQ, tc);
    } else if constexpr (GATHER) {
      if (tile >= job.tile_off[job.K]) break;  // the grid is sized by an upper bound
      int64_t lo = 0, hi = job.K - 1;            // knot: the last i with tile_off[i] <= tile
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (job.tile_off[mid] <= tile) lo = mid; else hi = mid - 1;
      }
      process_tile<W, MODE, false, false, true>(net, job, want_grad, lo,
                                                job.row_off[lo] + (tile - job.tile_off[lo]) * kTileQ, tc);
    } else {
      const int64_t kk = tile / nblk;
      process_tile<W, MODE, false>(net, job, want_grad, kk, (tile - kk * nblk) * kTileQ, tc);
    }
  }
}

// ----------------------------------------------------------------------------
// Table I training loss: per tile of 64 samples (sample i = knot i, point i)
//   forward      z_l, h_l                       (3 GEMMs W_l)
//   reverse      r_l = W_{l+1}^T g_{l+1}, g_l = r_l s'(z_l), r_4 = w_out    (3 GEMMs W^T)
//   tangent      zdot_1 = W_1 u, hdot_l = s'(z_l) zdot_l, zdot_{l+1} = W hdot (3 GEMMs W_l)
//   adjoint      zbar_4 = fbar w_out s'(z_4) + w_out s''(z_4) zdot_4,
//                zbar_l = hbar_l s'(z_l) + r_l s''(z_l) zdot_l, hbar_l = W^T zbar (3 GEMMs W^T)
// The weight gradient is then sum_i zbar_l h_{l-1}^T + g_l hdot_{l-1}^T per layer (and
// the input / output layers' equivalents), formed from the dumps by the GEMM and
// reduction kernels.  Pre-activations z, zdot and the products r are kept per
// workgroup in a register-order scratch (float4 k of thread t at (k * 256 + t) * 4),
// and every elementwise step streams them group by group, so at most one
// accumulator array is live.
// ----------------------------------------------------------------------------
__device__ __forceinline__ void silu_d12(float z, float& d1, float& d2) {
  const float t = __builtin_amdgcn_exp2f(-z * kLog2e);
  const float sg = __builtin_amdgcn_rcpf(1.0f + t);
  const float om = 1.0f - sg;
  d1 = sg + z * sg * om;                       // s'
  d2 = sg * om * (2.0f + z * (1.0f - 2.0f * sg));  // s''
}

template <int W>
__global__ __launch_bounds__(kThreads, 1) void table1_tiles(const DevNet net, const T1Job job, int64_t ntiles) {
  constexpr int MODE = kFP32;
  using G = Geo<W>;
  constexpr int MT = G::MT;
  constexpr int XF = G::XIN_FLOATS;
  __shared__ __attribute__((aligned(16))) char lds[G::LDS_BYTES];
  TileCtx<W, MODE> tc(lds, net, threadIdx.x);
  const Lane<W, MODE>& ln = tc.ln;
  const Bases<W, MODE>& b = tc.b;
  float* uin = tc.red;  // [64][9] tangent direction of the tile's samples
  const int tid = threadIdx.x;
  const size_t arr = (size_t)kThreads * 64;
  float* scr = job.scratch + (size_t)blockIdx.x * kT1ScratchArrays * arr;
  float* sZ = scr;             // z_1..z_4
  float* sZd = scr + 4 * arr;  // zdot_1..zdot_4
  float* sR = scr + 8 * arr;   // r_1..r_3
  const size_t layer = (size_t)W * job.ldb;
  // float4 idx of this thread in a scratch array (elements 4 (idx % 4) .. +3 of
  // accumulator (i, nt) with idx / 4 = i * 2 + nt)
  auto sget = [&](const float* base, int idx) {
    return *reinterpret_cast<const f32x4*>(base + ((size_t)idx * kThreads + tid) * 4);
  };
  auto sput = [&](float* base, int idx, const f32x4& v) {
    *reinterpret_cast<f32x4*>(base + ((size_t)idx * kThreads + tid) * 4) = v;
  };
  auto zero = [&](f32x16 (&x)[MT][2]) {
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int j = 0; j < 16; ++j) x[i][nt][j] = 0.f;
  };
  // a (accumulators) -> LDS tile, element by element through f(I, NT, j, value, z, zd, r),
  // with z / zd / r read from the scratch arrays when given (group by group)
  auto emit = [&](f32x16 (&a)[MT][2], const float* bz, const float* bzd, const float* br, auto&& f) {
    static_for<MT>([&](auto I) {
      static_for<2>([&](auto GP) {
        static_for<2>([&](auto NT) {
          float v[8];
#pragma unroll
          for (int hh = 0; hh < 2; ++hh) {
            const int idx = (I * 2 + NT) * 4 + 2 * GP + hh;
            const f32x4 zz = bz ? sget(bz, idx) : f32x4{0.f, 0.f, 0.f, 0.f};
            const f32x4 dd = bzd ? sget(bzd, idx) : f32x4{0.f, 0.f, 0.f, 0.f};
            const f32x4 rr = br ? sget(br, idx) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int j = 8 * GP + 4 * hh + u;
              v[4 * hh + u] = f(I, NT, j, a[I][NT][j], zz[u], dd[u], rr[u]);
            }
          }
          act_store_pair<W, MODE, I, GP, NT>(ln, v);
        });
        __builtin_amdgcn_sched_barrier(0);
      });
    });
  };
  auto put_all = [&](float* base, const f32x16 (&x)[MT][2]) {
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int k = 0; k < 4; ++k)
          sput(base, (i * 2 + nt) * 4 + k,
               f32x4{x[i][nt][4 * k], x[i][nt][4 * k + 1], x[i][nt][4 * k + 2], x[i][nt][4 * k + 3]});
  };

  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t q0 = tile * kTileQ;
    const int nvalid = (int)(job.B - q0 < kTileQ ? job.B - q0 : kTileQ);
    auto dumpl = [&](float* arrbase, int l) { dump_tile<W, MODE>(tc.act, arrbase + l * layer, job.ldb, q0, nvalid); };
    // ---- prologue: base-frame points, fbar and u of the tile's samples ----
    if (tid < kTileQ) {
      const int64_t q = q0 + tid;
      const bool ok = q < job.B;
      const int64_t qc = ok ? q : job.B - 1;
      const float* kn = job.knots + qc * kInDim;
      const float* pt = job.points + qc * 3;
      float sn, cs;
      sincosf(kn[2], &sn, &cs);
      const float ux = pt[0] - kn[0], uy = pt[1] - kn[1];
      float* x = tc.xin + tid * XF;
      x[0] = cs * ux + sn * uy;
      x[1] = -sn * ux + cs * uy;
      x[2] = pt[2];
      x[3] = cs;
      x[4] = sn;
#pragma unroll
      for (int c = 0; c < 6; ++c) x[5 + c] = kn[3 + c];
      x[11] = ok ? job.fbar[qc] : 0.f;
#pragma unroll
      for (int c = 0; c < 9; ++c) uin[tid * 9 + c] = ok ? job.u[c * job.ldb + qc] : 0.f;
#pragma unroll
      for (int c = 0; c < 3; ++c) job.V[c * job.ldb + q] = ok ? x[c] : 0.f;
#pragma unroll
      for (int c = 0; c < 6; ++c) job.V[(3 + c) * job.ldb + q] = ok ? x[5 + c] : 0.f;
    }
    __syncthreads();

    // ---- input layer: z_1 to the scratch, h_1 to LDS (8 rows at a time) ----
    static_for<MT>([&](auto I) {
      static_for<2>([&](auto GP) {
        f32x4 wa[8], wb[8];
        f32x2 wc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float* w = b.w1 + (16 * I + 8 * GP + q) * 12;
          wa[q] = *reinterpret_cast<const f32x4*>(w);
          wb[q] = *reinterpret_cast<const f32x4*>(w + 4);
          wc[q] = *reinterpret_cast<const f32x2*>(w + 8);
        }
        static_for<2>([&](auto NT) {
          const float* x = b.xin + NT * 32 * XF;
          float zv[8], hv[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const float c = arm_term(wa[q][3], wb[q][0], wb[q][1], wb[q][2], wb[q][3], wc[q][0], wc[q][1], x + 5);
            zv[q] = input_preact(c, wa[q][0], wa[q][1], wa[q][2], x);
            hv[q] = silu_only(zv[q]);
          }
          const int idx = (I * 2 + NT) * 4 + 2 * GP;
          sput(sZ, idx, f32x4{zv[0], zv[1], zv[2], zv[3]});
          sput(sZ, idx + 1, f32x4{zv[4], zv[5], zv[6], zv[7]});
          act_store_pair<W, MODE, I, GP, NT>(ln, hv);
        });
        __builtin_amdgcn_sched_barrier(0);
      });
    });
    __syncthreads();
    dumpl(job.H, 0);

    f32x16 a[MT][2];
    // ---- hidden layers forward: z to the scratch, h to LDS ----
    static_for<3>([&](auto L) {
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const f32x4 b4 = *reinterpret_cast<const f32x4*>(b.bh + L * W + 16 * i + 4 * g);
#pragma unroll
          for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int r = 0; r < 4; ++r) a[i][nt][4 * g + r] = b4[r];
        }
      layer_gemm<W, MODE>(a, stream_rsrc<W, MODE>(net.fwd[L]), b.voff, ln.act_r);
      __syncthreads();
      put_all(sZ + (L + 1) * arr, a);
      emit(a, nullptr, nullptr, nullptr, [&](int, int, int, float acc, float, float, float) { return silu_only(acc); });
      __syncthreads();
      dumpl(job.H, L + 1);
      __syncthreads();
    });
    // ---- reverse sweep: g_4 = w_out s'(z_4); r_l = W_{l+1}^T g_{l+1}; g_l = r_l s'(z_l) ----
    emit(a, sZ + 3 * arr, nullptr, nullptr, [&](int I, int, int j, float, float z, float, float) {
      float d1, d2;
      silu_d12(z, d1, d2);
      return b.w5[16 * I + j] * d1;
    });
    __syncthreads();
    dumpl(job.G, 3);
    static_for<3>([&](auto LL) {
      constexpr int L = 2 - LL;  // W_{L+2}^T g_{L+2} = r_{L+1}
      zero(a);
      layer_gemm<W, MODE>(a, stream_rsrc<W, MODE>(net.bwd[L]), b.voff, ln.act_r);
      __syncthreads();
      put_all(sR + L * arr, a);
      emit(a, sZ + L * arr, nullptr, nullptr, [&](int, int, int, float acc, float z, float, float) {
        float d1, d2;
        silu_d12(z, d1, d2);
        return acc * d1;
      });
      __syncthreads();
      dumpl(job.G, L);
      __syncthreads();
    });
    // ---- tangent pass along u: zdot_1 = W_1 u to the scratch, hdot_1 to LDS ----
    static_for<MT>([&](auto I) {
      static_for<2>([&](auto GP) {
        f32x4 wa[8], wb[8];
        f32x2 wc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const float* w = b.w1 + (16 * I + 8 * GP + q) * 12;
          wa[q] = *reinterpret_cast<const f32x4*>(w);
          wb[q] = *reinterpret_cast<const f32x4*>(w + 4);
          wc[q] = *reinterpret_cast<const f32x2*>(w + 8);
        }
        static_for<2>([&](auto NT) {
          const float* uu = uin + (32 * NT + ln.n0) * 9;
          const int idx = (I * 2 + NT) * 4 + 2 * GP;
          const f32x4 z0 = sget(sZ, idx), z1 = sget(sZ, idx + 1);
          float zd[8], hd[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            float t = wa[q][0] * uu[0];
            t += wa[q][1] * uu[1];
            t += wa[q][2] * uu[2];
            t += wb[q][0] * uu[3];
            t += wb[q][1] * uu[4];
            t += wb[q][2] * uu[5];
            t += wb[q][3] * uu[6];
            t += wc[q][0] * uu[7];
            t += wc[q][1] * uu[8];
            zd[q] = t;
            float d1, d2;
            silu_d12(q < 4 ? z0[q] : z1[q - 4], d1, d2);
            hd[q] = d1 * t;
          }
          sput(sZd, idx, f32x4{zd[0], zd[1], zd[2], zd[3]});
          sput(sZd, idx + 1, f32x4{zd[4], zd[5], zd[6], zd[7]});
          act_store_pair<W, MODE, I, GP, NT>(ln, hd);
        });
        __builtin_amdgcn_sched_barrier(0);
      });
    });
    __syncthreads();
    dumpl(job.Hd, 0);
    static_for<3>([&](auto L) {
      // zdot_{L+2} = W_{L+2} hdot_{L+1}; hdot_{L+2} = s'(z_{L+2}) zdot_{L+2}
      zero(a);
      layer_gemm<W, MODE>(a, stream_rsrc<W, MODE>(net.fwd[L]), b.voff, ln.act_r);
      __syncthreads();
      put_all(sZd + (L + 1) * arr, a);
      emit(a, sZ + (L + 1) * arr, nullptr, nullptr, [&](int, int, int, float acc, float z, float, float) {
        float d1, d2;
        silu_d12(z, d1, d2);
        return d1 * acc;
      });
      __syncthreads();
      dumpl(job.Hd, L + 1);
      __syncthreads();
    });
    // ---- adjoint of the primal ----
    emit(a, sZ + 3 * arr, sZd + 3 * arr, nullptr, [&](int I, int NT, int j, float, float z, float zd, float) {
      const float w5 = b.w5[16 * I + j];
      const float fb = b.xin[NT * 32 * XF + 11];
      float d1, d2;
      silu_d12(z, d1, d2);
      return (fb * w5) * d1 + w5 * d2 * zd;
    });
    __syncthreads();
    dumpl(job.Zb, 3);
    static_for<3>([&](auto LL) {
      constexpr int L = 2 - LL;  // hbar_{L+1} = W_{L+2}^T zbar_{L+2}
      zero(a);
      layer_gemm<W, MODE>(a, stream_rsrc<W, MODE>(net.bwd[L]), b.voff, ln.act_r);
      __syncthreads();
      emit(a, sZ + L * arr, sZd + L * arr, sR + L * arr, [&](int, int, int, float hb, float z, float zd, float r) {
        float d1, d2;
        silu_d12(z, d1, d2);
        return hb * d1 + r * d2 * zd;
      });
      __syncthreads();
      dumpl(job.Zb, L);
      __syncthreads();
    });
  }
}

hipError_t launch_table1_tiles(const DevNet& net, const T1Job& job, int grid, hipStream_t s) {
  if (net.width != 256 || net.mode != kFP32) return hipErrorInvalidValue;
  const int64_t ntiles = (job.B + kTileQ - 1) / kTileQ;
  hipLaunchKernelGGL(table1_tiles<256>, dim3((unsigned)grid), dim3(kThreads), 0, s, net, job, ntiles);
  return hipGetLastError();
}

// Per sample: loss terms and their derivatives (fixed-order sums over the batch).
__global__ __launch_bounds__(256) void table1_loss_kernel(const float* __restrict__ knots,
                                                          const float* __restrict__ points, const float* __restrict__ d,
                                                          const float* __restrict__ J, const float* __restrict__ fstar,
                                                          const float* __restrict__ Jstar, Minv9 mdiag, f32x4 lam,
                                                          int64_t B, int64_t ldb, float* __restrict__ fbar,
                                                          float* __restrict__ u, float* __restrict__ part) {
  __shared__ float red[4][256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float l4[4] = {0.f, 0.f, 0.f, 0.f};
  const float invn = 1.0f / (float)B;
  if (i < ldb) {
    float uu[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float fb = 0.f;
    if (i < B) {
      const float* Ji = J + i * 9;
      const float* Js = Jstar + i * 9;
      float nJ2 = 0.f, nJs2 = 0.f, dot = 0.f, nm2 = 0.f;
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        nJ2 += Ji[c] * Ji[c];
        nJs2 += Js[c] * Js[c];
        dot += Ji[c] * Js[c];
        nm2 += Ji[c] * Ji[c] / mdiag.v[c];
      }
      const float nJ = sqrtf(nJ2), nJs = sqrtf(nJs2), nm = sqrtf(nm2);
      const float cosv = dot / (nJ * nJs);
      const float rd = d[i] - fstar[i];
      l4[0] = rd * rd * invn;
      l4[1] = (1.f - cosv) * (1.f - cosv) * invn;
      l4[2] = (nm - 1.f) * (nm - 1.f) * invn;
      l4[3] = nJ2 * invn;
      fb = lam[0] * 2.f * rd * invn;
      float Jb[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        const float dcos = Js[c] / (nJ * nJs) - cosv * Ji[c] / nJ2;
        Jb[c] = invn * (lam[1] * (-2.f * (1.f - cosv) * dcos) + lam[2] * (2.f * (nm - 1.f) * Ji[c] / (mdiag.v[c] * nm)) +
                        lam[3] * 2.f * Ji[c]);
      }
      const float* kn = knots + i * 9;
      const float* pt = points + i * 3;
      float sn, cs;
      sincosf(kn[2], &sn, &cs);
      const float ux = pt[0] - kn[0], uy = pt[1] - kn[1];
      const float px = cs * ux + sn * uy, py = -sn * ux + cs * uy;
      uu[0] = -cs * Jb[0] - sn * Jb[1] + py * Jb[2];
      uu[1] = sn * Jb[0] - cs * Jb[1] - px * Jb[2];
#pragma unroll
      for (int c = 3; c < 9; ++c) uu[c] = Jb[c];
      fbar[i] = fb;
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) u[c * ldb + i] = uu[c];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = l4[k];
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[(int64_t)blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void table1_loss_sum_kernel(const float* __restrict__ part, int nblocks, f32x4 lam, float* __restrict__ losses) {
  if (threadIdx.x != 0) return;
  float t[4] = {0.f, 0.f, 0.f, 0.f};
  for (int k = 0; k < nblocks; ++k)
#pragma unroll
    for (int c = 0; c < 4; ++c) t[c] += part[k * 4 + c];
#pragma unroll
  for (int c = 0; c < 4; ++c) losses[c] = t[c];
  losses[4] = lam[0] * t[0] + lam[1] * t[1] + lam[2] * t[2] + lam[3] * t[3];
}

hipError_t launch_table1_loss(const float* knots, const float* points, const float* d, const float* J,
                              const float* fstar, const float* Jstar, const float* m_diag, const float* lambda,
                              int64_t B, int64_t ldb, float* fbar, float* u, float* part, float* losses,
                              hipStream_t s) {
  Minv9 md{};
  for (int c = 0; c < 9; ++c) md.v[c] = m_diag[c];
  const f32x4 lam = {lambda[0], lambda[1], lambda[2], lambda[3]};
  const int nb = (int)((ldb + 255) / 256);
  hipLaunchKernelGGL(table1_loss_kernel, dim3((unsigned)nb), dim3(256), 0, s, knots, points, d, J, fstar, Jstar, md,
                     lam, B, ldb, fbar, u, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(table1_loss_sum_kernel, dim3(1), dim3(64), 0, s, part, nb, lam, losses);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Persistent serving kernel.  Requests are published by the host in sequence
// order into ServeCtl (pinned host memory); every workgroup walks the sequence
// with its own cursor and claims tiles from the slot's (seq, count) word (a
// compare-and-swap re-tags it for a new request, a fetch_add hands out the
// rest), so a late workgroup can never run tiles of a request that has since
// been replaced in its slot under the wrong descriptor.  The first workgroup
// that stays idle ends the launch for all (the drain word); tiles not yet
// claimed then wait in the claim words for the next launch.
//
// Memory ordering is paid per request, not per tile: claims are relaxed; a
// workgroup acquires (system scope) once when it sees new publications; when it
// leaves a request (its next claim finds no tile left) it releases its output
// stores at agent scope once and adds the number of tiles it ran to the slot's
// done counter.  The workgroup whose addition completes the request acquires,
// decodes the per-knot minimum, restores the key scratch and publishes
// completion with a system-scope release store.  (Acquire and release at agent
// or system scope invalidate or write back the L2, which per tile would evict
// the packed weights.)
// ----------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T sys_relaxed(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <int W, int MODE>
__global__ __launch_bounds__(kThreads, 1) void serve_loop(const DevNet net, ServeCtl* ctl, ServeDev* dev,
                                                          uint64_t first_seq, uint64_t idle_ticks, uint32_t epoch) {
  __shared__ __attribute__((aligned(16))) char lds[Geo<W>::LDS_BYTES];
  __shared__ int64_t claim_info[3];  // claimed seq (or -1: exit, -2: none), tile, seq to finalize (or -1)
  __shared__ ServeDesc cur;          // the request this workgroup is working on
  __shared__ ServeDesc fin;          // a request this workgroup completes
  TileCtx<W, MODE> tc(lds, net, threadIdx.x);
  const int tid = threadIdx.x;
  uint64_t seq = first_seq;  // this workgroup's cursor in the request sequence
  uint64_t cur_seq = ~0ull;
  uint64_t idle_since = __builtin_amdgcn_s_memrealtime();
  const uint32_t slots = sys_relaxed(&ctl->slots);
  // thread 0's view of the queue
  uint64_t pub = 0, nt_seq = ~0ull;
  int64_t ntiles = 0;
  uint64_t open_count = 0;  // tiles of request cur_seq run here and not yet reported
  int backoff = 1;
  while (true) {
    if (tid == 0) {
      int64_t got_seq = -1, got_tile = 0, fin_seq = -1;
      bool leave = false;
      // Report the tiles of request cur_seq run here (the caller has established that
      // no further tile of it will be claimed here); the report that completes the
      // request makes this workgroup its finalizer.
      auto report = [&]() {
        const uint32_t s = (uint32_t)(cur_seq % slots);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this workgroup's stores and atomics
        const unsigned long long done =
            __hip_atomic_fetch_add(&dev->done[s], open_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + open_count;
        open_count = 0;
        if (done == cur.done_target) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every contributor's results
          fin = cur;
          fin_seq = (int64_t)cur_seq;
        }
      };
      while (true) {
        if (__hip_atomic_load(&dev->drain, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch) {
          // another workgroup ended this launch: claim nothing more
          if (open_count) report();
          leave = true;
          break;
        }
        if (seq >= pub) {
          const uint64_t p = sys_relaxed(&ctl->published);
          if (p > pub) {
            pub = p;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // system scope: the new descriptors
          }
        }
        if (seq < pub) {
          const uint32_t s = (uint32_t)(seq % slots);
          if (nt_seq != seq) {
            ntiles = sys_relaxed(&ctl->desc[s].ntiles);
            nt_seq = seq;
          }
          // Claim word of the slot: (request tag << 32) | tiles handed out.  The first
          // claimant of a request re-tags the word with a compare-and-swap; every other
          // claim is a fetch_add, which never has to be retried.
          unsigned long long v = __hip_atomic_load(&dev->claim[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const uint64_t s32 = seq & 0xffffffffull;
          bool moved_on = false;
          while (true) {
            const uint64_t vs = v >> 32, vc = v & 0xffffffffull;
            if (vs > s32) { moved_on = true; break; }  // slot already reused: seq is complete
            if (vs < s32) {                            // first claim of request seq
              if (__hip_atomic_compare_exchange_strong(&dev->claim[s], &v, (s32 << 32) | 1ull, __ATOMIC_RELAXED,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                got_seq = (int64_t)seq;
                got_tile = 0;
                break;
              }
              continue;  // v now holds the current word
            }
            if ((int64_t)vc >= ntiles) { moved_on = true; break; }
            const unsigned long long w =
                __hip_atomic_fetch_add(&dev->claim[s], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t ws = w >> 32, wc = w & 0xffffffffull;
            if (ws == s32) {
              if ((int64_t)wc < ntiles) { got_seq = (int64_t)seq; got_tile = (int64_t)wc; }
              else moved_on = true;
              break;
            }
            // Between the load and the add, request seq finished and a later request
            // took the slot: the add handed out tile wc of that request, which must be
            // run here.  Its tag is the low half of its sequence number.
            const uint64_t later = seq + ((ws - s32) & 0xffffffffull);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // its descriptor
            const int64_t lnt = sys_relaxed(&ctl->desc[s].ntiles);
            // (no tiles of seq can be unreported here: seq could not have completed)
            seq = later;
            if (pub < later + 1) pub = later + 1;
            nt_seq = later;
            ntiles = lnt;
            if ((int64_t)wc < lnt) { got_seq = (int64_t)later; got_tile = (int64_t)wc; }
            else moved_on = true;
            break;
          }
          if (got_seq >= 0) break;
          if (moved_on) {
            if (open_count && cur_seq == seq) report();  // leaving request seq
            ++seq;
            if (fin_seq >= 0) break;
          }
        } else {
          if (sys_relaxed(&ctl->stop)) {
            leave = true;
            break;
          }
          if (__builtin_amdgcn_s_memrealtime() - idle_since > idle_ticks) {
            // idle: end the launch for every workgroup
            __hip_atomic_store(&dev->drain, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (open_count) report();  // (none expected: every published request has been left)
            leave = true;
            break;
          }
          // idle: back off up to ~4 us between polls of host memory
          for (int i = 0; i < backoff; ++i) __builtin_amdgcn_s_sleep(16);
          backoff = backoff < 8 ? 2 * backoff : 8;
        }
      }
      backoff = 1;
      // -1: exit (after finalizing, if fin_seq is set), -2: nothing claimed but a request to finalize
      claim_info[0] = got_seq >= 0 ? got_seq : (fin_seq >= 0 && !leave ? -2 : -1);
      claim_info[1] = got_tile;
      claim_info[2] = fin_seq;
      if (got_seq >= 0 && (uint64_t)got_seq != cur_seq) {
        const ServeDesc* d = &ctl->desc[got_seq % slots];
        cur.knots = sys_relaxed(&d->knots);
        cur.points = sys_relaxed(&d->points);
        cur.K = sys_relaxed(&d->K);
        cur.Np = sys_relaxed(&d->Np);
        cur.nblk = sys_relaxed(&d->nblk);
        cur.ntiles = sys_relaxed(&d->ntiles);
        cur.done_target = sys_relaxed(&d->done_target);
        cur.d = sys_relaxed(&d->d);
        cur.J = sys_relaxed(&d->J);
        cur.minkey = sys_relaxed(&d->minkey);
        cur.dmin = sys_relaxed(&d->dmin);
        cur.argmin = sys_relaxed(&d->argmin);
        cur.want_grad = sys_relaxed(&d->want_grad);
        cur.seq = (uint64_t)got_seq;
        cur_seq = (uint64_t)got_seq;
      }
      if (got_seq >= 0) ++open_count;
    }
    __syncthreads();
    const int64_t gs = claim_info[0];
    if (claim_info[2] >= 0) {
      // this workgroup completed request fin.seq: per-knot minimum, key scratch restored
      if (fin.dmin) {
        for (int64_t k = tid; k < fin.K; k += kThreads) {
          const unsigned long long key = __hip_atomic_load(fin.minkey + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const uint32_t o = (uint32_t)(key >> 32);
          const uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
          fin.dmin[k] = __uint_as_float(u);
          fin.argmin[k] = key == ~0ull ? 0 : (int32_t)(uint32_t)(key & 0xffffffffu);
          fin.minkey[k] = ~0ull;
        }
      }
      __threadfence_system();
      __syncthreads();
      if (tid == 0)
        __hip_atomic_store(&ctl->complete[fin.seq % slots], fin.seq + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (gs == -1) break;
    if (gs < 0) continue;
    const int64_t t = claim_info[1];
    Job job{};
    job.knots = cur.knots;
    job.points = cur.points;
    job.K = cur.K;
    job.Np = cur.Np;
    job.d = cur.d;
    job.J = cur.J;
    job.minkey = cur.minkey;
    const int64_t kk = t / cur.nblk;
    process_tile<W, MODE, false>(net, job, cur.want_grad, kk, (t - kk * cur.nblk) * kTileQ, tc);
    if (tid == 0) idle_since = __builtin_amdgcn_s_memrealtime();
  }
}

template <int W, int MODE>
static hipError_t launch_serve_t(const DevNet& net, ServeCtl* ctl, ServeDev* dev, uint64_t first_seq,
                                 uint64_t idle_ticks, uint32_t epoch, int num_cu, hipStream_t s) {
  hipLaunchKernelGGL((serve_loop<W, MODE>), dim3(num_cu), dim3(kThreads), 0, s, net, ctl, dev, first_seq, idle_ticks,
                     epoch);
  return hipGetLastError();
}

hipError_t launch_serve(const DevNet& net, ServeCtl* ctl, ServeDev* dev, uint64_t first_seq, uint64_t idle_ticks,
                        uint32_t epoch, int num_cu, hipStream_t s) {
  if (net.width == 256) {
    switch (net.mode) {
      case kFP32: return launch_serve_t<256, kFP32>(net, ctl, dev, first_seq, idle_ticks, epoch, num_cu, s);
      case kBF16: return launch_serve_t<256, kBF16>(net, ctl, dev, first_seq, idle_ticks, epoch, num_cu, s);
      default: return launch_serve_t<256, kBF16X2>(net, ctl, dev, first_seq, idle_ticks, epoch, num_cu, s);
    }
  }
  switch (net.mode) {
    case kFP32: return launch_serve_t<512, kFP32>(net, ctl, dev, first_seq, idle_ticks, epoch, num_cu, s);
    case kBF16: return launch_serve_t<512, kBF16>(net, ctl, dev, first_seq, idle_ticks, epoch, num_cu, s);
    default: return launch_serve_t<512, kBF16X2>(net, ctl, dev, first_seq, idle_ticks, epoch, num_cu, s);
  }
}

// ----------------------------------------------------------------------------
// Packing and helper kernels
// ----------------------------------------------------------------------------
size_t packed_matrix_bytes(int width, int mode) {
  return (size_t)width * width * (mode == kFP32 ? 4 : 2);
}

// Output element -> source element.  Chunk order: [wave][kstep][i] with 64 lanes per chunk.
__global__ void pack_bf16_kernel(const float* __restrict__ src, __bf16* __restrict__ dst, int W, int transpose) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)W * W) return;
  const int MT = W / (32 * kWaves), NKB = W / 16;
  const int e = idx & 7;
  const int lane = (idx >> 3) & 63;
  int64_t chunk = idx >> 9;
  const int i = chunk % MT; chunk /= MT;
  const int kb = chunk % NKB; chunk /= NKB;
  const int wave = (int)chunk;
  const int row = 32 * (wave * MT + i) + (lane & 31);
  const int col = 16 * kb + 8 * (lane >> 5) + e;
  const float v = transpose ? src[(int64_t)col * W + row] : src[(int64_t)row * W + col];
  dst[idx] = (__bf16)v;
}

__global__ void pack_fp32_kernel(const float* __restrict__ src, float* __restrict__ dst, int W, int transpose) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)W * W) return;
  const int MT = W / (32 * kWaves), NK8 = W / 8;
  const int q = idx & 3;
  const int lane = (idx >> 2) & 63;
  int64_t chunk = idx >> 8;
  const int i = chunk % MT; chunk /= MT;
  const int j = chunk % NK8; chunk /= NK8;
  const int wave = (int)chunk;
  const int row = 32 * (wave * MT + i) + (lane & 31);
  const int col = 8 * j + 2 * q + (lane >> 5);
  dst[idx] = transpose ? src[(int64_t)col * W + row] : src[(int64_t)row * W + col];
}

hipError_t pack_matrix(const float* src, void* dst, int width, int mode, bool transpose, hipStream_t s) {
  const int64_t n = (int64_t)width * width;
  const int threads = 256;
  const int blocks = (int)((n + threads - 1) / threads);
  if (mode == kFP32)
    hipLaunchKernelGGL(pack_fp32_kernel, dim3(blocks), dim3(threads), 0, s, src, static_cast<float*>(dst), width,
                       transpose ? 1 : 0);
  else
    hipLaunchKernelGGL(pack_bf16_kernel, dim3(blocks), dim3(threads), 0, s, src, static_cast<__bf16*>(dst), width,
                       transpose ? 1 : 0);
  return hipGetLastError();
}

// Lane-major position of row R (see Bases).
__host__ __device__ inline int lane_major_pos(int R, int W) {
  const int MT = W / (32 * kWaves);
  const int wave = R / (32 * MT), rem = R % (32 * MT);
  const int i = rem / 32, g = (rem % 32) / 8, h = (rem % 8) / 4, r = rem % 4;
  return ((wave * 2 + h) * MT + i) * 16 + 4 * g + r;
}

__global__ void pack_input_kernel(const float* __restrict__ W1, const float* __restrict__ b1, float* __restrict__ w1p,
                                  int W) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= W) return;
  float* o = w1p + lane_major_pos(r, W) * 12;
  o[0] = W1[r * 9 + 0];
  o[1] = W1[r * 9 + 1];
  o[2] = W1[r * 9 + 2];
  o[3] = b1[r];
  for (int c = 3; c < 9; ++c) o[1 + c] = W1[r * 9 + c];
  o[10] = 0.f;
  o[11] = 0.f;
}

hipError_t pack_input_layer(const float* W1, const float* b1, float* w1p, int width, hipStream_t s) {
  hipLaunchKernelGGL(pack_input_kernel, dim3((width + 255) / 256), dim3(256), 0, s, W1, b1, w1p, width);
  return hipGetLastError();
}

__global__ void pack_rows_kernel(const float* __restrict__ src, float* __restrict__ dst, int W, int nvec) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= W * nvec) return;
  const int v = idx / W, r = idx % W;
  dst[v * W + lane_major_pos(r, W)] = src[v * W + r];
}

hipError_t pack_row_vectors(const float* src, float* dst, int width, int nvec, hipStream_t s) {
  const int n = width * nvec;
  hipLaunchKernelGGL(pack_rows_kernel, dim3((n + 255) / 256), dim3(256), 0, s, src, dst, width, nvec);
  return hipGetLastError();
}

__global__ void minkey_init_kernel(unsigned long long* k, int64_t K) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < K) k[i] = ~0ull;
}

hipError_t launch_fill_ones(unsigned long long* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(minkey_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_minkey_init(unsigned long long* minkey, int64_t K, hipStream_t s) {
  hipLaunchKernelGGL(minkey_init_kernel, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, minkey, K);
  return hipGetLastError();
}

__global__ void minkey_decode_kernel(const unsigned long long* __restrict__ key, int64_t K, float* dmin,
                                     int32_t* argmin, int64_t* kidx, int64_t* pidx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  const unsigned long long k = key[i];
  const uint32_t o = (uint32_t)(k >> 32);
  const uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
  if (dmin) dmin[i] = __uint_as_float(u);
  // every knot of a launch receives at least one key; an untouched slot would
  // decode to index 0 rather than an out-of-range point
  const int32_t j = (k == ~0ull) ? 0 : (int32_t)(uint32_t)(k & 0xffffffffu);
  if (argmin) argmin[i] = j;
  if (kidx) kidx[i] = i;
  if (pidx) pidx[i] = j;
}

hipError_t launch_minkey_decode(const unsigned long long* minkey, int64_t K, float* dmin, int32_t* argmin,
                                int64_t* kidx, int64_t* pidx, hipStream_t s) {
  hipLaunchKernelGGL(minkey_decode_kernel, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, minkey, K, dmin,
                     argmin, kidx, pidx);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Launch
// ----------------------------------------------------------------------------
template <int W, int MODE, bool PAIRS>
static hipError_t launch_t(const DevNet& net, const Job& job, bool want_grad, int num_cu, hipStream_t s) {
  constexpr int OCC = 1;
  const int64_t ntiles = PAIRS ? (job.npairs + kTileQ - 1) / kTileQ
                               : (job.tile_off ? job.ntiles_bound : job.K * ((job.Np + kTileQ - 1) / kTileQ));
  if (ntiles <= 0) return hipSuccess;
  const int64_t slots = (int64_t)num_cu * OCC;
  const int grid = (int)(ntiles < slots ? ntiles : slots);
  if constexpr (PAIRS && W == 256 && MODE != kBF16X2) {  // training: width 256, FP32 or BF16
    if (job.dumpH) {
      hipLaunchKernelGGL((fused_query<W, MODE, true, OCC, true>), dim3(grid), dim3(kThreads), 0, s, net, job, 1,
                         ntiles);
      return hipGetLastError();
    }
  }
  if (job.dumpH) return hipErrorInvalidValue;
  if constexpr (!PAIRS) {
    if (job.tile_off) {
      hipLaunchKernelGGL((fused_query<W, MODE, false, OCC, false, true>), dim3(grid), dim3(kThreads), 0, s, net, job,
                         want_grad ? 1 : 0, ntiles);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((fused_query<W, MODE, PAIRS, OCC>), dim3(grid), dim3(kThreads), 0, s, net, job,
                     want_grad ? 1 : 0, ntiles);
  return hipGetLastError();
}

template <int W, int MODE>
static hipError_t launch_m(const DevNet& net, const Job& job, bool pairs, bool want_grad, int num_cu, hipStream_t s) {
  return pairs ? launch_t<W, MODE, true>(net, job, want_grad, num_cu, s)
               : launch_t<W, MODE, false>(net, job, want_grad, num_cu, s);
}

template <int W>
static hipError_t launch_w(const DevNet& net, const Job& job, bool pairs, bool want_grad, int num_cu, hipStream_t s) {
  switch (net.mode) {
    case kFP32: return launch_m<W, kFP32>(net, job, pairs, want_grad, num_cu, s);
    case kBF16: return launch_m<W, kBF16>(net, job, pairs, want_grad, num_cu, s);
    default: return launch_m<W, kBF16X2>(net, job, pairs, want_grad, num_cu, s);
  }
}

hipError_t launch_fused(const DevNet& net, const Job& job, bool pairs, bool want_grad, int num_cu, hipStream_t s) {
  if (net.width == 256) return launch_w<256>(net, job, pairs, want_grad, num_cu, s);
  return launch_w<512>(net, job, pairs, want_grad, num_cu, s);
}

// ----------------------------------------------------------------------------
// Training: weight gradients.
//
// out[f][g] = sum_i G[f][i] H[g][i] over the batch, G and H in the blocked
// feature-major layout of dump_tile.  Workgroup (tile, chunk) computes a 128 x 128 block of out over
// one chunk of the batch with matrix cores (4 waves, 64 x 64 each) into
// partial[chunk]; a second kernel adds the chunks in index order, so the result
// does not depend on scheduling.
// ----------------------------------------------------------------------------
constexpr int kWgChunk = 2048;  // batch samples per chunk

int wgrad_chunks(int64_t B) { return (int)((B + kWgChunk - 1) / kWgChunk); }

template <int MODE>
struct WgFrag;
template <>
struct WgFrag<kFP32> {
  f32x4 a[2], b[2];
};
template <>
struct WgFrag<kBF16> {
  bf16x8 a[2], b[2];
};

// Blocks are dealt to the 8 XCDs round-robin (block b runs on XCD b % 8); the
// mapping below keeps the 4 output tiles of one (GEMM, chunk) on one XCD, so the
// chunk's rows of G and H come from HBM once and are shared through that L2.
template <int MODE>
__global__ __launch_bounds__(256) void wgrad_gemm_kernel(WgradJobs jobs, int Wd, int64_t ldb, int64_t B, int nchunks,
                                                         float* __restrict__ partial) {
  constexpr int kXcd = 8;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tiles_n = Wd / 128, ntile = tiles_n * tiles_n;
  const int64_t groups = (int64_t)jobs.n * nchunks;  // (GEMM, chunk) pairs
  const int64_t b = blockIdx.x;
  const int64_t per_xcd = (groups + kXcd - 1) / kXcd;  // groups served by each XCD
  const int64_t local = b / kXcd, xcd = b % kXcd;
  const int64_t grp = xcd * per_xcd + local / ntile;
  if (grp >= groups) return;
  const int tile = (int)(local % ntile);
  const int job = (int)(grp / nchunks), chunk = (int)(grp % nchunks);
  const int f0 = (tile / tiles_n) * 128 + (wave >> 1) * 64;  // rows of out (G features)
  const int g0 = (tile % tiles_n) * 128 + (wave & 1) * 64;   // cols of out (H features)
  const int64_t i0 = (int64_t)chunk * kWgChunk;
  const int64_t i1 = i0 + kWgChunk < B ? i0 + kWgChunk : B;
  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[a][c][j] = 0.f;
  const int m = lane & 31, kh = lane >> 5;
  using E = typename std::conditional<MODE == kFP32, float, __bf16>::type;
  constexpr int KS = MODE == kFP32 ? 8 : 16;  // samples per step
  const E* G = static_cast<const E*>(jobs.G[job]);
  const E* H = static_cast<const E*>(jobs.H[job]);
  // The 16-byte block of S samples of feature f starts at element ((i / S) W + f) S:
  // lane (m, kh) of a step reads block i / S + kh of its row, and the 32 lanes of
  // a half read 32 consecutive features, 512 contiguous bytes.
  constexpr int S = MODE == kFP32 ? 4 : 8;  // samples per 16-byte block (KS = 2 S)
  constexpr int U = 4;                      // steps per prefetch group
  const E* ga[2] = {G + (int64_t)(kh * Wd + f0 + m) * S, G + (int64_t)(kh * Wd + f0 + 32 + m) * S};
  const E* hb[2] = {H + (int64_t)(kh * Wd + g0 + m) * S, H + (int64_t)(kh * Wd + g0 + 32 + m) * S};
  auto load = [&](WgFrag<MODE>& f, int64_t i, int u) {
    const int64_t off = ((i + (int64_t)KS * u) / S) * Wd * S;  // first block of step u
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      if constexpr (MODE == kFP32) {
        f.a[t] = *reinterpret_cast<const f32x4*>(ga[t] + off);
        f.b[t] = *reinterpret_cast<const f32x4*>(hb[t] + off);
      } else {
        f.a[t] = *reinterpret_cast<const bf16x8*>(ga[t] + off);
        f.b[t] = *reinterpret_cast<const bf16x8*>(hb[t] + off);
      }
    }
  };
  auto mma = [&](const WgFrag<MODE>& f) {
    if constexpr (MODE == kFP32) {
      // lane (m, kh) holds samples 4 kh + q of the step; MFMA q pairs samples q and 4 + q
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int ta = 0; ta < 2; ++ta)
#pragma unroll
          for (int tb = 0; tb < 2; ++tb)
            acc[ta][tb] = __builtin_amdgcn_mfma_f32_32x32x2f32(f.a[ta][q], f.b[tb][q], acc[ta][tb], 0, 0, 0);
    } else {
#pragma unroll
      for (int ta = 0; ta < 2; ++ta)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb)
          acc[ta][tb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.a[ta], f.b[tb], acc[ta][tb], 0, 0, 0);
    }
  };
  // Rows hold zeros from B up to the next multiple of 64 and chunks start at
  // multiples of 64, so whole groups are read.  Double-buffered: the loads of the
  // next group are in flight while this one runs on the matrix cores.
  static_assert(U * KS <= kTileQ, "a group must not run past the zero-padded tail");
  WgFrag<MODE> cur[U], nxt[U];
  if (i0 < i1) {
#pragma unroll
    for (int u = 0; u < U; ++u) load(cur[u], i0, u);
  }
  for (int64_t i = i0; i < i1; i += U * KS) {
    if (i + U * KS < i1) {
#pragma unroll
      for (int u = 0; u < U; ++u) load(nxt[u], i + U * KS, u);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) mma(cur[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) cur[u] = nxt[u];
  }
  // C layout: lane (n = lane%32, half h) holds rows 8 (j/4) + 4 h + j%4 of column n
  float* out = partial + ((int64_t)job * nchunks + chunk) * Wd * Wd;
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int row = f0 + 32 * ta + 8 * (j >> 2) + 4 * kh + (j & 3);
        const int col = g0 + 32 * tb + m;
        out[(int64_t)row * Wd + col] = acc[ta][tb][j];
      }
}

// out_j[e] = sum over chunks (in index order) of partial[j][chunk][e], 4 elements per thread.
__global__ void sum_chunks_kernel(const float* __restrict__ partial, int nchunks, int64_t n, WgradJobs jobs, int accum) {
  const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  const int job = blockIdx.y;
  if (t >= n) return;
  const float* p = partial + (int64_t)job * nchunks * n + t;
  f32x4 s = {0.f, 0.f, 0.f, 0.f};
  for (int c = 0; c < nchunks; ++c) {
    const f32x4 v = *reinterpret_cast<const f32x4*>(p + (int64_t)c * n);
#pragma unroll
    for (int u = 0; u < 4; ++u) s[u] += v[u];
  }
  float* o = jobs.out[job] + t;
#pragma unroll
  for (int u = 0; u < 4; ++u) o[u] = accum ? o[u] + s[u] : s[u];
}

hipError_t launch_wgrad_gemm(const WgradJobs& jobs, int width, int mode, int64_t ldb, int64_t B, float* partial,
                             int nchunks, hipStream_t s, bool accumulate) {
  if (jobs.n < 1 || jobs.n > kWgMaxJobs || width % 128) return hipErrorInvalidValue;
  const int ntile = (width / 128) * (width / 128);
  const int64_t groups = (int64_t)jobs.n * nchunks;
  const int64_t per_xcd = (groups + 7) / 8;
  const unsigned grid = (unsigned)(8 * per_xcd * ntile);
  if (mode == kFP32)
    hipLaunchKernelGGL(wgrad_gemm_kernel<kFP32>, dim3(grid), dim3(256), 0, s, jobs, width, ldb, B, nchunks, partial);
  else
    hipLaunchKernelGGL(wgrad_gemm_kernel<kBF16>, dim3(grid), dim3(256), 0, s, jobs, width, ldb, B, nchunks, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)width * width;
  hipLaunchKernelGGL(sum_chunks_kernel, dim3((unsigned)((n / 4 + 255) / 256), (unsigned)jobs.n), dim3(256), 0, s,
                     partial, nchunks, n, jobs, accumulate ? 1 : 0);
  return hipGetLastError();
}

// Row reductions over the batch in two fixed-order passes, A in the blocked
// feature-major layout of dump_tile.  Pass 1: grid (256-row group, chunk of
// kRrChunk samples); a thread owns one row and walks the chunk's 16-byte blocks
// in order (a workgroup reads 4 KB contiguous per block), V is read uniformly.
// Pass 2 adds the chunks in index order.  The result does not depend on scheduling.
constexpr int kRrChunk = 512;
constexpr int kRrMaxC = 9;

int rr_chunks(int64_t B) { return (int)((B + kRrChunk - 1) / kRrChunk); }

template <bool BF>
__global__ __launch_bounds__(256) void rr_partial_kernel(const void* __restrict__ Av, int rows, int64_t B,
                                                          const float* __restrict__ V, int64_t ldv, int C,
                                                          float* __restrict__ partial) {
  constexpr int S = BF ? 8 : 4;  // samples per 16-byte block
  __shared__ float sv[kRrMaxC][kRrChunk];  // this chunk of V (zero past B)
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * kRrChunk;
  const int64_t i1 = i0 + kRrChunk < B ? i0 + kRrChunk : B;
  for (int c = 0; c < C; ++c)
    for (int k = threadIdx.x; k < kRrChunk; k += 256) sv[c][k] = i0 + k < i1 ? V[(int64_t)c * ldv + i0 + k] : 0.f;
  __syncthreads();
  if (r >= rows) return;
  float acc[kRrMaxC + 1];
#pragma unroll
  for (int c = 0; c <= kRrMaxC; ++c) acc[c] = 0.f;
  // NB blocks per round: their loads are issued together, then consumed in order
  constexpr int NB = 8;
  static_assert(NB * S <= kTileQ && kRrChunk % (NB * S) == 0, "rounds must stay in the zero-padded tail");
  typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 v8;
  for (int64_t i = i0; i < i1; i += NB * S) {
    float a[NB][S];
    // A round covers NB * S (64 or 32) samples from a multiple of that size below B,
    // so it stays inside the zero-padded tail (rows are zero from B to the next
    // multiple of 64): the loads need no condition and are issued together.
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int64_t blk = (((i + k * S) / S) * rows + r) * S;
      if constexpr (BF) {
        const v8 x = *reinterpret_cast<const v8*>(static_cast<const __bf16*>(Av) + blk);
#pragma unroll
        for (int u = 0; u < S; ++u) a[k][u] = (float)x[u];
      } else {
        const f32x4 x = *reinterpret_cast<const f32x4*>(static_cast<const float*>(Av) + blk);
#pragma unroll
        for (int u = 0; u < S; ++u) a[k][u] = x[u];
      }
    }
#pragma unroll
    for (int k = 0; k < NB; ++k)
#pragma unroll
      for (int u = 0; u < S; ++u) acc[kRrMaxC] += a[k][u];
    // V from LDS: every lane reads the same word (a broadcast)
    const int j0 = (int)(i - i0);
    for (int c = 0; c < C; ++c) {
      float t = acc[c];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const f32x4* vp = reinterpret_cast<const f32x4*>(&sv[c][j0 + k * S]);
#pragma unroll
        for (int h = 0; h < S / 4; ++h) {
          const f32x4 vv = vp[h];
#pragma unroll
          for (int u = 0; u < 4; ++u) t += a[k][4 * h + u] * vv[u];
        }
      }
      acc[c] = t;
    }
  }
  float* out = partial + ((int64_t)blockIdx.y * rows + r) * (kRrMaxC + 1);
#pragma unroll
  for (int c = 0; c <= kRrMaxC; ++c) out[c] = acc[c];
}

__global__ void rr_sum_kernel(const float* __restrict__ partial, int nchunks, int rows, int C, float* __restrict__ out,
                              float* __restrict__ bias, int accum) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = (int)(t / (kRrMaxC + 1)), c = (int)(t % (kRrMaxC + 1));
  if (r >= rows || (c >= C && c != kRrMaxC)) return;
  float s = 0.f;
#pragma unroll 8
  for (int k = 0; k < nchunks; ++k) s += partial[((int64_t)k * rows + r) * (kRrMaxC + 1) + c];
  if (c == kRrMaxC) {
    if (bias) bias[r] = accum ? bias[r] + s : s;
  } else if (out) {
    out[(int64_t)r * C + c] = accum ? out[(int64_t)r * C + c] + s : s;
  }
}

// One workgroup: out = sum_{i < n} x[i], strided per thread then a fixed tree.
__global__ __launch_bounds__(256) void vec_sum_kernel(const float* __restrict__ x, int64_t n, float* __restrict__ out) {
  __shared__ float red[256];
  float s = 0.f;
#pragma unroll 8
  for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_row_reduce(const void* A, bool a_is_bf16, int rows, int64_t B, const float* V, int64_t ldv, int C,
                             float* out, float* bias, float* partial, hipStream_t s, bool accumulate) {
  if (C > kRrMaxC || rows <= 0 || B <= 0) return hipErrorInvalidValue;
  const int nch = rr_chunks(B);
  const dim3 grid((unsigned)((rows + 255) / 256), (unsigned)nch);
  if (a_is_bf16)
    hipLaunchKernelGGL(rr_partial_kernel<true>, grid, dim3(256), 0, s, A, rows, B, V, ldv, C, partial);
  else
    hipLaunchKernelGGL(rr_partial_kernel<false>, grid, dim3(256), 0, s, A, rows, B, V, ldv, C, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)rows * (kRrMaxC + 1);
  hipLaunchKernelGGL(rr_sum_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, partial, nch, rows, C, out,
                     bias, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_vec_sum(const float* x, int64_t n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(vec_sum_kernel, dim3(1), dim3(256), 0, s, x, n, out);
  return hipGetLastError();
}

}  // namespace gcdf
