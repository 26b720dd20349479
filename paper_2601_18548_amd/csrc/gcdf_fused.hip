// Query, training and packing kernels for gfx950 (MI355X) and their launchers;
// the per-tile query body lives in gcdf_tile.h.
#include <algorithm>

#include "gcdf_tile.h"

namespace gcdf {

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
__global__ __launch_bounds__((Geo<W, kFP32>::THREADS), 1) void table1_tiles(const DevNet net, const T1Job job, int64_t ntiles) {
  constexpr int MODE = kFP32;
  using G = Geo<W, MODE>;
  constexpr int MT = G::MT;
  constexpr int XF = G::XIN_FLOATS;
  __shared__ __attribute__((aligned(16))) char lds[G::LDS_BYTES];
  __shared__ uint32_t ovf;  // (FP32: never set)
  TileCtx<W, MODE> tc(lds, &ovf, net, threadIdx.x);
  const Lane<W, MODE>& ln = tc.ln;
  const Bases<W, MODE>& b = tc.b;
  float* uin = tc.red;  // [64][9] tangent direction of the tile's samples
  const int tid = threadIdx.x;
  constexpr int NTH = G::THREADS;
  static_assert(NTH == kThreads, "gcdf_train_table1 sizes the scratch for kThreads threads per workgroup");
  const size_t arr = (size_t)NTH * 64;
  float* scr = job.scratch + (size_t)blockIdx.x * kT1ScratchArrays * arr;
  float* sZ = scr;             // z_1..z_4
  float* sZd = scr + 4 * arr;  // zdot_1..zdot_4
  float* sR = scr + 8 * arr;   // r_1..r_3
  const size_t layer = (size_t)W * job.ldb;
  // float4 idx of this thread in a scratch array (elements 4 (idx % 4) .. +3 of
  // accumulator (i, nt) with idx / 4 = i * 2 + nt)
  auto sget = [&](const float* base, int idx) {
    return *reinterpret_cast<const f32x4*>(base + ((size_t)idx * NTH + tid) * 4);
  };
  auto sput = [&](float* base, int idx, const f32x4& v) {
    *reinterpret_cast<f32x4*>(base + ((size_t)idx * NTH + tid) * 4) = v;
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
    auto dumpl = [&](float* arrbase, int l) { dump_tile<W, MODE>(tc.act, nullptr, arrbase + l * layer, job.ldb, q0, nvalid); };
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
      layer_gemm<W, MODE, MODE>(a, stream_rsrc<W, MODE>(net.fwd[L]), b.voff, ln.act_r);
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
      layer_gemm<W, MODE, MODE>(a, stream_rsrc<W, MODE>(net.bwd[L]), b.voff, ln.act_r);
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
      layer_gemm<W, MODE, MODE>(a, stream_rsrc<W, MODE>(net.fwd[L]), b.voff, ln.act_r);
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
      layer_gemm<W, MODE, MODE>(a, stream_rsrc<W, MODE>(net.bwd[L]), b.voff, ln.act_r);
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
  hipLaunchKernelGGL(table1_tiles<256>, dim3((unsigned)grid), dim3((Geo<256, kFP32>::THREADS)), 0, s, net, job, ntiles);
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
  // the blocks in order; unrolled so that 16 blocks' loads are in flight at once
#pragma unroll 16
  for (int k = 0; k < nblocks; ++k) {
    const f32x4 v = *reinterpret_cast<const f32x4*>(part + (int64_t)k * 4);
#pragma unroll
    for (int c = 0; c < 4; ++c) t[c] += v[c];
  }
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
// Packing and helper kernels
// ----------------------------------------------------------------------------
size_t packed_matrix_bytes(int width, int mode) {
  return (size_t)width * width * (mode == kFP32 ? 4 : 2);
}

// Output element -> source element.  Chunk order: [wave][kstep][i] with 64 lanes per chunk.
// Elements are rounded to BF16; with to_f16 the BF16 value is then stored as FP16
// (exact for magnitudes in [2^-17, 65504], the range gcdf_create admits).  Element e
// of lane (m, kh) in K step kb is column 16 kb + 8 kh + e, or with lane_order
// 16 kb + 8 (e / 4) + 4 kh + e % 4 (the order the split modes keep activations in).
__device__ __forceinline__ void pack_bf16_elem(const float* __restrict__ src, uint16_t* __restrict__ dst, int W,
                                               int64_t idx, int transpose, int to_f16, int lane_order) {
  const int MT = W / (32 * kWaves), NKB = W / 16;
  const int e = idx & 7;
  const int lane = (idx >> 3) & 63;
  int64_t chunk = idx >> 9;
  const int i = chunk % MT; chunk /= MT;
  const int kb = chunk % NKB; chunk /= NKB;
  const int wave = (int)chunk;
  const int row = 32 * (wave * MT + i) + (lane & 31);
  const int col = lane_order ? 16 * kb + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3) : 16 * kb + 8 * (lane >> 5) + e;
  const float v = transpose ? src[(int64_t)col * W + row] : src[(int64_t)row * W + col];
  const __bf16 vb = (__bf16)v;
  dst[idx] = to_f16 ? __builtin_bit_cast(uint16_t, (_Float16)(float)vb) : __builtin_bit_cast(uint16_t, vb);
}

__global__ void pack_bf16_kernel(const float* __restrict__ src, uint16_t* __restrict__ dst, int W, int transpose,
                                 int to_f16, int lane_order) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (int64_t)W * W) pack_bf16_elem(src, dst, W, idx, transpose, to_f16, lane_order);
}

__device__ __forceinline__ void pack_fp32_elem(const float* __restrict__ src, float* __restrict__ dst, int W,
                                               int64_t idx, int transpose) {
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

__global__ void pack_fp32_kernel(const float* __restrict__ src, float* __restrict__ dst, int W, int transpose) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (int64_t)W * W) pack_fp32_elem(src, dst, W, idx, transpose);
}

hipError_t pack_matrix(const float* src, void* dst, int width, int mode, bool transpose, hipStream_t s) {
  const int64_t n = (int64_t)width * width;
  const int threads = 256;
  const int blocks = (int)((n + threads - 1) / threads);
  if (mode == kFP32)
    hipLaunchKernelGGL(pack_fp32_kernel, dim3(blocks), dim3(threads), 0, s, src, static_cast<float*>(dst), width,
                       transpose ? 1 : 0);
  else  // the reverse sweep of kBF16X2F16 multiplies the transposed matrix in FP16
    hipLaunchKernelGGL(pack_bf16_kernel, dim3(blocks), dim3(threads), 0, s, src, static_cast<uint16_t*>(dst), width,
                       transpose ? 1 : 0, (transpose && mode == kBF16X2F16) ? 1 : 0,
                       (mode == kBF16X2 || mode == kBF16X2F16) ? 1 : 0);
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
                                  int W, int in_dim) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= W) return;
  const float* w = W1 + (size_t)r * in_dim;
  const int arm0 = in_dim - 6;  // the arm columns are the last six
  float* o = w1p + lane_major_pos(r, W) * 12;
  o[0] = w[0];
  o[1] = w[1];
  o[2] = w[2];
  o[3] = b1[r];
  for (int c = 0; c < 6; ++c) o[4 + c] = w[arm0 + c];
  o[10] = in_dim == kInDimSphere ? w[3] : 0.f;  // radius column
  o[11] = 0.f;
}

// Every packed array of a network in one launch: blockIdx.y = 0..5 the hidden
// matrices (y < 3: W_{y+2}, else W_{y-1}^T), 6 the row vectors b2, b3, b4, w_out,
// 7 the input layer; each block packs 256 elements.
__global__ __launch_bounds__(256) void pack_all_kernel(PackJob pj) {
  const int W = pj.width;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  if (y < 6) {
    if (idx >= (int64_t)W * W) return;
    const int l = y % 3;
    const bool tr = y >= 3;
    if (pj.mode == kFP32) {
      pack_fp32_elem(pj.Wl[l], static_cast<float*>(tr ? pj.bwd[l] : pj.fwd[l]), W, idx, tr ? 1 : 0);
    } else {
      pack_bf16_elem(pj.Wl[l], static_cast<uint16_t*>(tr ? pj.bwd[l] : pj.fwd[l]), W, idx, tr ? 1 : 0,
                     (tr && pj.mode == kBF16X2F16) ? 1 : 0, (pj.mode == kBF16X2 || pj.mode == kBF16X2F16) ? 1 : 0);
    }
  } else if (y == 6) {
    if (idx >= 4 * (int64_t)W) return;
    const int v = (int)(idx / W), r = (int)(idx % W);
    const float* src = v < 3 ? pj.bl[v] : pj.w5;
    float* dst = v < 3 ? pj.bh + (size_t)v * W : pj.w5p;
    dst[lane_major_pos(r, W)] = src[r];
  } else {
    if (idx >= W) return;
    const int r = (int)idx;
    const float* w = pj.W1 + (size_t)r * pj.in_dim;
    const int arm0 = pj.in_dim - 6;
    float* o = pj.w1p + lane_major_pos(r, W) * 12;
    o[0] = w[0];
    o[1] = w[1];
    o[2] = w[2];
    o[3] = pj.b1[r];
    for (int c = 0; c < 6; ++c) o[4 + c] = w[arm0 + c];
    o[10] = pj.in_dim == kInDimSphere ? w[3] : 0.f;
    o[11] = 0.f;
  }
}

// Index of element (row, col) in a packed matrix (the inverse of pack_bf16_elem
// with the natural K order, resp. pack_fp32_elem, without transposition).
__device__ __forceinline__ int64_t packed_index_bf16(int row, int col, int W) {
  const int MT = W / (32 * kWaves), NKB = W / 16;
  const int wave = row / (32 * MT), i = (row / 32) % MT;
  const int kb = col / 16, lane = row % 32 + 32 * ((col % 16) / 8), e = col % 8;
  return ((((int64_t)wave * NKB + kb) * MT + i) * 64 + lane) * 8 + e;
}
__device__ __forceinline__ int64_t packed_index_fp32(int row, int col, int W) {
  const int MT = W / (32 * kWaves), NK8 = W / 8;
  const int wave = row / (32 * MT), i = (row / 32) % MT;
  const int j = col / 8, lane = row % 32 + 32 * (col % 2), q = (col % 8) / 2;
  return ((((int64_t)wave * NK8 + j) * MT + i) * 64 + lane) * 4 + q;
}

// Adam over a network's flat parameters, every updated value also packed.  Blocks
// [0, 3 T) take the 32 x 32 tiles of the hidden matrices (T per matrix): p, g, m
// and v are read and written by rows (a wave covers two 128-byte rows), the new
// values go through LDS, and each packed block the tile covers (32 rows by 16
// BF16 or 8 FP32 columns, 1 KiB) is written in its own order, for the forward
// packing and for the transposed one.  Then the row vectors b2, b3, b4, w_out
// (256 per block) and the input layer (row r: W1[r][:], b1[r]; thread 0 also b_out).
template <int MODE>
__device__ __forceinline__ void adam_pack_tile(const PackJob& pj, float* __restrict__ p, const float* __restrict__ g,
                                               float* __restrict__ m, float* __restrict__ v, const AdamConsts& a,
                                               int y, int tile) {
  __shared__ float t_new[32][33];
  const int W = pj.width, tpr = W / 32;
  const int r0 = (tile / tpr) * 32, c0 = (tile % tpr) * 32;
  const int64_t base = (pj.Wl[y] - p) + (int64_t)r0 * W + c0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = threadIdx.x + 256 * k, r = e >> 5, c = e & 31;
    t_new[r][c] = adam_update(p, g, m, v, base + (int64_t)r * W + c, a);
  }
  __syncthreads();
  // packed position q of a block -> (row, col) inside the block
  constexpr int kCols = MODE == kFP32 ? 8 : 16, kPer = 32 * kCols;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int P = threadIdx.x + 256 * k, blk = P / kPer, q = P % kPer;
    int r, c;
    if constexpr (MODE == kFP32) {
      const int ln = q >> 2;
      r = ln & 31;
      c = blk * kCols + 2 * (q & 3) + (ln >> 5);
    } else {
      const int ln = q >> 3;
      r = ln & 31;
      c = blk * kCols + 8 * (ln >> 5) + (q & 7);
    }
    // forward packing: W[r0 + r][c0 + c]; transposed: W^T[c0 + r][r0 + c] = W[r0 + c][c0 + r]
    const float f = t_new[r][c], b = t_new[c][r];
    if constexpr (MODE == kFP32) {
      static_cast<float*>(pj.fwd[y])[packed_index_fp32(r0 + r, c0 + c, W)] = f;
      static_cast<float*>(pj.bwd[y])[packed_index_fp32(c0 + r, r0 + c, W)] = b;
    } else {
      static_cast<uint16_t*>(pj.fwd[y])[packed_index_bf16(r0 + r, c0 + c, W)] = __builtin_bit_cast(uint16_t, (__bf16)f);
      static_cast<uint16_t*>(pj.bwd[y])[packed_index_bf16(c0 + r, r0 + c, W)] = __builtin_bit_cast(uint16_t, (__bf16)b);
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void adam_pack_kernel(PackJob pj, float* __restrict__ p, const float* __restrict__ g,
                                                        float* __restrict__ m, float* __restrict__ v, int64_t b5_off,
                                                        AdamConsts a) {
  const int W = pj.width;
  const int T = (W / 32) * (W / 32), nrv = (4 * W + 255) / 256;
  const int b = blockIdx.x;
  if (b < 3 * T) {
    adam_pack_tile<MODE>(pj, p, g, m, v, a, b / T, b % T);
  } else if (b < 3 * T + nrv) {
    const int64_t idx = (int64_t)(b - 3 * T) * 256 + threadIdx.x;
    if (idx >= 4 * (int64_t)W) return;
    const int vi = (int)(idx / W), r = (int)(idx % W);
    const float* src = vi < 3 ? pj.bl[vi] : pj.w5;
    float* dst = vi < 3 ? pj.bh + (size_t)vi * W : pj.w5p;
    dst[lane_major_pos(r, W)] = adam_update(p, g, m, v, (src - p) + r, a);
  } else {
    const int64_t idx = (int64_t)(b - 3 * T - nrv) * 256 + threadIdx.x;
    if (idx >= W) return;
    const int r = (int)idx;
    const int64_t w0 = (pj.W1 - p) + (int64_t)r * kInDim;
    float w[kInDim];
#pragma unroll
    for (int c = 0; c < kInDim; ++c) w[c] = adam_update(p, g, m, v, w0 + c, a);
    float* o = pj.w1p + lane_major_pos(r, W) * 12;
    o[0] = w[0];
    o[1] = w[1];
    o[2] = w[2];
    o[3] = adam_update(p, g, m, v, (pj.b1 - p) + r, a);
    for (int c = 0; c < 6; ++c) o[4 + c] = w[3 + c];
    o[10] = 0.f;
    o[11] = 0.f;
    if (r == 0) adam_update(p, g, m, v, b5_off, a);
  }
}

hipError_t launch_adam_pack(const PackJob& pj, float* params, const float* grad, float* m, float* v,
                            const AdamConsts& a, int64_t b5_off, hipStream_t s) {
  if (pj.in_dim != kInDim || (pj.mode != kFP32 && pj.mode != kBF16) || pj.width % 32) return hipErrorInvalidValue;
  const int W = pj.width;
  const unsigned grid = (unsigned)(3 * (W / 32) * (W / 32) + (4 * W + 255) / 256 + (W + 255) / 256);
  if (pj.mode == kFP32)
    hipLaunchKernelGGL(adam_pack_kernel<kFP32>, dim3(grid), dim3(256), 0, s, pj, params, grad, m, v, b5_off, a);
  else
    hipLaunchKernelGGL(adam_pack_kernel<kBF16>, dim3(grid), dim3(256), 0, s, pj, params, grad, m, v, b5_off, a);
  return hipGetLastError();
}

hipError_t pack_network(const PackJob& pj, hipStream_t s) {
  if (pj.in_dim != kInDim && pj.in_dim != kInDimSphere) return hipErrorInvalidValue;
  const unsigned bx = (unsigned)(((int64_t)pj.width * pj.width + 255) / 256);
  hipLaunchKernelGGL(pack_all_kernel, dim3(bx, 8), dim3(256), 0, s, pj);
  return hipGetLastError();
}

hipError_t pack_input_layer(const float* W1, const float* b1, float* w1p, int width, int in_dim, hipStream_t s) {
  if (in_dim != kInDim && in_dim != kInDimSphere) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pack_input_kernel, dim3((width + 255) / 256), dim3(256), 0, s, W1, b1, w1p, width, in_dim);
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
                                     int32_t* argmin) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K) return;
  const unsigned long long k = key[i];
  const uint32_t o = (uint32_t)(k >> 32);
  const uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
  if (dmin) dmin[i] = __uint_as_float(u);
  // every knot of a launch receives at least one key; an untouched slot would
  // decode to index 0 rather than an out-of-range point
  if (argmin) argmin[i] = (k == ~0ull) ? 0 : (int32_t)(uint32_t)(k & 0xffffffffu);
}

hipError_t launch_minkey_decode(const unsigned long long* minkey, int64_t K, float* dmin, int32_t* argmin,
                                hipStream_t s) {
  hipLaunchKernelGGL(minkey_decode_kernel, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, minkey, K, dmin,
                     argmin);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Launch
// ----------------------------------------------------------------------------
hipError_t launch_fused(const DevNet& net, const Job& job, bool pairs, bool want_grad, int num_cu, hipStream_t s) {
  if (net.in_dim == kInDimSphere) return launch_fused_sphere(net, job, pairs, want_grad, num_cu, s);
  if (net.width == 256) return launch_w<256, false>(net, job, pairs, want_grad, num_cu, s);
  return launch_w<512, false>(net, job, pairs, want_grad, num_cu, s);
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
int64_t wgrad_chunk_len(int64_t B, int n, int width, int num_cu) {
  const int ntile = (width / 128) * (width / 128);
  const int64_t nch = std::max<int64_t>(1, num_cu / (ntile * std::max(n, 1)));
  const int64_t per = (B + nch - 1) / nch;
  return std::max<int64_t>(kTileQ, (per + kTileQ - 1) / kTileQ * kTileQ);
}

int64_t wgrad_partial_floats(int64_t B, int width, int num_cu) {
  int64_t most = 0;
  for (int n = 1; n <= kWgMaxJobs; ++n) {
    const int64_t L = wgrad_chunk_len(B, n, width, num_cu);
    most = std::max(most, n * ((B + L - 1) / L));
  }
  return most * width * width;
}

struct WgFrag {
  f32x4 a[2], b[2];
};

// Blocks are dealt to the 8 XCDs round-robin (block b runs on XCD b % 8); the
// mapping below keeps the 4 output tiles of one (GEMM, chunk) on one XCD, so the
// chunk's rows of G and H come from HBM once and are shared through that L2.
// FP32 (the BF16 product is wgrad_gemm_lds_kernel below).
template <int MODE>
__global__ __launch_bounds__(256) void wgrad_gemm_kernel(WgradJobs jobs, int Wd, int64_t ldb, int64_t B, int nchunks,
                                                         int64_t chunk_len, float* __restrict__ partial) {
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
  const int64_t i0 = (int64_t)chunk * chunk_len;
  const int64_t i1 = i0 + chunk_len < B ? i0 + chunk_len : B;
  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[a][c][j] = 0.f;
  const int m = lane & 31, kh = lane >> 5;
  static_assert(MODE == kFP32, "FP32 operands");
  using E = float;
  constexpr int KS = 8;  // samples per step
  const E* G = static_cast<const E*>(jobs.G[job]);
  const E* H = static_cast<const E*>(jobs.H[job]);
  // The 16-byte block of S samples of feature f starts at element ((i / S) W + f) S:
  // lane (m, kh) of a step reads block i / S + kh of its row, and the 32 lanes of
  // a half read 32 consecutive features, 512 contiguous bytes.
  constexpr int S = 4;  // samples per 16-byte block (KS = 2 S)
  constexpr int U = 4;  // steps per prefetch group
  const E* ga[2] = {G + (int64_t)(kh * Wd + f0 + m) * S, G + (int64_t)(kh * Wd + f0 + 32 + m) * S};
  const E* hb[2] = {H + (int64_t)(kh * Wd + g0 + m) * S, H + (int64_t)(kh * Wd + g0 + 32 + m) * S};
  auto load = [&](WgFrag& f, int64_t i, int u) {
    const int64_t off = ((i + (int64_t)KS * u) / S) * Wd * S;  // first block of step u
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      f.a[t] = *reinterpret_cast<const f32x4*>(ga[t] + off);
      f.b[t] = *reinterpret_cast<const f32x4*>(hb[t] + off);
    }
  };
  auto mma = [&](const WgFrag& f) {
    // lane (m, kh) holds samples 4 kh + q of the step; MFMA q pairs samples q and 4 + q
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int ta = 0; ta < 2; ++ta)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb)
          acc[ta][tb] = __builtin_amdgcn_mfma_f32_32x32x2f32(f.a[ta][q], f.b[tb][q], acc[ta][tb], 0, 0, 0);
  };
  // Rows hold zeros from B up to the next multiple of 64 and chunks start at
  // multiples of 64, so whole groups are read.  Double-buffered: the loads of the
  // next group are in flight while this one runs on the matrix cores.
  static_assert(U * KS <= kTileQ, "a group must not run past the zero-padded tail");
  WgFrag cur[U], nxt[U];
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

// BF16 form of the same product, the operands staged in LDS: per 64-sample group
// the workgroup's unique operand bytes (128 rows of G and 128 of H, 32 KiB) go
// from HBM straight into LDS (global_load_lds_dwordx4, no registers), two groups
// ahead in a ring of three, and the 4 waves read their fragments from there, so
// each byte crosses the compute unit's L1 once instead of twice.  Group piece P
// (1 KiB) = ((u 2 + X) 2 + kh) 2 + hf: step u of the group, operand X (G, H),
// 8-sample block kh of the step, rows 64 hf .. 64 hf + 63 of the block's 128;
// lane l of the copying wave fetches row 64 hf + l.
constexpr int kWgRing = 3;                   // groups in LDS
constexpr int kWgGroup = 64;                 // samples per group
constexpr int kWgGroupBytes = 32 * 1024;     // 32 pieces of 1 KiB
__global__ __launch_bounds__(256) void wgrad_gemm_lds_kernel(WgradJobs jobs, int Wd, int64_t B, int nchunks,
                                                             int64_t chunk_len, float* __restrict__ partial) {
  constexpr int kXcd = 8;
  __shared__ __attribute__((aligned(16))) char ring[kWgRing * kWgGroupBytes];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tiles_n = Wd / 128, ntile = tiles_n * tiles_n;
  const int64_t groups = (int64_t)jobs.n * nchunks;  // (GEMM, chunk) pairs
  const int64_t b = blockIdx.x;
  const int64_t per_xcd = (groups + kXcd - 1) / kXcd;
  const int64_t local = b / kXcd, xcd = b % kXcd;
  const int64_t grp = xcd * per_xcd + local / ntile;
  if (grp >= groups) return;
  const int tile = (int)(local % ntile);
  const int job = (int)(grp / nchunks), chunk = (int)(grp % nchunks);
  const int fb = (tile / tiles_n) * 128, gb = (tile % tiles_n) * 128;  // the block's rows of G and of H
  const int64_t i0 = (int64_t)chunk * chunk_len;
  const int64_t i1 = i0 + chunk_len < B ? i0 + chunk_len : B;
  // rows hold zeros from B to the next multiple of 64 and chunks start at multiples of 64
  const int ngr = (int)((i1 - i0 + kWgGroup - 1) / kWgGroup);
  const __bf16* G = static_cast<const __bf16*>(jobs.G[job]);
  const __bf16* H = static_cast<const __bf16*>(jobs.H[job]);
  // this wave copies pieces 8 wave .. 8 wave + 7 of every group
  auto issue = [&](int g) {
    char* slot = ring + (g % kWgRing) * kWgGroupBytes;
    const int64_t ib0 = (i0 + (int64_t)g * kWgGroup) / 8;  // first 8-sample block of the group
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int P = wave * 8 + j;
      const int hf = P & 1, kh = (P >> 1) & 1, X = (P >> 2) & 1, u = P >> 3;
      const __bf16* src = (X ? H : G) + ((ib0 + 2 * u + kh) * Wd + (X ? gb : fb) + 64 * hf + lane) * 8;
      __builtin_amdgcn_global_load_lds(static_cast<const void*>(src),
                                       (__attribute__((address_space(3))) void*)(slot + P * 1024), 16, 0, 0);
    }
  };
  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[a][c][j] = 0.f;
  const int m = lane & 31, kh = lane >> 5;
  const int wa = wave >> 1, wb = wave & 1;  // this wave's 64 x 64 quarter: rows 64 wa of G, 64 wb of H
  if (ngr > 0) issue(0);
  if (ngr > 1) issue(1);
  for (int g = 0; g < ngr; ++g) {
    // group g has landed once at most the next group's 8 copies are outstanding
    if (g + 1 < ngr) __builtin_amdgcn_s_waitcnt(0x3F78);  // vmcnt(8)
    else __builtin_amdgcn_s_waitcnt(0x3F70);              // vmcnt(0)
    // every wave's copies of group g are in LDS, and every wave has finished
    // reading group g - 1, whose slot the copies of group g + 2 take
    __builtin_amdgcn_s_barrier();
    if (g + 2 < ngr) issue(g + 2);
    const char* slot = ring + (g % kWgRing) * kWgGroupBytes;
    // all 16 fragments of the group first, then its 16 products
    bf16x8 af[4][2], bf[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        af[u][t] = *reinterpret_cast<const bf16x8*>(slot + ((((u * 2 + 0) * 2 + kh) * 2 + wa) * 1024) + (32 * t + m) * 16);
        bf[u][t] = *reinterpret_cast<const bf16x8*>(slot + ((((u * 2 + 1) * 2 + kh) * 2 + wb) * 1024) + (32 * t + m) * 16);
      }
    __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the products
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int ta = 0; ta < 2; ++ta)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb)
          acc[ta][tb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[u][ta], bf[u][tb], acc[ta][tb], 0, 0, 0);
  }
  // C layout: lane (n = lane%32, half h) holds rows 8 (j/4) + 4 h + j%4 of column n
  float* out = partial + ((int64_t)job * nchunks + chunk) * Wd * Wd;
#pragma unroll
  for (int ta = 0; ta < 2; ++ta)
#pragma unroll
    for (int tb = 0; tb < 2; ++tb)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int row = fb + 64 * wa + 32 * ta + 8 * (j >> 2) + 4 * kh + (j & 3);
        const int col = gb + 64 * wb + 32 * tb + m;
        out[(int64_t)row * Wd + col] = acc[ta][tb][j];
      }
}

// Entry (r, f) = sum over workgroups w of part[(r W + f) nparts + w]: one wave
// per entry, lane l adding workgroups l, l + 64, ... in order, then the 64 lane
// sums in a fixed butterfly (the result does not depend on scheduling).
__device__ __forceinline__ void part_sum_entry(const PartSum& ps, int j, int lane) {
  const int W = ps.width;
  if (j >= kTrainSumRows * W) return;
  const int r = j / W, f = j % W;
  if (!ps.out.base[r] || f >= ps.out.n[r]) return;
  const float* p = ps.part + (int64_t)j * ps.nparts;
  float s = 0.f;
  int w = lane;
  for (; w + 192 < ps.nparts; w += 256) {  // four loads in flight, added in order
    const float a0 = p[w], a1 = p[w + 64], a2 = p[w + 128], a3 = p[w + 192];
    s += a0;
    s += a1;
    s += a2;
    s += a3;
  }
  for (; w < ps.nparts; w += 64) s += p[w];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  if (lane == 0) ps.out.base[r][(int64_t)f * ps.out.stride[r]] = s;
}

// out_j[e] = sum over chunks (in index order) of partial[j][chunk][e], 4 elements per
// thread, blocks [j bx, (j + 1) bx) for GEMM j; the blocks after those: the training
// kernel's per-workgroup sums (PartSum), one wave per entry.
__global__ void sum_chunks_kernel(const float* __restrict__ partial, int nchunks, int64_t n, WgradJobs jobs, int accum,
                                  PartSum ps, int bx) {
  const int b = blockIdx.x;
  if (b >= jobs.n * bx) {
    part_sum_entry(ps, (b - jobs.n * bx) * (blockDim.x / 64) + (threadIdx.x >> 6), threadIdx.x & 63);
    return;
  }
  const int job = b / bx;
  const int64_t t = ((int64_t)(b % bx) * blockDim.x + threadIdx.x) * 4;
  if (t >= n) return;
  const float* p = partial + (int64_t)job * nchunks * n + t;
  f32x4 s = {0.f, 0.f, 0.f, 0.f};
  constexpr int U = 8;  // loads in flight; the sums still run over the chunks in order
  int c = 0;
  for (; c + U <= nchunks; c += U) {
    f32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = *reinterpret_cast<const f32x4*>(p + (int64_t)(c + u) * n);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) s[e] += v[u][e];
  }
  for (; c < nchunks; ++c) {
    const f32x4 v = *reinterpret_cast<const f32x4*>(p + (int64_t)c * n);
#pragma unroll
    for (int e = 0; e < 4; ++e) s[e] += v[e];
  }
  float* o = jobs.out[job] + t;
#pragma unroll
  for (int u = 0; u < 4; ++u) o[u] = accum ? o[u] + s[u] : s[u];
}

hipError_t launch_wgrad_gemm(const WgradJobs& jobs, int width, int mode, int64_t ldb, int64_t B, float* partial,
                             int num_cu, hipStream_t s, bool accumulate, const PartSum* ps) {
  if (jobs.n < 1 || jobs.n > kWgMaxJobs || width % 128 || B <= 0) return hipErrorInvalidValue;
  if (ps && (ps->nparts < 1 || ps->width < 1)) return hipErrorInvalidValue;
  const int64_t chunk_len = wgrad_chunk_len(B, jobs.n, width, num_cu);
  const int nchunks = (int)((B + chunk_len - 1) / chunk_len);
  const int ntile = (width / 128) * (width / 128);
  const int64_t groups = (int64_t)jobs.n * nchunks;
  const int64_t per_xcd = (groups + 7) / 8;
  const unsigned grid = (unsigned)(8 * per_xcd * ntile);
  if (mode == kFP32)
    hipLaunchKernelGGL(wgrad_gemm_kernel<kFP32>, dim3(grid), dim3(256), 0, s, jobs, width, ldb, B, nchunks, chunk_len,
                       partial);
  else
    hipLaunchKernelGGL(wgrad_gemm_lds_kernel, dim3(grid), dim3(256), 0, s, jobs, width, B, nchunks, chunk_len, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)width * width;
  const unsigned bx = (unsigned)((n / 4 + 255) / 256);
  const unsigned bps = ps ? (unsigned)((kTrainSumRows * ps->width + 3) / 4) : 0u;  // 4 entries per block
  hipLaunchKernelGGL(sum_chunks_kernel, dim3((unsigned)jobs.n * bx + bps), dim3(256), 0, s, partial, nchunks, n, jobs,
                     accumulate ? 1 : 0, ps ? *ps : PartSum{}, (int)bx);
  return hipGetLastError();
}

// Row reductions over the batch in two fixed-order passes, A in the blocked
// feature-major layout of dump_tile.  Pass 1: grid (256-row group, chunk of
// kRrChunk samples, job); a thread owns one row and walks the chunk's 16-byte
// blocks in order (a workgroup reads 4 KB contiguous per block), V is read
// uniformly.  Pass 2 adds the chunks in index order.  The result does not depend
// on scheduling.
constexpr int kRrChunk = 512;
constexpr int kRrMaxC = 9;

int rr_chunks(int64_t B) { return (int)((B + kRrChunk - 1) / kRrChunk); }

// Several row reductions in one pass each (see RrJobs): job j's partial sums at
// partial + j * job_stride, [chunk][row][kRrMaxC + 1] (the last slot the row sum).
// A job without A reduces a single row of ones (out = sum V).
template <bool BF>
__global__ __launch_bounds__(256) void rr_multi_partial_kernel(RrJobs jobs, int64_t B, int64_t ldv,
                                                               float* __restrict__ partial, int64_t job_stride) {
  constexpr int S = BF ? 8 : 4;
  __shared__ float sv[kRrMaxC][kRrChunk];
  const RrJob& jb = jobs.job[blockIdx.z];
  const int rows = jb.A ? jb.rows : 1, C = jb.C;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.x * 256 >= rows) return;  // a whole workgroup past this job's rows
  const int64_t i0 = (int64_t)blockIdx.y * kRrChunk;
  const int64_t i1 = i0 + kRrChunk < B ? i0 + kRrChunk : B;
  for (int c = 0; c < C; ++c)
    for (int k = threadIdx.x; k < kRrChunk; k += 256) sv[c][k] = i0 + k < i1 ? jb.V[(int64_t)c * ldv + i0 + k] : 0.f;
  __syncthreads();
  if (r >= rows) return;
  float acc[kRrMaxC + 1];
#pragma unroll
  for (int c = 0; c <= kRrMaxC; ++c) acc[c] = 0.f;
  constexpr int NB = 8;
  typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 v8;
  for (int64_t i = i0; i < i1; i += NB * S) {
    float a[NB][S];
    // rounds stay inside the zero-padded tail (chunks start at multiples of 64)
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      if (!jb.A) {
#pragma unroll
        for (int u = 0; u < S; ++u) a[k][u] = 1.f;  // V is zero past B
        continue;
      }
      const int64_t blk = (((i + k * S) / S) * rows + r) * S;
      if constexpr (BF) {
        const v8 x = *reinterpret_cast<const v8*>(static_cast<const __bf16*>(jb.A) + blk);
#pragma unroll
        for (int u = 0; u < S; ++u) a[k][u] = (float)x[u];
      } else {
        const f32x4 x = *reinterpret_cast<const f32x4*>(static_cast<const float*>(jb.A) + blk);
#pragma unroll
        for (int u = 0; u < S; ++u) a[k][u] = x[u];
      }
    }
#pragma unroll
    for (int k = 0; k < NB; ++k)
#pragma unroll
      for (int u = 0; u < S; ++u) acc[kRrMaxC] += a[k][u];
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
  float* out = partial + blockIdx.z * job_stride + ((int64_t)blockIdx.y * rows + r) * (kRrMaxC + 1);
#pragma unroll
  for (int c = 0; c <= kRrMaxC; ++c) out[c] = acc[c];
}

__global__ void rr_multi_sum_kernel(RrJobs jobs, const float* __restrict__ partial, int64_t job_stride, int nchunks) {
  const RrJob& jb = jobs.job[blockIdx.y];
  const int rows = jb.A ? jb.rows : 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = (int)(t / (kRrMaxC + 1)), c = (int)(t % (kRrMaxC + 1));
  if (r >= rows || (c >= jb.C && c != kRrMaxC)) return;
  const float* p = partial + blockIdx.y * job_stride;
  float s = 0.f;
#pragma unroll 8
  for (int k = 0; k < nchunks; ++k) s += p[((int64_t)k * rows + r) * (kRrMaxC + 1) + c];
  float* o = c == kRrMaxC ? jb.bias + r : (jb.out ? jb.out + (int64_t)r * jb.C + c : nullptr);
  if (c == kRrMaxC && !jb.bias) return;
  if (o) *o = jb.accumulate ? *o + s : s;
}

int64_t rr_multi_job_floats(int rows, int64_t B) { return (int64_t)rr_chunks(B) * rows * (kRrMaxC + 1); }

hipError_t launch_row_reduce_multi(const RrJobs& jobs, bool a_is_bf16, int64_t B, int64_t ldv, float* partial,
                                   hipStream_t s) {
  if (jobs.n < 1 || jobs.n > kRrMaxJobs || B <= 0) return hipErrorInvalidValue;
  int rmax = 1;
  for (int j = 0; j < jobs.n; ++j) {
    const RrJob& jb = jobs.job[j];
    if (jb.C > kRrMaxC || (jb.C > 0 && !jb.V) || (jb.A && jb.rows <= 0) || (!jb.A && jb.C < 1)) return hipErrorInvalidValue;
    if (jb.A && jb.rows > rmax) rmax = jb.rows;
  }
  const int nch = rr_chunks(B);
  const int64_t stride = rr_multi_job_floats(rmax, B);
  const dim3 grid((unsigned)((rmax + 255) / 256), (unsigned)nch, (unsigned)jobs.n);
  if (a_is_bf16)
    hipLaunchKernelGGL(rr_multi_partial_kernel<true>, grid, dim3(256), 0, s, jobs, B, ldv, partial, stride);
  else
    hipLaunchKernelGGL(rr_multi_partial_kernel<false>, grid, dim3(256), 0, s, jobs, B, ldv, partial, stride);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)rmax * (kRrMaxC + 1);
  hipLaunchKernelGGL(rr_multi_sum_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)jobs.n), dim3(256), 0, s, jobs,
                     partial, stride, nch);
  return hipGetLastError();
}


}  // namespace gcdf
