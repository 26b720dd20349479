// What the solver needs around the query: obstacle partitions and the sparsity
// pattern of the stacked GCDF constraint Jacobian (Sec. IV-A of the paper:
// partitions I_{M,i} of the obstacle points by reference base position, the
// knot-major constraint vector c_gcdf, and the projections P_i of each knot's
// dense gradient rows into the (sum m_i) x 2Nn Jacobian), and the single-step
// projection onto the zero set with the weighted eikonal norm (Theorem 1).
//
// Membership: point j is in partition i when its planar distance to reference
// base position i is within the radius, decided in float32 as
// rn(rn(dx*dx) + rn(dy*dy)) <= rn(r*r) with no fused multiply-add, so the count
// and fill passes (and any reimplementation) take the same decision.  Sphere
// obstacles (x, y, z, s) of the primitive-aware network are in range when they
// reach into the disc: the same test with r replaced by rn(r + s).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gcdf_internal.h"

namespace gcdf {
namespace {

constexpr int kPartThreads = 256;
constexpr int kPartPerThread = 16;  // count pass: points per thread per workgroup
constexpr int kFillPerThread = 4;   // fill pass: points per thread per round

__device__ __forceinline__ float squared(float r) {
#pragma clang fp contract(off)
  return r * r;
}

// r2 = rn(radius * radius), used as is for points
template <bool SPH>
__device__ __forceinline__ bool in_range(const float* __restrict__ points, int64_t j, float rx, float ry, float radius,
                                         float r2) {
#pragma clang fp contract(off)
  const float* p = points + (SPH ? 4 : 3) * j;
  const float dx = p[0] - rx;
  const float dy = p[1] - ry;
  const float lim = SPH ? squared(radius + p[3]) : r2;
  return dx * dx + dy * dy <= lim;
}

__global__ void zero_i64_kernel(int64_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// grid (chunks of kPartThreads * kPartPerThread points, N): counts[i] += members in the chunk.
template <bool SPH>
__global__ __launch_bounds__(kPartThreads) void partition_count_kernel(const float* __restrict__ ref, int64_t ref_stride,
                                                                       const float* __restrict__ points, int64_t M,
                                                                       float radius, int64_t* __restrict__ counts) {
  __shared__ int wsum[kPartThreads / 64];
  const int64_t i = blockIdx.y;
  const float rx = ref[i * ref_stride], ry = ref[i * ref_stride + 1], r2 = squared(radius);
  const int64_t j0 = (int64_t)blockIdx.x * kPartThreads * kPartPerThread + threadIdx.x;
  int c = 0;
#pragma unroll 4
  for (int u = 0; u < kPartPerThread; ++u) {
    const int64_t j = j0 + (int64_t)u * kPartThreads;
    if (j < M && in_range<SPH>(points, j, rx, ry, radius, r2)) ++c;
  }
  for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kPartThreads / 64; ++w) t += wsum[w];
    if (t) atomicAdd(reinterpret_cast<unsigned long long*>(counts + i), (unsigned long long)t);
  }
}

// One workgroup: offsets[0] = 0, offsets[i+1] = counts[0] + ... + counts[i], in place
// (counts live at offsets + 1).
__global__ __launch_bounds__(kPartThreads) void partition_scan_kernel(int64_t* __restrict__ offsets, int64_t N) {
  __shared__ int64_t buf[kPartThreads];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) {
    carry = 0;
    offsets[0] = 0;
  }
  __syncthreads();
  for (int64_t b = 0; b < N; b += kPartThreads) {
    const int64_t i = b + threadIdx.x;
    int64_t v = i < N ? offsets[i + 1] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kPartThreads; o <<= 1) {  // inclusive Hillis-Steele scan
      const int64_t add = threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
      __syncthreads();
      buf[threadIdx.x] += add;
      __syncthreads();
    }
    const int64_t base = carry;
    if (i < N) offsets[i + 1] = base + buf[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == kPartThreads - 1) carry = base + buf[kPartThreads - 1];
    __syncthreads();
  }
}

// One workgroup per partition, rounds of kPartThreads * kFillPerThread points in
// ascending order; inside a round point j = j0 + u * 256 + wave * 64 + lane, ranked
// by (u, wave, lane) with ballots, so the indices come out ascending.
template <bool SPH>
__global__ __launch_bounds__(kPartThreads) void partition_fill_kernel(const float* __restrict__ ref, int64_t ref_stride,
                                                                      const float* __restrict__ points, int64_t M,
                                                                      float radius, const int64_t* __restrict__ offsets,
                                                                      int32_t* __restrict__ idx, int64_t capacity) {
  constexpr int kW = kPartThreads / 64;
  __shared__ int wcnt[2][kFillPerThread][kW];
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float rx = ref[i * ref_stride], ry = ref[i * ref_stride + 1], r2 = squared(radius);
  const int64_t base = offsets[i];
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  int64_t run = 0;
  int buf = 0;
  for (int64_t j0 = 0; j0 < M; j0 += kPartThreads * kFillPerThread, buf ^= 1) {
    bool in[kFillPerThread];
    int rank[kFillPerThread];
#pragma unroll
    for (int u = 0; u < kFillPerThread; ++u) {
      const int64_t j = j0 + u * kPartThreads + threadIdx.x;
      in[u] = j < M && in_range<SPH>(points, j, rx, ry, radius, r2);
      const uint64_t m = __ballot(in[u]);
      rank[u] = __popcll(m & below);
      if (lane == 0) wcnt[buf][u][wave] = __popcll(m);
    }
    __syncthreads();
    int total = 0;
#pragma unroll
    for (int u = 0; u < kFillPerThread; ++u)
#pragma unroll
      for (int w = 0; w < kW; ++w) total += wcnt[buf][u][w];
#pragma unroll
    for (int u = 0; u < kFillPerThread; ++u) {
      int off = 0;  // members of this round ranked before (u, wave)
#pragma unroll
      for (int uu = 0; uu < kFillPerThread; ++uu)
#pragma unroll
        for (int w = 0; w < kW; ++w)
          if (uu < u || (uu == u && w < wave)) off += wcnt[buf][uu][w];
      if (in[u]) {
        const int64_t pos = base + run + off + rank[u];
        if (pos < capacity) idx[pos] = (int32_t)(j0 + u * kPartThreads + threadIdx.x);
      }
    }
    run += total;
    // wcnt[buf] is rewritten two rounds later, after the next round's barrier
  }
}

// One workgroup: tile_off[0] = 0, tile_off[i+1] = tile_off[i] + ceil(m_i / 64) with
// m_i = offsets[i+1] - offsets[i] (the gathered tiles of the CSR query).  Thread t
// takes the contiguous knots [t L, (t + 1) L), L = ceil(N / 1024): it sums their
// tile counts, the workgroup scans the 1024 sums, and the thread writes its
// knots' offsets from its base (two passes over the offsets, two barriers per
// scan step, however large N is).
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void csr_tile_offsets_kernel(const int64_t* __restrict__ offsets, int64_t N,
                                                                        int64_t* __restrict__ tile_off) {
  __shared__ int64_t buf[kScanThreads];
  const int t = threadIdx.x;
  const int64_t L = (N + kScanThreads - 1) / kScanThreads;
  const int64_t i0 = t * L < N ? t * L : N;
  const int64_t i1 = i0 + L < N ? i0 + L : N;
  auto tiles = [&](int64_t i) {
    const int64_t m = offsets[i + 1] - offsets[i];
    return m > 0 ? (m + kTileQ - 1) / kTileQ : (int64_t)0;
  };
  int64_t sum = 0;
#pragma unroll 8
  for (int64_t i = i0; i < i1; ++i) sum += tiles(i);
  buf[t] = sum;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {  // inclusive scan of the segment sums
    const int64_t add = t >= o ? buf[t - o] : 0;
    __syncthreads();
    buf[t] += add;
    __syncthreads();
  }
  int64_t run = buf[t] - sum;  // tiles of the knots before this segment
  if (t == 0) tile_off[0] = 0;
#pragma unroll 8
  for (int64_t i = i0; i < i1; ++i) {
    run += tiles(i);
    tile_off[i + 1] = run;
  }
}

// Thread per row r in [0, total]: row_ptr and the n_conf column indices of row r.
__global__ void jacobian_pattern_kernel(const int64_t* __restrict__ offsets, int64_t N, int64_t total,
                                        int32_t state_dim, int64_t col0, int64_t* __restrict__ row_ptr,
                                        int32_t* __restrict__ cols) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r > total) return;
  row_ptr[r] = (int64_t)kInDim * r;
  if (r == total) return;
  int64_t lo = 0, hi = N - 1;  // the last i with offsets[i] <= r
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (offsets[mid] <= r) lo = mid; else hi = mid - 1;
  }
  const int32_t c0 = (int32_t)(col0 + (int64_t)state_dim * lo);
#pragma unroll
  for (int c = 0; c < kInDim; ++c) cols[kInDim * r + c] = c0 + c;
}

// Knot of stacked row r: dense rows are knot-major with Np points per knot; CSR
// rows take the last i < N with offsets[i] <= r.
__device__ __forceinline__ int64_t row_knot(const int64_t* __restrict__ offsets, int64_t N, int64_t Np, int64_t r) {
  if (!offsets) return r / Np;
  int64_t lo = 0, hi = N - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (offsets[mid] <= r) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Theorem 1: q_z = q - f M^{-1} J and |J|_{M^{-1}} per row.  A block stages its
// 256 rows of J (9 floats each) through LDS so that the global loads and the q_z
// stores are contiguous dword accesses; the kernel is bound by HBM (80 B per row).
__global__ __launch_bounds__(256) void project_kernel(const float* __restrict__ knots, int64_t N, int64_t Np,
                                                      const int64_t* __restrict__ offsets, int64_t rows,
                                                      const float* __restrict__ f, const float* __restrict__ J,
                                                      Minv9 minv, float* __restrict__ qz, float* __restrict__ eik) {
  constexpr int R = 256;
  __shared__ float tile[R * kInDim];
  const int64_t r0 = (int64_t)blockIdx.x * R;
  const int n = rows - r0 < R ? (int)(rows - r0) : R;
  const int lim = n * kInDim;
  const float* Jb = J + r0 * kInDim;
#pragma unroll
  for (int u = 0; u < kInDim; ++u) {
    const int t = u * R + threadIdx.x;
    tile[t] = t < lim ? Jb[t] : 0.f;
  }
  __syncthreads();
  float out[kInDim];
  const int me = threadIdx.x;
  if (me < n) {
    const int64_t r = r0 + me;
    const float* kn = knots + row_knot(offsets, N, Np, r) * kInDim;
    const float fr = f[r];
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < kInDim; ++c) {
      const float j = tile[me * kInDim + c];
      const float t = j * minv.v[c];
      out[c] = kn[c] - fr * t;
      s += t * j;
    }
    if (eik) eik[r] = sqrtf(s);
  }
  if (!qz) return;
  __syncthreads();
  if (me < n) {
#pragma unroll
    for (int c = 0; c < kInDim; ++c) tile[me * kInDim + c] = out[c];
  }
  __syncthreads();
  float* Qb = qz + r0 * kInDim;
#pragma unroll
  for (int u = 0; u < kInDim; ++u) {
    const int t = u * R + threadIdx.x;
    if (t < lim) Qb[t] = tile[t];
  }
}

}  // namespace

hipError_t launch_project(const float* knots, int64_t N, int64_t Np, const int64_t* offsets, int64_t rows,
                          const float* f, const float* J, const Minv9& minv, float* qz, float* eik, hipStream_t s) {
  hipLaunchKernelGGL(project_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, knots, N, Np, offsets,
                     rows, f, J, minv, qz, eik);
  return hipGetLastError();
}

hipError_t launch_partition_count(const float* ref, int64_t N, int64_t ref_stride, const float* points, int64_t M,
                                  bool spheres, float radius, int64_t* offsets, hipStream_t s) {
  hipLaunchKernelGGL(zero_i64_kernel, dim3((unsigned)((N + 1 + 255) / 256)), dim3(256), 0, s, offsets, N + 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t per = (int64_t)kPartThreads * kPartPerThread;
  const int64_t chunks = (M + per - 1) / per;
  for (int64_t n0 = 0; n0 < N; n0 += 65535) {  // grid.y limit
    const int64_t n = N - n0 < 65535 ? N - n0 : 65535;
    if (spheres)
      hipLaunchKernelGGL(partition_count_kernel<true>, dim3((unsigned)chunks, (unsigned)n), dim3(kPartThreads), 0, s,
                         ref + n0 * ref_stride, ref_stride, points, M, radius, offsets + 1 + n0);
    else
      hipLaunchKernelGGL(partition_count_kernel<false>, dim3((unsigned)chunks, (unsigned)n), dim3(kPartThreads), 0, s,
                         ref + n0 * ref_stride, ref_stride, points, M, radius, offsets + 1 + n0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(partition_scan_kernel, dim3(1), dim3(kPartThreads), 0, s, offsets, N);
  return hipGetLastError();
}

hipError_t launch_partition_fill(const float* ref, int64_t N, int64_t ref_stride, const float* points, int64_t M,
                                 bool spheres, float radius, const int64_t* offsets, int32_t* idx, int64_t capacity,
                                 hipStream_t s) {
  if (spheres)
    hipLaunchKernelGGL(partition_fill_kernel<true>, dim3((unsigned)N), dim3(kPartThreads), 0, s, ref, ref_stride,
                       points, M, radius, offsets, idx, capacity);
  else
    hipLaunchKernelGGL(partition_fill_kernel<false>, dim3((unsigned)N), dim3(kPartThreads), 0, s, ref, ref_stride,
                       points, M, radius, offsets, idx, capacity);
  return hipGetLastError();
}

hipError_t launch_csr_tile_offsets(const int64_t* offsets, int64_t N, int64_t* tile_off, hipStream_t s) {
  hipLaunchKernelGGL(csr_tile_offsets_kernel, dim3(1), dim3(kScanThreads), 0, s, offsets, N, tile_off);
  return hipGetLastError();
}

hipError_t launch_jacobian_pattern(const int64_t* offsets, int64_t N, int64_t total, int32_t state_dim, int64_t col0,
                                   int64_t* row_ptr, int32_t* cols, hipStream_t s) {
  const int64_t rows = total + 1;
  hipLaunchKernelGGL(jacobian_pattern_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, offsets, N,
                     total, state_dim, col0, row_ptr, cols);
  return hipGetLastError();
}

}  // namespace gcdf
