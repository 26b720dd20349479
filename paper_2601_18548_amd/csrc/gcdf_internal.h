// Internal interface between the C-ABI host code and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gcdf {

constexpr int kInDim = 9;
constexpr int kTileQ = 64;   // queries per tile (two 32-wide MFMA column blocks)
constexpr int kWaves = 4;    // waves per workgroup, one per SIMD
constexpr int kThreads = 64 * kWaves;

enum Mode : int { kFP32 = 0, kBF16 = 1, kBF16X2 = 2 };

// Device-resident network in kernel layout.
// Row-indexed arrays are in the kernel's lane-major row order (pack_input_layer,
// pack_row_vectors).
struct DevNet {
  int width;
  int mode;
  const float* w1p;   // [width][12]: W1[r][0..2], b1[r], W1[r][3..8], 0, 0
  const float* bh;    // [depth-1][width]: b2, b3, b4
  const float* w5;    // [width]
  float b5;
  const void* fwd[3]; // W2, W3, W4 as matrix-core A fragments (see pack_matrix)
  const void* bwd[3]; // W2^T, W3^T, W4^T, same layout
};

// What one fused launch computes.
struct Job {
  const float* knots;        // [K][9]
  const float* points;       // [Np][3]
  int64_t K, Np;
  // pair list (pairs mode): pair i = (knots[kidx[i]], points[pidx[i]]); NULL index arrays
  // mean pair i = (knots[i], points[i]).
  const int64_t* kidx;
  const int64_t* pidx;
  int64_t npairs;
  float* d;                  // dense: [K][Np]; pairs: [npairs]      (nullable)
  float* J;                  // dense: [K][Np][9]; pairs: [npairs][9] (nullable)
  unsigned long long* minkey;// dense only: [K] ordered (distance, index) keys (nullable)
};

// Packed fragment bytes for one width x width matrix.
size_t packed_matrix_bytes(int width, int mode);

// Convert a row-major float32 width x width matrix (device) into the kernel's
// A-fragment layout (device), transposing first if `transpose`.
hipError_t pack_matrix(const float* src, void* dst, int width, int mode, bool transpose, hipStream_t s);

// Build w1p (device) from W1 [width][9] and b1 [width] (device).
hipError_t pack_input_layer(const float* W1, const float* b1, float* w1p, int width, hipStream_t s);

// Reorder nvec consecutive row vectors of length width into lane-major row order.
hipError_t pack_row_vectors(const float* src, float* dst, int width, int nvec, hipStream_t s);

// Launch the fused query kernel (dense all-pairs if !pairs, else the pair list).
hipError_t launch_fused(const DevNet& net, const Job& job, bool pairs, bool want_grad, int num_cu, hipStream_t s);

// minkey[i] = all ones, for i < K (fill kernel; graph-capture safe).
hipError_t launch_minkey_init(unsigned long long* minkey, int64_t K, hipStream_t s);

// Decode keys into dmin / argmin; if kidx/pidx given, also write the argmin
// pair list (kidx[i] = i, pidx[i] = argmin[i]).
hipError_t launch_minkey_decode(const unsigned long long* minkey, int64_t K, float* dmin, int32_t* argmin,
                                int64_t* kidx, int64_t* pidx, hipStream_t s);

}  // namespace gcdf
