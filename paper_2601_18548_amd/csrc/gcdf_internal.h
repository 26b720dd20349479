// Internal interface between the C-ABI host code and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gcdf {

constexpr int kInDim = 9;         // configuration coordinates per knot (x, y, yaw, a1..a6)
constexpr int kInDimSphere = 10;  // network inputs for sphere obstacles: [p', r, a]
constexpr int kTileQ = 64;   // queries per tile (two 32-wide MFMA column blocks)
constexpr int kWaves = 4;    // row groups of the packed weights; waves per workgroup in FP32 (BF16: 8)
constexpr int kThreads = 64 * kWaves;

// kBF16X2F16: forward layers as kBF16X2, reverse sweep as single-pass FP16
// products (transposed weights packed in FP16).
enum Mode : int { kFP32 = 0, kBF16 = 1, kBF16X2 = 2, kBF16X2F16 = 3 };

// Device-resident network in kernel layout.
// Row-indexed arrays are in the kernel's lane-major row order (pack_input_layer,
// pack_row_vectors).
struct DevNet {
  int width;
  int mode;
  int in_dim;         // 9: point obstacles [Np][3]; 10: spheres [Np][4], input [p', r, a]
  const float* w1p;   // [width][12]: W1[r][p'x, p'y, p'z], b1[r], W1[r][a1..a6], W1[r][radius] (0 when in_dim 9), 0
  const float* bh;    // [depth-1][width]: b2, b3, b4
  const float* w5;    // [width]
  const float* b5p;   // device pointer to the output bias
  const void* fwd[3]; // W2, W3, W4 as matrix-core A fragments (see pack_matrix)
  const void* bwd[3]; // W2^T, W3^T, W4^T, same layout
  // kBF16X2F16: set to 1 (host-visible memory) by any query whose d is finite but
  // whose J is not, i.e. the FP16 reverse sweep overflowed (nullable)
  uint32_t* overflow;
};

// What one fused launch computes.
struct Job {
  const float* knots;        // [K][9]
  const float* points;       // [Np][3]
  int64_t K, Np;
  // pair list (pairs mode): pair i = (knots[kidx[i]], points[pidx[i]]); NULL index arrays
  // mean pair i = (knots[i], points[i]).  pidx32, when set, replaces pidx (32-bit point
  // indices, e.g. a per-knot argmin array: pair i = (knots[i], points[argmin[i]])).
  const int64_t* kidx;
  const int64_t* pidx;
  const int32_t* pidx32;
  int64_t npairs;
  // CSR pairs (pairs mode, when csr_off is set): pair r belongs to the knot i with
  // csr_off[i] <= r < csr_off[i+1] (i < csr_n) and to point csr_idx[r]; a point index
  // outside [0, Np) yields NaN outputs for that pair.
  const int64_t* csr_off;
  int64_t csr_n;
  const int32_t* csr_idx;
  // Gathered knot tiles (dense mode, when tile_off is set): knot i owns rows
  // row_off[i] .. row_off[i+1]-1, row r pairing it with point pgather[r]; its rows
  // form tile_off[i+1] - tile_off[i] tiles of up to 64 (tile_off[0] = 0), so no tile
  // mixes knots; d and J are indexed by row; ntiles_bound >= tile_off[K] sizes the grid.
  const int64_t* tile_off;
  const int64_t* row_off;
  const int32_t* pgather;
  int64_t ntiles_bound;
  float* d;                  // dense: [K][Np]; pairs: [npairs]      (nullable)
  float* J;                  // dense: [K][Np][9]; pairs: [npairs][9] (nullable)
  unsigned long long* minkey;// dense only: [K] ordered (distance, index) keys (nullable)
  // training (pairs mode): the reverse sweep is seeded with seed[i] = dL/dd_i instead
  // of 1, and the tile's layer inputs h_{l+1} (dumpH[l]) and back-propagated
  // gradients dL/dz_{l+1} (dumpG[l]), l = 0..3, are written as [W x ldb] arrays in
  // the blocked feature-major layout (element (f, i) at ((i / S) W + f) S + i % S,
  // S = 16 bytes of samples); dumpV[c][i] = network input c (FP32), row stride ldb
  // (a multiple of 64).
  const float* seed;
  void* dumpH;
  void* dumpG;
  float* dumpV;
  int64_t ldb;
  // fused MSE loss (training, seed NULL, target set): each tile finishes d before its
  // reverse sweep and seeds it with dL/dd_i = mse_scale (d_i - target_i), written to
  // seed_out[i], and writes sq_out[i] = inv_b (d_i - target_i)^2 (i < npairs; both
  // nullable).
  const float* target;
  float* seed_out;
  float* sq_out;
  float mse_scale, inv_b;
  // training, pure BF16: per-workgroup sums [kTrainSumRows][W][grid] (rows:
  // sum_i g_l for l = 1..4; sum_i seed_i h4_i; sum_i g1_i v_c(i) for the nine
  // inputs c; sum_i seed_i; the fused loss), so that h4 and g1 are not written
  float* bias_part;
};
constexpr int kTrainSumRows = 16;

// Packed fragment bytes for one width x width matrix.
size_t packed_matrix_bytes(int width, int mode);

// Convert a row-major float32 width x width matrix (device) into the kernel's
// A-fragment layout (device), transposing first if `transpose`.
hipError_t pack_matrix(const float* src, void* dst, int width, int mode, bool transpose, hipStream_t s);

// Build w1p (device) from W1 [width][in_dim] and b1 [width] (device).
hipError_t pack_input_layer(const float* W1, const float* b1, float* w1p, int width, int in_dim, hipStream_t s);

// Reorder nvec consecutive row vectors of length width into lane-major row order.
hipError_t pack_row_vectors(const float* src, float* dst, int width, int nvec, hipStream_t s);

// Every packed array of a network (pack_matrix of W2..W4 and their transposes,
// pack_row_vectors of b2, b3, b4 and w_out, pack_input_layer) in one launch.
struct PackJob {
  int width, mode, in_dim;
  const float* W1;     // [width][in_dim]
  const float* b1;     // [width]
  const float* Wl[3];  // W2, W3, W4 (row-major, width x width)
  const float* bl[3];  // b2, b3, b4
  const float* w5;     // w_out [width]
  void* fwd[3];        // packed W2..W4
  void* bwd[3];        // packed W2^T..W4^T
  float* bh;           // [3][width] lane-major
  float* w5p;          // [width] lane-major
  float* w1p;          // [width][12]
};
hipError_t pack_network(const PackJob& pj, hipStream_t s);

// Obstacle partitions: offsets[i+1] - offsets[i] = number of points within `radius`
// (planar distance) of reference base position i (ref + i * ref_stride), offsets[0] = 0.
// spheres: points hold (x, y, z, s) and the limit is radius + s.
hipError_t launch_partition_count(const float* ref, int64_t N, int64_t ref_stride, const float* points, int64_t M,
                                  bool spheres, float radius, int64_t* offsets, hipStream_t s);
// idx[offsets[i] + k] = k-th point (ascending) of partition i; entries at positions >=
// capacity are not written.
hipError_t launch_partition_fill(const float* ref, int64_t N, int64_t ref_stride, const float* points, int64_t M,
                                 bool spheres, float radius, const int64_t* offsets, int32_t* idx, int64_t capacity,
                                 hipStream_t s);
// tile_off[0] = 0, tile_off[i+1] = tile_off[i] + ceil((offsets[i+1] - offsets[i]) / 64).
hipError_t launch_csr_tile_offsets(const int64_t* offsets, int64_t N, int64_t* tile_off, hipStream_t s);
// Sparsity pattern of the stacked constraint Jacobian: row_ptr[r] = n_conf * r (r <= total),
// cols[n_conf * r + c] = col0 + state_dim * knot(r) + c.
hipError_t launch_jacobian_pattern(const int64_t* offsets, int64_t N, int64_t total, int32_t state_dim, int64_t col0,
                                   int64_t* row_ptr, int32_t* cols, hipStream_t s);

// Single-step projection (Theorem 1) over stacked rows r < rows: the knot of row r
// is r / Np (offsets == NULL, dense knot-major rows) or the CSR row's knot;
// qz[r] = knot - f[r] * minv .* J[r] and eik[r] = sqrt(sum_c minv_c J[r][c]^2)
// (either output may be NULL).
struct Minv9 {
  float v[kInDim];
};
hipError_t launch_project(const float* knots, int64_t N, int64_t Np, const int64_t* offsets, int64_t rows,
                          const float* f, const float* J, const Minv9& minv, float* qz, float* eik, hipStream_t s);

// Launch the fused query kernel (dense all-pairs if !pairs, else the pair list).
hipError_t launch_fused(const DevNet& net, const Job& job, bool pairs, bool want_grad, int num_cu, hipStream_t s);
// The same for a sphere network (net.in_dim == 10; points hold (x, y, z, r)); no training.
hipError_t launch_fused_sphere(const DevNet& net, const Job& job, bool pairs, bool want_grad, int num_cu,
                               hipStream_t s);

// minkey[i] = all ones, for i < K (fill kernel; graph-capture safe).
hipError_t launch_minkey_init(unsigned long long* minkey, int64_t K, hipStream_t s);

// Decode keys into dmin / argmin.
hipError_t launch_minkey_decode(const unsigned long long* minkey, int64_t K, float* dmin, int32_t* argmin,
                                hipStream_t s);

// ----------------------------------------------------------------------------
// Serving: a persistent kernel claims tiles of published requests.
// ----------------------------------------------------------------------------
constexpr int kMaxSlots = 256;

// One request as the device sees it (written by the host before publication).
// The host rewrites a slot's descriptor only after its previous request has
// completed, seqlock-style: seq = kDescWriting, the fields, then seq = the new
// request's number.  A reader that finds seq != the request it wants (before or
// after reading a field) knows that request has completed.
constexpr uint64_t kDescWriting = ~0ull;
struct ServeDesc {
  uint64_t seq;         // request sequence number; slot = seq % slots
  const float* knots;
  const float* points;
  int64_t K, Np, nblk, ntiles;
  uint64_t done_target; // value of the slot's cumulative done counter when this request is complete
  float* d;
  float* J;
  unsigned long long* minkey;  // [K], all ones on entry; restored to all ones on completion
  float* dmin;
  int32_t* argmin;
  float* Jmin;                 // [K][9] J at the argmin pairs (NULL: not wanted; needs dmin)
  int32_t want_grad;
  int32_t pad;
};

// Control block in pinned, coherent host memory (host <-> device).
struct ServeCtl {
  uint64_t published;              // number of requests published (host writes, release)
  uint32_t stop;                   // host: exit when no work is claimable
  uint32_t slots;                  // number of request slots in use (<= kMaxSlots)
  uint32_t fault;                  // device: a protocol invariant failed (the host stops serving)
  uint32_t pad;
  uint64_t complete[kMaxSlots];    // seq + 1 of the last request completed in each slot (device writes)
  ServeDesc desc[kMaxSlots];
};

// Claim / completion counters in device memory.
struct ServeDev {
  unsigned long long claim[kMaxSlots];  // (seq << 32) | tiles claimed of request seq
  unsigned long long done[kMaxSlots];   // tiles finished in the slot, cumulative over its requests
  uint32_t drain;                       // epoch of the launch that is draining (0: none yet)
};

// Launch the persistent serving kernel; it processes published requests from
// sequence number first_seq on and returns once `stop` is set or a workgroup has
// found no work for idle_ticks of the 100 MHz real-time counter.  Exit is
// collective: that workgroup writes `epoch` (non-zero, distinct per launch) into
// dev->drain, and every workgroup stops claiming at its next claim, reports the
// tiles it ran and returns, so a launch never lingers with part of its grid.
// Tiles left unclaimed stay in the claim words for the next launch.
hipError_t launch_serve(const DevNet& net, ServeCtl* ctl, ServeDev* dev, uint64_t first_seq, uint64_t idle_ticks,
                        uint32_t epoch, int num_cu, hipStream_t s);

hipError_t launch_fill_ones(unsigned long long* p, int64_t n, hipStream_t s);

// ----------------------------------------------------------------------------
// Training: weight gradients from the dumped H / G (element type = bf16 for the
// BF16 modes, float for FP32).
// ----------------------------------------------------------------------------
// Up to kWgMaxJobs products in one launch: out_j[f][g] = sum_{i < B} G_j[f][i] H_j[g][i]
// for f, g < width (a multiple of 128), via split-K partial sums in `partial`
// (wgrad_partial_floats(B, width, num_cu) floats) reduced in a fixed order.  Rows
// of G and H have stride ldb and hold zeros from B up to the next multiple of 64.
// The batch is cut into as few chunks as keep one workgroup per (product, chunk,
// 128 x 128 output tile) within num_cu, so every workgroup runs in one round.
constexpr int kWgMaxJobs = 3;
struct WgradJobs {
  const void* G[kWgMaxJobs];
  const void* H[kWgMaxJobs];
  float* out[kWgMaxJobs];
  int n;
};
// The training kernel's per-workgroup sums (Job::bias_part, nparts workgroups)
// added in a fixed order: entry f < n[r] of row r goes to base[r][f * stride[r]]
// (rows with a NULL base are dropped).
struct PartOut {
  float* base[kTrainSumRows];
  int stride[kTrainSumRows];
  int n[kTrainSumRows];
};
struct PartSum {
  const float* part;
  int nparts, width;
  PartOut out;
};
// ps (optional): those sums too, in the launch that adds the chunks.
hipError_t launch_wgrad_gemm(const WgradJobs& jobs, int width, int mode, int64_t ldb, int64_t B, float* partial,
                             int num_cu, hipStream_t s, bool accumulate = false, const PartSum* ps = nullptr);
// samples per chunk (a multiple of 64) for n products, and the floats of `partial`
// any launch of up to kWgMaxJobs products over at most B samples needs
int64_t wgrad_chunk_len(int64_t B, int n, int width, int num_cu);
int64_t wgrad_partial_floats(int64_t B, int width, int num_cu);
// Row reductions over a batch: for each row r < rows, out[r][c] = sum_i A[r][i] V[c][i]
// (c < C <= 9, V row stride ldv, V[c] holding at least B entries) and
// bias[r] = sum_i A[r][i] (out / bias may be NULL), i < B, with A (rows x batch) in
// the blocked feature-major layout of the training dumps (NULL: a single row of
// ones); chunked partial sums added in a fixed order.  Up to kRrMaxJobs of them in
// one pass of two launches, sharing ldv; no job writes another's outputs, and a job
// with `accumulate` adds to what its outputs hold.  partial needs
// n * rr_multi_job_floats(max rows, B) floats.
int rr_chunks(int64_t B);
constexpr int kRrMaxJobs = 7;
struct RrJob {
  const void* A;
  int rows;
  const float* V;
  int C;
  float* out;
  float* bias;
  int accumulate;  // 1: add to out / bias instead of overwriting them
};
struct RrJobs {
  RrJob job[kRrMaxJobs];
  int n;
};
int64_t rr_multi_job_floats(int rows, int64_t B);
hipError_t launch_row_reduce_multi(const RrJobs& jobs, bool a_is_bf16, int64_t B, int64_t ldv, float* partial,
                                   hipStream_t s);
// Workgroups of a one-shot fused_query launch over ntiles tiles: one per compute
// unit (each holds one), fewer for small launches.  Training's per-workgroup sums
// are indexed by it.
inline int fused_grid(int64_t ntiles, int num_cu) { return (int)(ntiles < num_cu ? ntiles : num_cu); }


// Table I training loss (width 256, FP32): per 64-sample tile, the forward, the
// reverse sweep for e = dF/dv, the tangent pass along u and the reverse mode through
// both programs (see table1_tiles).  Dumps (blocked feature-major, [W x ldb] each):
//   H[l] = h_{l+1}, G[l] = g_{l+1} (reverse sweep, = d/dz of the tangent output),
//   Hd[l] = hdot_{l+1} (tangent), Zb[l] = zbar_{l+1} (adjoint of the primal), l = 0..3;
// V[c][i] = network input c.  scratch: per workgroup of the grid, 11 arrays of
// kThreads * 64 floats (pre-activations, tangent pre-activations, reverse products).
struct T1Job {
  const float* knots;
  const float* points;
  int64_t B, ldb;
  const float* fbar;  // [B] dL/dF per sample
  const float* u;     // [9][ldb] A^T dL/dJ per sample (input-space tangent direction)
  float* H;
  float* G;
  float* Hd;
  float* Zb;
  float* V;
  float* scratch;
};
constexpr int kT1ScratchArrays = 11;
hipError_t launch_table1_tiles(const DevNet& net, const T1Job& job, int grid, hipStream_t s);
// Per-sample loss terms and their derivatives: from d[i], J[i][9] (the query), targets
// fstar, Jstar, m_diag (9) and lambda (4): fbar[i] = dL/dd_i, u[c][i] (row stride ldb,
// zero from B to ldb), and losses[0..3] = the four averaged terms, losses[4] = total,
// summed in a fixed order (part: 4 * ceil(ldb / 256) floats of scratch).
hipError_t launch_table1_loss(const float* knots, const float* points, const float* d, const float* J,
                              const float* fstar, const float* Jstar, const float* m_diag, const float* lambda,
                              int64_t B, int64_t ldb, float* fbar, float* u, float* part, float* losses,
                              hipStream_t s);

// Adam step over n floats (see gcdf_adam_step).
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, int64_t step, hipStream_t s);

// One Adam update of element i in torch.optim.Adam's operation order (no weight
// decay, no amsgrad); lr_corr = lr / (1 - b1^t), inv_sqrt_bc2 = 1 / sqrt(1 - b2^t).
struct AdamConsts {
  float lr_corr, b1, b2, inv_sqrt_bc2, eps;
  static AdamConsts make(float lr, float b1, float b2, float eps, int64_t step);
};
__device__ __forceinline__ float adam_update(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                             float* __restrict__ v, int64_t i, const AdamConsts& a) {
  const float gi = g[i];
  const float mi = a.b1 * m[i] + (1.0f - a.b1) * gi;
  const float vi = a.b2 * v[i] + (1.0f - a.b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float denom = sqrtf(vi) * a.inv_sqrt_bc2 + a.eps;
  const float pi = p[i] - a.lr_corr * (mi / denom);
  p[i] = pi;
  return pi;
}
// Adam over the flat parameters of a point network (pj's source pointers point into
// params; grad, m, v share its layout; b_out at params[b5_off]) with every updated
// value also written to pj's packed arrays, in one launch, so the packing of the
// next forward is done.  FP32 and pure-BF16 packings (the training precisions).
hipError_t launch_adam_pack(const PackJob& pj, float* params, const float* grad, float* m, float* v,
                            const AdamConsts& a, int64_t b5_off, hipStream_t s);

}  // namespace gcdf
