// Training form of libgcdf: weight gradients behind the C ABI (include/gcdf.h).
//
// forward : the pair-list query kernel (sample i = knot i, point i), weights
//           packed on the device from the FP32 master copy at every call;
// backward: the same kernel in training mode -- forward recomputed per tile,
//           reverse sweep seeded with dL/dd_i, layer inputs h_l and gradients
//           g_l = dL/dz_l written in a blocked feature-major layout -- then
//             dW_l = G_l H_{l-1}^T       (matrix cores, split-K, fixed-order sum),
//             dW_1 = G_1 V^T, db_l = sum_i G_l, dw_out = H_4 seed, db_out = sum seed
//           (fixed-order row reductions);
// mse     : the backward's launches with the loss L = mean_i (d_i - y_i)^2 fused in:
//           each tile finishes d before its reverse sweep and seeds it with
//           dL/dd_i = 2 (d_i - y_i) / B, so no separate forward runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "gcdf.h"
#include "gcdf_internal.h"
#include "gcdf_serve.h"

struct gcdf_trainer {
  int W = 0, mode = 0, device = 0, num_cu = 0;
  int64_t max_batch = 0, ldb = 0;
  gcdf::DevNet net{};
  void* wbuf = nullptr;
  size_t mbytes = 0, off_m = 0;
  void* dumpH = nullptr;
  void* dumpG = nullptr;
  float* dumpV = nullptr;
  float* mse = nullptr;  // fused MSE: per-sample seeds [ldb], then loss terms [ldb]
  float* bias_part = nullptr;  // BF16: the training kernel's per-workgroup sums [kTrainSumRows][W][num_cu]
  float* partial = nullptr;
  const float* packed_from = nullptr;  // params pointer of the last packing
  // Table I loss workspace (allocated at its first use)
  float* t1 = nullptr;  // d, J, fbar, u, partial sums, Hd, Zb, per-workgroup scratch
  size_t t1_bytes = 0;
};

namespace {

gcdf_status tfail(gcdf_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return gcdf::set_error(st, buf);
}

struct Offsets {
  size_t W1, b1, Wl[3], bl[3], w5, b5, total;
  explicit Offsets(int W) {
    size_t o = 0;
    W1 = o; o += (size_t)W * 9;
    b1 = o; o += W;
    for (int l = 0; l < 3; ++l) { Wl[l] = o; o += (size_t)W * W; bl[l] = o; o += W; }
    w5 = o; o += W;
    b5 = o; o += 1;
    total = o;
  }
};

struct DevGuard {
  int prev = -1;
  explicit DevGuard(int d) {
    if (hipGetDevice(&prev) == hipSuccess && prev != d) (void)hipSetDevice(d);
  }
  ~DevGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// The packing of params into the trainer's packed arrays.
gcdf::PackJob pack_job(const gcdf_trainer* tr, const float* params) {
  const Offsets o(tr->W);
  char* base = static_cast<char*>(tr->wbuf);
  gcdf::PackJob pj{};
  pj.width = tr->W;
  pj.mode = tr->mode;
  pj.in_dim = gcdf::kInDim;
  pj.W1 = params + o.W1;
  pj.b1 = params + o.b1;
  for (int l = 0; l < 3; ++l) {
    pj.Wl[l] = params + o.Wl[l];
    pj.bl[l] = params + o.bl[l];
    pj.fwd[l] = base + tr->off_m + (size_t)l * tr->mbytes;
    pj.bwd[l] = base + tr->off_m + (size_t)(3 + l) * tr->mbytes;
  }
  pj.w5 = params + o.w5;
  pj.bh = const_cast<float*>(tr->net.bh);
  pj.w5p = const_cast<float*>(tr->net.w5);
  pj.w1p = const_cast<float*>(tr->net.w1p);
  return pj;
}

hipError_t pack(gcdf_trainer* tr, const float* params, hipStream_t s) {
  hipError_t e = gcdf::pack_network(pack_job(tr, params), s);
  tr->net.b5p = params + Offsets(tr->W).b5;
  tr->packed_from = e == hipSuccess ? params : nullptr;
  return e;
}

gcdf_status check(const gcdf_trainer* tr, const float* params, const float* knots, const float* points, int64_t B) {
  if (!tr) return tfail(GCDF_EINVAL, "trainer is NULL");
  if (!params || !knots || !points) return tfail(GCDF_EINVAL, "params/knots/points pointer is NULL");
  if (B <= 0 || B > tr->max_batch) return tfail(GCDF_EINVAL, "batch %lld outside [1, %lld]", (long long)B, (long long)tr->max_batch);
  return GCDF_OK;
}

// The training-mode query over the batch as a pair list (sample i = knot i, point i).
gcdf::Job training_job(const gcdf_trainer* tr, const float* knots, const float* points, int64_t B) {
  gcdf::Job job{};
  job.knots = knots;
  job.points = points;
  job.K = B;
  job.Np = B;
  job.npairs = B;
  job.dumpH = tr->dumpH;
  job.dumpG = tr->dumpG;
  job.ldb = tr->ldb;
  if (tr->mode == GCDF_FP32) {
    job.dumpV = tr->dumpV;  // for dW1, reduced from the dumps
  } else {
    job.bias_part = tr->bias_part;  // the kernel sums what needs no GEMM
  }
  return job;
}

// After the training-mode query: the weight gradients from its dumps and the
// per-sample seeds dL/dd; with sq set, also *loss = sum_i sq[i].
hipError_t weight_gradients(gcdf_trainer* tr, int64_t B, const float* seed, const float* sq, float* loss, float* grad,
                            hipStream_t s) {
  const int W = tr->W;
  const Offsets o(W);
  const size_t esz = tr->mode == GCDF_FP32 ? 4 : 2;
  const size_t layer = (size_t)W * tr->ldb * esz;
  auto H = [&](int l) { return static_cast<const char*>(tr->dumpH) + l * layer; };
  auto G = [&](int l) { return static_cast<const char*>(tr->dumpG) + l * layer; };
  const bool bf = tr->mode != GCDF_FP32;
  const int gmode = bf ? gcdf::kBF16 : gcdf::kFP32;
  // dW_{l+1} = G_{l+1} H_l^T for the hidden layers 2..4, one launch
  gcdf::WgradJobs wj{};
  wj.n = 3;
  for (int l = 0; l < 3; ++l) {
    wj.G[l] = G(l + 1);
    wj.H[l] = H(l);
    wj.out[l] = grad + o.Wl[l];
  }
  const int64_t ntiles = (B + gcdf::kTileQ - 1) / gcdf::kTileQ;
  if (bf) {
    // everything else was summed per workgroup by the training kernel: the launch
    // that adds the GEMMs' chunks also adds the workgroups' sums (bias gradients,
    // dw_out, dW1 column by column, db_out, loss)
    gcdf::PartSum ps{};
    ps.part = tr->bias_part;
    ps.nparts = gcdf::fused_grid(ntiles, tr->num_cu);
    ps.width = W;
    float* rows[5] = {grad + o.b1, grad + o.bl[0], grad + o.bl[1], grad + o.bl[2], grad + o.w5};
    for (int r = 0; r < 5; ++r) ps.out.base[r] = rows[r], ps.out.stride[r] = 1, ps.out.n[r] = W;
    for (int c = 0; c < 9; ++c) ps.out.base[5 + c] = grad + o.W1 + c, ps.out.stride[5 + c] = 9, ps.out.n[5 + c] = W;
    ps.out.base[14] = grad + o.b5, ps.out.stride[14] = 1, ps.out.n[14] = 1;
    ps.out.base[15] = loss, ps.out.stride[15] = 1, ps.out.n[15] = 1;
    return gcdf::launch_wgrad_gemm(wj, W, gmode, tr->ldb, B, tr->partial, tr->num_cu, s, false, &ps);
  }
  hipError_t e = gcdf::launch_wgrad_gemm(wj, W, gmode, tr->ldb, B, tr->partial, tr->num_cu, s);
  // FP32: one pass over the batch for the rest (the partial buffer is free again:
  // this follows the GEMMs' chunk sum on the stream): input layer dW1 = G_1 V^T and
  // db1 = sum G_1; db_l = sum G_l; output layer dw_out = H_4 seed, db_out = sum seed;
  // the loss.  (Single-row V operands ignore the shared row stride ldb.)
  gcdf::RrJobs rj{};
  rj.n = sq ? 7 : 6;
  rj.job[0] = {G(0), W, tr->dumpV, 9, grad + o.W1, grad + o.b1, 0};
  for (int l = 0; l < 3; ++l) rj.job[1 + l] = {G(l + 1), W, nullptr, 0, nullptr, grad + o.bl[l], 0};
  rj.job[4] = {H(3), W, seed, 1, grad + o.w5, nullptr, 0};
  rj.job[5] = {nullptr, 1, seed, 1, grad + o.b5, nullptr, 0};
  if (sq) rj.job[6] = {nullptr, 1, sq, 1, loss, nullptr, 0};
  if (e == hipSuccess) e = gcdf::launch_row_reduce_multi(rj, false, B, tr->ldb, tr->partial, s);
  return e;
}

}  // namespace

extern "C" {

int64_t gcdf_param_count(int32_t width) { return width > 0 ? (int64_t)Offsets(width).total : 0; }

gcdf_status gcdf_trainer_create(int32_t width, int32_t precision, int32_t device, int64_t max_batch,
                                gcdf_trainer** out) {
  if (!out) return tfail(GCDF_EINVAL, "out is NULL");
  *out = nullptr;
  if (width != 256) return tfail(GCDF_EINVAL, "training is built for width 256 (got %d)", width);
  if (precision != GCDF_FP32 && precision != GCDF_BF16)
    return tfail(GCDF_EINVAL, "training precision must be GCDF_FP32 or GCDF_BF16");
  if (max_batch <= 0 || max_batch > ((int64_t)1 << 30)) return tfail(GCDF_EINVAL, "max_batch out of range");
  int dev = device;
  if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return tfail(GCDF_EDEVICE, "no current HIP device");
  DevGuard g(dev);
  gcdf_trainer* tr = new gcdf_trainer;
  tr->W = width;
  tr->mode = precision;
  tr->device = dev;
  tr->max_batch = max_batch;
  tr->ldb = (max_batch + gcdf::kTileQ - 1) / gcdf::kTileQ * gcdf::kTileQ;
  hipError_t e = hipDeviceGetAttribute(&tr->num_cu, hipDeviceAttributeMultiprocessorCount, dev);
  const int W = width;
  auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
  tr->mbytes = align(gcdf::packed_matrix_bytes(W, precision));
  const size_t off_w1 = 0, off_bh = align((size_t)W * 12 * 4), off_w5 = off_bh + align((size_t)3 * W * 4);
  tr->off_m = off_w5 + align((size_t)W * 4);
  const size_t esz = precision == GCDF_FP32 ? 4 : 2;
  const size_t dump = (size_t)4 * W * tr->ldb * esz;
  if (e == hipSuccess) e = hipMalloc(&tr->wbuf, tr->off_m + 6 * tr->mbytes);
  if (e == hipSuccess) e = hipMalloc(&tr->dumpH, dump);
  if (e == hipSuccess) e = hipMalloc(&tr->dumpG, dump);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&tr->dumpV), (size_t)9 * tr->ldb * 4);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&tr->mse), (size_t)2 * tr->ldb * 4);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&tr->bias_part), (size_t)std::max(tr->num_cu, 1) * gcdf::kTrainSumRows * W * 4);
  const size_t part = std::max({(size_t)gcdf::wgrad_partial_floats(max_batch, W, tr->num_cu),
                                 (size_t)gcdf::rr_chunks(max_batch) * W * 10,
                                 (size_t)gcdf::kRrMaxJobs * gcdf::rr_multi_job_floats(W, max_batch)});
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&tr->partial), part * 4);
  if (e != hipSuccess) {
    gcdf_trainer_destroy(tr);
    return tfail(GCDF_ENOMEM, "trainer allocation failed: %s", hipGetErrorString(e));
  }
  char* base = static_cast<char*>(tr->wbuf);
  tr->net.width = W;
  tr->net.mode = precision;
  tr->net.in_dim = gcdf::kInDim;  // training takes point networks
  tr->net.w1p = reinterpret_cast<float*>(base + off_w1);
  tr->net.bh = reinterpret_cast<float*>(base + off_bh);
  tr->net.w5 = reinterpret_cast<float*>(base + off_w5);
  for (int l = 0; l < 3; ++l) {
    tr->net.fwd[l] = base + tr->off_m + (size_t)l * tr->mbytes;
    tr->net.bwd[l] = base + tr->off_m + (size_t)(3 + l) * tr->mbytes;
  }
  *out = tr;
  return GCDF_OK;
}

void gcdf_trainer_destroy(gcdf_trainer* tr) {
  if (!tr) return;
  DevGuard g(tr->device);
  (void)hipFree(tr->wbuf);
  (void)hipFree(tr->dumpH);
  (void)hipFree(tr->dumpG);
  (void)hipFree(tr->dumpV);
  (void)hipFree(tr->mse);
  (void)hipFree(tr->bias_part);
  (void)hipFree(tr->partial);
  (void)hipFree(tr->t1);
  delete tr;
}

gcdf_status gcdf_train_forward(gcdf_trainer* tr, const float* params, const float* knots, const float* points,
                               int64_t B, float* d, void* stream) {
  gcdf_status st = check(tr, params, knots, points, B);
  if (st != GCDF_OK) return st;
  if (!d) return tfail(GCDF_EINVAL, "d is NULL");
  DevGuard g(tr->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = pack(tr, params, s);
  gcdf::Job job{};
  job.knots = knots;
  job.points = points;
  job.K = B;
  job.Np = B;
  job.npairs = B;
  job.d = d;
  if (e == hipSuccess) e = gcdf::launch_fused(tr->net, job, true, false, tr->num_cu, s);
  return e == hipSuccess ? GCDF_OK : tfail(GCDF_EDEVICE, "gcdf_train_forward: %s", hipGetErrorString(e));
}

gcdf_status gcdf_train_backward(gcdf_trainer* tr, const float* params, const float* knots, const float* points,
                                int64_t B, const float* grad_d, float* grad, int32_t reuse_packed, void* stream) {
  gcdf_status st = check(tr, params, knots, points, B);
  if (st != GCDF_OK) return st;
  if (!grad_d || !grad) return tfail(GCDF_EINVAL, "grad_d or grad_params is NULL");
  DevGuard g(tr->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = (reuse_packed && tr->packed_from == params) ? hipSuccess : pack(tr, params, s);
  gcdf::Job job = training_job(tr, knots, points, B);
  job.seed = grad_d;
  if (e == hipSuccess) e = gcdf::launch_fused(tr->net, job, true, true, tr->num_cu, s);
  if (e == hipSuccess) e = weight_gradients(tr, B, grad_d, nullptr, nullptr, grad, s);
  return e == hipSuccess ? GCDF_OK : tfail(GCDF_EDEVICE, "gcdf_train_backward: %s", hipGetErrorString(e));
}

gcdf_status gcdf_train_mse(gcdf_trainer* tr, const float* params, const float* knots, const float* points, int64_t B,
                           const float* target, float* loss, float* grad, float* d, int32_t reuse_packed,
                           void* stream) {
  gcdf_status st = check(tr, params, knots, points, B);
  if (st != GCDF_OK) return st;
  if (!target || !loss || !grad) return tfail(GCDF_EINVAL, "target, loss or grad_params is NULL");
  DevGuard g(tr->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = (reuse_packed && tr->packed_from == params) ? hipSuccess : pack(tr, params, s);
  gcdf::Job job = training_job(tr, knots, points, B);
  float* seed = tr->mse;
  float* sq = tr->mse + tr->ldb;
  job.target = target;
  if (tr->mode == GCDF_FP32) {  // the seeds and loss terms for the reductions from the dumps
    job.seed_out = seed;
    job.sq_out = sq;
  }
  job.mse_scale = (float)(2.0 / (double)B);
  job.inv_b = (float)(1.0 / (double)B);
  job.d = d;
  if (e == hipSuccess) e = gcdf::launch_fused(tr->net, job, true, true, tr->num_cu, s);
  if (e == hipSuccess) e = weight_gradients(tr, B, seed, sq, loss, grad, s);
  return e == hipSuccess ? GCDF_OK : tfail(GCDF_EDEVICE, "gcdf_train_mse: %s", hipGetErrorString(e));
}

gcdf_status gcdf_train_table1(gcdf_trainer* tr, const float* params, const float* knots, const float* points,
                              int64_t B, const float* fstar, const float* Jstar, const float* m_diag,
                              const float* lambda, float* losses, float* grad, void* stream) {
  gcdf_status st = check(tr, params, knots, points, B);
  if (st != GCDF_OK) return st;
  if (!fstar || !Jstar || !m_diag || !lambda || !losses || !grad)
    return tfail(GCDF_EINVAL, "NULL argument to gcdf_train_table1");
  if (tr->mode != GCDF_FP32) return tfail(GCDF_EINVAL, "the Table I loss is built for a GCDF_FP32 trainer");
  for (int c = 0; c < 9; ++c)
    if (!(m_diag[c] > 0.f) || !std::isfinite(m_diag[c])) return tfail(GCDF_EINVAL, "m_diag must be finite and > 0");
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(lambda[k])) return tfail(GCDF_EINVAL, "lambda must be finite");
  DevGuard g(tr->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int W = tr->W;
  const int64_t ldb = tr->ldb;
  const size_t layer = (size_t)W * ldb;
  const int grid = tr->num_cu;
  const size_t arr = (size_t)gcdf::kThreads * 64;
  // workspace: d [ldb], J [9 ldb], fbar [ldb], u [9 ldb], part [4 ceil(ldb/256)], Hd, Zb [4 layer each],
  // scratch [grid * 11 * arr]
  const size_t n_d = ldb, n_J = 9 * ldb, n_f = ldb, n_u = 9 * ldb, n_p = 4 * ((ldb + 255) / 256) + 8;
  const size_t n_dump = 4 * layer, n_s = (size_t)grid * gcdf::kT1ScratchArrays * arr;
  const size_t need = 4 * (n_d + n_J + n_f + n_u + n_p + 2 * n_dump + n_s);
  if (!tr->t1) {
    if (hipMalloc(reinterpret_cast<void**>(&tr->t1), need) != hipSuccess) {
      tr->t1 = nullptr;
      return tfail(GCDF_ENOMEM, "Table I workspace allocation (%zu bytes) failed", need);
    }
    tr->t1_bytes = need;
  }
  float* d = tr->t1;
  float* J = d + n_d;
  float* fbar = J + n_J;
  float* u = fbar + n_f;
  float* part = u + n_u;
  float* Hd = part + n_p;
  float* Zb = Hd + n_dump;
  float* scratch = Zb + n_dump;
  float* H = static_cast<float*>(tr->dumpH);
  float* Gs = static_cast<float*>(tr->dumpG);
  const Offsets o(W);
  hipError_t e = pack(tr, params, s);
  // 1. the query over the samples: d and J
  gcdf::Job qj{};
  qj.knots = knots;
  qj.points = points;
  qj.K = B;
  qj.Np = B;
  qj.npairs = B;
  qj.d = d;
  qj.J = J;
  if (e == hipSuccess) e = gcdf::launch_fused(tr->net, qj, true, true, tr->num_cu, s);
  // 2. loss terms, dL/dF and u = A^T dL/dJ per sample
  if (e == hipSuccess)
    e = gcdf::launch_table1_loss(knots, points, d, J, fstar, Jstar, m_diag, lambda, B, ldb, fbar, u, part, losses, s);
  // 3. per tile: forward, reverse, tangent, adjoint (dumps)
  gcdf::T1Job tj{};
  tj.knots = knots;
  tj.points = points;
  tj.B = B;
  tj.ldb = ldb;
  tj.fbar = fbar;
  tj.u = u;
  tj.H = H;
  tj.G = Gs;
  tj.Hd = Hd;
  tj.Zb = Zb;
  tj.V = tr->dumpV;
  tj.scratch = scratch;
  const int64_t ntiles = (B + gcdf::kTileQ - 1) / gcdf::kTileQ;
  if (e == hipSuccess) e = gcdf::launch_table1_tiles(tr->net, tj, (int)std::min<int64_t>(grid, ntiles), s);
  // 4. dW_l = sum zbar_l h_{l-1}^T + g_l hdot_{l-1}^T for the hidden layers
  gcdf::WgradJobs a{}, b{};
  a.n = b.n = 3;
  for (int l = 0; l < 3; ++l) {
    a.G[l] = Zb + (l + 1) * layer;
    a.H[l] = H + l * layer;
    b.G[l] = Gs + (l + 1) * layer;
    b.H[l] = Hd + l * layer;
    a.out[l] = b.out[l] = grad + o.Wl[l];
  }
  if (e == hipSuccess) e = gcdf::launch_wgrad_gemm(a, W, gcdf::kFP32, ldb, B, tr->partial, tr->num_cu, s, false);
  if (e == hipSuccess) e = gcdf::launch_wgrad_gemm(b, W, gcdf::kFP32, ldb, B, tr->partial, tr->num_cu, s, true);
  // 5. the rest in two passes over the batch (fixed-order row reductions, the second
  //    adding to the first's outputs): input layer dW_1 = sum zbar_1 v^T + g_1 u^T,
  //    db_1 = sum zbar_1; db_l = sum zbar_l; output layer dw_out = sum fbar h_4 + hdot_4,
  //    db_out = sum fbar.  (v and u share the row stride ldb.)
  gcdf::RrJobs r1{}, r2{};
  r1.n = 6;
  r1.job[0] = {Zb, W, tr->dumpV, 9, grad + o.W1, grad + o.b1, 0};
  for (int l = 0; l < 3; ++l) r1.job[1 + l] = {Zb + (l + 1) * layer, W, nullptr, 0, nullptr, grad + o.bl[l], 0};
  r1.job[4] = {H + 3 * layer, W, fbar, 1, grad + o.w5, nullptr, 0};
  r1.job[5] = {nullptr, 1, fbar, 1, grad + o.b5, nullptr, 0};
  r2.n = 2;
  r2.job[0] = {Gs, W, u, 9, grad + o.W1, nullptr, 1};
  r2.job[1] = {Hd + 3 * layer, W, nullptr, 0, nullptr, grad + o.w5, 1};
  if (e == hipSuccess) e = gcdf::launch_row_reduce_multi(r1, false, B, ldb, tr->partial, s);
  if (e == hipSuccess) e = gcdf::launch_row_reduce_multi(r2, false, B, ldb, tr->partial, s);
  return e == hipSuccess ? GCDF_OK : tfail(GCDF_EDEVICE, "gcdf_train_table1: %s", hipGetErrorString(e));
}

gcdf_status gcdf_train_adam_step(gcdf_trainer* tr, float* params, const float* grad, float* m, float* v, float lr,
                                 float beta1, float beta2, float eps, int64_t step, void* stream) {
  if (!tr || !params || !grad || !m || !v) return tfail(GCDF_EINVAL, "NULL pointer to gcdf_train_adam_step");
  if (step < 1) return tfail(GCDF_EINVAL, "step must be >= 1");
  if (!std::isfinite(lr) || !std::isfinite(eps) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f))
    return tfail(GCDF_EINVAL, "lr / eps must be finite and betas in [0, 1)");
  DevGuard g(tr->device);
  const Offsets o(tr->W);
  const hipError_t e = gcdf::launch_adam_pack(pack_job(tr, params), params, grad, m, v,
                                              gcdf::AdamConsts::make(lr, beta1, beta2, eps, step), (int64_t)o.b5,
                                              static_cast<hipStream_t>(stream));
  tr->net.b5p = params + o.b5;
  tr->packed_from = e == hipSuccess ? params : nullptr;
  return e == hipSuccess ? GCDF_OK : tfail(GCDF_EDEVICE, "gcdf_train_adam_step: %s", hipGetErrorString(e));
}

gcdf_status gcdf_adam_step(float* params, const float* grad, float* m, float* v, int64_t n, float lr, float beta1,
                           float beta2, float eps, int64_t step, void* stream) {
  if (!params || !grad || !m || !v) return tfail(GCDF_EINVAL, "NULL pointer to gcdf_adam_step");
  if (n < 0 || step < 1) return tfail(GCDF_EINVAL, "n must be >= 0 and step >= 1");
  if (!std::isfinite(lr) || !std::isfinite(eps) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f))
    return tfail(GCDF_EINVAL, "lr / eps must be finite and betas in [0, 1)");
  if (n == 0) return GCDF_OK;
  const hipError_t e = gcdf::launch_adam(params, grad, m, v, n, lr, beta1, beta2, eps, step,
                                         static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GCDF_OK : tfail(GCDF_EDEVICE, "gcdf_adam_step: %s", hipGetErrorString(e));
}

}  // extern "C"
