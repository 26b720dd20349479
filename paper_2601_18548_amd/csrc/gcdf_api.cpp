// C-ABI of libgcdf: contexts, argument checking, weight packing and launches.
// The query semantics are documented in include/gcdf.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gcdf.h"
#include "gcdf_internal.h"
#include "gcdf_serve.h"

#include <mutex>

namespace {

thread_local std::string g_err;

// Per-knot minimum keys of gcdf_query_noalloc, which allocates nothing: a
// file-scope device array, one copy per GPU (held until the process ends).  Its
// name is only a host-side stand-in; kernels get the device address that
// hipGetSymbolAddress returns for the current device (g_noalloc_keys).
constexpr int64_t kNoAllocMaxKnots = 1 << 16;  // 512 KiB of keys
static __device__ __align__(256) unsigned long long scratch[kNoAllocMaxKnots];
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
unsigned long long* g_noalloc_keys[kMaxDevices];  // device address of `scratch` per device
hipError_t g_noalloc_err[kMaxDevices];            // hipGetSymbolAddress's result per device
bool g_noalloc_done[kMaxDevices];

gcdf_status fail(gcdf_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

gcdf_status hip_fail(hipError_t e, const char* what) {
  return fail(GCDF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kHeader = 32;

}  // namespace

struct gcdf_ctx {
  gcdf_config cfg{};
  int device = 0;
  int num_cu = 0;
  gcdf::DevNet net{};
  void* wbuf = nullptr;               // all packed weights
  unsigned long long* minkey = nullptr;  // [max_knots]
  int64_t* tile_off = nullptr;        // [max_knots + 1] (CSR query)
  unsigned long long* noalloc_keys = nullptr;  // this device's `scratch` (gcdf_query_noalloc)
  hipError_t noalloc_err = hipSuccess;         // why noalloc_keys is NULL
  uint32_t* overflow = nullptr;       // pinned host word written by the device (GCDF_BF16X2_F16)
  gcdf::Server* server = nullptr;
};

namespace {

// RAII: make `dev` current for the scope of a call, restoring the caller's device.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// The sticky FP16-overflow flag of a GCDF_BF16X2_F16 context: reported (and
// cleared) by the first query call or poll that sees it.
gcdf_status take_overflow(gcdf_ctx* ctx) {
  if (ctx->overflow && __atomic_exchange_n(ctx->overflow, 0u, __ATOMIC_ACQ_REL) != 0)
    return fail(GCDF_ERANGE, "an earlier query's FP16 reverse sweep overflowed: its J holds Inf/NaN "
                             "(back-propagated values beyond the FP16 range of the GCDF_BF16X2_F16 precision)");
  return GCDF_OK;
}

gcdf_status check_query(gcdf_ctx* ctx, const float* knots, int64_t K, const float* points, int64_t Np) {
  if (!ctx) return fail(GCDF_EINVAL, "ctx is NULL");
  if (gcdf_status st = take_overflow(ctx); st != GCDF_OK) return st;
  if (!knots || !points) return fail(GCDF_EINVAL, "knots/points pointer is NULL");
  if (K <= 0 || Np <= 0) return fail(GCDF_EINVAL, "K and Np must be positive (K=%lld, Np=%lld)", (long long)K, (long long)Np);
  if (K > INT64_MAX / 9 / Np) return fail(GCDF_EINVAL, "K*Np*9 overflows int64");
  return GCDF_OK;
}

// Device address of `scratch` on device `dev`, which must be current: looked up
// once per device (the first context created on it) and kept.
unsigned long long* noalloc_keys_for(int dev, hipError_t* err) {
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_done[dev]) {
    void* p = nullptr;
    g_noalloc_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_noalloc_keys[dev] = g_noalloc_err[dev] == hipSuccess ? static_cast<unsigned long long*>(p) : nullptr;
    g_noalloc_done[dev] = true;
  }
  *err = g_noalloc_err[dev];
  return g_noalloc_keys[dev];
}

}  // namespace

namespace gcdf {

// Enqueue a dense query on `s` (used by the eval calls and the serving loop).
hipError_t enqueue_dense(const gcdf_ctx* ctx, const Job& job, bool want_grad, hipStream_t s) {
  return launch_fused(ctx->net, job, false, want_grad, ctx->num_cu, s);
}

const DevNet& ctx_net(const gcdf_ctx* ctx) { return ctx->net; }
int ctx_num_cu(const gcdf_ctx* ctx) { return ctx->num_cu; }
int ctx_device(const gcdf_ctx* ctx) { return ctx->device; }

}  // namespace gcdf

extern "C" {

const char* gcdf_last_error(const gcdf_ctx*) { return g_err.c_str(); }

gcdf_status gcdf_create(const gcdf_config* cfg, const void* blob, size_t bytes, gcdf_ctx** out) {
  if (!cfg || !blob || !out) return fail(GCDF_EINVAL, "NULL argument to gcdf_create");
  *out = nullptr;
  if (cfg->width != 256 && cfg->width != 512) return fail(GCDF_EINVAL, "width must be 256 or 512 (got %d)", cfg->width);
  if (cfg->depth != 4) return fail(GCDF_EINVAL, "depth must be 4 (got %d)", cfg->depth);
  if (cfg->precision < GCDF_FP32 || cfg->precision > GCDF_BF16X2_F16)
    return fail(GCDF_EINVAL, "unknown precision %d", cfg->precision);
  if (cfg->max_knots < 0) return fail(GCDF_EINVAL, "max_knots must be >= 0");
  const int W = cfg->width;
  if (bytes < kHeader) return fail(GCDF_EINVAL, "weight blob is %zu bytes, shorter than its header", bytes);
  const uint32_t* hdr = static_cast<const uint32_t*>(blob);
  // in_dim 9: point obstacles, input [p', a]; 10: sphere obstacles, input [p', r, a]
  const int in_dim = (int)hdr[2];
  if (std::memcmp(blob, "GCDF", 4) != 0 || hdr[1] != 1 || (in_dim != gcdf::kInDim && in_dim != gcdf::kInDimSphere) ||
      (int)hdr[3] != W || (int)hdr[4] != 4)
    return fail(GCDF_EINVAL, "weight blob header does not match (magic/version/in_dim/width/depth)");
  // blob: header + W1, b1, (W2, b2) .. (W4, b4), w_out, b_out
  const size_t nfloat = (size_t)W * in_dim + W + 3 * ((size_t)W * W + W) + W + 1;
  if (bytes != kHeader + 4 * nfloat) return fail(GCDF_EINVAL, "weight blob is %zu bytes, expected %zu", bytes, kHeader + 4 * nfloat);
  if (cfg->precision == GCDF_BF16X2_F16) {
    // The reverse sweep holds the BF16-rounded hidden weights as FP16: every one
    // must round to a finite FP16 value (|w| < 65408 rounds to at most 65280).
    const char* p = static_cast<const char*>(blob) + kHeader + 4 * ((size_t)W * in_dim + W);
    for (int l = 0; l < 3; ++l, p += 4 * ((size_t)W * W + W))
      for (size_t i = 0; i < (size_t)W * W; ++i) {
        float v;
        std::memcpy(&v, p + 4 * i, 4);
        if (!(std::fabs(v) < 65408.0f))
          return fail(GCDF_EINVAL, "precision BF16X2_F16: hidden weight W%d[%zu] = %g is not finite in FP16", l + 2, i, (double)v);
      }
  }

  int dev = cfg->device;
  if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return fail(GCDF_EDEVICE, "no current HIP device");
  DeviceGuard guard(dev);
  if (!guard.ok) return fail(GCDF_EDEVICE, "hipSetDevice(%d) failed", dev);

  gcdf_ctx* c = new gcdf_ctx;
  c->cfg = *cfg;
  if (c->cfg.max_knots == 0) c->cfg.max_knots = 1 << 20;
  c->device = dev;
  hipError_t e = hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipDeviceGetAttribute");
  }
  const int mode = cfg->precision;
  const size_t mbytes = gcdf::packed_matrix_bytes(W, mode);
  auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t off_w1 = 0;
  const size_t off_bh = align(off_w1 + (size_t)W * 12 * 4);
  const size_t off_w5 = align(off_bh + (size_t)3 * W * 4);
  const size_t off_b5 = align(off_w5 + (size_t)W * 4);
  const size_t off_m = align(off_b5 + 4);
  const size_t total = off_m + 6 * align(mbytes);
  const size_t ws = (size_t)c->cfg.max_knots * (8 + 8) + 8;
  float* staging = nullptr;
  e = hipMalloc(&c->wbuf, total);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&c->minkey), ws);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&staging), 4 * nfloat);
  if (e != hipSuccess) {
    hipFree(staging);
    gcdf_destroy(c);
    return fail(GCDF_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
  }
  c->tile_off = reinterpret_cast<int64_t*>(c->minkey + c->cfg.max_knots);
  hipStream_t s = nullptr;
  e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMemcpyAsync(staging, static_cast<const char*>(blob) + kHeader, 4 * nfloat, hipMemcpyHostToDevice, s);
  char* base = static_cast<char*>(c->wbuf);
  // offsets of the source arrays inside staging (floats)
  const float* W1 = staging;
  const float* b1 = W1 + (size_t)W * in_dim;
  const float* Wl[3];
  const float* bl[3];
  {
    const float* p = b1 + W;
    for (int l = 0; l < 3; ++l) {
      Wl[l] = p;
      bl[l] = p + (size_t)W * W;
      p = bl[l] + W;
    }
  }
  const float* w5src = bl[2] + W;
  float* w1p = reinterpret_cast<float*>(base + off_w1);
  float* bh = reinterpret_cast<float*>(base + off_bh);
  float* w5 = reinterpret_cast<float*>(base + off_w5);
  // biases b2..b4 are not contiguous in the blob: reorder them one by one
  if (e == hipSuccess) e = gcdf::pack_input_layer(W1, b1, w1p, W, in_dim, s);
  for (int l = 0; l < 3 && e == hipSuccess; ++l) e = gcdf::pack_row_vectors(bl[l], bh + (size_t)l * W, W, 1, s);
  if (e == hipSuccess) e = gcdf::pack_row_vectors(w5src, w5, W, 1, s);
  if (e == hipSuccess) e = hipMemcpyAsync(base + off_b5, staging + nfloat - 1, 4, hipMemcpyDeviceToDevice, s);
  for (int l = 0; l < 3 && e == hipSuccess; ++l) {
    void* f = base + off_m + (size_t)l * align(mbytes);
    void* b = base + off_m + (size_t)(3 + l) * align(mbytes);
    e = gcdf::pack_matrix(Wl[l], f, W, mode, false, s);
    if (e == hipSuccess) e = gcdf::pack_matrix(Wl[l], b, W, mode, true, s);
    c->net.fwd[l] = f;
    c->net.bwd[l] = b;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (s) hipStreamDestroy(s);
  hipFree(staging);
  if (e != hipSuccess) {
    gcdf_destroy(c);
    return hip_fail(e, "weight packing");
  }
  c->net.width = W;
  c->net.mode = mode;
  c->net.in_dim = in_dim;
  c->net.w1p = w1p;
  c->net.bh = bh;
  c->net.w5 = w5;
  c->net.b5p = reinterpret_cast<const float*>(base + off_b5);
  // the no-allocation entry point's key array on this device (only that entry
  // point depends on it, so a failed lookup is reported there)
  c->noalloc_keys = noalloc_keys_for(dev, &c->noalloc_err);
  if (mode == GCDF_BF16X2_F16) {
    e = hipHostMalloc(reinterpret_cast<void**>(&c->overflow), sizeof(uint32_t), hipHostMallocCoherent);
    if (e != hipSuccess) {
      c->overflow = nullptr;
      gcdf_destroy(c);
      return fail(GCDF_ENOMEM, "pinned host allocation failed: %s", hipGetErrorString(e));
    }
    *c->overflow = 0;
    c->net.overflow = c->overflow;
  }
  if (cfg->serve_mem_budget > 0) {
    gcdf_status st = gcdf::server_start(c, cfg->serve_mem_budget, cfg->serve_slots > 0 ? cfg->serve_slots : 64, &c->server);
    if (st != GCDF_OK) {
      std::string msg = g_err;
      gcdf_destroy(c);
      g_err = msg;
      return st;
    }
  }
  *out = c;
  return GCDF_OK;
}

void gcdf_destroy(gcdf_ctx* ctx) {
  if (!ctx) return;
  DeviceGuard guard(ctx->device);
  if (ctx->server) gcdf::server_stop(ctx->server);
  hipFree(ctx->wbuf);
  hipFree(ctx->minkey);
  if (ctx->overflow) {
    (void)hipDeviceSynchronize();  // no kernel of this context may still write the word
    hipHostFree(ctx->overflow);
  }
  delete ctx;
}

}  // extern "C"

namespace {
// gcdf_query with the per-knot key array `keys` (capacity key_cap knots), which
// the minimum clears (all ones) before use.
gcdf_status query_impl(gcdf_ctx* ctx, const float* knots, int64_t K, const float* points, int64_t Np, float* d,
                       float* J, float* dmin, int32_t* argmin, float* Jmin, unsigned long long* keys,
                       int64_t key_cap, const char* cap_name, void* stream) {
  const bool want_min = dmin || argmin;
  if (!d && !J && !want_min) return fail(GCDF_EINVAL, "no output requested");
  if (want_min && !(dmin && argmin)) return fail(GCDF_EINVAL, "dmin and argmin must be given together");
  if (Jmin && !want_min) return fail(GCDF_EINVAL, "Jmin needs dmin and argmin");
  if (want_min && K > key_cap)
    return fail(GCDF_EINVAL, "K=%lld exceeds %s=%lld", (long long)K, cap_name, (long long)key_cap);
  if (want_min && Np > INT32_MAX) return fail(GCDF_EINVAL, "Np=%lld exceeds 2^31-1", (long long)Np);
  DeviceGuard guard(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (want_min) e = gcdf::launch_minkey_init(keys, K, s);
  gcdf::Job job{};
  job.knots = knots;
  job.points = points;
  job.K = K;
  job.Np = Np;
  job.d = d;
  job.J = J;
  job.minkey = want_min ? keys : nullptr;
  if (e == hipSuccess) e = gcdf::launch_fused(ctx->net, job, false, J != nullptr, ctx->num_cu, s);
  if (e == hipSuccess && want_min) e = gcdf::launch_minkey_decode(keys, K, dmin, argmin, s);
  if (e == hipSuccess && Jmin) {
    // the K pairs (knot i, point argmin[i]) through the pair-list kernel
    gcdf::Job pj{};
    pj.knots = knots;
    pj.points = points;
    pj.K = K;
    pj.Np = Np;
    pj.pidx32 = argmin;
    pj.npairs = K;
    pj.J = Jmin;
    e = gcdf::launch_fused(ctx->net, pj, true, true, ctx->num_cu, s);
  }
  return e == hipSuccess ? GCDF_OK : hip_fail(e, "gcdf_query launch");
}
}  // namespace

extern "C" {

gcdf_status gcdf_query(gcdf_ctx* ctx, const float* knots, int64_t K, const float* points, int64_t Np, float* d,
                       float* J, float* dmin, int32_t* argmin, float* Jmin, void* stream) {
  gcdf_status st = check_query(ctx, knots, K, points, Np);
  if (st != GCDF_OK) return st;
  return query_impl(ctx, knots, K, points, Np, d, J, dmin, argmin, Jmin, ctx->minkey, ctx->cfg.max_knots,
                    "max_knots", stream);
}

gcdf_status gcdf_query_noalloc(gcdf_ctx* ctx, const float* knots, int64_t K, const float* points, int64_t Np,
                               float* d, float* J, float* dmin, int32_t* argmin, float* Jmin, void* stream) {
  gcdf_status st = check_query(ctx, knots, K, points, Np);
  if (st != GCDF_OK) return st;
  if (!ctx->noalloc_keys)
    return fail(GCDF_EDEVICE, "the no-allocation key array has no device address: %s",
                hipGetErrorString(ctx->noalloc_err));
  return query_impl(ctx, knots, K, points, Np, d, J, dmin, argmin, Jmin, ctx->noalloc_keys, kNoAllocMaxKnots,
                    "the no-allocation limit", stream);
}

gcdf_status gcdf_eval(gcdf_ctx* ctx, const float* knots, int64_t K, const float* points, int64_t Np, float* d,
                      void* stream) {
  if (!d) return fail(GCDF_EINVAL, "d is NULL");
  return gcdf_query(ctx, knots, K, points, Np, d, nullptr, nullptr, nullptr, nullptr, stream);
}

gcdf_status gcdf_eval_grad(gcdf_ctx* ctx, const float* knots, int64_t K, const float* points, int64_t Np, float* d,
                           float* J, void* stream) {
  if (!d || !J) return fail(GCDF_EINVAL, "d or J is NULL");
  return gcdf_query(ctx, knots, K, points, Np, d, J, nullptr, nullptr, nullptr, stream);
}

gcdf_status gcdf_knot_min(gcdf_ctx* ctx, const float* knots, int64_t K, const float* points, int64_t Np, float* dmin,
                          int32_t* argmin, float* Jmin, void* stream) {
  if (!dmin || !argmin) return fail(GCDF_EINVAL, "dmin or argmin is NULL");
  return gcdf_query(ctx, knots, K, points, Np, nullptr, nullptr, dmin, argmin, Jmin, stream);
}

gcdf_status gcdf_partition_count(gcdf_ctx* ctx, const float* ref, int64_t N, int64_t ref_stride, const float* points,
                                 int64_t Np, float radius, int64_t* offsets, void* stream) {
  if (!ctx) return fail(GCDF_EINVAL, "ctx is NULL");
  if (!ref || !points || !offsets) return fail(GCDF_EINVAL, "ref/points/offsets pointer is NULL");
  if (N <= 0 || Np <= 0) return fail(GCDF_EINVAL, "N and Np must be positive (N=%lld, Np=%lld)", (long long)N, (long long)Np);
  if (Np > INT32_MAX) return fail(GCDF_EINVAL, "Np=%lld exceeds 2^31-1", (long long)Np);
  if (ref_stride < 2) return fail(GCDF_EINVAL, "ref_stride must be >= 2 (got %lld)", (long long)ref_stride);
  if (!(radius >= 0.f) || radius > 3.0e38f) return fail(GCDF_EINVAL, "radius must be finite and >= 0");
  DeviceGuard guard(ctx->device);
  hipError_t e = gcdf::launch_partition_count(ref, N, ref_stride, points, Np, ctx->net.in_dim == gcdf::kInDimSphere,
                                              radius, offsets, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GCDF_OK : hip_fail(e, "gcdf_partition_count launch");
}

gcdf_status gcdf_partition_fill(gcdf_ctx* ctx, const float* ref, int64_t N, int64_t ref_stride, const float* points,
                                int64_t Np, float radius, const int64_t* offsets, int32_t* idx, int64_t capacity,
                                void* stream) {
  if (!ctx) return fail(GCDF_EINVAL, "ctx is NULL");
  if (!ref || !points || !offsets) return fail(GCDF_EINVAL, "ref/points/offsets pointer is NULL");
  if (N <= 0 || Np <= 0) return fail(GCDF_EINVAL, "N and Np must be positive (N=%lld, Np=%lld)", (long long)N, (long long)Np);
  if (Np > INT32_MAX) return fail(GCDF_EINVAL, "Np=%lld exceeds 2^31-1", (long long)Np);
  if (ref_stride < 2) return fail(GCDF_EINVAL, "ref_stride must be >= 2 (got %lld)", (long long)ref_stride);
  if (!(radius >= 0.f) || radius > 3.0e38f) return fail(GCDF_EINVAL, "radius must be finite and >= 0");
  if (capacity < 0 || (capacity > 0 && !idx)) return fail(GCDF_EINVAL, "idx is NULL or capacity < 0");
  if (capacity == 0) return GCDF_OK;
  DeviceGuard guard(ctx->device);
  hipError_t e = gcdf::launch_partition_fill(ref, N, ref_stride, points, Np, ctx->net.in_dim == gcdf::kInDimSphere,
                                             radius, offsets, idx, capacity, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GCDF_OK : hip_fail(e, "gcdf_partition_fill launch");
}

gcdf_status gcdf_eval_grad_csr(gcdf_ctx* ctx, const float* knots, int64_t N, const float* points, int64_t Np,
                               const int64_t* offsets, const int32_t* idx, int64_t total, float* c, float* J,
                               void* stream) {
  gcdf_status st = check_query(ctx, knots, N, points, Np);
  if (st != GCDF_OK) return st;
  if (Np > INT32_MAX) return fail(GCDF_EINVAL, "Np=%lld exceeds 2^31-1", (long long)Np);
  if (total < 0) return fail(GCDF_EINVAL, "total must be >= 0");
  if (total > INT64_MAX / 9) return fail(GCDF_EINVAL, "total*9 overflows int64");
  if (!c) return fail(GCDF_EINVAL, "c is NULL");
  if (total == 0) return GCDF_OK;
  if (!offsets || !idx) return fail(GCDF_EINVAL, "offsets/idx pointer is NULL");
  if (N > ctx->cfg.max_knots)
    return fail(GCDF_EINVAL, "N=%lld exceeds max_knots=%lld", (long long)N, (long long)ctx->cfg.max_knots);
  DeviceGuard guard(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // each knot's rows run as gathered dense tiles (one knot per tile): the arm term
  // of the input layer is computed once per tile, as in the dense query
  hipError_t e = gcdf::launch_csr_tile_offsets(offsets, N, ctx->tile_off, s);
  gcdf::Job job{};
  job.knots = knots;
  job.points = points;
  job.K = N;
  job.Np = Np;
  job.tile_off = ctx->tile_off;
  job.row_off = offsets;
  job.pgather = idx;
  job.ntiles_bound = (total + gcdf::kTileQ - 1) / gcdf::kTileQ + N;
  job.d = c;
  job.J = J;
  if (e == hipSuccess) e = gcdf::launch_fused(ctx->net, job, false, J != nullptr, ctx->num_cu, s);
  return e == hipSuccess ? GCDF_OK : hip_fail(e, "gcdf_eval_grad_csr launch");
}

gcdf_status gcdf_jacobian_pattern(gcdf_ctx* ctx, const int64_t* offsets, int64_t N, int64_t total, int32_t state_dim,
                                  int64_t col0, int64_t* row_ptr, int32_t* cols, void* stream) {
  if (!ctx) return fail(GCDF_EINVAL, "ctx is NULL");
  if (!offsets || !row_ptr || (total > 0 && !cols)) return fail(GCDF_EINVAL, "offsets/row_ptr/cols pointer is NULL");
  if (N <= 0 || total < 0) return fail(GCDF_EINVAL, "N must be positive and total >= 0");
  if (state_dim < 9) return fail(GCDF_EINVAL, "state_dim must be >= 9 (got %d)", state_dim);
  if (col0 < 0 || col0 > INT32_MAX - (int64_t)state_dim * N)
    return fail(GCDF_EINVAL, "columns col0 + state_dim*N exceed 2^31-1");
  if (total >= ((int64_t)1 << 38)) return fail(GCDF_EINVAL, "total=%lld too large", (long long)total);
  DeviceGuard guard(ctx->device);
  hipError_t e = gcdf::launch_jacobian_pattern(offsets, N, total, state_dim, col0, row_ptr, cols,
                                               static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GCDF_OK : hip_fail(e, "gcdf_jacobian_pattern launch");
}

namespace {
gcdf_status project_common(gcdf_ctx* ctx, const float* knots, int64_t N, int64_t Np, const int64_t* offsets,
                           int64_t rows, const float* f, const float* J, const float* m_diag, float* qz, float* eik,
                           void* stream) {
  if (!ctx) return fail(GCDF_EINVAL, "ctx is NULL");
  if (!knots || !f || !J || !m_diag) return fail(GCDF_EINVAL, "knots/f/J/m_diag pointer is NULL");
  if (!qz && !eik) return fail(GCDF_EINVAL, "no output requested");
  gcdf::Minv9 minv{};
  for (int c = 0; c < 9; ++c) {
    if (!(m_diag[c] > 0.f) || m_diag[c] > 3.0e38f) return fail(GCDF_EINVAL, "m_diag[%d] must be finite and > 0", c);
    minv.v[c] = 1.0f / m_diag[c];
  }
  if (rows == 0) return GCDF_OK;
  DeviceGuard guard(ctx->device);
  hipError_t e = gcdf::launch_project(knots, N, Np, offsets, rows, f, J, minv, qz, eik,
                                      static_cast<hipStream_t>(stream));
  return e == hipSuccess ? GCDF_OK : hip_fail(e, "gcdf_project launch");
}
}  // namespace

gcdf_status gcdf_project(gcdf_ctx* ctx, const float* knots, int64_t K, int64_t Np, const float* d, const float* J,
                         const float* m_diag, float* qz, float* eik, void* stream) {
  if (K <= 0 || Np <= 0) return fail(GCDF_EINVAL, "K and Np must be positive (K=%lld, Np=%lld)", (long long)K, (long long)Np);
  if (K > INT64_MAX / 9 / Np) return fail(GCDF_EINVAL, "K*Np*9 overflows int64");
  if (K * Np >= ((int64_t)1 << 38)) return fail(GCDF_EINVAL, "K*Np too large");
  return project_common(ctx, knots, K, Np, nullptr, K * Np, d, J, m_diag, qz, eik, stream);
}

gcdf_status gcdf_project_csr(gcdf_ctx* ctx, const float* knots, int64_t N, const int64_t* offsets, int64_t total,
                             const float* c, const float* J, const float* m_diag, float* qz, float* eik,
                             void* stream) {
  if (N <= 0 || total < 0) return fail(GCDF_EINVAL, "N must be positive and total >= 0");
  if (total >= ((int64_t)1 << 38)) return fail(GCDF_EINVAL, "total=%lld too large", (long long)total);
  if (total > 0 && !offsets) return fail(GCDF_EINVAL, "offsets is NULL");
  return project_common(ctx, knots, N, 1, offsets, total, c, J, m_diag, qz, eik, stream);
}

gcdf_status gcdf_submit(gcdf_ctx* ctx, const gcdf_request* req, uint64_t* ticket) {
  if (!ctx || !req || !ticket) return fail(GCDF_EINVAL, "NULL argument to gcdf_submit");
  if (!ctx->server) return fail(GCDF_EINVAL, "serving is disabled (serve_mem_budget == 0)");
  return gcdf::server_submit(ctx->server, req, ticket);
}

gcdf_status gcdf_poll(gcdf_ctx* ctx, uint64_t ticket) {
  if (!ctx) return fail(GCDF_EINVAL, "ctx is NULL");
  if (!ctx->server) return fail(GCDF_EINVAL, "serving is disabled (serve_mem_budget == 0)");
  if (gcdf_status st = take_overflow(ctx); st != GCDF_OK) return st;
  return gcdf::server_poll(ctx->server, ticket);
}

}  // extern "C"

namespace gcdf {
gcdf_status set_error(gcdf_status st, const char* msg) {
  g_err = msg;
  return st;
}
}  // namespace gcdf
