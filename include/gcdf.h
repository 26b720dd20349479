/*
 * libgcdf: batched neural GCDF queries on MI355X (gfx950).
 *
 * The query is the one a trajectory optimiser makes for every (knot, obstacle
 * point) pair of the GCDF collision constraints f(p_j, q_i) - delta >= 0
 * (eq. optimization-in-general, Sec. IV-A of Li et al., "Fast and Safe
 * Trajectory Optimization for Mobile Manipulators With Neural Configuration
 * Space Distance Field"):
 *
 *   1. express point p_j in the base frame of knot q_i = (x, y, yaw, a1..a6):
 *      p' = R(yaw)^T (p - (x, y, 0)) (Sec. III-B; Sec. IV-A treats the base
 *      pose as the origin and biases the obstacle points into that frame);
 *   2. evaluate the distance network on [p', a1..a6] (Sec. III-C network):
 *      an MLP 9 -> width x depth -> 1 with SiLU hidden activations;
 *   3. differentiate it with respect to the full configuration (x, y, yaw,
 *      a1..a6) by reverse mode through the network and the chain rule through
 *      the point coordinates (Sec. III-B);
 *   4. reduce by minimum over the points of each knot.
 *
 * Results are knot-major as the constraint vector c_gcdf and its dense
 * gradient matrix are stacked (eq. cdf_constraints_vector, Sec. IV-A):
 *   d[i*Np + j]          distance for knot i, point j
 *   J[(i*Np + j)*9 + c]  d d / d q_i[c], c in (x, y, yaw, a1..a6)
 *
 * Sphere obstacles (the primitive-aware GCDF over (q, p, r) of the closing
 * discussion, Sec. VII): a context created from a blob with in_dim = 10 takes
 * obstacles as spheres float32[Np][4] = (x, y, z, r) and evaluates the
 * network on [p', r, a1..a6]; the radius is not moved by the base-frame
 * transform, and J is still the gradient over the 9 configuration
 * coordinates.  Every query, partition and serving call below then reads
 * 4 floats per obstacle where it says "points".
 *
 * Memory: every knots/points/output pointer is DEVICE memory owned by the
 * caller (e.g. a torch tensor).  knots is float32[K][9] (x, y, yaw, a1..a6),
 * points is float32[Np][3] world coordinates (float32[Np][4] spheres for an
 * in_dim 10 network).  The library never frees caller
 * memory.  Calls are asynchronous on the caller's HIP stream (hipStream_t
 * passed as void*; NULL = the null stream) and never synchronise the host;
 * the caller synchronises the stream before reading outputs.
 *
 * Errors: every call returns a gcdf_status and never aborts or throws across
 * the ABI.  The message for the last failed call on the calling thread is
 * available from gcdf_last_error().  Device faults surface as GCDF_EDEVICE at
 * the call that observes them.
 *
 * Threads: the query calls on one context may be issued by one thread at a
 * time and on one stream at a time (they share the context's per-knot
 * workspace); gcdf_submit / gcdf_poll are thread-safe.
 */
#ifndef GCDF_H
#define GCDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GCDF_OK = 0,
    GCDF_PENDING = 1, /* gcdf_poll: request not finished yet */
    GCDF_EINVAL = 2,  /* bad argument (message says which) */
    GCDF_ENOMEM = 3,  /* device allocation failed, or a request can never fit the serving budget */
    GCDF_EDEVICE = 4, /* HIP runtime error */
    GCDF_EBUSY = 5,   /* serving queue full */
    GCDF_ERANGE = 6   /* GCDF_BF16X2_F16: an earlier query's reverse sweep overflowed FP16 (see below) */
} gcdf_status;

typedef enum {
    GCDF_FP32 = 0,   /* all layers in FP32 (matrix cores, FP32 in and out) */
    GCDF_BF16 = 1,   /* hidden layers on BF16 matrix cores, FP32 accumulate (fast; ~1e-2 error) */
    GCDF_BF16X2 = 2, /* as BF16 with each activation split into hi + lo BF16 parts (FP32-class error) */
    GCDF_BF16X2_F16 = 3 /* forward layers as BF16X2; the reverse sweep multiplies FP16 back-propagated
                         * values (scaled by 2^6) by the BF16-rounded transposed weights held as FP16:
                         * one product instead of two per reverse fragment, d as BF16X2, Jacobian
                         * relative error a few 1e-3 (under 1e-2).  Hidden weights must satisfy
                         * |w| < 65408; values back-propagated beyond ~1e3 in magnitude
                         * overflow FP16.  A query whose d is finite but whose J is not
                         * sets a flag of the context; the next query call (gcdf_eval,
                         * gcdf_eval_grad, gcdf_knot_min, gcdf_query, gcdf_eval_grad_csr)
                         * or gcdf_poll that sees it clears it and returns GCDF_ERANGE
                         * without doing anything else (a poll's ticket stays valid).
                         * The flag is written by the device: synchronise the stream of
                         * the overflowing call before relying on the next call to
                         * report it. */
} gcdf_precision;

typedef struct {
    int32_t width;          /* hidden width: 256 or 512 */
    int32_t depth;          /* hidden SiLU layers: 4 */
    int32_t precision;      /* gcdf_precision */
    int32_t device;         /* HIP device ordinal; -1 = the calling thread's current device */
    int64_t max_knots;      /* capacity of the per-knot minimum workspace; 0 = 1<<20 */
    size_t serve_mem_budget;/* device bytes the serving loop may reserve for requests; 0 = serving off */
    int32_t serve_slots;    /* max requests in flight in the serving loop; 0 = 64 */
    int32_t reserved[7];
} gcdf_config;

typedef struct gcdf_ctx gcdf_ctx;

/* Create a context from a weight blob (host memory, copied; the caller keeps
 * ownership).  Blob format, little-endian: "GCDF", u32 version = 1,
 * u32 in_dim = 9 (points, input [p', a]) or 10 (spheres, input [p', r, a]),
 * u32 width, u32 depth, 3 reserved u32, then float32 arrays
 * W1 (width x in_dim), b1, W2 (width x width), b2, ..., W_depth, b_depth,
 * w_out (1 x width), b_out, each matrix row-major (out x in) -- the network of
 * Sec. III-C.  For the BF16 precisions W2..W_depth are rounded to BF16
 * (round-to-nearest-even); blobs whose hidden matrices already lie on the BF16
 * grid are multiplied exactly (GCDF_BF16X2_F16: also in FP16, for |w| >= 2^-17;
 * smaller weights round by at most 2^-25).  Errors: EINVAL (bad config or blob:
 * width not 256/512, depth != 4, in_dim not 9 or 10, size mismatch; for
 * GCDF_BF16X2_F16 a hidden weight with |w| >= 65408 or not finite), ENOMEM,
 * EDEVICE. */
gcdf_status gcdf_create(const gcdf_config* cfg, const void* weight_blob, size_t blob_bytes, gcdf_ctx** out);

/* Destroy a context: waits for in-flight serving requests, then frees every
 * device buffer the library owns.  NULL is ignored. */
void gcdf_destroy(gcdf_ctx* ctx);

/* Message of the last failed call on the calling thread (library-owned, valid
 * until the next failing call on that thread).  ctx may be NULL. */
const char* gcdf_last_error(const gcdf_ctx* ctx);

/* Distance d (float32[K][Np]) for all pairs (steps 1-2).
 * EINVAL: NULL pointer, K <= 0, Np <= 0, or K*Np*9 overflowing int64. */
gcdf_status gcdf_eval(gcdf_ctx* ctx, const float* knots, int64_t K, const float* points, int64_t Np,
                      float* d, void* stream);

/* Distance d (float32[K][Np]) and configuration gradient J (float32[K][Np][9])
 * for all pairs (steps 1-3).  Errors as gcdf_eval. */
gcdf_status gcdf_eval_grad(gcdf_ctx* ctx, const float* knots, int64_t K, const float* points, int64_t Np,
                           float* d, float* J, void* stream);

/* Per-knot minimum over points (step 4) without materialising d or J:
 * dmin (float32[K]) = min_j d[i][j], argmin (int32[K]) = lowest j attaining it,
 * and, if Jmin != NULL, Jmin (float32[K][9]) = J[i][argmin[i]].  Values are
 * bitwise equal to the minimum over gcdf_eval_grad's d on the same inputs.
 * EINVAL also when K > cfg.max_knots or Np > 2^31 - 1. */
gcdf_status gcdf_knot_min(gcdf_ctx* ctx, const float* knots, int64_t K, const float* points, int64_t Np,
                          float* dmin, int32_t* argmin, float* Jmin, void* stream);

/* All four steps in one pass: every non-NULL output among d (float32[K][Np]),
 * J (float32[K][Np][9]) and dmin/argmin (float32[K], int32[K], given together)
 * comes from the same fused launch; Jmin (float32[K][9], needs dmin/argmin)
 * adds a pass over the K argmin pairs.  Results are bitwise equal to those of
 * gcdf_eval_grad and gcdf_knot_min.  EINVAL if no output is requested, if only
 * one of dmin/argmin is given, or as gcdf_knot_min for the minimum. */
gcdf_status gcdf_query(gcdf_ctx* ctx, const float* knots, int64_t K, const float* points, int64_t Np,
                       float* d, float* J, float* dmin, int32_t* argmin, float* Jmin, void* stream);

/* gcdf_query for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same outputs, bitwise, from the same kernels, but the per-knot minimum keys
 * live in a fixed array of 65,536 keys (512 KiB) that the library holds on
 * each GPU until the process ends, instead of the context's workspace.  The
 * call allocates nothing.  Every call on one GPU (from any context) shares that
 * GPU's array, which keeps the last call's contents; the minimum clears the
 * keys it uses before each launch, so consecutive calls are independent, but
 * calls that overlap on one GPU (other streams or threads) race and may
 * return wrong minima.  Arguments, layout and ownership as gcdf_query.
 * EINVAL as gcdf_query, and when the minimum is requested with K > 65,536;
 * EDEVICE if the array has no device address on the context's device. */
gcdf_status gcdf_query_noalloc(gcdf_ctx* ctx, const float* knots, int64_t K, const float* points, int64_t Np,
                               float* d, float* J, float* dmin, int32_t* argmin, float* Jmin, void* stream);

/* ------------------------------------------------------------------------ */
/* Obstacle partitions and the sparse constraint Jacobian.                   */
/*                                                                           */
/* Sec. IV-A of the paper: the obstacle points are split into N overlapping  */
/* partitions I_{M,i}, one per time step, holding the points within a range  */
/* of that step's reference base position; the GCDF constraints are stacked  */
/* knot by knot into c_gcdf (length m_1 + ... + m_N), and each knot's dense  */
/* gradient rows are placed by the projection P_i at the columns of q_i      */
/* inside the state x_i = [q_i, v_i] of the (sum m_i) x 2Nn Jacobian.        */
/* Partitions are in CSR form: offsets int64[N+1] (offsets[0] = 0), idx      */
/* int32[offsets[N]] with the points of partition i, ascending, at           */
/* idx[offsets[i] .. offsets[i+1]-1].  All arrays are device memory owned by */
/* the caller; the calls are asynchronous on `stream`.                       */
/* ------------------------------------------------------------------------ */

/* Partition sizes.  Reference base position i is (ref[i*ref_stride],
 * ref[i*ref_stride+1]) (ref_stride = 9 takes the (x, y) of a knots array);
 * point j (points float32[Np][3]) is in partition i when
 * dx*dx + dy*dy <= radius*radius, evaluated in float32 with every product and
 * the sum rounded (no fused multiply-add), dx = px - x_i, dy = py - y_i.
 * For a sphere context (points float32[Np][4], (x, y, z, s)) the sphere is in
 * partition i when it reaches into the disc: radius*radius is replaced by
 * t*t with t = radius + s, rounded the same way.
 * Writes offsets int64[N+1].  The caller reads offsets[N] (the total) to size
 * idx.  EINVAL: NULL pointers, N <= 0, Np <= 0 or > 2^31 - 1, ref_stride < 2,
 * radius negative or not finite. */
gcdf_status gcdf_partition_count(gcdf_ctx* ctx, const float* ref, int64_t N, int64_t ref_stride,
                                 const float* points, int64_t Np, float radius, int64_t* offsets,
                                 void* stream);

/* Partition members: idx[offsets[i] + k] = the k-th point (ascending index)
 * of partition i, for offsets from gcdf_partition_count with the same
 * arguments.  Positions >= capacity are not written (compare offsets[N] with
 * capacity).  EINVAL as gcdf_partition_count, or idx NULL with capacity > 0. */
gcdf_status gcdf_partition_fill(gcdf_ctx* ctx, const float* ref, int64_t N, int64_t ref_stride,
                                const float* points, int64_t Np, float radius, const int64_t* offsets,
                                int32_t* idx, int64_t capacity, void* stream);

/* The stacked constraint vector and its dense gradient rows over CSR
 * partitions: row r (0 <= r < total) pairs knot i, the last i with
 * offsets[i] <= r (empty partitions are skipped), with point idx[r];
 * c[r] (float32[total]) = d of that pair and, if J != NULL, J[r][0..8]
 * (float32[total][9]) = its configuration gradient, bitwise equal to the
 * entries gcdf_eval_grad gives for the same pair.  total = offsets[N]; idx
 * holds total entries.  A point index outside [0, Np) gives NaN in its row.
 * total == 0 is a no-op.  EINVAL as gcdf_eval_grad, or Np > 2^31 - 1, c NULL,
 * total < 0. */
gcdf_status gcdf_eval_grad_csr(gcdf_ctx* ctx, const float* knots, int64_t N, const float* points, int64_t Np,
                               const int64_t* offsets, const int32_t* idx, int64_t total, float* c, float* J,
                               void* stream);

/* Sparsity pattern of the (total) x (col0 + N*state_dim) constraint Jacobian
 * in CSR form whose values array is J of gcdf_eval_grad_csr as it stands:
 * row_ptr int64[total+1] with row_ptr[r] = 9r, and cols int32[9*total] with
 * cols[9r + c] = col0 + state_dim*i + c for the knot i of row r (state_dim = 18
 * for x_i = [q_i, v_i]).  EINVAL: NULL pointers, N <= 0, total < 0,
 * state_dim < 9, col0 < 0 or col0 + state_dim*N > 2^31 - 1. */
gcdf_status gcdf_jacobian_pattern(gcdf_ctx* ctx, const int64_t* offsets, int64_t N, int64_t total,
                                  int32_t state_dim, int64_t col0, int64_t* row_ptr, int32_t* cols,
                                  void* stream);

/* Single-step projection onto the zero set and the weighted eikonal norm
 * (Theorem 1): for a pair with distance f and configuration gradient J,
 *   qz = q - f * M^{-1} J,    eik = |J|_{M^{-1}} = sqrt(sum_c J_c^2 / m_c),
 * with q the pair's knot and M = diag(m_diag), m_diag a HOST float[9] of finite
 * positive weights (for a true GCDF, eik = 1 and qz lies on the zero set).
 * Rows follow gcdf_eval_grad's layout: d float32[K][Np], J float32[K][Np][9],
 * qz float32[K][Np][9], eik float32[K][Np]; either output may be NULL (not
 * both).  Computed in float32 (q_c - f * (J_c * (1/m_c))).  EINVAL: NULL
 * inputs, no output, K or Np <= 0, a weight not finite and positive. */
gcdf_status gcdf_project(gcdf_ctx* ctx, const float* knots, int64_t K, int64_t Np, const float* d,
                         const float* J, const float* m_diag, float* qz, float* eik, void* stream);

/* The same over the stacked CSR rows of gcdf_eval_grad_csr (c float32[total],
 * J float32[total][9], qz float32[total][9], eik float32[total]); row r uses
 * the knot of its partition.  Bitwise equal to gcdf_project's entries for the
 * same pairs.  total == 0 is a no-op. */
gcdf_status gcdf_project_csr(gcdf_ctx* ctx, const float* knots, int64_t N, const int64_t* offsets,
                             int64_t total, const float* c, const float* J, const float* m_diag, float* qz,
                             float* eik, void* stream);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of trajectory-optimisation requests.         */
/* ------------------------------------------------------------------------ */

/* One request: the pairs of K knots x Np points, with any subset of outputs
 * (NULL = not wanted; at least one of d, J, dmin must be given).  All pointers
 * are device memory owned by the caller and must stay valid until gcdf_poll
 * returns GCDF_OK (or an error) for the request's ticket.  The outputs are
 * bitwise equal to those of gcdf_query on the same inputs, whatever else the
 * serving loop runs at the same time. */
typedef struct {
    const float* knots;
    int64_t K;
    const float* points;
    int64_t Np;
    float* d;        /* float32[K][Np] */
    float* J;        /* float32[K][Np][9] */
    float* dmin;     /* float32[K] */
    int32_t* argmin; /* int32[K]  (given together with dmin) */
    float* Jmin;     /* float32[K][9]: J at (knot i, point argmin[i]); needs dmin/argmin */
} gcdf_request;

/* Queue a request and return at once with its ticket.  The serving loop
 * admits queued requests while in-flight slots and the memory budget allow,
 * and runs all admitted requests' tiles in shared persistent launches on the
 * library's own stream, which is not ordered after any caller stream: every
 * write to the request's input and output buffers must have completed before
 * the call (synchronise the streams that produce or initialise them), and the
 * buffers must not be touched again until gcdf_poll returns GCDF_OK.
 * ENOMEM: the request alone exceeds serve_mem_budget.  EBUSY: too many queued.
 * EINVAL: bad request (NULL knots/points, K or Np <= 0, no output, only one of
 * dmin/argmin, Jmin without them) or serving disabled (serve_mem_budget == 0). */
gcdf_status gcdf_submit(gcdf_ctx* ctx, const gcdf_request* req, uint64_t* ticket);

/* GCDF_OK when the ticket's outputs are complete and visible to the caller's
 * later stream work, GCDF_PENDING while not, EINVAL for an unknown ticket
 * (including one already reported complete), EDEVICE on a device error. */
gcdf_status gcdf_poll(gcdf_ctx* ctx, uint64_t ticket);

/* ------------------------------------------------------------------------ */
/* Training form: gradients of the distance network's weights.               */
/* ------------------------------------------------------------------------ */

/* Sample i of a batch is the pair (knots[i], points[i]): one knot and one
 * point per sample, the network evaluated on [R(yaw)^T (p - t), a] as in the
 * query (the network of Sec. III-C, trained on (point, configuration) pairs).
 * Training covers the point network (in_dim 9) only. */
typedef struct gcdf_trainer gcdf_trainer;

/* Number of float32 parameters of a width-W, depth-4 network: the weight-blob
 * payload W1 (W x 9), b1, W2, b2, W3, b3, W4, b4, w_out (1 x W), b_out. */
int64_t gcdf_param_count(int32_t width);

/* Create a trainer for width 256 with precision GCDF_FP32 or GCDF_BF16 (hidden
 * layers on BF16 matrix cores from FP32 master weights) for batches up to
 * max_batch samples.  Owns its device workspace (activation and gradient
 * dumps, ~W * max_batch * 16 bytes for BF16).  EINVAL / ENOMEM / EDEVICE. */
gcdf_status gcdf_trainer_create(int32_t width, int32_t precision, int32_t device, int64_t max_batch,
                                gcdf_trainer** out);
void gcdf_trainer_destroy(gcdf_trainer* tr);

/* d[i] = network distance of sample i (device float32[B]).  params: device
 * float32[gcdf_param_count(W)] (FP32 master weights, read at the call). */
gcdf_status gcdf_train_forward(gcdf_trainer* tr, const float* params, const float* knots, const float* points,
                               int64_t B, float* d, void* stream);

/* grad_params (device float32[gcdf_param_count(W)], overwritten) =
 * sum_i grad_d[i] * d d_i / d params: the reverse mode of the network, seeded
 * with the per-sample loss gradient.  Deterministic (fixed reduction order).
 * reuse_packed != 0 asserts that params (same pointer) has not changed since
 * the last forward or backward call on this trainer, whose packed copy of the
 * weights is then reused; with 0 (or another pointer) the weights are packed
 * again. */
gcdf_status gcdf_train_backward(gcdf_trainer* tr, const float* params, const float* knots, const float* points,
                                int64_t B, const float* grad_d, float* grad_params, int32_t reuse_packed,
                                void* stream);

/* Training with the mean squared error fused in: L = (1/B) sum_i (d_i - y_i)^2
 * over the samples (knot i, point i), with d the network distance, and its weight
 * gradient, from one training-mode pass (no separate forward).  Each 64-sample
 * tile finishes d before its reverse sweep and seeds the sweep with
 * dL/dd_i = 2 (d_i - y_i) / B; otherwise as gcdf_train_backward (deterministic;
 * the weights are packed from params unless reuse_packed is 1 and params is the
 * pointer this trainer last packed or updated with gcdf_train_adam_step, and was
 * not changed since).  target: device float32[B];
 * loss: device float32[1]; grad_params: device, overwritten; d: device
 * float32[B] for the distances, or NULL.  EINVAL: NULL tr, params, knots,
 * points, target, loss or grad_params, or B outside [1, max_batch].  The
 * trainer's buffers make concurrent calls on one trainer race. */
gcdf_status gcdf_train_mse(gcdf_trainer* tr, const float* params, const float* knots, const float* points, int64_t B,
                           const float* target, float* loss, float* grad_params, float* d, int32_t reuse_packed,
                           void* stream);

/* The training loss of Table I (Sec. III-C) over the samples (knot i, point i)
 * and its weight gradient.  With F the network distance and J = dF/dq the
 * configuration gradient of the query (chain rule through the base frame):
 *   L_dist = mean (F - fstar)^2,  L_grad = mean (1 - cos(J, Jstar))^2,
 *   L_eikonal = mean (|J|_{M^-1} - 1)^2,  L_tension = mean |J|^2,
 * total = sum_k lambda[k] L_k (lambda = (5, 0.1, 0.01, 0.01) in Sec. V-A).
 * fstar float32[B], Jstar float32[B][9] (device); m_diag (9 weights of M) and
 * lambda (4) are HOST float arrays.  losses: device float32[5] = the four terms
 * and the total; grad_params (device, overwritten) = d total / d params.  The
 * gradient is exact reverse mode through the query and its Jacobian (a tangent
 * pass along A^T dL/dJ, then the adjoint of both programs), deterministic.  FP32
 * trainers only (EINVAL otherwise); the first call allocates a workspace of about
 * 16 W max_batch floats plus per-CU scratch (ENOMEM if that fails). */
gcdf_status gcdf_train_table1(gcdf_trainer* tr, const float* params, const float* knots, const float* points,
                              int64_t B, const float* fstar, const float* Jstar, const float* m_diag,
                              const float* lambda, float* losses, float* grad_params, void* stream);

/* gcdf_adam_step over a trainer's flat parameter vector (gcdf_param_count(width)
 * floats; grad, m and v in the same layout) that also packs the updated weights
 * into the trainer, in one launch, so that the next gcdf_train_mse or
 * gcdf_train_backward with reuse_packed = 1 and the same params pointer needs no
 * packing.  Same arithmetic and EINVAL cases as gcdf_adam_step (NULL tr too). */
gcdf_status gcdf_train_adam_step(gcdf_trainer* tr, float* params, const float* grad, float* m, float* v, float lr,
                                 float beta1, float beta2, float eps, int64_t step, void* stream);

/* One Adam step (the optimiser of the paper's training, Sec. V-A) over n device
 * floats, in torch.optim.Adam's arithmetic (no weight decay, no amsgrad):
 *   m = beta1 m + (1 - beta1) g;  v = beta2 v + (1 - beta2) g^2;
 *   p -= (lr / (1 - beta1^step)) * m / (sqrt(v) / sqrt(1 - beta2^step) + eps).
 * params, m, v are updated in place (m and v start at zero); step counts from 1.
 * EINVAL: NULL pointers, n < 0, step < 1, lr or eps not finite, beta outside [0, 1). */
gcdf_status gcdf_adam_step(float* params, const float* grad, float* m, float* v, int64_t n, float lr, float beta1,
                           float beta2, float eps, int64_t step, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GCDF_H */
