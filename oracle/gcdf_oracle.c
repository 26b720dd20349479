/*
 * FP64 CPU oracle for the batched neural GCDF query.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code with the HIP library.
 *
 * What it computes (Li et al., "Fast and Safe Trajectory Optimization for
 * Mobile Manipulators With Neural Configuration Space Distance Field"):
 *
 *   For a knot configuration q = (x, y, yaw, a1..a6) and a world point p,
 *   - the point is expressed in the base frame of the knot (Sec. III-B:
 *     base translation handled by moving obstacle points into the base
 *     frame; Sec. IV-A: the base pose is treated as the origin and the
 *     obstacle points are biased into that frame).  The base x axis points
 *     at angle yaw (the base kinematics in eq. optimization-in-general).
 *     p' = R(yaw)^T (p - t), t = (x, y, 0).
 *   - the distance network (Sec. III-C, "Network Architecture"): an MLP on
 *     the concatenation [p', arm joints] with SiLU hidden layers,
 *     d = w_out . h_L + b_out, h_l = SiLU(W_l h_{l-1} + b_l), h_0 = [p', a].
 *   - the derivative of d with respect to the full configuration, by the
 *     chain rule through the point coordinates (Sec. III-B), ordered
 *     (x, y, yaw, a1..a6): the gradient the constraint Jacobian stacks
 *     row by row (Sec. IV-A, dense gradient matrix).
 *   - per knot, the minimum over points and the lowest index attaining it
 *     (the constraint f - delta >= 0 of eq. optimization-in-general holds
 *     for all points iff it holds for the minimum).
 *
 * Everything is the plain definition: double precision, straight loops, no
 * blocking and no library calls beyond exp().  SiLU(z) = z * s(z) with
 * s(z) = 1 / (1 + exp(-z)); its derivative s(z) * (1 + z * (1 - s(z))).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IN_DIM 9

typedef struct {
    int width;
    int depth;            /* number of SiLU hidden layers */
    const float* mat[16]; /* mat[l]: out x in, row-major; mat[depth] is the 1 x width output row */
    const float* bias[16];
} net_t;

/* Parse the little-endian weight blob: "GCDF", version 1, in_dim 9, width,
 * depth, 3 reserved u32, then float32 W1, b1, ..., W_depth, b_depth, w_out, b_out. */
static int parse_blob(const void* blob, size_t bytes, net_t* n) {
    const uint32_t* h = (const uint32_t*)blob;
    if (bytes < 32 || memcmp(blob, "GCDF", 4) != 0) return -1;
    if (h[1] != 1 || h[2] != IN_DIM) return -1;
    n->width = (int)h[3];
    n->depth = (int)h[4];
    if (n->width <= 0 || n->depth < 1 || n->depth > 15) return -1;
    const float* f = (const float*)((const char*)blob + 32);
    size_t used = 0;
    for (int l = 0; l <= n->depth; ++l) {
        int fi = (l == 0) ? IN_DIM : n->width;
        int fo = (l == n->depth) ? 1 : n->width;
        n->mat[l] = f + used;
        used += (size_t)fo * fi;
        n->bias[l] = f + used;
        used += (size_t)fo;
    }
    if (32 + used * 4 != bytes) return -1;
    return 0;
}

static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }
static double silu(double z) { return z * sigmoid(z); }
static double silu_prime(double z) {
    double s = sigmoid(z);
    return s * (1.0 + z * (1.0 - s));
}

/* Base-frame transform of one point for one knot (p' = R(yaw)^T (p - t)). */
static void to_base_frame(const double* q, const double* p, double pp[3]) {
    double c = cos(q[2]), s = sin(q[2]);
    double ux = p[0] - q[0];
    double uy = p[1] - q[1];
    pp[0] = c * ux + s * uy;
    pp[1] = -s * ux + c * uy;
    pp[2] = p[2];
}

/* Chain rule from the network-input gradient e = dd/d[p', a] to the
 * configuration gradient J = dd/d(x, y, yaw, a1..a6).
 *   dp'x/dx = -c, dp'y/dx =  s;  dp'x/dy = -s, dp'y/dy = -c;
 *   dp'x/dyaw = p'y, dp'y/dyaw = -p'x;  the arm part passes through. */
static void chain_rule(const double* q, const double pp[3], const double e[IN_DIM], double J[IN_DIM]) {
    double c = cos(q[2]), s = sin(q[2]);
    J[0] = -(c * e[0] - s * e[1]);
    J[1] = -(s * e[0] + c * e[1]);
    J[2] = e[0] * pp[1] - e[1] * pp[0];
    for (int i = 3; i < IN_DIM; ++i) J[i] = e[i];
}

/* Network value at input v; if e != NULL also dd/dv by reverse mode.
 * z and h must each hold depth*width doubles (pre-activations and SiLU
 * outputs per hidden layer), g and t width doubles each. */
static double mlp(const net_t* n, const double v[IN_DIM], double* e, double* z, double* h, double* g, double* t) {
    const int W = n->width, L = n->depth;
    /* forward: z_1 = W_1 v + b_1; z_l = W_l h_{l-1} + b_l; h_l = SiLU(z_l) */
    for (int r = 0; r < W; ++r) {
        double acc = n->bias[0][r];
        for (int c = 0; c < IN_DIM; ++c) acc += (double)n->mat[0][r * IN_DIM + c] * v[c];
        z[r] = acc;
        h[r] = silu(acc);
    }
    for (int l = 1; l < L; ++l) {
        const double* hin = h + (size_t)(l - 1) * W;
        double* zo = z + (size_t)l * W;
        double* ho = h + (size_t)l * W;
        for (int r = 0; r < W; ++r) {
            double acc = n->bias[l][r];
            for (int c = 0; c < W; ++c) acc += (double)n->mat[l][(size_t)r * W + c] * hin[c];
            zo[r] = acc;
            ho[r] = silu(acc);
        }
    }
    const double* zl = z + (size_t)(L - 1) * W;
    const double* hl = h + (size_t)(L - 1) * W;
    double d = n->bias[L][0];
    for (int c = 0; c < W; ++c) d += (double)n->mat[L][c] * hl[c];
    if (!e) return d;
    /* reverse: g_L = w_out * SiLU'(z_L); g_{l-1} = (W_l^T g_l) * SiLU'(z_{l-1}); e = W_1^T g_1 */
    for (int c = 0; c < W; ++c) g[c] = (double)n->mat[L][c] * silu_prime(zl[c]);
    for (int l = L - 1; l >= 1; --l) {
        const double* zin = z + (size_t)(l - 1) * W;
        for (int c = 0; c < W; ++c) {
            double acc = 0.0;
            for (int r = 0; r < W; ++r) acc += (double)n->mat[l][(size_t)r * W + c] * g[r];
            t[c] = acc * silu_prime(zin[c]);
        }
        memcpy(g, t, sizeof(double) * W);
    }
    for (int c = 0; c < IN_DIM; ++c) {
        double acc = 0.0;
        for (int r = 0; r < W; ++r) acc += (double)n->mat[0][r * IN_DIM + c] * g[r];
        e[c] = acc;
    }
    return d;
}

/* ------------------------------------------------------------------------ */
/* exported                                                                  */
/* ------------------------------------------------------------------------ */

/* Number of OpenMP threads a call with nthreads (0 = default) will use. */
int gcdf_ref_threads(int nthreads) {
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* Base-frame transform for n (knot, point) pairs taken row by row. */
void gcdf_ref_transform(const double* knots, const double* points, int64_t n, double* pprime) {
    for (int64_t i = 0; i < n; ++i) to_base_frame(knots + 9 * i, points + 3 * i, pprime + 3 * i);
}

/* Chain rule for n pairs: e (n x 9, base-frame input gradient) -> J (n x 9). */
void gcdf_ref_chain(const double* knots, const double* points, const double* e, int64_t n, double* J) {
    for (int64_t i = 0; i < n; ++i) {
        double pp[3];
        to_base_frame(knots + 9 * i, points + 3 * i, pp);
        chain_rule(knots + 9 * i, pp, e + 9 * i, J + 9 * i);
    }
}

/* Network value (and input gradient if e != NULL) at n inputs v (n x 9). */
int gcdf_ref_mlp(const void* blob, size_t bytes, const double* v, int64_t n, double* d, double* e, int nthreads) {
    net_t net;
    if (parse_blob(blob, bytes, &net)) return -1;
    const int W = net.width;
#pragma omp parallel num_threads(gcdf_ref_threads(nthreads))
    {
        double* z = (double*)malloc(sizeof(double) * (size_t)W * (2 * net.depth + 2));
        double* h = z + (size_t)W * net.depth;
        double* g = h + (size_t)W * net.depth;
        double* t = g + W;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) d[i] = mlp(&net, v + 9 * i, e ? e + 9 * i : NULL, z, h, g, t);
        free(z);
    }
    return 0;
}

/* All (knot, point) pairs, knot-major: d[k*Np + j], J[(k*Np + j)*9 + c] (J may be NULL).
 * Inputs in double precision. */
int gcdf_ref_eval_grad_f64(const void* blob, size_t bytes, const double* knots, int64_t K,
                           const double* points, int64_t Np, double* d, double* J, int nthreads) {
    net_t net;
    if (parse_blob(blob, bytes, &net)) return -1;
    const int W = net.width;
#pragma omp parallel num_threads(gcdf_ref_threads(nthreads))
    {
        double* z = (double*)malloc(sizeof(double) * (size_t)W * (2 * net.depth + 2));
        double* h = z + (size_t)W * net.depth;
        double* g = h + (size_t)W * net.depth;
        double* t = g + W;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < K * Np; ++i) {
            const double* q = knots + 9 * (i / Np);
            const double* p = points + 3 * (i % Np);
            double v[IN_DIM], e[IN_DIM];
            to_base_frame(q, p, v);
            for (int c = 3; c < IN_DIM; ++c) v[c] = q[c];
            d[i] = mlp(&net, v, J ? e : NULL, z, h, g, t);
            if (J) chain_rule(q, v, e, J + 9 * i);
        }
        free(z);
    }
    return 0;
}

static double* widen(const float* a, int64_t n) {
    double* o = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) o[i] = (double)a[i];
    return o;
}

/* Same with the library's float32 inputs, widened exactly to double. */
int gcdf_ref_eval_grad(const void* blob, size_t bytes, const float* knots, int64_t K,
                       const float* points, int64_t Np, double* d, double* J, int nthreads) {
    double* kd = widen(knots, 9 * K);
    double* pd = widen(points, 3 * Np);
    int rc = gcdf_ref_eval_grad_f64(blob, bytes, kd, K, pd, Np, d, J, nthreads);
    free(kd);
    free(pd);
    return rc;
}

/* Same as gcdf_ref_eval_grad on a list of (knot index, point index) pairs. */
int gcdf_ref_eval_pairs(const void* blob, size_t bytes, const float* knots, const float* points,
                        const int64_t* kidx, const int64_t* pidx, int64_t n, double* d, double* J, int nthreads) {
    net_t net;
    if (parse_blob(blob, bytes, &net)) return -1;
    const int W = net.width;
#pragma omp parallel num_threads(gcdf_ref_threads(nthreads))
    {
        double* z = (double*)malloc(sizeof(double) * (size_t)W * (2 * net.depth + 2));
        double* h = z + (size_t)W * net.depth;
        double* g = h + (size_t)W * net.depth;
        double* t = g + W;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double q[IN_DIM], p[3];
            for (int c = 0; c < IN_DIM; ++c) q[c] = (double)knots[9 * kidx[i] + c];
            for (int c = 0; c < 3; ++c) p[c] = (double)points[3 * pidx[i] + c];
            double v[IN_DIM], e[IN_DIM];
            to_base_frame(q, p, v);
            for (int c = 3; c < IN_DIM; ++c) v[c] = q[c];
            d[i] = mlp(&net, v, J ? e : NULL, z, h, g, t);
            if (J) chain_rule(q, v, e, J + 9 * i);
        }
        free(z);
    }
    return 0;
}

/* Per-knot minimum over the points of d (K x Np) and the lowest index attaining it. */
void gcdf_ref_knot_min(const double* d, int64_t K, int64_t Np, double* dmin, int32_t* argmin) {
    for (int64_t k = 0; k < K; ++k) {
        double best = d[k * Np];
        int32_t bj = 0;
        for (int64_t j = 1; j < Np; ++j)
            if (d[k * Np + j] < best) { best = d[k * Np + j]; bj = (int32_t)j; }
        dmin[k] = best;
        argmin[k] = bj;
    }
}

/* Mean-squared-error training loss over n samples (knot i, point i) with
 * targets y, and its gradient with respect to every weight and bias.
 * grad is laid out exactly like the blob's float payload (W1, b1, ...,
 * w_out, b_out).  Straight sequential sums over the samples.
 * Returns the loss; NaN on a malformed blob. */
double gcdf_ref_mse_grad(const void* blob, size_t bytes, const double* knots, const double* points,
                         const double* y, int64_t n, double* grad) {
    net_t net;
    if (parse_blob(blob, bytes, &net)) return NAN;
    const int W = net.width, L = net.depth;
    /* offsets of each parameter array inside grad */
    size_t off_m[16], off_b[16], total = 0;
    for (int l = 0; l <= L; ++l) {
        int fi = (l == 0) ? IN_DIM : W;
        int fo = (l == L) ? 1 : W;
        off_m[l] = total;
        total += (size_t)fo * fi;
        off_b[l] = total;
        total += (size_t)fo;
    }
    memset(grad, 0, sizeof(double) * total);
    double* z = (double*)malloc(sizeof(double) * (size_t)W * L);
    double* h = (double*)malloc(sizeof(double) * (size_t)W * L);
    double* g = (double*)malloc(sizeof(double) * W);
    double* t = (double*)malloc(sizeof(double) * W);
    double loss = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double* q = knots + 9 * i;
        double v[IN_DIM];
        to_base_frame(q, points + 3 * i, v);
        for (int c = 3; c < IN_DIM; ++c) v[c] = q[c];
        double d = mlp(&net, v, NULL, z, h, g, t);
        double r = d - y[i];
        loss += r * r / (double)n;
        double dd = 2.0 * r / (double)n; /* dL/dd */
        /* output layer */
        const double* zl = z + (size_t)(L - 1) * W;
        const double* hl = h + (size_t)(L - 1) * W;
        grad[off_b[L]] += dd;
        for (int c = 0; c < W; ++c) grad[off_m[L] + c] += dd * hl[c];
        for (int c = 0; c < W; ++c) g[c] = dd * (double)net.mat[L][c] * silu_prime(zl[c]);
        /* hidden layers l = L-1 .. 1 (0-based mats), g holds dL/dz_{l+1} */
        for (int l = L - 1; l >= 1; --l) {
            const double* zin = z + (size_t)(l - 1) * W;
            const double* hin = h + (size_t)(l - 1) * W;
            for (int r2 = 0; r2 < W; ++r2) {
                grad[off_b[l] + r2] += g[r2];
                for (int c = 0; c < W; ++c) grad[off_m[l] + (size_t)r2 * W + c] += g[r2] * hin[c];
            }
            for (int c = 0; c < W; ++c) {
                double acc = 0.0;
                for (int r2 = 0; r2 < W; ++r2) acc += (double)net.mat[l][(size_t)r2 * W + c] * g[r2];
                t[c] = acc * silu_prime(zin[c]);
            }
            memcpy(g, t, sizeof(double) * W);
        }
        /* input layer */
        for (int r2 = 0; r2 < W; ++r2) {
            grad[off_b[0] + r2] += g[r2];
            for (int c = 0; c < IN_DIM; ++c) grad[off_m[0] + (size_t)r2 * IN_DIM + c] += g[r2] * v[c];
        }
    }
    free(z);
    free(h);
    free(g);
    free(t);
    return loss;
}
