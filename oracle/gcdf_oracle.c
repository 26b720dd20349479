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
 *   - the primitive-aware variant of the closing discussion (Sec. VII): the
 *     obstacle is a sphere (p, r) and the network reads (q, p, r).  Input
 *     width 10, in the order [p', r, a]: the radius is a property of the
 *     obstacle, unchanged by the rigid base-frame motion, so it passes
 *     through the transform, and the configuration gradient is still the
 *     chain rule through p' alone.  A blob's in_dim (9 or 10) selects the
 *     variant; obstacles then hold 3 or 4 floats (x, y, z[, r]).
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

#define IN_DIM 9   /* configuration coordinates (x, y, yaw, a1..a6) */
#define MAX_IN 10  /* network inputs: 9, or 10 with an obstacle radius */

typedef struct {
    int in_dim;           /* 9: [p', a];  10: [p', r, a] */
    int width;
    int depth;            /* number of SiLU hidden layers */
    const float* mat[16]; /* mat[l]: out x in, row-major; mat[depth] is the 1 x width output row */
    const float* bias[16];
} net_t;

/* Parse the little-endian weight blob: "GCDF", version 1, in_dim (9 or 10),
 * width, depth, 3 reserved u32, then float32 W1, b1, ..., W_depth, b_depth,
 * w_out, b_out. */
static int parse_blob(const void* blob, size_t bytes, net_t* n) {
    const uint32_t* h = (const uint32_t*)blob;
    if (bytes < 32 || memcmp(blob, "GCDF", 4) != 0) return -1;
    if (h[1] != 1 || (h[2] != IN_DIM && h[2] != MAX_IN)) return -1;
    n->in_dim = (int)h[2];
    n->width = (int)h[3];
    n->depth = (int)h[4];
    if (n->width <= 0 || n->depth < 1 || n->depth > 15) return -1;
    const float* f = (const float*)((const char*)blob + 32);
    size_t used = 0;
    for (int l = 0; l <= n->depth; ++l) {
        int fi = (l == 0) ? n->in_dim : n->width;
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

/* Chain rule from the network-input gradient e = dd/d[p', (r,) a] (in_dim
 * entries) to the configuration gradient J = dd/d(x, y, yaw, a1..a6).
 *   dp'x/dx = -c, dp'y/dx =  s;  dp'x/dy = -s, dp'y/dy = -c;
 *   dp'x/dyaw = p'y, dp'y/dyaw = -p'x;  the arm part passes through; the
 *   radius does not depend on the configuration. */
static void chain_rule(const double* q, const double pp[3], const double* e, int in_dim, double J[IN_DIM]) {
    double c = cos(q[2]), s = sin(q[2]);
    J[0] = -(c * e[0] - s * e[1]);
    J[1] = -(s * e[0] + c * e[1]);
    J[2] = e[0] * pp[1] - e[1] * pp[0];
    for (int i = 3; i < IN_DIM; ++i) J[i] = e[in_dim - IN_DIM + i];
}

/* Network input for knot q and obstacle p (x, y, z, and r when in_dim is 10):
 * v = [p', (r,) a]; pp receives p'. */
static void network_input(int in_dim, const double* q, const double* p, double* v, double pp[3]) {
    to_base_frame(q, p, pp);
    for (int c = 0; c < 3; ++c) v[c] = pp[c];
    if (in_dim == MAX_IN) v[3] = p[3];
    for (int c = 3; c < IN_DIM; ++c) v[in_dim - IN_DIM + c] = q[c];
}

/* Network value at input v (in_dim entries); if e != NULL also dd/dv by reverse mode.
 * z and h must each hold depth*width doubles (pre-activations and SiLU
 * outputs per hidden layer), g and t width doubles each. */
static double mlp(const net_t* n, const double* v, double* e, double* z, double* h, double* g, double* t) {
    const int W = n->width, L = n->depth, NI = n->in_dim;
    /* forward: z_1 = W_1 v + b_1; z_l = W_l h_{l-1} + b_l; h_l = SiLU(z_l) */
    for (int r = 0; r < W; ++r) {
        double acc = n->bias[0][r];
        for (int c = 0; c < NI; ++c) acc += (double)n->mat[0][r * NI + c] * v[c];
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
    for (int c = 0; c < NI; ++c) {
        double acc = 0.0;
        for (int r = 0; r < W; ++r) acc += (double)n->mat[0][r * NI + c] * g[r];
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
        chain_rule(knots + 9 * i, pp, e + 9 * i, IN_DIM, J + 9 * i);
    }
}

/* Network input width of a blob (9 or 10), or -1 if malformed. */
int gcdf_ref_in_dim(const void* blob, size_t bytes) {
    net_t net;
    return parse_blob(blob, bytes, &net) ? -1 : net.in_dim;
}

/* Network value (and input gradient if e != NULL) at n inputs v (n x in_dim). */
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
        for (int64_t i = 0; i < n; ++i)
            d[i] = mlp(&net, v + (size_t)net.in_dim * i, e ? e + (size_t)net.in_dim * i : NULL, z, h, g, t);
        free(z);
    }
    return 0;
}

/* All (knot, obstacle) pairs, knot-major: d[k*Np + j], J[(k*Np + j)*9 + c] (J may be NULL).
 * Inputs in double precision; obstacles hold in_dim - 6 values (x, y, z[, r]). */
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
            const double* p = points + (size_t)(net.in_dim - 6) * (i % Np);
            double v[MAX_IN], e[MAX_IN], pp[3];
            network_input(net.in_dim, q, p, v, pp);
            d[i] = mlp(&net, v, J ? e : NULL, z, h, g, t);
            if (J) chain_rule(q, pp, e, net.in_dim, J + 9 * i);
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
    const int in_dim = gcdf_ref_in_dim(blob, bytes);
    if (in_dim < 0) return -1;
    double* kd = widen(knots, 9 * K);
    double* pd = widen(points, (int64_t)(in_dim - 6) * Np);
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
        const int pd = net.in_dim - 6;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double q[IN_DIM], p[4];
            for (int c = 0; c < IN_DIM; ++c) q[c] = (double)knots[9 * kidx[i] + c];
            for (int c = 0; c < pd; ++c) p[c] = (double)points[pd * pidx[i] + c];
            double v[MAX_IN], e[MAX_IN], pp[3];
            network_input(net.in_dim, q, p, v, pp);
            d[i] = mlp(&net, v, J ? e : NULL, z, h, g, t);
            if (J) chain_rule(q, pp, e, net.in_dim, J + 9 * i);
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
    if (parse_blob(blob, bytes, &net) || net.in_dim != IN_DIM) return NAN;
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

/* ------------------------------------------------------------------------ */
/* Training loss of Table I (Sec. III-C) and its weight gradient.            */
/*                                                                          */
/* Per sample i with prediction f, configuration gradient J = dF/dq (the    */
/* query's chain rule) and targets f*, J*:                                   */
/*   L_dist    = (f - f*)^2                                                  */
/*   L_grad    = (1 - cos(J, J*))^2                                          */
/*   L_eikonal = (|J|_{M^-1} - 1)^2,  |J|_{M^-1} = sqrt(sum_c J_c^2 / m_c)   */
/*   L_tension = |J|^2                                                       */
/* each averaged over the samples; total = sum_k lambda_k L_k (eq. total_lo, */
/* weights of Sec. V-A).  The eikonal and tension terms act on the          */
/* prediction (the table's hat convention is read as "prediction").         */
/*                                                                          */
/* Gradient: the loss depends on the weights through f and through          */
/* J = A e, e = d f / d v (A: the chain rule, independent of the weights).  */
/* With fbar = dL/df and u = A^T dL/dJ, dL/dW = fbar df/dW + d(u . e)/dW,   */
/* and u . e is the forward-mode derivative of f along the input direction   */
/* u.  So: forward, reverse for e, tangent pass along u, then reverse mode  */
/* through the primal and the tangent program together:                     */
/*   hbar_L = fbar w_out,  tbar_L = w_out                                     */
/*   per layer: zdot_bar = tbar * s'(z) (= the reverse sweep's g),           */
/*              zbar = hbar * s'(z) + tbar * s''(z) * zdot,                  */
/*              dW += zbar h_prev^T + zdot_bar hdot_prev^T, db += zbar,      */
/*              hbar_prev = W^T zbar, tbar_prev = W^T zdot_bar;              */
/*   input layer: dW_1 += zbar v^T + zdot_bar u^T, db_1 += zbar.             */
/* s = SiLU, s'' = sigma (1 - sigma) (2 + z (1 - 2 sigma)).                 */
/* ------------------------------------------------------------------------ */
static double silu_second(double z) {
    double s = sigmoid(z);
    return s * (1.0 - s) * (2.0 + z * (1.0 - 2.0 * s));
}

double gcdf_ref_table1_grad(const void* blob, size_t bytes, const double* knots, const double* points,
                            const double* fstar, const double* Jstar, const double* m_diag, const double* lambda,
                            int64_t n, double* losses, double* grad) {
    net_t net;
    if (parse_blob(blob, bytes, &net) || net.in_dim != IN_DIM) return NAN;
    const int W = net.width, L = net.depth;
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
    for (int k = 0; k < 4; ++k) losses[k] = 0.0;
    /* per layer (1..L, stored 0-based): z, h, zdot, hdot, g (= zdot_bar), r (= tbar) */
    double* z = (double*)malloc(sizeof(double) * (size_t)W * L);
    double* h = (double*)malloc(sizeof(double) * (size_t)W * L);
    double* zd = (double*)malloc(sizeof(double) * (size_t)W * L);
    double* hd = (double*)malloc(sizeof(double) * (size_t)W * L);
    double* g = (double*)malloc(sizeof(double) * (size_t)W * L);
    double* r = (double*)malloc(sizeof(double) * (size_t)W * L);
    double* hbar = (double*)malloc(sizeof(double) * W);
    double* zbar = (double*)malloc(sizeof(double) * W);
    const double inv_n = 1.0 / (double)n;
    for (int64_t i = 0; i < n; ++i) {
        const double* q = knots + 9 * i;
        double v[IN_DIM];
        to_base_frame(q, points + 3 * i, v);
        for (int c = 3; c < IN_DIM; ++c) v[c] = q[c];
        /* forward */
        for (int l = 0; l < L; ++l) {
            const int fi = (l == 0) ? IN_DIM : W;
            const double* in = (l == 0) ? v : h + (size_t)(l - 1) * W;
            for (int o = 0; o < W; ++o) {
                double acc = net.bias[l][o];
                for (int c = 0; c < fi; ++c) acc += (double)net.mat[l][(size_t)o * fi + c] * in[c];
                z[(size_t)l * W + o] = acc;
                h[(size_t)l * W + o] = silu(acc);
            }
        }
        double f = net.bias[L][0];
        for (int c = 0; c < W; ++c) f += (double)net.mat[L][c] * h[(size_t)(L - 1) * W + c];
        /* reverse for e = df/dv: r_L = w_out, g_l = r_l * s'(z_l), r_{l-1} = W_l^T g_l */
        for (int c = 0; c < W; ++c) r[(size_t)(L - 1) * W + c] = (double)net.mat[L][c];
        for (int l = L - 1; l >= 0; --l) {
            for (int c = 0; c < W; ++c) g[(size_t)l * W + c] = r[(size_t)l * W + c] * silu_prime(z[(size_t)l * W + c]);
            if (l == 0) break;
            for (int c = 0; c < W; ++c) {
                double acc = 0.0;
                for (int o = 0; o < W; ++o) acc += (double)net.mat[l][(size_t)o * W + c] * g[(size_t)l * W + o];
                r[(size_t)(l - 1) * W + c] = acc;
            }
        }
        double e[IN_DIM], J[IN_DIM];
        for (int c = 0; c < IN_DIM; ++c) {
            double acc = 0.0;
            for (int o = 0; o < W; ++o) acc += (double)net.mat[0][(size_t)o * IN_DIM + c] * g[o];
            e[c] = acc;
        }
        chain_rule(q, v, e, IN_DIM, J);
        /* losses and their derivatives in f and J */
        const double* Js = Jstar + 9 * i;
        double nJ2 = 0.0, nJs2 = 0.0, dot = 0.0, nm2 = 0.0;
        for (int c = 0; c < IN_DIM; ++c) {
            nJ2 += J[c] * J[c];
            nJs2 += Js[c] * Js[c];
            dot += J[c] * Js[c];
            nm2 += J[c] * J[c] / m_diag[c];
        }
        const double nJ = sqrt(nJ2), nJs = sqrt(nJs2), nm = sqrt(nm2);
        const double cosv = dot / (nJ * nJs);
        const double rd = f - fstar[i];
        losses[0] += rd * rd * inv_n;
        losses[1] += (1.0 - cosv) * (1.0 - cosv) * inv_n;
        losses[2] += (nm - 1.0) * (nm - 1.0) * inv_n;
        losses[3] += nJ2 * inv_n;
        const double fbar = lambda[0] * 2.0 * rd * inv_n;
        double Jbar[IN_DIM];
        for (int c = 0; c < IN_DIM; ++c) {
            const double dcos = Js[c] / (nJ * nJs) - cosv * J[c] / nJ2;
            Jbar[c] = inv_n * (lambda[1] * (-2.0 * (1.0 - cosv) * dcos) +
                               lambda[2] * (2.0 * (nm - 1.0) * J[c] / (m_diag[c] * nm)) + lambda[3] * 2.0 * J[c]);
        }
        /* u = A^T Jbar (transpose of the chain rule) */
        const double cy = cos(q[2]), sy = sin(q[2]);
        double u[IN_DIM];
        u[0] = -cy * Jbar[0] - sy * Jbar[1] + v[1] * Jbar[2];
        u[1] = sy * Jbar[0] - cy * Jbar[1] - v[0] * Jbar[2];
        u[2] = 0.0;
        for (int c = 3; c < IN_DIM; ++c) u[c] = Jbar[c];
        /* tangent pass along u */
        for (int l = 0; l < L; ++l) {
            const int fi = (l == 0) ? IN_DIM : W;
            const double* in = (l == 0) ? u : hd + (size_t)(l - 1) * W;
            for (int o = 0; o < W; ++o) {
                double acc = 0.0;
                for (int c = 0; c < fi; ++c) acc += (double)net.mat[l][(size_t)o * fi + c] * in[c];
                zd[(size_t)l * W + o] = acc;
                hd[(size_t)l * W + o] = silu_prime(z[(size_t)l * W + o]) * acc;
            }
        }
        /* reverse through primal and tangent; seeds fbar (for f) and 1 (for u . e) */
        grad[off_b[L]] += fbar;
        for (int c = 0; c < W; ++c) {
            grad[off_m[L] + c] += fbar * h[(size_t)(L - 1) * W + c] + hd[(size_t)(L - 1) * W + c];
            hbar[c] = fbar * (double)net.mat[L][c];
        }
        for (int l = L - 1; l >= 0; --l) {
            const double* zl = z + (size_t)l * W;
            for (int c = 0; c < W; ++c)
                zbar[c] = hbar[c] * silu_prime(zl[c]) + r[(size_t)l * W + c] * silu_second(zl[c]) * zd[(size_t)l * W + c];
            const double* gl = g + (size_t)l * W; /* zdot_bar */
            const int fi = (l == 0) ? IN_DIM : W;
            const double* hin = (l == 0) ? v : h + (size_t)(l - 1) * W;
            const double* hdin = (l == 0) ? u : hd + (size_t)(l - 1) * W;
            for (int o = 0; o < W; ++o) {
                grad[off_b[l] + o] += zbar[o];
                for (int c = 0; c < fi; ++c) grad[off_m[l] + (size_t)o * fi + c] += zbar[o] * hin[c] + gl[o] * hdin[c];
            }
            if (l == 0) break;
            for (int c = 0; c < W; ++c) {
                double acc = 0.0;
                for (int o = 0; o < W; ++o) acc += (double)net.mat[l][(size_t)o * W + c] * zbar[o];
                hbar[c] = acc;
            }
        }
    }
    free(z); free(h); free(zd); free(hd); free(g); free(r); free(hbar); free(zbar);
    return lambda[0] * losses[0] + lambda[1] * losses[1] + lambda[2] * losses[2] + lambda[3] * losses[3];
}
