/*
 * FP64 reference renderer for the object-aware Gaussian rasterization hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product path never does.  It shares no code,
 * header, table or constant generator with the HIP library.
 *
 * What it computes (plain definitions, no tiling, no sorting tricks):
 *   - Each Gaussian is the "same shape" primitive as the object quadric of
 *     Sec. III-A, Eq. (2): mean mu, rotation R(q), scale s = exp(l).
 *   - Image formation is the alpha blending of colour and depth the method
 *     renders with (Sec. III-D, text around Eq. (12)), in the EWA-splatting form
 *     inherited from 3D Gaussian Splatting: project the mean, push the 3D
 *     covariance through the perspective Jacobian, and blend front to back.
 *   - The per-object instance channel ins_k (Eq. (12)) is read as the
 *     transmittance-weighted sum of the blend weights of object k's Gaussians,
 *     so that sum_k ins_k + T_final = 1 and ins_k lies in [0,1].
 *   - Every Gaussian is evaluated at every listed pixel: the pixel's result is
 *     defined by the contribution rule, not by which tiles a splat touches.
 *
 * Contribution rule at a pixel sample s = (u + 1/2, v + 1/2):
 *   d = s - m, Q = A dx^2 + 2 B dx dy + C dy^2 with (A,B,C) the conic (inverse
 *   of the 2D covariance).  The Gaussian contributes iff Q <= q_max and
 *   alpha = min(alpha_max, o * exp(-Q/2)) >= alpha_min.  Blending runs over the
 *   visible Gaussians in order of increasing camera depth (ties by index); it
 *   stops before the Gaussian that would bring the transmittance below t_min.
 *
 * The backward pass is the analytic adjoint of that forward with the set of
 * blended Gaussians held fixed, chained through the projection to the stored
 * parameters (mean, log-scale, quaternion, opacity logit, colour).
 *
 * Parameter layout: params[14][n] (row-major, row r holds component r of every
 * Gaussian): rows 0-2 mean, 3-5 log-scale, 6-9 quaternion (w,x,y,z),
 * 10 opacity logit, 11-13 colour.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double R[9];      /* world -> camera rotation, row-major */
    double t[3];      /* world -> camera translation */
    double fx, fy, cx, cy;
    int32_t width, height;
} ocam;

typedef struct {
    double z_near, dilation, q_max, alpha_min, alpha_max, t_min;
    double bg[3];
} ocfg;

/* Per-Gaussian projected quantities. */
typedef struct {
    int visible;
    double x, y, z;          /* camera-frame mean */
    double mx, my;           /* 2D mean in pixels */
    double s00, s01, s11;    /* 2D covariance incl. dilation */
    double A, B, C;          /* conic = inverse 2D covariance */
    double ex, ey;           /* 3-sigma extents */
    double o;                /* opacity */
    double R[9];             /* rotation from the normalised quaternion */
    double s[3];             /* scales */
    double qn[4];            /* normalised quaternion */
    double qnorm;
    double S3[9];            /* world covariance */
    double ux, uy;           /* x/z, y/z as used in the Jacobian (limited) */
    int ux_clamped, uy_clamped;
} oproj;

static void clamp_ratio(double u, double lim, double* out, int* clamped) {
    *clamped = 0;
    *out = u;
    if (u > lim) { *out = lim; *clamped = 1; }
    if (u < -lim) { *out = -lim; *clamped = 1; }
}

#define NPAR 14

static void quat_to_rot(const double q[4], double R[9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* Projection of one Gaussian (EWA splatting). */
static void project_one(const double* params, int64_t n, int64_t i, const ocam* cam,
                        const ocfg* cfg, oproj* p) {
    double mu[3], l[3], q[4];
    for (int k = 0; k < 3; ++k) mu[k] = params[k * n + i];
    for (int k = 0; k < 3; ++k) l[k] = params[(3 + k) * n + i];
    for (int k = 0; k < 4; ++k) q[k] = params[(6 + k) * n + i];
    double eta = params[10 * n + i];
    memset(p, 0, sizeof(*p));
    const double* W = cam->R;
    p->x = W[0] * mu[0] + W[1] * mu[1] + W[2] * mu[2] + cam->t[0];
    p->y = W[3] * mu[0] + W[4] * mu[1] + W[5] * mu[2] + cam->t[1];
    p->z = W[6] * mu[0] + W[7] * mu[1] + W[8] * mu[2] + cam->t[2];
    p->o = 1.0 / (1.0 + exp(-eta));
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    p->qnorm = qn;
    for (int k = 0; k < 4; ++k) p->qn[k] = q[k] / qn;
    quat_to_rot(p->qn, p->R);
    for (int k = 0; k < 3; ++k) p->s[k] = exp(l[k]);
    /* Sigma3 = R diag(s^2) R^T */
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += p->R[a * 3 + k] * p->s[k] * p->s[k] * p->R[b * 3 + k];
            p->S3[a * 3 + b] = acc;
        }
    if (!(p->z > cfg->z_near)) { p->visible = 0; return; }
    double z = p->z;
    p->mx = cam->fx * p->x / z + cam->cx;
    p->my = cam->fy * p->y / z + cam->cy;
    /* J = d(pixel)/d(camera point), evaluated with x/z and y/z limited to 1.3
     * times the half field of view (the linearisation is meaningless far
     * outside the view); T2 = J W */
    clamp_ratio(p->x / z, 1.3 * 0.5 * cam->width / cam->fx, &p->ux, &p->ux_clamped);
    clamp_ratio(p->y / z, 1.3 * 0.5 * cam->height / cam->fy, &p->uy, &p->uy_clamped);
    double J[6] = {cam->fx / z, 0, -cam->fx * p->ux / z,
                   0, cam->fy / z, -cam->fy * p->uy / z};
    double T2[6];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += J[a * 3 + k] * W[k * 3 + b];
            T2[a * 3 + b] = acc;
        }
    double S2[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k)
                for (int m = 0; m < 3; ++m) acc += T2[a * 3 + k] * p->S3[k * 3 + m] * T2[b * 3 + m];
            S2[a * 2 + b] = acc;
        }
    p->s00 = S2[0] + cfg->dilation;
    p->s01 = 0.5 * (S2[1] + S2[2]);
    p->s11 = S2[3] + cfg->dilation;
    double det = p->s00 * p->s11 - p->s01 * p->s01;
    if (!(det > 0)) { p->visible = 0; return; }
    p->A = p->s11 / det;
    p->B = -p->s01 / det;
    p->C = p->s00 / det;
    p->ex = 3.0 * sqrt(p->s00);
    p->ey = 3.0 * sqrt(p->s11);
    p->visible = 1;
}

/* out[n][16]: visible, x, y, z, mx, my, s00, s01, s11, A, B, C, ex, ey, o, pad */
void oracle_project(int64_t n, const double* params, const ocam* cam, const ocfg* cfg, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        oproj p;
        project_one(params, n, i, cam, cfg, &p);
        double* o = out + i * 16;
        o[0] = p.visible; o[1] = p.x; o[2] = p.y; o[3] = p.z; o[4] = p.mx; o[5] = p.my;
        o[6] = p.s00; o[7] = p.s01; o[8] = p.s11; o[9] = p.A; o[10] = p.B; o[11] = p.C;
        o[12] = p.ex; o[13] = p.ey; o[14] = p.o; o[15] = 0;
    }
}

/* Depth order of the visible Gaussians: by z ascending, ties by index. */
static const oproj* g_sort_proj;
static int cmp_depth(const void* a, const void* b) {
    int64_t i = *(const int64_t*)a, j = *(const int64_t*)b;
    double zi = g_sort_proj[i].z, zj = g_sort_proj[j].z;
    if (zi < zj) return -1;
    if (zi > zj) return 1;
    return (i < j) ? -1 : (i > j);
}

static int64_t build_order(int64_t n, const oproj* pr, int64_t* order) {
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (pr[i].visible) order[m++] = i;
    g_sort_proj = pr;
    qsort(order, (size_t)m, sizeof(int64_t), cmp_depth);
    return m;
}

static double rel_margin(double v, double thr) { return fabs(v - thr) / fabs(thr); }

/*
 * Forward render of the listed pixels (pix[j] = v * W + u).
 * Outputs (per listed pixel j): C[3][npix], D[npix], Tf[npix], P[K][npix] (may be NULL),
 * last[npix] (index of the last blended Gaussian or -1), nblend[npix],
 * margin[npix] = smallest relative distance of any threshold decision taken
 * at the pixel (Q vs q_max, alpha vs alpha_min, T' vs t_min) to its threshold,
 * margin_clamp[npix] = smallest relative distance of an unclamped alpha to
 * alpha_max (it changes gradients, not values), and depth_gap[npix] = smallest
 * relative depth difference between consecutive contributors (the order of two
 * contributors at almost the same depth is a discrete decision too; its scale
 * is the resolution of the depth values, not the threshold band).
 */
int oracle_render(int64_t n, const double* params, const int32_t* ids, const ocam* cam,
                  const ocfg* cfg, int K, int64_t npix, const int64_t* pix,
                  double* C, double* D, double* Tf, double* P, int64_t* last, int32_t* nblend,
                  double* margin, double* margin_clamp, double* depth_gap) {
    oproj* pr = (oproj*)malloc(sizeof(oproj) * (size_t)(n > 0 ? n : 1));
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!pr || !order) { free(pr); free(order); return -1; }
    for (int64_t i = 0; i < n; ++i) project_one(params, n, i, cam, cfg, &pr[i]);
    int64_t m = build_order(n, pr, order);
    int W = cam->width;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < npix; ++j) {
        double su = (double)(pix[j] % W) + 0.5, sv = (double)(pix[j] / W) + 0.5;
        double T = 1.0, c[3] = {0, 0, 0}, d = 0, mg = INFINITY, mgc = INFINITY, gapmin = INFINITY;
        double prev_z = -INFINITY;
        int64_t lst = -1;
        int32_t nb = 0;
        if (P) for (int k = 0; k < K; ++k) P[(int64_t)k * npix + j] = 0;
        for (int64_t r = 0; r < m; ++r) {
            const oproj* g = &pr[order[r]];
            double dx = su - g->mx, dy = sv - g->my;
            double Q = g->A * dx * dx + 2.0 * g->B * dx * dy + g->C * dy * dy;
            double mq = rel_margin(Q, cfg->q_max);
            if (mq < mg) mg = mq;
            if (Q > cfg->q_max) continue;
            double araw = g->o * exp(-0.5 * Q);
            double mc = rel_margin(araw, cfg->alpha_max);
            if (mc < mgc) mgc = mc;
            double a = araw < cfg->alpha_max ? araw : cfg->alpha_max;
            double ma = rel_margin(a, cfg->alpha_min);
            if (ma < mg) mg = ma;
            if (a < cfg->alpha_min) continue;
            /* a contributor: check the depth gap to the previous contributor */
            if (prev_z > -INFINITY) {
                double gap = fabs(g->z - prev_z) / fabs(g->z);
                if (gap < gapmin) gapmin = gap;
            }
            prev_z = g->z;
            double Tn = T * (1.0 - a);
            double mt = rel_margin(Tn, cfg->t_min);
            if (mt < mg) mg = mt;
            if (Tn < cfg->t_min) break;
            double w = a * T;
            int64_t gi = order[r];
            for (int k = 0; k < 3; ++k) c[k] += w * params[(11 + k) * n + gi];
            d += w * g->z;
            if (P) {
                int id = ids[gi];
                if (id >= 0 && id < K) P[(int64_t)id * npix + j] += w;
            }
            T = Tn;
            lst = gi;
            ++nb;
        }
        for (int k = 0; k < 3; ++k) C[(int64_t)k * npix + j] = c[k] + T * cfg->bg[k];
        D[j] = d;
        Tf[j] = T;
        if (last) last[j] = lst;
        if (nblend) nblend[j] = nb;
        if (margin) margin[j] = mg;
        if (margin_clamp) margin_clamp[j] = mgc;
        if (depth_gap) depth_gap[j] = gapmin;
    }
    free(pr);
    free(order);
    return 0;
}

/* d R(q) / d q_c for the normalised quaternion (w,x,y,z); out[c][9]. */
static void drot_dq(const double q[4], double dR[4][9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    /* R00 = 1-2(y^2+z^2) */
    double d[4][9] = {
        /* d/dw */ {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0},
        /* d/dx */ {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x},
        /* d/dy */ {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y},
        /* d/dz */ {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0},
    };
    memcpy(dR, d, sizeof(d));
}

/*
 * Chain rule from the 2D quantities of one Gaussian to its parameters.
 * g2d = {dmx, dmy, dA, dB, dC, dopacity, dr, dg, db, dz}; grads[14][n] accumulated.
 */
static void project_backward_one(const double* params, int64_t n, int64_t i, const ocam* cam,
                                 const oproj* p, const double g2d[10], double* grads) {
    const double* W = cam->R;
    double fx = cam->fx, fy = cam->fy, x = p->x, y = p->y, z = p->z;
    double a = p->s00, b = p->s01, c = p->s11;
    double det = a * c - b * b, det2 = det * det;
    double dA = g2d[2], dB = g2d[3], dC = g2d[4];
    /* conic A = c/det, B = -b/det, C = a/det with det = a c - b^2 */
    double da = dA * (-c * c / det2) + dB * (b * c / det2) + dC * (1.0 / det - a * c / det2);
    double db = dA * (2 * b * c / det2) + dB * (-1.0 / det - 2 * b * b / det2) + dC * (2 * a * b / det2);
    double dc = dA * (1.0 / det - a * c / det2) + dB * (a * b / det2) + dC * (-a * a / det2);
    /* symmetric gradient of Sigma2 (b appears in both off-diagonal slots) */
    double G2[4] = {da, 0.5 * db, 0.5 * db, dc};
    double J[6] = {fx / z, 0, -fx * p->ux / z, 0, fy / z, -fy * p->uy / z};
    double T2[6];
    for (int r = 0; r < 2; ++r)
        for (int s = 0; s < 3; ++s) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += J[r * 3 + k] * W[k * 3 + s];
            T2[r * 3 + s] = acc;
        }
    /* dSigma3 = T2^T G2 T2 ; dT2 = 2 G2 T2 Sigma3 */
    double G3[9];
    for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) {
            double acc = 0;
            for (int u = 0; u < 2; ++u)
                for (int v = 0; v < 2; ++v) acc += T2[u * 3 + r] * G2[u * 2 + v] * T2[v * 3 + s];
            G3[r * 3 + s] = acc;
        }
    double T2S[6], dT2[6];
    for (int r = 0; r < 2; ++r)
        for (int s = 0; s < 3; ++s) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += T2[r * 3 + k] * p->S3[k * 3 + s];
            T2S[r * 3 + s] = acc;
        }
    for (int r = 0; r < 2; ++r)
        for (int s = 0; s < 3; ++s) {
            double acc = 0;
            for (int u = 0; u < 2; ++u) acc += G2[r * 2 + u] * T2S[u * 3 + s];
            dT2[r * 3 + s] = 2.0 * acc;
        }
    /* dJ = dT2 W^T */
    double dJ[6];
    for (int r = 0; r < 2; ++r)
        for (int s = 0; s < 3; ++s) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += dT2[r * 3 + k] * W[s * 3 + k];
            dJ[r * 3 + s] = acc;
        }
    double dpx = 0, dpy = 0, dpz = 0;
    /* J entries: J00 = fx/z, J02 = -fx ux/z, J11 = fy/z, J12 = -fy uy/z with
     * ux = x/z (or the constant limit when clamped), likewise uy */
    dpz += dJ[0] * (-fx / (z * z)) + dJ[4] * (-fy / (z * z));
    if (p->ux_clamped) {
        dpz += dJ[2] * (fx * p->ux / (z * z));
    } else {
        dpx += dJ[2] * (-fx / (z * z));
        dpz += dJ[2] * (2 * fx * x / (z * z * z));
    }
    if (p->uy_clamped) {
        dpz += dJ[5] * (fy * p->uy / (z * z));
    } else {
        dpy += dJ[5] * (-fy / (z * z));
        dpz += dJ[5] * (2 * fy * y / (z * z * z));
    }
    /* 2D mean */
    dpx += g2d[0] * fx / z;
    dpz += g2d[0] * (-fx * x / (z * z));
    dpy += g2d[1] * fy / z;
    dpz += g2d[1] * (-fy * y / (z * z));
    /* rendered depth */
    dpz += g2d[9];
    /* mean: p = W mu + t */
    for (int k = 0; k < 3; ++k) grads[k * n + i] += W[0 * 3 + k] * dpx + W[1 * 3 + k] * dpy + W[2 * 3 + k] * dpz;
    /* Sigma3 = M M^T, M = R diag(s): dM = 2 G3 M */
    double M[9], dM[9];
    for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) M[r * 3 + s] = p->R[r * 3 + s] * p->s[s];
    for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += G3[r * 3 + k] * M[k * 3 + s];
            dM[r * 3 + s] = 2.0 * acc;
        }
    double dR[9];
    for (int s = 0; s < 3; ++s) {
        double ds = 0;
        for (int r = 0; r < 3; ++r) {
            ds += dM[r * 3 + s] * p->R[r * 3 + s];
            dR[r * 3 + s] = dM[r * 3 + s] * p->s[s];
        }
        grads[(3 + s) * n + i] += ds * p->s[s];
    }
    double dRq[4][9];
    drot_dq(p->qn, dRq);
    double dqn[4];
    for (int k = 0; k < 4; ++k) {
        double acc = 0;
        for (int e = 0; e < 9; ++e) acc += dRq[k][e] * dR[e];
        dqn[k] = acc;
    }
    double dot = 0;
    for (int k = 0; k < 4; ++k) dot += p->qn[k] * dqn[k];
    for (int k = 0; k < 4; ++k) grads[(6 + k) * n + i] += (dqn[k] - p->qn[k] * dot) / p->qnorm;
    grads[10 * n + i] += g2d[5] * p->o * (1.0 - p->o);
    for (int k = 0; k < 3; ++k) grads[(11 + k) * n + i] += g2d[6 + k];
}

/*
 * Adjoint of oracle_render for the listed pixels.  Upstream gradients per
 * listed pixel: gC[3][npix], gD[npix], gP[K][npix] (may be NULL), gT[npix].
 * Writes grads[14][n] (overwritten) and, if g2d_out is not NULL, the per-Gaussian
 * 2D gradients g2d_out[n][10].
 */
int oracle_render_backward(int64_t n, const double* params, const int32_t* ids, const ocam* cam,
                           const ocfg* cfg, int K, int64_t npix, const int64_t* pix,
                           const double* gC, const double* gD, const double* gP, const double* gT,
                           double* grads, double* g2d_out) {
    oproj* pr = (oproj*)malloc(sizeof(oproj) * (size_t)(n > 0 ? n : 1));
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!pr || !order) { free(pr); free(order); return -1; }
    for (int64_t i = 0; i < n; ++i) project_one(params, n, i, cam, cfg, &pr[i]);
    int64_t m = build_order(n, pr, order);
    int W = cam->width;
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double* acc = (double*)calloc((size_t)nthr * (size_t)(n > 0 ? n : 1) * 10, sizeof(double));
    if (!acc) { free(pr); free(order); return -1; }
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* my = acc + (size_t)tid * (size_t)n * 10;
        int64_t cap = 64;
        int64_t* lst = (int64_t*)malloc(sizeof(int64_t) * cap);
        double* la = (double*)malloc(sizeof(double) * cap * 6);
#pragma omp for schedule(dynamic, 16)
        for (int64_t j = 0; j < npix; ++j) {
            double su = (double)(pix[j] % W) + 0.5, sv = (double)(pix[j] / W) + 0.5;
            /* forward, recording the blended list */
            double T = 1.0;
            int64_t nb = 0;
            for (int64_t r = 0; r < m; ++r) {
                const oproj* g = &pr[order[r]];
                double dx = su - g->mx, dy = sv - g->my;
                double Q = g->A * dx * dx + 2.0 * g->B * dx * dy + g->C * dy * dy;
                if (Q > cfg->q_max) continue;
                double G = exp(-0.5 * Q);
                double araw = g->o * G;
                int clamped = !(araw < cfg->alpha_max);
                double a = clamped ? cfg->alpha_max : araw;
                if (a < cfg->alpha_min) continue;
                double Tn = T * (1.0 - a);
                if (Tn < cfg->t_min) break;
                if (nb == cap) {
                    cap *= 2;
                    lst = (int64_t*)realloc(lst, sizeof(int64_t) * cap);
                    la = (double*)realloc(la, sizeof(double) * cap * 6);
                }
                lst[nb] = order[r];
                la[nb * 6 + 0] = a;
                la[nb * 6 + 1] = T;      /* transmittance before this Gaussian */
                la[nb * 6 + 2] = G;
                la[nb * 6 + 3] = dx;
                la[nb * 6 + 4] = dy;
                la[nb * 6 + 5] = clamped;
                ++nb;
                T = Tn;
            }
            double gc[3] = {gC[j], gC[npix + j], gC[2 * npix + j]};
            double gd = gD ? gD[j] : 0.0;
            double gt = gT ? gT[j] : 0.0;
            /* S = sum over later blended of w v, plus the background / T_final term */
            double S = T * (gc[0] * cfg->bg[0] + gc[1] * cfg->bg[1] + gc[2] * cfg->bg[2] + gt);
            for (int64_t b = nb - 1; b >= 0; --b) {
                int64_t gi = lst[b];
                const oproj* g = &pr[gi];
                double a = la[b * 6 + 0], Ti = la[b * 6 + 1], G = la[b * 6 + 2];
                double dx = la[b * 6 + 3], dy = la[b * 6 + 4];
                int clamped = la[b * 6 + 5] != 0;
                double w = a * Ti;
                double v = gc[0] * params[11 * n + gi] + gc[1] * params[12 * n + gi] +
                           gc[2] * params[13 * n + gi] + gd * g->z;
                int id = ids[gi];
                if (gP && id >= 0 && id < K) v += gP[(int64_t)id * npix + j];
                double dalpha = Ti * v - S / (1.0 - a);
                S += w * v;
                double* o = my + gi * 10;
                o[6] += gc[0] * w;
                o[7] += gc[1] * w;
                o[8] += gc[2] * w;
                o[9] += gd * w;
                if (!clamped) {
                    double dQ = dalpha * (-0.5 * a);
                    o[5] += dalpha * G;
                    o[0] += dQ * (-2.0 * (g->A * dx + g->B * dy));
                    o[1] += dQ * (-2.0 * (g->B * dx + g->C * dy));
                    o[2] += dQ * dx * dx;
                    o[3] += dQ * 2.0 * dx * dy;
                    o[4] += dQ * dy * dy;
                }
            }
        }
        free(lst);
        free(la);
    }
    memset(grads, 0, sizeof(double) * NPAR * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        double g[10] = {0};
        for (int t = 0; t < nthr; ++t)
            for (int k = 0; k < 10; ++k) g[k] += acc[((size_t)t * n + i) * 10 + k];
        if (g2d_out) memcpy(g2d_out + i * 10, g, sizeof(g));
        if (pr[i].visible) project_backward_one(params, n, i, cam, &pr[i], g, grads);
    }
    free(acc);
    free(pr);
    free(order);
    return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
