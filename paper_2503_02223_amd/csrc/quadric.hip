// Per-object dual quadric from 2D boxes (Eq. (1)) and its decoupling into
// centre, rotation and semi-axes (Eq. (2)-(3)), in FP64.
//
// One wavefront per object.  Each box edge line l seen by camera P gives the
// plane pi = P^T l; pi^T Q* pi = 0 is one row of a linear system in the 10
// unique entries of Q*.  Lane r % 64 holds row r, so the one-sided (Hestenes)
// Jacobi SVD rotates column pairs with three wave-wide dot products per pair,
// and lanes 0-9 carry the rows of the accumulated right rotation V.  The
// solution is the column of V whose rotated column of A has the least norm.
#include "dqo_device.hpp"

namespace dqo {

constexpr int kQRows = 4;  // rows per lane: up to 256 equations per object
constexpr int kQSweeps = 60;

__device__ __forceinline__ double wave_sum_all(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix (one thread).
__device__ void sym3_eigen(double A[9], double ev[3], double Vm[9]) {
    for (int i = 0; i < 9; ++i) Vm[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 50; ++sweep) {
        const double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        const double diag = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
        if (off <= 1e-34 * diag || off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                const double apq = A[p * 3 + q];
                if (apq == 0.0) continue;
                const double app = A[p * 3 + p], aqq = A[q * 3 + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 3; ++k) {  // A <- J^T A J
                    const double akp = A[k * 3 + p], akq = A[k * 3 + q];
                    A[k * 3 + p] = c * akp - s * akq;
                    A[k * 3 + q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    const double apk = A[p * 3 + k], aqk = A[q * 3 + k];
                    A[p * 3 + k] = c * apk - s * aqk;
                    A[q * 3 + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    const double vkp = Vm[k * 3 + p], vkq = Vm[k * 3 + q];
                    Vm[k * 3 + p] = c * vkp - s * vkq;
                    Vm[k * 3 + q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < 3; ++i) ev[i] = A[i * 4];
    // ascending order
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2 - i; ++j)
            if (ev[j] > ev[j + 1]) {
                const double t = ev[j];
                ev[j] = ev[j + 1];
                ev[j + 1] = t;
                for (int k = 0; k < 3; ++k) {
                    const double u = Vm[k * 3 + j];
                    Vm[k * 3 + j] = Vm[k * 3 + j + 1];
                    Vm[k * 3 + j + 1] = u;
                }
            }
}

__global__ __launch_bounds__(64) void fit_quadric_kernel(int n_obj, int n_views, int64_t n_boxes, const double* __restrict__ boxes,
                                                         const int32_t* __restrict__ box_obj,
                                                         const int32_t* __restrict__ box_view,
                                                         const double* __restrict__ P,
                                                         const int32_t* __restrict__ img_wh, double border,
                                                         double* __restrict__ Qo, double* __restrict__ muo,
                                                         double* __restrict__ Ro, double* __restrict__ axo,
                                                         int32_t* __restrict__ status) {
    const int k = blockIdx.x;
    const int lane = threadIdx.x;
    double a[kQRows][10];
#pragma unroll
    for (int s = 0; s < kQRows; ++s)
#pragma unroll
        for (int j = 0; j < 10; ++j) a[s][j] = 0.0;
    int nrows = 0;
    for (int64_t b = 0; b < n_boxes; ++b) {
        if (box_obj[b] != k) continue;
        const int v = box_view[b];
        if (v < 0 || v >= n_views) continue;
        const double x0 = boxes[4 * b], y0 = boxes[4 * b + 1], x1 = boxes[4 * b + 2], y1 = boxes[4 * b + 3];
        double lines[4][3];
        int nl = 0;
        const bool chk = img_wh != nullptr;
        const double Wv = chk ? (double)img_wh[2 * v] : 0.0, Hv = chk ? (double)img_wh[2 * v + 1] : 0.0;
        if (!chk || x0 > border) { lines[nl][0] = 1; lines[nl][1] = 0; lines[nl][2] = -x0; ++nl; }
        if (!chk || x1 < Wv - border) { lines[nl][0] = 1; lines[nl][1] = 0; lines[nl][2] = -x1; ++nl; }
        if (!chk || y0 > border) { lines[nl][0] = 0; lines[nl][1] = 1; lines[nl][2] = -y0; ++nl; }
        if (!chk || y1 < Hv - border) { lines[nl][0] = 0; lines[nl][1] = 1; lines[nl][2] = -y1; ++nl; }
        const double* Pv = P + 12 * v;
        for (int li = 0; li < nl; ++li) {
            const int r = nrows++;
            if (r < 64 * kQRows && (r & 63) == lane) {
                double pi[4];
                for (int c = 0; c < 4; ++c)
                    pi[c] = Pv[c] * lines[li][0] + Pv[4 + c] * lines[li][1] + Pv[8 + c] * lines[li][2];
                const double nrm = sqrt(pi[0] * pi[0] + pi[1] * pi[1] + pi[2] * pi[2] + pi[3] * pi[3]);
                for (int c = 0; c < 4; ++c) pi[c] /= nrm;
                const double row[10] = {pi[0] * pi[0],     2 * pi[0] * pi[1], 2 * pi[0] * pi[2], 2 * pi[0] * pi[3],
                                        pi[1] * pi[1],     2 * pi[1] * pi[2], 2 * pi[1] * pi[3], pi[2] * pi[2],
                                        2 * pi[2] * pi[3], pi[3] * pi[3]};
                const int s = r >> 6;
#pragma unroll
                for (int ss = 0; ss < kQRows; ++ss)
                    if (ss == s)
#pragma unroll
                        for (int j = 0; j < 10; ++j) a[ss][j] = row[j];
            }
        }
    }
    double vrow[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) vrow[j] = (lane == j) ? 1.0 : 0.0;
    if (nrows < 9) {
        if (lane < 16) Qo[16 * k + lane] = 0.0;
        if (lane < 3) { muo[3 * k + lane] = 0.0; axo[3 * k + lane] = 0.0; }
        if (lane < 9) Ro[9 * k + lane] = (lane % 4 == 0) ? 1.0 : 0.0;
        if (lane == 0) status[k] = DQO_QUADRIC_DEGENERATE;
        return;
    }
    for (int sweep = 0; sweep < kQSweeps; ++sweep) {
        bool rotated = false;
#pragma unroll
        for (int p = 0; p < 9; ++p) {
#pragma unroll
            for (int q = p + 1; q < 10; ++q) {
                double al = 0, be = 0, ga = 0;
#pragma unroll
                for (int s = 0; s < kQRows; ++s) {
                    al += a[s][p] * a[s][p];
                    be += a[s][q] * a[s][q];
                    ga += a[s][p] * a[s][q];
                }
                al = wave_sum_all(al);
                be = wave_sum_all(be);
                ga = wave_sum_all(ga);
                if (fabs(ga) > 1e-15 * sqrt(al * be) && ga != 0.0) {
                    rotated = true;
                    const double zeta = (be - al) / (2.0 * ga);
                    const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
#pragma unroll
                    for (int s = 0; s < kQRows; ++s) {
                        const double ap = a[s][p], aq = a[s][q];
                        a[s][p] = c * ap - sn * aq;
                        a[s][q] = sn * ap + c * aq;
                    }
                    const double vp = vrow[p], vq = vrow[q];
                    vrow[p] = c * vp - sn * vq;
                    vrow[q] = sn * vp + c * vq;
                }
            }
        }
        if (!rotated) break;
    }
    double sig[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) {
        double s2 = 0;
#pragma unroll
        for (int s = 0; s < kQRows; ++s) s2 += a[s][j] * a[s][j];
        sig[j] = sqrt(wave_sum_all(s2));
    }
    int jmin = 0;
    double smax = sig[0];
#pragma unroll
    for (int j = 1; j < 10; ++j) {
        if (sig[j] < sig[jmin]) jmin = j;
        smax = fmax(smax, sig[j]);
    }
    double s2nd = INFINITY;
#pragma unroll
    for (int j = 0; j < 10; ++j)
        if (j != jmin) s2nd = fmin(s2nd, sig[j]);
    double mine = 0;
#pragma unroll
    for (int j = 0; j < 10; ++j)
        if (j == jmin) mine = vrow[j];
    double q[10];
#pragma unroll
    for (int i = 0; i < 10; ++i) q[i] = __shfl(mine, i);
    if (lane != 0) return;
    int st = DQO_QUADRIC_OK;
    if (s2nd <= 1e-10 * smax) st = DQO_QUADRIC_DEGENERATE;
    double Qm[16] = {q[0], q[1], q[2], q[3], q[1], q[4], q[5], q[6], q[2], q[5], q[7], q[8], q[3], q[6], q[8], q[9]};
    double qabs = 0;
    for (int i = 0; i < 10; ++i) qabs = fmax(qabs, fabs(q[i]));
    double mu[3] = {0, 0, 0}, ax[3] = {0, 0, 0}, Rm[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    if (st == DQO_QUADRIC_OK) {
        if (fabs(Qm[15]) <= 1e-12 * qabs) {
            st = DQO_QUADRIC_NOT_ELLIPSOID;
        } else {
            const double sc = -1.0 / Qm[15];
            for (int i = 0; i < 16; ++i) Qm[i] *= sc;
            for (int i = 0; i < 3; ++i) mu[i] = -Qm[i * 4 + 3];
            double M[9];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    M[i * 3 + j] = 0.5 * (Qm[i * 4 + j] + Qm[j * 4 + i]) + mu[i] * mu[j];
            double ev[3], Vm[9];
            sym3_eigen(M, ev, Vm);
            const double det = Vm[0] * (Vm[4] * Vm[8] - Vm[5] * Vm[7]) - Vm[1] * (Vm[3] * Vm[8] - Vm[5] * Vm[6]) +
                               Vm[2] * (Vm[3] * Vm[7] - Vm[4] * Vm[6]);
            if (det < 0)
                for (int i = 0; i < 3; ++i) Vm[i * 3] = -Vm[i * 3];
            if (!(ev[0] > 0)) {
                st = DQO_QUADRIC_NOT_ELLIPSOID;
            } else {
                for (int i = 0; i < 3; ++i) ax[i] = sqrt(ev[i]);
                for (int i = 0; i < 9; ++i) Rm[i] = Vm[i];
            }
        }
    }
    for (int i = 0; i < 16; ++i) Qo[16 * k + i] = (st == DQO_QUADRIC_DEGENERATE) ? 0.0 : Qm[i];
    for (int i = 0; i < 3; ++i) {
        muo[3 * k + i] = (st == DQO_QUADRIC_OK) ? mu[i] : 0.0;
        axo[3 * k + i] = ax[i];
    }
    for (int i = 0; i < 9; ++i) Ro[9 * k + i] = Rm[i];
    status[k] = st;
}

// Boxes of the objects in rendered id maps: one workgroup per view reduces the
// per-object min/max pixel coordinates in LDS, then writes its K boxes.
__global__ __launch_bounds__(256) void id_boxes_kernel(const int32_t* __restrict__ id_map, int W, int H, int K,
                                                       double* __restrict__ boxes, int32_t* __restrict__ box_obj,
                                                       int32_t* __restrict__ box_view) {
    __shared__ int s_box[DQO_MAX_K][4];
    const int v = blockIdx.x;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        s_box[k][0] = W;
        s_box[k][1] = H;
        s_box[k][2] = -1;
        s_box[k][3] = -1;
    }
    __syncthreads();
    const int32_t* im = id_map + (int64_t)v * W * H;
    for (int64_t i = threadIdx.x; i < (int64_t)W * H; i += blockDim.x) {
        const int k = im[i];
        if (k < 0 || k >= K) continue;
        const int u = (int)(i % W), y = (int)(i / W);
        atomicMin(&s_box[k][0], u);
        atomicMin(&s_box[k][1], y);
        atomicMax(&s_box[k][2], u);
        atomicMax(&s_box[k][3], y);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const int64_t b = (int64_t)v * K + k;
        const bool seen = s_box[k][2] >= 0;
        boxes[4 * b + 0] = seen ? (double)s_box[k][0] : 0.0;
        boxes[4 * b + 1] = seen ? (double)s_box[k][1] : 0.0;
        boxes[4 * b + 2] = seen ? (double)(s_box[k][2] + 1) : 0.0;
        boxes[4 * b + 3] = seen ? (double)(s_box[k][3] + 1) : 0.0;
        box_obj[b] = seen ? k : -1;
        box_view[b] = v;
    }
}

hipError_t launch_id_boxes(const int32_t* id_map, int n_views, int W, int H, int K, double* boxes, int32_t* box_obj,
                           int32_t* box_view, hipStream_t st) {
    hipLaunchKernelGGL(id_boxes_kernel, dim3(n_views), dim3(256), 0, st, id_map, W, H, K, boxes, box_obj, box_view);
    return hipGetLastError();
}

hipError_t launch_fit_quadric(int n_obj, int64_t n_boxes, const double* boxes, const int32_t* box_obj,
                              const int32_t* box_view, int n_views, const double* P, const int32_t* img_wh,
                              double border, double* Q, double* mu, double* R, double* axes, int32_t* status,
                              hipStream_t st) {
    if (n_obj == 0) return hipSuccess;
    hipLaunchKernelGGL(fit_quadric_kernel, dim3(n_obj), dim3(64), 0, st, n_obj, n_views, n_boxes, boxes, box_obj, box_view, P,
                       img_wh, border, Q, mu, R, axes, status);
    return hipGetLastError();
}

}  // namespace dqo
