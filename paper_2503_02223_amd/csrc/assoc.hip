// Object-level association scores (Sec. III-B, Eq. (4)-(6)), in FP64, batched
// over the detections of any number of frames: IoU between the clipped
// tangent box of each object's projected dual quadric (C* = P Q* P^T) and
// each detection of the frame it belongs to; the coarse match of every
// detection; the occlusion overlap ratio of detection pairs of one frame; and
// the quadric distance of Eq. (5) between two sets of quadrics.
#include "dqo_device.hpp"

namespace dqo {

// Clipped tangent box of the quadric (mu, R, axes) in camera P (3x4 row
// major); false when its projection is not an ellipse in front of the camera.
__device__ bool quadric_box(const double* mu, const double* R, const double* ax, const double* P, double W, double H,
                            double b[4]) {
    double G[3][4];
    for (int r = 0; r < 3; ++r) {
        for (int m = 0; m < 3; ++m) G[r][m] = P[4 * r] * R[m] + P[4 * r + 1] * R[3 + m] + P[4 * r + 2] * R[6 + m];
        G[r][3] = P[4 * r] * mu[0] + P[4 * r + 1] * mu[1] + P[4 * r + 2] * mu[2] + P[4 * r + 3];
    }
    const double w[3] = {ax[0] * ax[0], ax[1] * ax[1], ax[2] * ax[2]};
    auto C = [&](int i, int j) {
        return w[0] * G[i][0] * G[j][0] + w[1] * G[i][1] * G[j][1] + w[2] * G[i][2] * G[j][2] - G[i][3] * G[j][3];
    };
    const double s = C(2, 2);
    if (!(s < 0.0)) return false;
    const double c00 = C(0, 0) / s, c02 = C(0, 2) / s, c11 = C(1, 1) / s, c12 = C(1, 2) / s;
    const double dx2 = c02 * c02 - c00, dy2 = c12 * c12 - c11;
    if (!(dx2 > 0.0) || !(dy2 > 0.0)) return false;
    const double dx = sqrt(dx2), dy = sqrt(dy2);
    b[0] = c02 - dx;
    b[1] = c12 - dy;
    b[2] = c02 + dx;
    b[3] = c12 + dy;
    const double lim[4] = {W, H, W, H};
    for (int i = 0; i < 4; ++i) b[i] = b[i] < 0.0 ? 0.0 : (b[i] > lim[i] ? lim[i] : b[i]);
    return true;
}

__device__ double box_iou(const double* b, const double* o) {
    const double iw = (b[2] < o[2] ? b[2] : o[2]) - (b[0] > o[0] ? b[0] : o[0]);
    const double ih = (b[3] < o[3] ? b[3] : o[3]) - (b[1] > o[1] ? b[1] : o[1]);
    if (!(iw > 0.0) || !(ih > 0.0)) return 0.0;
    const double I = iw * ih;
    return I / ((b[2] - b[0]) * (b[3] - b[1]) + (o[2] - o[0]) * (o[3] - o[1]) - I);
}

// iou[k][j]: one thread per (object, detection).
__global__ __launch_bounds__(256) void assoc_iou_kernel(int n_obj, int64_t n_det, const double* __restrict__ mu,
                                                        const double* __restrict__ R, const double* __restrict__ ax,
                                                        const double* __restrict__ boxes,
                                                        const int32_t* __restrict__ det_frame, int n_frames,
                                                        const double* __restrict__ P,
                                                        const int32_t* __restrict__ img_wh,
                                                        double* __restrict__ iou) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)n_obj * n_det) return;
    const int k = (int)(t / n_det);
    const int64_t j = t - (int64_t)k * n_det;
    const int f = det_frame[j];
    double v = 0.0;
    if (f >= 0 && f < n_frames) {
        double b[4];
        if (quadric_box(mu + 3 * k, R + 9 * k, ax + 3 * k, P + 12 * f, (double)img_wh[2 * f],
                        (double)img_wh[2 * f + 1], b))
            v = box_iou(b, boxes + 4 * j);
    }
    iou[t] = v;
}

// match[j]: the object of largest IoU (lowest index among equals) if it
// reaches iou_min, else -1.
__global__ __launch_bounds__(256) void assoc_match_kernel(int n_obj, int64_t n_det, const double* __restrict__ iou,
                                                          double iou_min, int32_t* __restrict__ match) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n_det) return;
    double best = -1.0;
    int arg = -1;
    for (int k = 0; k < n_obj; ++k) {
        const double v = iou[(int64_t)k * n_det + j];
        if (v > best) {
            best = v;
            arg = k;
        }
    }
    match[j] = (arg >= 0 && best >= iou_min) ? arg : -1;
}

// occ[i][j] = |B_i n B_j| / |B_j| for detections of the same frame with
// |B_j| < |B_i|, else 0.
__global__ __launch_bounds__(256) void assoc_occ_kernel(int64_t n_det, const double* __restrict__ boxes,
                                                        const int32_t* __restrict__ det_frame,
                                                        double* __restrict__ occ) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_det * n_det) return;
    const int64_t i = t / n_det, j = t - i * n_det;
    const double* bi = boxes + 4 * i;
    const double* bj = boxes + 4 * j;
    const double ai = (bi[2] - bi[0]) * (bi[3] - bi[1]), aj = (bj[2] - bj[0]) * (bj[3] - bj[1]);
    double v = 0.0;
    if (i != j && det_frame[i] == det_frame[j] && aj < ai && aj > 0.0) {
        const double iw = (bi[2] < bj[2] ? bi[2] : bj[2]) - (bi[0] > bj[0] ? bi[0] : bj[0]);
        const double ih = (bi[3] < bj[3] ? bi[3] : bj[3]) - (bi[1] > bj[1] ? bi[1] : bj[1]);
        if (iw > 0.0 && ih > 0.0) v = iw * ih / aj;
    }
    occ[t] = v;
}

// Eq. (5): qd[a][b] = exp(-tau (||mu_a - mu_b|| + ||S_a - S_b||_F)), S = R diag(axes^2) R^T.
__global__ __launch_bounds__(256) void quadric_distance_kernel(int na, const double* __restrict__ mu_a,
                                                               const double* __restrict__ R_a,
                                                               const double* __restrict__ ax_a, int nb,
                                                               const double* __restrict__ mu_b,
                                                               const double* __restrict__ R_b,
                                                               const double* __restrict__ ax_b, double tau,
                                                               double* __restrict__ qd) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)na * nb) return;
    const int a = (int)(t / nb), b = (int)(t - (int64_t)a * nb);
    double dm = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double d = mu_a[3 * a + i] - mu_b[3 * b + i];
        dm += d * d;
    }
    double ds = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double sa = 0.0, sb = 0.0;
            for (int m = 0; m < 3; ++m) {
                sa += R_a[9 * a + 3 * i + m] * R_a[9 * a + 3 * j + m] * ax_a[3 * a + m] * ax_a[3 * a + m];
                sb += R_b[9 * b + 3 * i + m] * R_b[9 * b + 3 * j + m] * ax_b[3 * b + m] * ax_b[3 * b + m];
            }
            ds += (sa - sb) * (sa - sb);
        }
    qd[t] = exp(-tau * (sqrt(dm) + sqrt(ds)));
}

// The decisions of Sec. III-B: the QD filter of each coarse match (Eq. (5))
// and the parent of each detection in the occlusion merge (Eq. (6)): the
// same-label detection whose larger box holds it by a ratio above t_occ with
// a QD above qd_occ, the largest ratio winning, then the lowest index.  One
// thread per detection; for a fixed i the threads read consecutive columns.
__global__ __launch_bounds__(256) void decide_parent_kernel(int64_t n_det, int n_obj, const int32_t* __restrict__ match,
                                                            const double* __restrict__ qd_obs,
                                                            const double* __restrict__ occ,
                                                            const double* __restrict__ qd_det,
                                                            const int32_t* __restrict__ label, double qd_min,
                                                            double t_occ, double qd_occ, int32_t* __restrict__ fine,
                                                            int32_t* __restrict__ parent) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n_det) return;
    const int k = match[j];
    fine[j] = (k >= 0 && k < n_obj && qd_obs[j * n_obj + k] >= qd_min) ? k : -1;
    const int32_t lj = label[j];
    double best = -1.0;
    int32_t arg = -1;
    for (int64_t i = 0; i < n_det; ++i) {
        const double t = occ[i * n_det + j];
        if (label[i] == lj && t > t_occ && qd_det[i * n_det + j] > qd_occ && t > best) {
            best = t;
            arg = (int32_t)i;
        }
    }
    parent[j] = arg;
}

// The end of each detection's parent chain and the object it updates.  A
// parent's box is strictly larger, so a chain has fewer than n_det links;
// the loop is bounded by n_det all the same.
__global__ __launch_bounds__(256) void decide_root_kernel(int64_t n_det, const int32_t* __restrict__ fine,
                                                          const int32_t* __restrict__ parent,
                                                          int32_t* __restrict__ root, int32_t* __restrict__ obj) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n_det) return;
    int64_t r = j;
    for (int64_t s = 0; s < n_det; ++s) {
        const int32_t p = parent[r];
        if (p < 0 || p >= n_det) break;
        r = p;
    }
    root[j] = (int32_t)r;
    obj[j] = fine[r];
}

static unsigned grid_of(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_associate(int n_obj, const double* mu, const double* R, const double* ax, int64_t n_det,
                            const double* boxes, const int32_t* det_frame, int n_frames, const double* P,
                            const int32_t* img_wh, double iou_min, double* iou, int32_t* match, double* occ,
                            hipStream_t st) {
    if (n_det == 0) return hipSuccess;
    if (n_obj > 0)
        hipLaunchKernelGGL(assoc_iou_kernel, dim3(grid_of((int64_t)n_obj * n_det)), dim3(256), 0, st, n_obj, n_det,
                           mu, R, ax, boxes, det_frame, n_frames, P, img_wh, iou);
    hipLaunchKernelGGL(assoc_match_kernel, dim3(grid_of(n_det)), dim3(256), 0, st, n_obj, n_det, (const double*)iou,
                       iou_min, match);
    if (occ)
        hipLaunchKernelGGL(assoc_occ_kernel, dim3(grid_of(n_det * n_det)), dim3(256), 0, st, n_det, boxes, det_frame,
                           occ);
    return hipGetLastError();
}

hipError_t launch_quadric_distance(int na, const double* mu_a, const double* R_a, const double* ax_a, int nb,
                                   const double* mu_b, const double* R_b, const double* ax_b, double tau, double* qd,
                                   hipStream_t st) {
    if ((int64_t)na * nb == 0) return hipSuccess;
    hipLaunchKernelGGL(quadric_distance_kernel, dim3(grid_of((int64_t)na * nb)), dim3(256), 0, st, na, mu_a, R_a,
                       ax_a, nb, mu_b, R_b, ax_b, tau, qd);
    return hipGetLastError();
}

hipError_t launch_associate_decide(int64_t n_det, int n_obj, const int32_t* match, const double* qd_obs,
                                   const double* occ, const double* qd_det, const int32_t* label, double qd_min,
                                   double t_occ, double qd_occ, int32_t* fine, int32_t* parent, int32_t* root,
                                   int32_t* obj, hipStream_t st) {
    if (n_det == 0) return hipSuccess;
    hipLaunchKernelGGL(decide_parent_kernel, dim3(grid_of(n_det)), dim3(256), 0, st, n_det, n_obj, match, qd_obs, occ,
                       qd_det, label, qd_min, t_occ, qd_occ, fine, parent);
    hipLaunchKernelGGL(decide_root_kernel, dim3(grid_of(n_det)), dim3(256), 0, st, n_det, (const int32_t*)fine,
                       (const int32_t*)parent, root, obj);
    return hipGetLastError();
}

}  // namespace dqo
