// Quadric pose refinement by the IoU loss of Eq. (9), in FP64.
//
// An object's quadric is theta = (mu, q, log-axes): Q* = Z diag(a^2, b^2, c^2, -1) Z^T,
// Z = [[R(q / |q|), mu], [0, 1]].  For a box seen by camera P, the dual conic
// is C* = G diag(w) G^T with G = P Z and w = (a^2, b^2, c^2, -1) (Eq. (4)),
// its tangent box is clipped to the image, and the object's loss is the sum
// over its boxes of 1 - IoU with the observed box.
//
// One wavefront per object.  The object's boxes (and their cameras) are
// staged in LDS once; lane i evaluates boxes i, i + 64, ... and back-
// propagates to (mu, R, w); a butterfly reduction leaves identical totals in
// every lane, so every lane performs the same Adam step on its own copy of
// theta and the whole optimisation runs in one launch with no barrier.
#include "dqo_device.hpp"

namespace dqo {

constexpr int kRefineMaxBoxes = 256;

struct RefineHp {
    int iterations;
    double lr_mu, lr_rot, lr_axes;
    double beta1, beta2, eps;
};

struct BoxSet {
    double obs[kRefineMaxBoxes][4];
    double P[kRefineMaxBoxes][12];
    double wh[kRefineMaxBoxes][2];  // image size for clipping; negative: no clipping
    int32_t idx[kRefineMaxBoxes];   // index of the box in the caller's arrays
};

__device__ __forceinline__ double rf_wave_sum(double v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);  // a + b == b + a: every lane ends equal
    return v;
}

__device__ void rot_from_unit_quat(const double q[4], double R[9]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z);
    R[1] = 2 * (x * y - w * z);
    R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);
    R[4] = 1 - 2 * (x * x + z * z);
    R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);
    R[7] = 2 * (y * z + w * x);
    R[8] = 1 - 2 * (x * x + y * y);
}

// Quaternion (w, x, y, z) of a rotation matrix (Shepperd's method: the
// largest of the four squared components is taken from the diagonal).
__device__ void quat_from_rot(const double R[9], double q[4]) {
    const double tr = R[0] + R[4] + R[8];
    if (tr >= R[0] && tr >= R[4] && tr >= R[8]) {
        const double s = 2.0 * sqrt(1.0 + tr);
        q[0] = 0.25 * s;
        q[1] = (R[7] - R[5]) / s;
        q[2] = (R[2] - R[6]) / s;
        q[3] = (R[3] - R[1]) / s;
    } else if (R[0] >= R[4] && R[0] >= R[8]) {
        const double s = 2.0 * sqrt(1.0 + R[0] - R[4] - R[8]);
        q[0] = (R[7] - R[5]) / s;
        q[1] = 0.25 * s;
        q[2] = (R[1] + R[3]) / s;
        q[3] = (R[2] + R[6]) / s;
    } else if (R[4] >= R[8]) {
        const double s = 2.0 * sqrt(1.0 + R[4] - R[0] - R[8]);
        q[0] = (R[2] - R[6]) / s;
        q[1] = (R[1] + R[3]) / s;
        q[2] = 0.25 * s;
        q[3] = (R[5] + R[7]) / s;
    } else {
        const double s = 2.0 * sqrt(1.0 + R[8] - R[0] - R[4]);
        q[0] = (R[3] - R[1]) / s;
        q[1] = (R[2] + R[6]) / s;
        q[2] = (R[5] + R[7]) / s;
        q[3] = 0.25 * s;
    }
}

// Quantities of theta shared by all boxes of an iteration.
struct ThetaView {
    double mu[3], qh[4], nq, R[9], w[3];
};

__device__ void theta_view(const double th[10], ThetaView& tv) {
    for (int i = 0; i < 3; ++i) tv.mu[i] = th[i];
    tv.nq = sqrt(th[3] * th[3] + th[4] * th[4] + th[5] * th[5] + th[6] * th[6]);
    for (int i = 0; i < 4; ++i) tv.qh[i] = th[3 + i] / tv.nq;
    rot_from_unit_quat(tv.qh, tv.R);
    for (int i = 0; i < 3; ++i) tv.w[i] = exp(2.0 * th[7 + i]);
}

// 1 - IoU of one box; with `acc` set, its gradient with respect to mu, R and
// w is added to acc[0..2], acc[3..11] (row-major R), acc[12..14].
__device__ double box_term(const ThetaView& tv, const double* __restrict__ P, const double* __restrict__ o,
                           const double* __restrict__ wh, double* acc, double* iou_out) {
    // M = P3 R, g = P3 mu + p4
    double M[3][3], g[3];
    for (int r = 0; r < 3; ++r) {
        for (int m = 0; m < 3; ++m) M[r][m] = P[4 * r] * tv.R[m] + P[4 * r + 1] * tv.R[3 + m] + P[4 * r + 2] * tv.R[6 + m];
        g[r] = P[4 * r] * tv.mu[0] + P[4 * r + 1] * tv.mu[1] + P[4 * r + 2] * tv.mu[2] + P[4 * r + 3];
    }
    auto Cij = [&](int i, int j) {
        return tv.w[0] * M[i][0] * M[j][0] + tv.w[1] * M[i][1] * M[j][1] + tv.w[2] * M[i][2] * M[j][2] - g[i] * g[j];
    };
    const double C00 = Cij(0, 0), C02 = Cij(0, 2), C11 = Cij(1, 1), C12 = Cij(1, 2), s = Cij(2, 2);
    *iou_out = 0.0;
    if (!(s < 0.0)) return 1.0;  // not an ellipse in front of the camera
    const double c00 = C00 / s, c02 = C02 / s, c11 = C11 / s, c12 = C12 / s;
    const double dx2 = c02 * c02 - c00, dy2 = c12 * c12 - c11;
    if (!(dx2 > 0.0) || !(dy2 > 0.0)) return 1.0;
    const double dx = sqrt(dx2), dy = sqrt(dy2);
    double b[4] = {c02 - dx, c12 - dy, c02 + dx, c12 + dy};
    bool pass[4] = {true, true, true, true};
    if (wh[0] >= 0.0) {
        const double lim[4] = {wh[0], wh[1], wh[0], wh[1]};
        for (int i = 0; i < 4; ++i) {
            if (b[i] < 0.0) { b[i] = 0.0; pass[i] = false; }
            else if (b[i] > lim[i]) { b[i] = lim[i]; pass[i] = false; }
        }
    }
    const bool px0 = b[0] > o[0], px1 = b[2] < o[2], py0 = b[1] > o[1], py1 = b[3] < o[3];
    const double iw = (px1 ? b[2] : o[2]) - (px0 ? b[0] : o[0]);
    const double ih = (py1 ? b[3] : o[3]) - (py0 ? b[1] : o[1]);
    if (!(iw > 0.0) || !(ih > 0.0)) return 1.0;
    const double I = iw * ih;
    const double bw = b[2] - b[0], bh = b[3] - b[1];
    const double U = bw * bh + (o[2] - o[0]) * (o[3] - o[1]) - I;
    const double iou = I / U;
    *iou_out = iou;
    if (!acc) return 1.0 - iou;
    // d(1 - IoU): dI and dA (predicted area) coefficients
    const double gI = -(U + I) / (U * U), gA = I / (U * U);
    double gb[4];
    gb[0] = gI * (px0 ? -ih : 0.0) + gA * (-bh);
    gb[2] = gI * (px1 ? ih : 0.0) + gA * bh;
    gb[1] = gI * (py0 ? -iw : 0.0) + gA * (-bw);
    gb[3] = gI * (py1 ? iw : 0.0) + gA * bw;
    for (int i = 0; i < 4; ++i)
        if (!pass[i]) gb[i] = 0.0;
    // x0 = c02 - dx, x1 = c02 + dx, dx = sqrt(c02^2 - c00) (and y likewise)
    const double gdx = gb[2] - gb[0], gdy = gb[3] - gb[1];
    const double gc02 = gb[0] + gb[2] + gdx * c02 / dx, gc00 = -gdx / (2.0 * dx);
    const double gc12 = gb[1] + gb[3] + gdy * c12 / dy, gc11 = -gdy / (2.0 * dy);
    // c = C / s
    const double gC00 = gc00 / s, gC02 = gc02 / s, gC11 = gc11 / s, gC12 = gc12 / s;
    const double gs = -(gc00 * c00 + gc02 * c02 + gc11 * c11 + gc12 * c12) / s;
    // S = G_hat + G_hat^T for the used entries of the symmetric C*
    const double S[3][3] = {{2 * gC00, 0.0, gC02}, {0.0, 2 * gC11, gC12}, {gC02, gC12, 2 * gs}};
    // dL/dw_m = sum_ij G_hat_ij M_im M_jm;  dL/dM_m = w_m S M_m;  dL/dg = -S g
    double gM[3][3];
    for (int m = 0; m < 3; ++m) {
        const double m0 = M[0][m], m1 = M[1][m], m2 = M[2][m];
        acc[12 + m] += gC00 * m0 * m0 + gC02 * m0 * m2 + gC11 * m1 * m1 + gC12 * m1 * m2 + gs * m2 * m2;
        for (int r = 0; r < 3; ++r) gM[r][m] = tv.w[m] * (S[r][0] * m0 + S[r][1] * m1 + S[r][2] * m2);
    }
    double gg[3];
    for (int r = 0; r < 3; ++r) gg[r] = -(S[r][0] * g[0] + S[r][1] * g[1] + S[r][2] * g[2]);
    // M = P3 R: dL/dR = P3^T dL/dM;  g = P3 mu + p4: dL/dmu = P3^T dL/dg
    for (int i = 0; i < 3; ++i) {
        acc[i] += P[i] * gg[0] + P[4 + i] * gg[1] + P[8 + i] * gg[2];
        for (int m = 0; m < 3; ++m) acc[3 + 3 * i + m] += P[i] * gM[0][m] + P[4 + i] * gM[1][m] + P[8 + i] * gM[2][m];
    }
    return 1.0 - iou;
}

// Loss and gradient of the object's theta over its staged boxes (every lane
// returns the same totals).
__device__ double object_loss_grad(const double th[10], const BoxSet& bs, int nb, double grad[10], double* box_iou) {
    ThetaView tv;
    theta_view(th, tv);
    double acc[15];
    for (int i = 0; i < 15; ++i) acc[i] = 0.0;
    double J = 0.0;
    for (int i = (int)threadIdx.x; i < nb; i += kWave) {
        double iou;
        J += box_term(tv, bs.P[i], bs.obs[i], bs.wh[i], grad ? acc : nullptr, &iou);
        if (box_iou) box_iou[bs.idx[i]] = iou;
    }
    J = rf_wave_sum(J);
    if (!grad) return J;
    for (int i = 0; i < 15; ++i) acc[i] = rf_wave_sum(acc[i]);
    for (int i = 0; i < 3; ++i) grad[i] = acc[i];
    // R(q_hat): derivative of the unit-quaternion rotation formula
    const double* gR = acc + 3;
    const double w = tv.qh[0], x = tv.qh[1], y = tv.qh[2], z = tv.qh[3];
    double gq[4];
    gq[0] = 2 * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
    gq[1] = 2 * (y * gR[1] + z * gR[2] + y * gR[3] - 2 * x * gR[4] - w * gR[5] + z * gR[6] + w * gR[7] - 2 * x * gR[8]);
    gq[2] = 2 * (-2 * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] + z * gR[7] - 2 * y * gR[8]);
    gq[3] = 2 * (-2 * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2 * z * gR[4] + y * gR[5] + x * gR[6] + y * gR[7]);
    // q_hat = q / |q|
    const double dot = gq[0] * tv.qh[0] + gq[1] * tv.qh[1] + gq[2] * tv.qh[2] + gq[3] * tv.qh[3];
    for (int i = 0; i < 4; ++i) grad[3 + i] = (gq[i] - tv.qh[i] * dot) / tv.nq;
    // w_m = exp(2 l_m)
    for (int m = 0; m < 3; ++m) grad[7 + m] = 2.0 * tv.w[m] * acc[12 + m];
    return J;
}

// Stage the boxes of object k in LDS, in ascending box order.  Returns their
// count (which may exceed kRefineMaxBoxes: then only the first are staged).
__device__ int stage_boxes(int k, int n_views, int64_t n_boxes, const double* __restrict__ boxes,
                           const int32_t* __restrict__ box_obj, const int32_t* __restrict__ box_view,
                           const double* __restrict__ P, const int32_t* __restrict__ img_wh, BoxSet& bs) {
    const int lane = threadIdx.x;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    int nb = 0;
    for (int64_t b0 = 0; b0 < n_boxes; b0 += kWave) {
        const int64_t b = b0 + lane;
        int v = -1;
        bool mine = false;
        if (b < n_boxes) {
            v = box_view[b];
            mine = box_obj[b] == k && v >= 0 && v < n_views;
        }
        const uint64_t bal = __ballot(mine);
        const int pos = nb + (int)__popcll(bal & lt);
        if (mine && pos < kRefineMaxBoxes) {
            for (int c = 0; c < 4; ++c) bs.obs[pos][c] = boxes[4 * b + c];
            for (int c = 0; c < 12; ++c) bs.P[pos][c] = P[12 * v + c];
            bs.wh[pos][0] = img_wh ? (double)img_wh[2 * v] : -1.0;
            bs.wh[pos][1] = img_wh ? (double)img_wh[2 * v + 1] : -1.0;
            bs.idx[pos] = (int32_t)b;
        }
        nb += (int)__popcll(bal);
    }
    __syncthreads();
    return nb;
}

__global__ __launch_bounds__(kWave) void quadric_iou_grad_kernel(int n_views, int64_t n_boxes,
                                                                 const double* __restrict__ boxes,
                                                                 const int32_t* __restrict__ box_obj,
                                                                 const int32_t* __restrict__ box_view,
                                                                 const double* __restrict__ P,
                                                                 const int32_t* __restrict__ img_wh,
                                                                 const double* __restrict__ theta,
                                                                 double* __restrict__ loss, double* __restrict__ grad,
                                                                 double* __restrict__ box_iou) {
    __shared__ BoxSet bs;
    const int k = blockIdx.x, lane = threadIdx.x;
    const int nb = stage_boxes(k, n_views, n_boxes, boxes, box_obj, box_view, P, img_wh, bs);
    if (nb > kRefineMaxBoxes) {
        if (lane == 0) loss[k] = __builtin_nan("");
        if (lane < 10) grad[10 * k + lane] = __builtin_nan("");
        return;
    }
    double th[10], g[10];
    for (int i = 0; i < 10; ++i) th[i] = theta[10 * k + i];
    const double J = object_loss_grad(th, bs, nb, g, box_iou);
    if (lane == 0) loss[k] = J;
    if (lane < 10) {
        double gi = g[0];
        for (int i = 1; i < 10; ++i)
            if (lane == i) gi = g[i];
        grad[10 * k + lane] = gi;
    }
}

__global__ __launch_bounds__(kWave) void refine_quadric_kernel(int n_views, int64_t n_boxes,
                                                               const double* __restrict__ boxes,
                                                               const int32_t* __restrict__ box_obj,
                                                               const int32_t* __restrict__ box_view,
                                                               const double* __restrict__ P,
                                                               const int32_t* __restrict__ img_wh,
                                                               const int32_t* __restrict__ status, RefineHp hp,
                                                               double* __restrict__ mu_io, double* __restrict__ R_io,
                                                               double* __restrict__ ax_io, double* __restrict__ Qo,
                                                               double* __restrict__ loss,
                                                               double* __restrict__ box_iou) {
    __shared__ BoxSet bs;
    const int k = blockIdx.x, lane = threadIdx.x;
    const double nan = __builtin_nan("");
    if (status && status[k] != DQO_QUADRIC_OK) {
        if (lane < 2) loss[2 * k + lane] = nan;
        return;
    }
    const int nb = stage_boxes(k, n_views, n_boxes, boxes, box_obj, box_view, P, img_wh, bs);
    if (nb > kRefineMaxBoxes) {
        if (lane < 2) loss[2 * k + lane] = nan;
        return;
    }
    double th[10], m[10], v[10], g[10];
    {
        double R0[9], q0[4];
        for (int i = 0; i < 9; ++i) R0[i] = R_io[9 * k + i];
        quat_from_rot(R0, q0);
        for (int i = 0; i < 3; ++i) th[i] = mu_io[3 * k + i];
        for (int i = 0; i < 4; ++i) th[3 + i] = q0[i];
        for (int i = 0; i < 3; ++i) th[7 + i] = log(ax_io[3 * k + i]);
    }
    for (int i = 0; i < 10; ++i) m[i] = v[i] = 0.0;
    const double lr[10] = {hp.lr_mu, hp.lr_mu, hp.lr_mu, hp.lr_rot, hp.lr_rot,
                           hp.lr_rot, hp.lr_rot, hp.lr_axes, hp.lr_axes, hp.lr_axes};
    double J0 = 0.0;
    for (int t = 1; t <= hp.iterations; ++t) {
        const double J = object_loss_grad(th, bs, nb, g, nullptr);
        if (t == 1) J0 = J;
        const double bc1 = 1.0 - pow(hp.beta1, (double)t), bc2 = 1.0 - pow(hp.beta2, (double)t);
        for (int i = 0; i < 10; ++i) {
            m[i] = hp.beta1 * m[i] + (1.0 - hp.beta1) * g[i];
            v[i] = hp.beta2 * v[i] + (1.0 - hp.beta2) * g[i] * g[i];
            th[i] = th[i] - lr[i] * (m[i] / bc1) / (sqrt(v[i] / bc2) + hp.eps);
        }
    }
    const double Jf = object_loss_grad(th, bs, nb, nullptr, box_iou);
    if (hp.iterations == 0) J0 = Jf;
    ThetaView tv;
    theta_view(th, tv);
    if (lane == 0) {
        loss[2 * k] = J0;
        loss[2 * k + 1] = Jf;
        for (int i = 0; i < 3; ++i) {
            mu_io[3 * k + i] = th[i];
            ax_io[3 * k + i] = sqrt(tv.w[i]);
        }
        for (int i = 0; i < 9; ++i) R_io[9 * k + i] = tv.R[i];
        if (Qo) {
            // Q* = Z diag(w, -1) Z^T: [[R diag(w) R^T - mu mu^T, -mu], [-mu^T, -1]]
            double* Q = Qo + 16 * k;
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j)
                    Q[4 * i + j] = tv.w[0] * tv.R[3 * i] * tv.R[3 * j] + tv.w[1] * tv.R[3 * i + 1] * tv.R[3 * j + 1] +
                                   tv.w[2] * tv.R[3 * i + 2] * tv.R[3 * j + 2] - th[i] * th[j];
                Q[4 * i + 3] = -th[i];
                Q[12 + i] = -th[i];
            }
            Q[15] = -1.0;
        }
    }
}

hipError_t launch_quadric_iou_grad(int n_obj, int n_views, int64_t n_boxes, const double* boxes,
                                   const int32_t* box_obj, const int32_t* box_view, const double* P,
                                   const int32_t* img_wh, const double* theta, double* loss, double* grad,
                                   double* box_iou, hipStream_t st) {
    if (n_obj == 0) return hipSuccess;
    hipLaunchKernelGGL(quadric_iou_grad_kernel, dim3(n_obj), dim3(kWave), 0, st, n_views, n_boxes, boxes, box_obj,
                       box_view, P, img_wh, theta, loss, grad, box_iou);
    return hipGetLastError();
}

hipError_t launch_refine_quadrics(int n_obj, int n_views, int64_t n_boxes, const double* boxes,
                                  const int32_t* box_obj, const int32_t* box_view, const double* P,
                                  const int32_t* img_wh, const int32_t* status, const dqo_refine_cfg& c, double* mu,
                                  double* R, double* axes, double* Q, double* loss, double* box_iou, hipStream_t st) {
    if (n_obj == 0) return hipSuccess;
    RefineHp hp;
    hp.iterations = c.iterations;
    hp.lr_mu = c.lr_mu;
    hp.lr_rot = c.lr_rot;
    hp.lr_axes = c.lr_axes;
    hp.beta1 = c.beta1;
    hp.beta2 = c.beta2;
    hp.eps = c.eps;
    hipLaunchKernelGGL(refine_quadric_kernel, dim3(n_obj), dim3(kWave), 0, st, n_views, n_boxes, boxes, box_obj,
                       box_view, P, img_wh, status, hp, mu, R, axes, Q, loss, box_iou);
    return hipGetLastError();
}

}  // namespace dqo
