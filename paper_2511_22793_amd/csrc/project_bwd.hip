// Backward of the projection (Sec. 3.2 and Sec. 4.2) in FP64: from the
// per-Gaussian gradients with respect to the pixel-space centre (p_x, p_y),
// the conic (A, B, C), the opacity and the attenuation, accumulated by the
// blend backward, to the raw parameters (mean, log-scale, unnormalised
// quaternion, opacity logit).  One thread per Gaussian; the queries of a
// batch are summed inside the thread, so the result is deterministic.
//
//   conic = inverse(Sigma'),  dL/dSigma' = -conic . G . conic  (G symmetric,
//                                           off-diagonal dL/dB / 2)
//   Sigma' = K diag(s^2) K^T + eps I,  K = J V R(q/|q|),  s = exp(l)
//   J = d(p_x, p_y)/dt at t = V (mu - x_rx)
//   a = 1 / max(|mu - x_ref|, r_near)^p,  opacity = sigmoid(o)
#include "common.h"

namespace gs {

struct View3b {
    double m[9];
};

__global__ __launch_bounds__(256) void k_project_bwd(
    int n, int nq, const float* __restrict__ mean, const float* __restrict__ log_scale,
    const float* __restrict__ quat, const float* __restrict__ opac, const float* __restrict__ rx_all,
    const float* __restrict__ tx_all, View3b V, int H, int W, float rnear, double eps, double apow, int aref,
    const uint32_t* __restrict__ status, size_t s_status, const float* __restrict__ g2d, size_t s_g2d,
    float* __restrict__ d_mean, float* __restrict__ d_log_scale, float* __restrict__ d_quat,
    float* __restrict__ d_opac)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double mx = mean[i], my = mean[n + i], mz = mean[2 * n + i];
    const double l[3] = {log_scale[i], log_scale[n + i], log_scale[2 * n + i]};
    const double q0[4] = {quat[i], quat[n + i], quat[2 * n + i], quat[3 * n + i]};
    const double o = opac[i];
    double gm[3] = {0, 0, 0}, gl[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, go = 0.0;
    const double PI = 3.14159265358979323846;
    const double* v = V.m;
    for (int q = 0; q < nq; ++q) {
        if (status[q * s_status + i] != ST_VISIBLE) continue;
        const float* gg = g2d + q * s_g2d + (size_t)i * 8;
        const double dpx = gg[0], dpy = gg[1], dA = gg[2], dB = gg[3], dC = gg[4], dsig = gg[5], datt = gg[6];
        const float* rxp = rx_all + 3 * q;
        const float* txp = tx_all ? tx_all + 3 * q : rxp;
        // opacity = sigmoid(o)
        const double sigma = 1.0 / (1.0 + exp(-o));
        go += dsig * sigma * (1.0 - sigma);
        // attenuation 1 / max(d, r_near)^p
        {
            const float* ref = aref ? txp : rxp;
            const double e[3] = {mx - ref[0], my - ref[1], mz - ref[2]};
            const double d = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
            if (d > (double)rnear && apow != 0.0) {
                const double att = pow(d, -apow);
                const double k = datt * (-apow * att / d) / d;
                for (int a = 0; a < 3; ++a) gm[a] += k * e[a];
            }
        }
        // forward quantities
        const double qn = sqrt(q0[0] * q0[0] + q0[1] * q0[1] + q0[2] * q0[2] + q0[3] * q0[3]);
        const double w = q0[0] / qn, x = q0[1] / qn, y = q0[2] / qn, z = q0[3] / qn;
        const double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                                {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                                {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
        double M[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) M[a][b] = v[3 * a] * R[0][b] + v[3 * a + 1] * R[1][b] + v[3 * a + 2] * R[2][b];
        const double s2[3] = {exp(2 * l[0]), exp(2 * l[1]), exp(2 * l[2])};
        const double dw[3] = {mx - rxp[0], my - rxp[1], mz - rxp[2]};
        const double tx = v[0] * dw[0] + v[1] * dw[1] + v[2] * dw[2];
        const double ty = v[3] * dw[0] + v[4] * dw[1] + v[5] * dw[2];
        const double tz = v[6] * dw[0] + v[7] * dw[1] + v[8] * dw[2];
        const double r2 = tx * tx + ty * ty + tz * tz;
        const double rho_true = sqrt(tx * tx + tz * tz);
        const double r = sqrt(r2);
        const bool clamped = rho_true < 1e-6 * r;
        const double rho = clamped ? 1e-6 * r : rho_true;
        const double rho2 = rho * rho;
        const double kx = W / (2.0 * PI), ky = 2.0 * H / PI;
        const double J[2][3] = {{kx * tz / rho2, 0.0, -kx * tx / rho2},
                                {-ky * tx * ty / (r2 * rho), ky * rho / r2, -ky * tz * ty / (r2 * rho)}};
        double K[2][3];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b) K[a][b] = J[a][0] * M[0][b] + J[a][1] * M[1][b] + J[a][2] * M[2][b];
        double a00 = eps, a01 = 0.0, a11 = eps;
        for (int b = 0; b < 3; ++b) {
            a00 += K[0][b] * K[0][b] * s2[b];
            a01 += K[0][b] * K[1][b] * s2[b];
            a11 += K[1][b] * K[1][b] * s2[b];
        }
        const double det = a00 * a11 - a01 * a01;
        const double CA = a11 / det, CB = -a01 / det, CC = a00 / det;
        // dL/dSigma' = -conic G conic, G = [[dA, dB/2], [dB/2, dC]]
        const double G00 = dA, G01 = 0.5 * dB, G11 = dC;
        // X = conic G
        const double X00 = CA * G00 + CB * G01, X01 = CA * G01 + CB * G11;
        const double X10 = CB * G00 + CC * G01, X11 = CB * G01 + CC * G11;
        const double S00 = -(X00 * CA + X01 * CB);
        const double S01 = -(X00 * CB + X01 * CC);
        const double S11 = -(X10 * CB + X11 * CC);
        // Sigma' = K diag(s2) K^T: dK = 2 S K diag(s2), ds2_b = (K^T S K)_bb
        double dK[2][3];
        for (int b = 0; b < 3; ++b) {
            dK[0][b] = 2.0 * (S00 * K[0][b] + S01 * K[1][b]) * s2[b];
            dK[1][b] = 2.0 * (S01 * K[0][b] + S11 * K[1][b]) * s2[b];
            const double ds2 = K[0][b] * K[0][b] * S00 + 2.0 * K[0][b] * K[1][b] * S01 + K[1][b] * K[1][b] * S11;
            gl[b] += 2.0 * s2[b] * ds2;
        }
        // K = J M: dJ = dK M^T, dM = J^T dK
        double dJ[2][3], dM[3][3];
        for (int a = 0; a < 2; ++a)
            for (int k = 0; k < 3; ++k) dJ[a][k] = dK[a][0] * M[k][0] + dK[a][1] * M[k][1] + dK[a][2] * M[k][2];
        for (int k = 0; k < 3; ++k)
            for (int b = 0; b < 3; ++b) dM[k][b] = J[0][k] * dK[0][b] + J[1][k] * dK[1][b];
        // M = V R: dR = V^T dM
        double dR[3][3];
        for (int m = 0; m < 3; ++m)
            for (int b = 0; b < 3; ++b) dR[m][b] = v[m] * dM[0][b] + v[3 + m] * dM[1][b] + v[6 + m] * dM[2][b];
        // R(w, x, y, z) of the unit quaternion
        const double gw = 2.0 * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] - y * dR[2][0] + x * dR[2][1]);
        const double gx = 2.0 * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - 2.0 * x * dR[1][1] - w * dR[1][2] +
                                 z * dR[2][0] + w * dR[2][1] - 2.0 * x * dR[2][2]);
        const double gy = 2.0 * (-2.0 * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] -
                                 w * dR[2][0] + z * dR[2][1] - 2.0 * y * dR[2][2]);
        const double gz = 2.0 * (-2.0 * z * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] -
                                 2.0 * z * dR[1][1] + y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
        // normalisation q^ = q / |q|
        const double dot = w * gw + x * gx + y * gy + z * gz;
        gq[0] += (gw - w * dot) / qn;
        gq[1] += (gx - x * dot) / qn;
        gq[2] += (gy - y * dot) / qn;
        gq[3] += (gz - z * dot) / qn;
        // view-space offset: through the centre (J) and through J itself
        double gt[3];
        for (int k = 0; k < 3; ++k) gt[k] = dpx * J[0][k] + dpy * J[1][k];
        if (!clamped) {
            const double rho4 = rho2 * rho2, r4 = r2 * r2, rho3 = rho2 * rho;
            // J00 = kx z / rho^2, J02 = -kx x / rho^2
            gt[0] += dJ[0][0] * (-2.0 * kx * tx * tz / rho4) + dJ[0][2] * (-kx * (tz * tz - tx * tx) / rho4);
            gt[2] += dJ[0][0] * (kx * (tx * tx - tz * tz) / rho4) + dJ[0][2] * (2.0 * kx * tx * tz / rho4);
            // J11 = ky rho / r^2
            gt[0] += dJ[1][1] * (ky * tx * (r2 - 2.0 * rho2) / (rho * r4));
            gt[1] += dJ[1][1] * (-2.0 * ky * rho * ty / r4);
            gt[2] += dJ[1][1] * (ky * tz * (r2 - 2.0 * rho2) / (rho * r4));
            // J10 = -ky x y / (r^2 rho)
            gt[0] += -ky * dJ[1][0] * (ty / (r2 * rho) - 2.0 * tx * tx * ty / (r4 * rho) - tx * tx * ty / (r2 * rho3));
            gt[1] += -ky * dJ[1][0] * (tx / (r2 * rho) - 2.0 * tx * ty * ty / (r4 * rho));
            gt[2] += -ky * dJ[1][0] * (-2.0 * tx * ty * tz / (r4 * rho) - tx * ty * tz / (r2 * rho3));
            // J12 = -ky z y / (r^2 rho)
            gt[0] += -ky * dJ[1][2] * (-2.0 * tx * ty * tz / (r4 * rho) - tx * ty * tz / (r2 * rho3));
            gt[1] += -ky * dJ[1][2] * (tz / (r2 * rho) - 2.0 * tz * ty * ty / (r4 * rho));
            gt[2] += -ky * dJ[1][2] * (ty / (r2 * rho) - 2.0 * tz * tz * ty / (r4 * rho) - tz * tz * ty / (r2 * rho3));
        }
        // t = V (mu - x_rx): dmu = V^T dt
        for (int a = 0; a < 3; ++a) gm[a] += v[a] * gt[0] + v[3 + a] * gt[1] + v[6 + a] * gt[2];
    }
    d_opac[i] = (float)go;
    for (int a = 0; a < 3; ++a) d_mean[a * n + i] = (float)gm[a];
    for (int a = 0; a < 3; ++a) d_log_scale[a * n + i] = (float)gl[a];
    for (int a = 0; a < 4; ++a) d_quat[a * n + i] = (float)gq[a];
}

void launch_project_bwd(const gs_scene& sc, const gs_queries& qs, const gs_grid& g, const gs_params& p,
                        const Layout& L, char* ws, float* d_mean, float* d_log_scale, float* d_quat, float* d_opac,
                        hipStream_t s)
{
    View3b V;
    for (int k = 0; k < 9; ++k) V.m[k] = g.view[k];
    hipLaunchKernelGGL(k_project_bwd, dim3((L.n + 255) / 256), dim3(256), 0, s, L.n, L.nq, sc.mean, sc.log_scale,
                       sc.quat, sc.opacity_logit, qs.rx, qs.tx, V, L.H, L.W, p.r_near, (double)p.dilation,
                       (double)p.atten_power, p.atten_ref, (const uint32_t*)(ws + L.status), L.s_status / 4,
                       (const float*)(ws + L.g2d), L.s_g2d / 4, d_mean, d_log_scale, d_quat, d_opac);
}

}  // namespace gs
