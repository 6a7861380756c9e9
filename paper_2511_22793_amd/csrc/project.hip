// Projection of 3D Gaussians onto the receiver-centred equirectangular grid
// (paper Sec. 3.2 and Sec. 4.2): activation, view transform, culling, the
// equirectangular map, the EWA projected covariance Sigma' = J V Sigma V^T J^T
// plus dilation, attenuation, the opacity-aware support rectangle and its
// tile set.  One thread per (Gaussian, query); SoA loads are coalesced.
#include "common.h"

namespace gs {

struct View3 {
    double m[9];
};

// FP32 distance key: every operation rounded once to single precision, in
// the order ((dx^2 + dy^2) + dz^2) then sqrt.  Each step is evaluated in
// FP64 and rounded to FP32; with 53 >= 2*24 + 2 significand bits that double
// rounding gives the correctly rounded single-precision result.
__device__ __forceinline__ float r32_key(float mx, float my, float mz, float rx, float ry, float rz)
{
#pragma clang fp contract(off)
    const float dx = (float)((double)mx - (double)rx);
    const float dy = (float)((double)my - (double)ry);
    const float dz = (float)((double)mz - (double)rz);
    const float xx = (float)((double)dx * (double)dx);
    const float yy = (float)((double)dy * (double)dy);
    const float zz = (float)((double)dz * (double)dz);
    const float s = (float)((double)xx + (double)yy);
    const float s2 = (float)((double)s + (double)zz);
    return (float)__builtin_sqrt((double)s2);
}

__global__ __launch_bounds__(256) void k_project(
    int n, const float* __restrict__ mean, const float* __restrict__ log_scale,
    const float* __restrict__ quat, const float* __restrict__ opac, const float* __restrict__ rx_all,
    const float* __restrict__ tx_all, View3 V, int H, int W, int tw, int th, int TX, float amin,
    float rnear, double eps, double apow, int aref, double margin, GRec* __restrict__ rec, size_t s_rec,
    int4* __restrict__ rect, size_t s_rect, uint32_t* __restrict__ status, size_t s_status,
    uint4* __restrict__ tinfo, size_t s_tinfo, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
    size_t s_keys, uint32_t* __restrict__ flags, size_t s_flags)
{
    const int q = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    rec += q * s_rec;
    rect += q * s_rect;
    status += q * s_status;
    tinfo += q * s_tinfo;
    keys += q * s_keys;
    vals += q * s_keys;
    flags += q * s_flags;
    const float* rxp = rx_all + 3 * q;
    const float* txp = tx_all ? tx_all + 3 * q : rxp;

    uint32_t st = ST_INVALID;
    bool in = i < n;
    if (in) {
        const float fx = mean[i], fy = mean[n + i], fz = mean[2 * n + i];
        const float rxf = rxp[0], ryf = rxp[1], rzf = rxp[2];
        const float key = r32_key(fx, fy, fz, rxf, ryf, rzf);
        const double l0 = log_scale[i], l1 = log_scale[n + i], l2 = log_scale[2 * n + i];
        double qw = quat[i], qx = quat[n + i], qy = quat[2 * n + i], qz = quat[3 * n + i];
        const double o = opac[i];
        const double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        GRec R{};
        int4 rc = make_int4(0, -1, 0, -1);
        uint4 ti = make_uint4(0, 0, 0, 0);
        const bool finite_in = isfinite(fx) && isfinite(fy) && isfinite(fz) && isfinite(l0) &&
                               isfinite(l1) && isfinite(l2) && isfinite(qw) && isfinite(qx) &&
                               isfinite(qy) && isfinite(qz) && isfinite(o) && qn > 0.0 &&
                               isfinite(key);
        if (!finite_in) {
            st = ST_INVALID;
        } else if (key < rnear) {
            st = ST_NEAR;
        } else {
            const double sigma = 1.0 / (1.0 + exp(-o));
            R.sigma = (float)sigma;
            if (sigma < (double)amin) {
                st = ST_FAINT;
            } else {
                qw /= qn; qx /= qn; qy /= qn; qz /= qn;
                // rotation of the unit quaternion, then Sigma = R diag(s^2) R^T
                const double r00 = 1 - 2 * (qy * qy + qz * qz), r01 = 2 * (qx * qy - qw * qz),
                             r02 = 2 * (qx * qz + qw * qy);
                const double r10 = 2 * (qx * qy + qw * qz), r11 = 1 - 2 * (qx * qx + qz * qz),
                             r12 = 2 * (qy * qz - qw * qx);
                const double r20 = 2 * (qx * qz - qw * qy), r21 = 2 * (qy * qz + qw * qx),
                             r22 = 1 - 2 * (qx * qx + qy * qy);
                const double s0 = exp(2 * l0), s1 = exp(2 * l1), s2 = exp(2 * l2);
                // M = V R, so V Sigma V^T = M diag(s^2) M^T
                const double* v = V.m;
                double M[3][3];
                const double Rm[3][3] = {{r00, r01, r02}, {r10, r11, r12}, {r20, r21, r22}};
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b)
                        M[a][b] = v[3 * a] * Rm[0][b] + v[3 * a + 1] * Rm[1][b] + v[3 * a + 2] * Rm[2][b];
                const double dxw = (double)fx - rxf, dyw = (double)fy - ryf, dzw = (double)fz - rzf;
                const double x = v[0] * dxw + v[1] * dyw + v[2] * dzw;
                const double y = v[3] * dxw + v[4] * dyw + v[5] * dzw;
                const double z = v[6] * dxw + v[7] * dyw + v[8] * dzw;
                const double rr2 = x * x + y * y + z * z;
                const double r = sqrt(rr2);
                const double PI = 3.14159265358979323846;
                const double az = atan2(x, z);
                const double el = asin(y / r);
                const double px = (az / PI + 1.0) * (0.5 * W);
                const double py = el * (2.0 * H / PI);
                double rho = sqrt(x * x + z * z);
                rho = rho < 1e-6 * r ? 1e-6 * r : rho;
                const double kx = W / (2.0 * PI), ky = 2.0 * H / PI;
                const double irho2 = 1.0 / (rho * rho);
                const double j00 = kx * z * irho2, j02 = -kx * x * irho2;
                const double c = ky / (rr2 * rho);
                const double j10 = -c * x * y, j11 = ky * rho / rr2, j12 = -c * z * y;
                // K = J M (2x3); Sigma' = K diag(s^2) K^T + eps I
                double K0[3], K1[3];
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    K0[b] = j00 * M[0][b] + j02 * M[2][b];
                    K1[b] = j10 * M[0][b] + j11 * M[1][b] + j12 * M[2][b];
                }
                const double a00 = K0[0] * K0[0] * s0 + K0[1] * K0[1] * s1 + K0[2] * K0[2] * s2 + eps;
                const double a01 = K0[0] * K1[0] * s0 + K0[1] * K1[1] * s1 + K0[2] * K1[2] * s2;
                const double a11 = K1[0] * K1[0] * s0 + K1[1] * K1[1] * s1 + K1[2] * K1[2] * s2 + eps;
                const double det = a00 * a11 - a01 * a01;
                const double id = 1.0 / det;
                const float* ref = aref ? txp : rxp;
                const double e0 = (double)fx - ref[0], e1 = (double)fy - ref[1], e2 = (double)fz - ref[2];
                double dist = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
                dist = dist < (double)rnear ? (double)rnear : dist;
                const double att = apow == 2.0 ? 1.0 / (dist * dist) : (apow == 0.0 ? 1.0 : pow(dist, -apow));
                const double qmax = 2.0 * log(sigma / (double)amin);
                const double ex = sqrt(qmax * a00), ey = sqrt(qmax * a11);
                R.px = px; R.py = py;
                R.ca = a11 * id; R.cb = -a01 * id; R.cc = a00 * id;
                R.att = (float)att;
                if (!(det > 0.0) || !isfinite(px) || !isfinite(py) || !isfinite(ex) || !isfinite(ey) ||
                    !isfinite(R.ca) || !isfinite(R.cb) || !isfinite(R.cc) || !isfinite(att)) {
                    st = ST_INVALID;
                } else {
                    double rlo = ceil(py - ey - margin - 0.5), rhi = floor(py + ey + margin - 0.5);
                    rlo = rlo < 0.0 ? 0.0 : rlo;
                    rhi = rhi > H - 1 ? (double)(H - 1) : rhi;
                    if (rlo > rhi) {
                        st = ST_OFFGRID;
                    } else {
                        const double clo = ceil(px - ex - margin - 0.5), chi = floor(px + ex + margin - 0.5);
                        int c0, c1;
                        if (chi - clo + 1.0 >= (double)W) { c0 = 0; c1 = W - 1; }
                        else { c0 = (int)clo; c1 = (int)chi; }
                        const int r0 = (int)rlo, r1 = (int)rhi;
                        rc = make_int4(c0, c1, r0, r1);
                        // tile set: rows r0..r1, columns c0..c1 modulo W (one or two ranges)
                        const int ty0 = r0 / th, ty1 = r1 / th;
                        int xa0, xa1, xb0 = 1, xb1 = 0;
                        if (c1 - c0 + 1 >= W) {
                            xa0 = 0; xa1 = TX - 1;
                        } else {
                            int a = c0 % W;
                            a += a < 0 ? W : 0;
                            const int b = a + (c1 - c0);
                            if (b < W) {
                                xa0 = a / tw; xa1 = b / tw;
                            } else {
                                const int wrap_hi = (b - W) / tw, start = a / tw;
                                if (wrap_hi + 1 >= start) { xa0 = 0; xa1 = TX - 1; }
                                else { xa0 = start; xa1 = TX - 1; xb0 = 0; xb1 = wrap_hi; }
                            }
                        }
                        const int ncols = (xa1 - xa0 + 1) + (xb1 >= xb0 ? xb1 - xb0 + 1 : 0);
                        ti = make_uint4((uint32_t)xa0 | ((uint32_t)xa1 << 16), (uint32_t)xb0 | ((uint32_t)xb1 << 16),
                                        (uint32_t)ty0 | ((uint32_t)ty1 << 16), (uint32_t)(ncols * (ty1 - ty0 + 1)));
                        st = ST_VISIBLE;
                    }
                }
            }
        }
        rec[i] = R;
        rect[i] = rc;
        status[i] = st;
        tinfo[i] = ti;
        keys[i] = st == ST_VISIBLE ? __float_as_uint(key) : 0xFFFFFFFFu;
        vals[i] = (uint32_t)i;
    }
    // wave-aggregated counters
    const unsigned long long vis = __ballot(in && st == ST_VISIBLE);
    const unsigned long long bad = __ballot(in && st == ST_INVALID);
    if ((threadIdx.x & 63) == 0) {
        if (vis) atomicAdd(&flags[FL_NVIS], (uint32_t)__popcll(vis));
        if (bad) atomicAdd(&flags[FL_INVALID], (uint32_t)__popcll(bad));
    }
}

void launch_project(const gs_scene& sc, const gs_queries& qs, const gs_grid& g, const gs_params& p,
                    const Layout& L, char* ws, hipStream_t s)
{
    View3 V;
    for (int k = 0; k < 9; ++k) V.m[k] = g.view[k];
    dim3 grid((L.n + 255) / 256, L.nq);
    hipLaunchKernelGGL(k_project, grid, dim3(256), 0, s, L.n, sc.mean, sc.log_scale, sc.quat,
                       sc.opacity_logit, qs.rx, qs.tx, V, L.H, L.W, L.tw, L.th, L.TX, p.alpha_min,
                       p.r_near, (double)p.dilation, (double)p.atten_power, p.atten_ref, (double)p.margin,
                       (GRec*)(ws + L.rec), L.s_rec / sizeof(GRec), (int4*)(ws + L.rect), L.s_rect / sizeof(int4),
                       (uint32_t*)(ws + L.status), L.s_status / 4, (uint4*)(ws + L.tinfo),
                       L.s_tinfo / sizeof(uint4), (uint32_t*)(ws + L.keys_a), (uint32_t*)(ws + L.vals_a),
                       L.s_keys / 4, (uint32_t*)(ws + L.flags), L.s_flags / 4);
}

}  // namespace gs
