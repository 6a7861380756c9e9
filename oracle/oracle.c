/*
 * Reference renderer for the hemispherical RF splatting method: plain, slow,
 * FP64, one pixel at a time.  TEST INFRASTRUCTURE ONLY: only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load this
 * file.  It shares no source with the GPU library.
 *
 * What it computes (paper Sec. 3.2, Sec. 4.1 and Sec. 4.2, Eq. (3)):
 *   1. activation: s = exp(l), q^ = q/|q|, sigma = 1/(1+exp(-o)),
 *      Sigma = R(q^) diag(s^2) R(q^)^T                          (Sec. 3.2)
 *   2. view transform t = V (mu - x_rx)                        (Sec. 4.2)
 *   3. equirectangular projection
 *        p_x = (atan2(t_x, t_z)/pi + 1) W/2,
 *        p_y = 2 asin(t_y/|t|) H/pi                              (Sec. 4.2)
 *   4. projected covariance Sigma' = J V Sigma V^T J^T + eps I, J the
 *      Jacobian of step 3 with respect to t                      (Sec. 4.2)
 *   5. per pixel, every Gaussian in ascending distance from the receiver,
 *      front-to-back compositing S = sum_i alpha_i prod_{j<i}(1-alpha_j) u_i
 *      with alpha_i = sigma_i G'_i and u_i the attenuated attribute  (Eq. (3))
 *
 * Readings where the paper is silent (each is a parameter):
 *   - distance key: r32 = fl32(sqrt(fl32(fl32(dx^2)+fl32(dy^2))+fl32(dz^2)))
 *     with dx = fl32(mu_x - rx_x) etc.; order = ascending (r32, index).
 *     This file must be compiled with -ffp-contract=off so that the float
 *     expression is evaluated exactly in that order without fusion.
 *   - alpha = min(alpha_max, sigma G); a pair with alpha < alpha_min is
 *     skipped; compositing stops before adding the Gaussian that would take
 *     the transmittance below T_min.
 *   - attenuation a_i = 1 / max(d_i, r_near)^p, d_i the distance from the
 *     mean to the receiver (ref=0) or the transmitter (ref=1).
 *   - Gaussians with r32 < r_near, or with non-finite / degenerate
 *     parameters, are dropped.
 *   - pixel centres at (c + 1/2, row + 1/2); the azimuth offset is wrapped
 *     into [-W/2, W/2); the elevation offset is not wrapped.
 *   - Jacobian: rho = sqrt(t_x^2 + t_z^2) is clamped below at 1e-6 |t|.
 *
 * Parameter vector prm[] (double):
 *   0 alpha_min  1 alpha_max  2 T_min  3 dilation (px^2)  4 r_near (m)
 *   5 atten_power  6 atten_ref (0 = rx, 1 = tx)  7 rect margin (px)
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PRM_AMIN 0
#define PRM_AMAX 1
#define PRM_TMIN 2
#define PRM_EPS 3
#define PRM_RNEAR 4
#define PRM_APOW 5
#define PRM_AREF 6
#define PRM_MARGIN 7

/* per-Gaussian FP64 record */
enum {
    R_PX = 0, R_PY, R_CA, R_CB, R_CC, R_SIG, R_ATT, R_EX, R_EY,
    R_S00, R_S01, R_S11, R_DIST, R_QMAX, R_AZ, R_EL, NREC
};

/* culling status */
enum { ST_VISIBLE = 0, ST_NEAR = 1, ST_FAINT = 2, ST_OFFGRID = 3, ST_INVALID = 4 };

/* ---- the distance key, single precision, no contraction ---------------- */
float orc_r32(float mx, float my, float mz, float rx, float ry, float rz)
{
    volatile float dx = mx - rx, dy = my - ry, dz = mz - rz;
    volatile float xx = dx * dx, yy = dy * dy, zz = dz * dz;
    volatile float s = xx + yy;
    volatile float s2 = s + zz;
    return sqrtf(s2);
}

static int finite3(double a, double b, double c) { return isfinite(a) && isfinite(b) && isfinite(c); }

/* Steps 1-4 for every Gaussian.  rect[4*i] = (c0, c1, r0, r1): the pixel
 * columns c0..c1 (may extend past [0, W) and then wrap) and rows r0..r1 whose
 * centres lie within the opacity-aware support ellipse plus `margin` px.  */
int orc_project(int n, const float* mean, const float* log_scale, const float* quat,
                const float* opac, const float* rx, const float* tx, const double* V,
                int H, int W, const double* prm, double* rec, float* r32, int* rect, int* status)
{
    const double PI = 3.14159265358979323846;
    const double amin = prm[PRM_AMIN], eps = prm[PRM_EPS];
    const double rnear = prm[PRM_RNEAR], apow = prm[PRM_APOW], margin = prm[PRM_MARGIN];
    const int aref = (int)prm[PRM_AREF];
    const double kx = W / (2.0 * PI), ky = 2.0 * H / PI;
    int nvis = 0;
    for (int i = 0; i < n; ++i) {
        double* R_ = rec + (size_t)i * NREC;
        for (int k = 0; k < NREC; ++k) R_[k] = 0.0;
        rect[4 * i + 0] = 0; rect[4 * i + 1] = -1; rect[4 * i + 2] = 0; rect[4 * i + 3] = -1;
        const double mx = mean[i], my = mean[n + i], mz = mean[2 * n + i];
        const double l0 = log_scale[i], l1 = log_scale[n + i], l2 = log_scale[2 * n + i];
        double qw = quat[i], qx = quat[n + i], qy = quat[2 * n + i], qz = quat[3 * n + i];
        const double o = opac[i];
        r32[i] = orc_r32(mean[i], mean[n + i], mean[2 * n + i], rx[0], rx[1], rx[2]);
        double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
        if (!finite3(mx, my, mz) || !finite3(l0, l1, l2) || !finite3(qw, qx, qy) || !isfinite(qz) ||
            !isfinite(o) || !(qn > 0.0) || !isfinite(r32[i])) {
            status[i] = ST_INVALID;
            continue;
        }
        if (r32[i] < (float)rnear) { status[i] = ST_NEAR; continue; }
        const double sigma = 1.0 / (1.0 + exp(-o));
        R_[R_SIG] = sigma;
        if (sigma < amin) { status[i] = ST_FAINT; continue; }
        qw /= qn; qx /= qn; qy /= qn; qz /= qn;
        /* rotation matrix of the unit quaternion (w, x, y, z) */
        double Rm[3][3] = {
            {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
            {2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)},
            {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
        const double s2[3] = {exp(2 * l0), exp(2 * l1), exp(2 * l2)};
        double Sg[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0;
                for (int k = 0; k < 3; ++k) acc += Rm[a][k] * s2[k] * Rm[b][k];
                Sg[a][b] = acc;
            }
        /* view transform */
        const double d[3] = {mx - (double)rx[0], my - (double)rx[1], mz - (double)rx[2]};
        double t[3];
        for (int a = 0; a < 3; ++a) t[a] = V[3 * a] * d[0] + V[3 * a + 1] * d[1] + V[3 * a + 2] * d[2];
        double Sv[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0;
                for (int k = 0; k < 3; ++k)
                    for (int m = 0; m < 3; ++m) acc += V[3 * a + k] * Sg[k][m] * V[3 * b + m];
                Sv[a][b] = acc;
            }
        const double x = t[0], y = t[1], z = t[2];
        const double r = sqrt(x * x + y * y + z * z);
        const double az = atan2(x, z);
        const double el = asin(y / r);
        const double px = (az / PI + 1.0) * W / 2.0;
        const double py = 2.0 * el * H / PI;
        double rho = sqrt(x * x + z * z);
        if (rho < 1e-6 * r) rho = 1e-6 * r;
        const double r2 = r * r;
        const double J[2][3] = {{kx * z / (rho * rho), 0.0, -kx * x / (rho * rho)},
                                {-ky * x * y / (r2 * rho), ky * rho / r2, -ky * z * y / (r2 * rho)}};
        double Sp[2][2];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                double acc = 0;
                for (int k = 0; k < 3; ++k)
                    for (int m = 0; m < 3; ++m) acc += J[a][k] * Sv[k][m] * J[b][m];
                Sp[a][b] = acc;
            }
        Sp[0][0] += eps;
        Sp[1][1] += eps;
        const double det = Sp[0][0] * Sp[1][1] - Sp[0][1] * Sp[1][0];
        /* attenuation */
        const float* ref = aref ? tx : rx;
        const double e0 = mx - ref[0], e1 = my - ref[1], e2 = mz - ref[2];
        double dist = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
        double dcl = dist < rnear ? rnear : dist;
        const double att = 1.0 / pow(dcl, apow);
        const double qmax = 2.0 * log(sigma / amin);
        const double ex = sqrt(qmax * Sp[0][0]), ey = sqrt(qmax * Sp[1][1]);
        R_[R_PX] = px; R_[R_PY] = py;
        R_[R_CA] = Sp[1][1] / det; R_[R_CB] = -Sp[0][1] / det; R_[R_CC] = Sp[0][0] / det;
        R_[R_ATT] = att; R_[R_EX] = ex; R_[R_EY] = ey;
        R_[R_S00] = Sp[0][0]; R_[R_S01] = Sp[0][1]; R_[R_S11] = Sp[1][1];
        R_[R_DIST] = r; R_[R_QMAX] = qmax; R_[R_AZ] = az; R_[R_EL] = el;
        if (!(det > 0.0) || !isfinite(px) || !isfinite(py) || !isfinite(ex) || !isfinite(ey) ||
            !isfinite(R_[R_CA]) || !isfinite(R_[R_CB]) || !isfinite(R_[R_CC]) || !isfinite(att)) {
            status[i] = ST_INVALID;
            continue;
        }
        /* rows whose centre lies within the support (+margin) */
        double rlo = ceil(py - ey - margin - 0.5), rhi = floor(py + ey + margin - 0.5);
        if (rlo < 0) rlo = 0;
        if (rhi > H - 1) rhi = H - 1;
        if (rlo > rhi) { status[i] = ST_OFFGRID; continue; }
        double clo = ceil(px - ex - margin - 0.5), chi = floor(px + ex + margin - 0.5);
        int c0, c1;
        if (chi - clo + 1 >= W) { c0 = 0; c1 = W - 1; }
        else { c0 = (int)clo; c1 = (int)chi; }
        rect[4 * i + 0] = c0; rect[4 * i + 1] = c1;
        rect[4 * i + 2] = (int)rlo; rect[4 * i + 3] = (int)rhi;
        status[i] = ST_VISIBLE;
        ++nvis;
    }
    return nvis;
}

/* ---- depth order: visible Gaussians ascending by (r32, index) ---------- */
static const float* g_sort_keys;
static int cmp_key(const void* a, const void* b)
{
    int i = *(const int*)a, j = *(const int*)b;
    float ki = g_sort_keys[i], kj = g_sort_keys[j];
    if (ki < kj) return -1;
    if (ki > kj) return 1;
    return (i > j) - (i < j);
}

int orc_order(int n, const float* r32, const int* status, int* order)
{
    int m = 0;
    for (int i = 0; i < n; ++i)
        if (status[i] == ST_VISIBLE) order[m++] = i;
    g_sort_keys = r32;
    qsort(order, m, sizeof(int), cmp_key);
    return m;
}

/* ---- per-pixel compositing --------------------------------------------- */
typedef struct {
    int n, nvis, F, cplx, H, W;
    const double* rec;
    const int* order;
    const float* attr;
    const double* prm;
    const int* pix;
    int npix;
    double* out;
    double* T_final;
    int* n_contrib;
    double* absacc;
    unsigned char* ambig;
    double* flipb;
    unsigned char* live;
    int* scratch; /* per thread: 2 * nvis + 8 ints when live is set */
    int thread, nthreads;
    const int* tile_off; /* non-NULL: tiled variant */
    const int* tile_list;
    int tw, th;
} job_t;

/* A decision counts as ambiguous when its value lies within 1e-5 of its
 * threshold, relative: an FP32 evaluation of the same decision carries a few
 * roundings in alpha = sigma G (~6e-7 relative) and, in the transmittance, a
 * product of ~30 rounded factors (1 - alpha), each carrying alpha's error
 * scaled by alpha / (1 - alpha): up to ~1e-5. */
#define AMB_ALPHA 1e-5
#define AMB_T 1e-5
static int near_rel(double v, double thr, double m) { return fabs(v - thr) <= m * fabs(thr); }

/* |u_{g,f}| of every channel f of Gaussian g: attenuation times the modulus */
static void mag_u(const job_t* J, int g, double att, double* m)
{
    const int C = J->cplx ? 2 : 1;
    const float* v = J->attr + (size_t)g * J->F * C;
    for (int f = 0; f < J->F; ++f) {
        double s = 0.0;
        for (int c = 0; c < C; ++c) s += (double)v[f * C + c] * (double)v[f * C + c];
        m[f] = fabs(att) * sqrt(s);
    }
}

/* clamped alpha of a pair, 0 when below alpha_min */
static double alpha_of(double sg, double amin, double amax)
{
    const double a = sg < amax ? sg : amax;
    return a < amin ? 0.0 : a;
}

/* One pixel over `list` (Eq. (3)).  Besides the output, the final
 * transmittance and the contributor count, it records:
 *  absacc[f] = sum_i T_i alpha_i |u_i,f| (the absolute-sum magnitude A);
 *  ambig     = some decision (alpha >= alpha_min, the T_min stop, the
 *              alpha_max clamp, the seam wrap of a reaching Gaussian) lies
 *              within 1e-5 relative of its threshold;
 *  flipb[f]  = an upper bound of how far an evaluation that takes any of
 *              those decisions the other way can move out_f: a flipped
 *              alpha test or wrap changes alpha_i by d (<= alpha_min(1+1e-5)
 *              for the test, |alpha(wrap 1) - alpha(wrap 2)| for the wrap),
 *              which moves the term T_i alpha_i u_i by d T_i |u_i| and scales
 *              every later term by (1 - alpha_i)/(1 - alpha_i +- d): at most
 *              d A more; a flipped stop adds or drops T_i alpha_i u_i (the
 *              next entry then stops either way, as alpha >= alpha_min >>
 *              1e-5); after a flipped alpha the stop may also move by one
 *              entry either way (the last accepted term, or the term that
 *              stopped the walk at T / (1 - sum d)).  Plus 1e-5 A for the
 *              ordinary rounding of the compared evaluation.  The clamp at
 *              alpha_max is continuous in the value: it adds nothing. */
static void shade_pixel(const job_t* J, int row, int col, const int* list, int len)
{
    const double amin = J->prm[PRM_AMIN], amax = J->prm[PRM_AMAX], tmin = J->prm[PRM_TMIN];
    const int F = J->F, C = J->cplx ? 2 : 1, W = J->W, H = J->H;
    const size_t HW = (size_t)H * W, pix = (size_t)row * W + col;
    double acc[2 * 512], aab[512], direct[512], um[512], last[512];
    for (int k = 0; k < F * C; ++k) acc[k] = 0.0;
    for (int f = 0; f < F; ++f) aab[f] = direct[f] = last[f] = 0.0;
    double T = 1.0, dsum = 0.0;
    int cnt = 0, ncand = 0;
    unsigned char amb = 0;
    int* taken = J->live ? J->scratch : NULL;   /* taken entries, then candidates from the top */
    int* cand = J->live ? J->scratch + len + 4 : NULL;
    for (int k = 0; k < len; ++k) {
        const int g = list[k];
        const double* R_ = J->rec + (size_t)g * NREC;
        double dx = (col + 0.5) - R_[R_PX];
        if (dx >= 0.5 * W) dx -= W;
        else if (dx < -0.5 * W) dx += W;
        const double dy = (row + 0.5) - R_[R_PY];
        const double q = R_[R_CA] * dx * dx + 2.0 * R_[R_CB] * dx * dy + R_[R_CC] * dy * dy;
        const double sg = R_[R_SIG] * exp(-0.5 * q);
        double dflip = 0.0;
        if (fabs(fabs(dx) - 0.5 * W) < 1e-4) {
            /* offset on the seam: ambiguous only if either wrap reaches the support */
            const double dx2 = dx < 0 ? dx + W : dx - W;
            const double q2 = R_[R_CA] * dx2 * dx2 + 2.0 * R_[R_CB] * dx2 * dy + R_[R_CC] * dy * dy;
            const double qm = q < q2 ? q : q2;
            if (R_[R_SIG] * exp(-0.5 * qm) >= 0.5 * amin) {
                amb |= 8;
                dflip = fabs(alpha_of(sg, amin, amax) - alpha_of(R_[R_SIG] * exp(-0.5 * q2), amin, amax));
            }
        }
        if (near_rel(sg, amin, AMB_ALPHA)) { amb |= 1; dflip += amin * (1.0 + AMB_ALPHA); }
        if (near_rel(sg, amax, AMB_ALPHA)) amb |= 2;
        if (dflip > 0.0) {
            if (cand) cand[ncand++] = g;
            mag_u(J, g, R_[R_ATT], um);
            for (int f = 0; f < F; ++f) direct[f] += dflip * T * um[f];
            dsum += dflip;
        }
        const double alpha = sg < amax ? sg : amax;
        if (alpha < amin) continue;
        const double Tn = T * (1.0 - alpha);
        const int stop_amb = near_rel(Tn, tmin, AMB_T);
        if (stop_amb || (Tn < tmin && dsum > 0.0)) {
            mag_u(J, g, R_[R_ATT], um);
            /* the flipped stop adds or drops this term; after a flipped
             * alpha the walk's transmittance here is at most T / (1 - dsum) */
            const double Tb = (Tn < tmin && dsum > 0.0) ? T / (1.0 - (dsum < 0.5 ? dsum : 0.5)) : T;
            for (int f = 0; f < F; ++f) direct[f] += Tb * alpha * um[f];
            if (stop_amb) amb |= 4;
            if (cand) cand[ncand++] = g;
        }
        if (Tn < tmin) break;
        const double w = T * alpha * R_[R_ATT];
        const float* v = J->attr + (size_t)g * F * C;
        for (int f = 0; f < F; ++f) {
            double mag = 0.0;
            for (int c = 0; c < C; ++c) {
                acc[f * C + c] += w * (double)v[f * C + c];
                mag += (double)v[f * C + c] * (double)v[f * C + c];
            }
            last[f] = fabs(w) * sqrt(mag);
            aab[f] += last[f];
        }
        if (taken) taken[cnt] = g;
        T = Tn;
        ++cnt;
    }
    if (J->live) {
        for (int k = 0; k < cnt; ++k) __atomic_fetch_or(&J->live[taken[k]], amb ? 2 : 1, __ATOMIC_RELAXED);
        if (amb)
            for (int k = 0; k < ncand; ++k) __atomic_fetch_or(&J->live[cand[k]], 2, __ATOMIC_RELAXED);
    }
    for (int f = 0; f < F; ++f)
        for (int c = 0; c < C; ++c) {
            J->out[((size_t)f * HW + pix) * C + c] = acc[f * C + c];
            /* absolute-sum magnitude sum_i T_i alpha_i |u_i,f| (complex modulus) */
            if (J->absacc && c == 0) J->absacc[(size_t)f * HW + pix] = aab[f];
        }
    if (J->flipb)
        for (int f = 0; f < F; ++f)
            J->flipb[(size_t)f * HW + pix] =
                amb ? 1e-5 * aab[f] + direct[f] + dsum * aab[f] + (dsum > 0.0 ? last[f] : 0.0) : 0.0;
    J->T_final[pix] = T;
    J->n_contrib[pix] = cnt;
    if (J->ambig) J->ambig[pix] = amb;
}

static void render_rows(const job_t* J);

static void* render_worker(void* arg)
{
    job_t* J = (job_t*)arg;
    if (J->live) {
        int m = J->nvis > 0 ? J->nvis : 1;
        if (J->tile_off) m = J->n;
        J->scratch = (int*)malloc(sizeof(int) * (2 * (size_t)m + 8));
    }
    render_rows(J);
    free(J->scratch);
    J->scratch = NULL;
    return NULL;
}

static void render_rows(const job_t* J)
{
    if (J->tile_off) {
        const int TX = (J->W + J->tw - 1) / J->tw, TY = (J->H + J->th - 1) / J->th;
        for (int t = J->thread; t < TX * TY; t += J->nthreads) {
            const int ty = t / TX, tx = t % TX;
            const int* list = J->tile_list + J->tile_off[t];
            const int len = J->tile_off[t + 1] - J->tile_off[t];
            for (int row = ty * J->th; row < (ty + 1) * J->th && row < J->H; ++row)
                for (int col = tx * J->tw; col < (tx + 1) * J->tw && col < J->W; ++col)
                    shade_pixel(J, row, col, list, len);
        }
    } else if (J->pix) {
        for (int k = J->thread; k < J->npix; k += J->nthreads)
            shade_pixel(J, J->pix[k] / J->W, J->pix[k] % J->W, J->order, J->nvis);
    } else {
        for (int row = J->thread; row < J->H; row += J->nthreads)
            for (int col = 0; col < J->W; ++col) shade_pixel(J, row, col, J->order, J->nvis);
    }
}

static int run_jobs(job_t* base, int nthreads)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    job_t jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = *base;
        jobs[t].thread = t;
        jobs[t].nthreads = nthreads;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, render_worker, &jobs[t]);
    render_worker(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    return 0;
}

/* Untiled render: every pixel (or only the pixels in pix[0..npix) when pix is
 * non-NULL) walks the full depth order.  out is [F][H][W][C] (C = 2 when
 * complex), absacc [F][H][W] (may be NULL), T_final and n_contrib [H][W],
 * ambig [H][W] (may be NULL) flags pixels with a decision within 1e-5 of its
 * threshold, flipb [F][H][W] (may be NULL) bounds what flipping those
 * decisions can change (see shade_pixel).  live [n] (may be NULL, zeroed by
 * the caller) gets bit 0 for a Gaussian taken at some unambiguous pixel and
 * bit 1 for one taken, or whose decision is ambiguous, at an ambiguous
 * pixel.  Unlisted pixels are left untouched.  */
int orc_render(int n, const double* rec, const int* order, int nvis, const float* attr, int F,
               int cplx, int H, int W, const double* prm, const int* pix, int npix, double* out,
               double* T_final, int* n_contrib, double* absacc, unsigned char* ambig, double* flipb,
               unsigned char* live, int nthreads)
{
    if (F < 1 || F > 512) return -1;
    job_t J;
    memset(&J, 0, sizeof J);
    J.n = n; J.nvis = nvis; J.F = F; J.cplx = cplx; J.H = H; J.W = W;
    J.rec = rec; J.order = order; J.attr = attr; J.prm = prm; J.pix = pix; J.npix = npix;
    J.out = out; J.T_final = T_final; J.n_contrib = n_contrib; J.absacc = absacc; J.ambig = ambig;
    J.flipb = flipb;
    J.live = live;
    return run_jobs(&J, nthreads);
}

/* ---- binning: tile sets from integer rectangles ------------------------- */
/* Tile columns touched by the column interval [c0, c1] (wrapping mod W).
 * Returns the number of column ranges (1 or 2) written to rng[0..3]. */
static int tile_cols(int c0, int c1, int W, int tw, int* rng)
{
    const int TX = (W + tw - 1) / tw;
    if (c1 - c0 + 1 >= W) { rng[0] = 0; rng[1] = TX - 1; return 1; }
    int a = ((c0 % W) + W) % W;
    int b = a + (c1 - c0);
    if (b < W) { rng[0] = a / tw; rng[1] = b / tw; return 1; }
    int lo2 = (b - W) / tw, hi1 = a / tw;
    if (lo2 + 1 >= hi1) { rng[0] = 0; rng[1] = TX - 1; return 1; }
    rng[0] = hi1; rng[1] = TX - 1;
    rng[2] = 0; rng[3] = lo2;
    return 2;
}

int orc_tiles_of(const int* rect, int W, int H, int tw, int th, int* ty0, int* ty1, int* rng)
{
    *ty0 = rect[2] / th;
    *ty1 = rect[3] / th;
    (void)H;
    return tile_cols(rect[0], rect[1], W, tw, rng);
}

/* Per-tile lists: for each tile, the Gaussians of `order` whose rectangle
 * covers it, in `order`'s order.  tile_off has TX*TY+1 entries.  Returns the
 * number of (tile, Gaussian) pairs; list is written only if cap suffices.  */
long orc_bin(int nvis, const int* order, const int* rect, int H, int W, int tw, int th,
             int* tile_off, int* list, long cap)
{
    const int TX = (W + tw - 1) / tw, TY = (H + th - 1) / th, T = TX * TY;
    int* cnt = (int*)calloc((size_t)T + 1, sizeof(int));
    for (int k = 0; k < nvis; ++k) {
        int ty0, ty1, rng[4];
        int nr = orc_tiles_of(rect + 4 * order[k], W, H, tw, th, &ty0, &ty1, rng);
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int r = 0; r < nr; ++r)
                for (int tx = rng[2 * r]; tx <= rng[2 * r + 1]; ++tx) cnt[ty * TX + tx]++;
    }
    long P = 0;
    for (int t = 0; t < T; ++t) {
        tile_off[t] = (int)P;
        P += cnt[t];
    }
    tile_off[T] = (int)P;
    if (list && P <= cap) {
        for (int t = 0; t < T; ++t) cnt[t] = tile_off[t];
        for (int k = 0; k < nvis; ++k) {
            int g = order[k], ty0, ty1, rng[4];
            int nr = orc_tiles_of(rect + 4 * g, W, H, tw, th, &ty0, &ty1, rng);
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int r = 0; r < nr; ++r)
                    for (int tx = rng[2 * r]; tx <= rng[2 * r + 1]; ++tx) list[cnt[ty * TX + tx]++] = g;
        }
    }
    free(cnt);
    return P;
}

/* Tiled render: each pixel walks only its tile's list.  Same outputs as
 * orc_render; used to show that tiling changes nothing.  */
int orc_render_tiled(int n, const double* rec, const int* tile_off, const int* tile_list,
                     int tw, int th, const float* attr, int F, int cplx, int H, int W,
                     const double* prm, double* out, double* T_final, int* n_contrib, int nthreads)
{
    if (F < 1 || F > 512) return -1;
    job_t J;
    memset(&J, 0, sizeof J);
    J.n = n; J.F = F; J.cplx = cplx; J.H = H; J.W = W;
    J.rec = rec; J.attr = attr; J.prm = prm;
    J.out = out; J.T_final = T_final; J.n_contrib = n_contrib;
    J.tile_off = tile_off; J.tile_list = tile_list; J.tw = tw; J.th = th;
    return run_jobs(&J, nthreads);
}

int orc_nrec(void) { return NREC; }
