/*
 * Plain FP64 CPU oracle of the Gaussian-splatting hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library.  The GPU product path never includes,
 * links or calls anything here, and nothing here comes from the GPU path.
 *
 * What is computed.  Section 4 of the paper ("Distributed Gaussian Splatting")
 * lists the operators of one training step: spherical-harmonic colour and
 * projection per Gaussian (for every camera of the batch), then per camera a
 * depth sort, the rasteriser and an image-space loss, and the backward passes
 * of all of them (gradient accumulation in the rasteriser backward).  The
 * paper states none of their formulas; it takes them from 3D Gaussian
 * Splatting (Kerbl et al. 2023, its citation for the method).  This file
 * writes those formulas out one Gaussian / one pixel at a time in double
 * precision, with no blocking, fusion or reordering:
 *
 *   projection  Sigma = R S S^T R^T, p = W mu + t, EWA 2-D covariance
 *               Sigma2 = J W Sigma W^T J^T + eps2d I, conic = Sigma2^{-1},
 *               radii (3-sigma box; opacity-aware and eigenvalue-square
 *               variants), tile rectangle;
 *   colour      real spherical harmonics up to degree 3 along the ray from
 *               the camera centre, plus 0.5, clamped at 0;
 *   binning     one (tile | depth) key per (Gaussian, tile) pair, stably
 *               sorted, ties in Gaussian order;
 *   compositing front to back, alpha = min(0.99, sigma exp(power)), skip
 *               alpha < 1/255, stop when transmittance would fall below 1e-4;
 *   backward    the exact derivative of the above with discrete decisions
 *               (culling, clamps, skips, stops, list membership) frozen.
 *
 * Readings where the paper is silent (all follow 3D Gaussian Splatting):
 * thresholds are the float32 values 1/255f, 0.99f, 1e-4f, 1.3f promoted to
 * double; quaternions are (w, x, y, z); cameras use OpenCV axes; pixel (i, j)
 * has its centre at (i + 0.5, j + 0.5); radii bound the 3-sigma box of each
 * axis by default; the tile rectangle and the depth key bits are taken in float32
 * arithmetic from the float32-rounded mean, radius and depth; SH use the real
 * orthonormal basis with the Condon-Shortley phase.
 *
 * Layouts: per-Gaussian inputs are planar [C][N]; one view per call.
 *
 * Threads.  By default every function runs on one thread.  or_set_threads(n)
 * spreads the independent iterations (Gaussians of the projection and its
 * backward, pixel rows of the compositing) over n OpenMP threads with the
 * same arithmetic per iteration; in the compositing backward the per-Gaussian
 * sums are then accumulated atomically, so their order (and the last bits of
 * those FP64 sums) depends on the thread schedule.  The tests use one thread;
 * the benchmark's CPU baseline times both one thread and all host cores.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int g_threads = 1;

/* number of threads of the parallel loops below (1: serial) */
void or_set_threads(int n) { g_threads = n < 1 ? 1 : n; }

/* processors OpenMP sees (1 without OpenMP) */
int or_num_procs(void)
{
#ifdef _OPENMP
    return omp_get_num_procs();
#else
    return 1;
#endif
}

#define OR_ALPHA_MIN ((double)(1.0f / 255.0f))
#define OR_ALPHA_MAX ((double)0.99f)
#define OR_T_MIN ((double)1e-4f)
#define OR_CLIP ((double)1.3f)

int or_abi_version(void) { return 3; }

/* ------------------------------------------------------------------------- */
/* Real spherical harmonics (orthonormal, Condon-Shortley phase) as sums of    */
/* monomials x^a y^b z^c of the unit direction.  Index l*l + l + m.            */
/* ------------------------------------------------------------------------- */
typedef struct { int j; double coef; int a, b, c; } sh_term;

static int sh_table(sh_term* t)
{
    const double pi = 3.14159265358979323846;
    const double c0 = 0.5 / sqrt(pi);
    const double c1 = sqrt(3.0 / (4.0 * pi));
    const double c2a = 0.5 * sqrt(15.0 / pi);
    const double c2b = 0.25 * sqrt(5.0 / pi);
    const double c2c = 0.25 * sqrt(15.0 / pi);
    const double c3a = 0.25 * sqrt(35.0 / (2.0 * pi));
    const double c3b = 0.5 * sqrt(105.0 / pi);
    const double c3c = 0.25 * sqrt(21.0 / (2.0 * pi));
    const double c3d = 0.25 * sqrt(7.0 / pi);
    const double c3e = 0.25 * sqrt(105.0 / pi);
    int n = 0;
#define T(J, C, A, B, CC) do { t[n].j = (J); t[n].coef = (C); t[n].a = (A); t[n].b = (B); t[n].c = (CC); n++; } while (0)
    T(0, c0, 0, 0, 0);
    T(1, -c1, 0, 1, 0);                    /* l=1 m=-1: -c1 y */
    T(2, c1, 0, 0, 1);                     /* l=1 m= 0:  c1 z */
    T(3, -c1, 1, 0, 0);                    /* l=1 m=+1: -c1 x */
    T(4, c2a, 1, 1, 0);                    /* l=2 m=-2:  c2a xy */
    T(5, -c2a, 0, 1, 1);                   /* l=2 m=-1: -c2a yz */
    T(6, 2 * c2b, 0, 0, 2); T(6, -c2b, 2, 0, 0); T(6, -c2b, 0, 2, 0); /* c2b (2zz-xx-yy) */
    T(7, -c2a, 1, 0, 1);                   /* l=2 m=+1: -c2a xz */
    T(8, c2c, 2, 0, 0); T(8, -c2c, 0, 2, 0);  /* c2c (xx-yy) */
    T(9, -3 * c3a, 2, 1, 0); T(9, c3a, 0, 3, 0);            /* -c3a y(3xx-yy) */
    T(10, c3b, 1, 1, 1);                                   /*  c3b xyz */
    T(11, -4 * c3c, 0, 1, 2); T(11, c3c, 2, 1, 0); T(11, c3c, 0, 3, 0);  /* -c3c y(4zz-xx-yy) */
    T(12, 2 * c3d, 0, 0, 3); T(12, -3 * c3d, 2, 0, 1); T(12, -3 * c3d, 0, 2, 1); /* c3d z(2zz-3xx-3yy) */
    T(13, -4 * c3c, 1, 0, 2); T(13, c3c, 3, 0, 0); T(13, c3c, 1, 2, 0);  /* -c3c x(4zz-xx-yy) */
    T(14, c3e, 2, 0, 1); T(14, -c3e, 0, 2, 1);             /*  c3e z(xx-yy) */
    T(15, -c3a, 3, 0, 0); T(15, 3 * c3a, 1, 2, 0);         /* -c3a x(xx-3yy) */
#undef T
    return n;
}

static double ipow(double x, int k)
{
    double r = 1.0;
    for (int i = 0; i < k; i++) r *= x;
    return r;
}

/* Y[j] for j < K, and (if dY != NULL) the partials dY[j][0..2] of the
 * monomial form with respect to the direction components. */
static void sh_eval(int K, const double d[3], double* Y, double (*dY)[3])
{
    sh_term t[32];
    int n = sh_table(t);
    for (int j = 0; j < K; j++) {
        Y[j] = 0.0;
        if (dY) dY[j][0] = dY[j][1] = dY[j][2] = 0.0;
    }
    for (int i = 0; i < n; i++) {
        if (t[i].j >= K) continue;
        int a = t[i].a, b = t[i].b, c = t[i].c;
        Y[t[i].j] += t[i].coef * ipow(d[0], a) * ipow(d[1], b) * ipow(d[2], c);
        if (dY) {
            if (a) dY[t[i].j][0] += t[i].coef * a * ipow(d[0], a - 1) * ipow(d[1], b) * ipow(d[2], c);
            if (b) dY[t[i].j][1] += t[i].coef * b * ipow(d[0], a) * ipow(d[1], b - 1) * ipow(d[2], c);
            if (c) dY[t[i].j][2] += t[i].coef * c * ipow(d[0], a) * ipow(d[1], b) * ipow(d[2], c - 1);
        }
    }
}

/* exported for the basis pins: Y (K values) at one direction */
void or_sh_basis(int K, const double* d, double* Y) { sh_eval(K, d, Y, NULL); }

/* ------------------------------------------------------------------------- */
/* Small matrix helpers (row-major).                                           */
/* ------------------------------------------------------------------------- */
static void mat_mul(const double* A, const double* B, double* C, int n, int k, int m)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < m; j++) {
            double s = 0.0;
            for (int l = 0; l < k; l++) s += A[i * k + l] * B[l * m + j];
            C[i * m + j] = s;
        }
}

static void mat_t(const double* A, double* B, int n, int m)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < m; j++) B[j * n + i] = A[i * m + j];
}

/* rotation matrix of a unit quaternion (w, x, y, z) */
static void quat_rot(const double q[4], double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

void or_quat_rot(const double* q, double* R)
{
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double qh[4] = {q[0] / n, q[1] / n, q[2] / n, q[3] / n};
    quat_rot(qh, R);
}

static int finite_all(const double* a, int n)
{
    for (int i = 0; i < n; i++)
        if (!isfinite(a[i])) return 0;
    return 1;
}

/* distance of x to the nearest integer, relative to max(|x|, 1) */
static double int_margin(double x)
{
    double r = fabs(x - nearbyint(x));
    double s = fabs(x) > 1.0 ? fabs(x) : 1.0;
    return r / s;
}

static double rel_margin(double x, double thr)
{
    return fabs(x - thr) / fabs(thr);
}

/* tile rectangle of one splat in float32 arithmetic (reading R8) */
static void tile_rect(float u, float v, int rx, int ry, int tile, int W, int H, int r[4])
{
    int TX = (W + tile - 1) / tile, TY = (H + tile - 1) / tile;
    float ts = (float)tile;
    float fx0 = floorf((u - (float)rx) / ts);
    float fx1 = floorf((u + (float)rx) / ts) + 1.0f;
    float fy0 = floorf((v - (float)ry) / ts);
    float fy1 = floorf((v + (float)ry) / ts) + 1.0f;
    fx0 = fx0 < 0.0f ? 0.0f : (fx0 > (float)TX ? (float)TX : fx0);
    fx1 = fx1 < 0.0f ? 0.0f : (fx1 > (float)TX ? (float)TX : fx1);
    fy0 = fy0 < 0.0f ? 0.0f : (fy0 > (float)TY ? (float)TY : fy0);
    fy1 = fy1 < 0.0f ? 0.0f : (fy1 > (float)TY ? (float)TY : fy1);
    r[0] = (int)fx0; r[1] = (int)fy0; r[2] = (int)fx1; r[3] = (int)fy1;
}

void or_tile_rect(float u, float v, int rx, int ry, int tile, int W, int H, int32_t* r)
{
    int rr[4];
    tile_rect(u, v, rx, ry, tile, W, H, rr);
    for (int i = 0; i < 4; i++) r[i] = rr[i];
}

/* tile rectangles of n Gaussians: radii [2][n]; out [n][4] = x0, y0, x1, y1
 * (all zero where the radii are zero, i.e. culled) */
void or_tile_rects(int64_t n, const float* u, const float* v, const int32_t* radii, int tile, int W, int H,
                   int32_t* out)
{
    for (int64_t g = 0; g < n; g++) {
        int rr[4] = {0, 0, 0, 0};
        if (radii[g] > 0 || radii[n + g] > 0) tile_rect(u[g], v[g], radii[g], radii[n + g], tile, W, H, rr);
        for (int i = 0; i < 4; i++) out[4 * g + i] = rr[i];
    }
}

/* ------------------------------------------------------------------------- */
/* Projection + SH colour, forward, one view.                                  */
/* ------------------------------------------------------------------------- */
typedef struct {
    double z, x, y;            /* camera-space mean */
    double u, v;               /* pixel-space mean */
    double cov[3];             /* Sigma2: a, b, c */
    double conic[3];           /* A, B, C */
    double sigma;
    double rgb[3];
    int clamp[3];
    int rx, ry;
    int tiles;
    int visible;
    double margin;             /* smallest relative distance to a decision boundary */
    double margin_img;         /* the same over the decisions that can change an image discontinuously
                                  (visibility, radii, tile rectangle); the Jacobian and colour clamps
                                  are continuous in value */
    /* quantities reused by the backward */
    double R[9], s[3], qn[4], qnorm, Wr[9], J[6], Sc[9], dirv[3], dnorm, d[3];
    int clx, cly;
    double rxz, ryz;
} proj_t;

static void project_one(int64_t g, int64_t N, int K, const double* means, const double* log_scales,
                        const double* quats, const double* opac, const double* sh,
                        const double* vm, const double* intr, int W, int H,
                        double near_, double far_, double eps2d, int tile, int radius_mode, proj_t* P)
{
    memset(P, 0, sizeof(*P));
    P->margin = INFINITY;
    P->margin_img = INFINITY;
    double mu[3] = {means[g], means[N + g], means[2 * N + g]};
    double ls[3] = {log_scales[g], log_scales[N + g], log_scales[2 * N + g]};
    double q[4] = {quats[g], quats[N + g], quats[2 * N + g], quats[3 * N + g]};
    double o = opac[g];
    int ok = finite_all(mu, 3) && finite_all(ls, 3) && finite_all(q, 4) && isfinite(o);
    for (int j = 0; ok && j < K; j++)
        for (int c = 0; c < 3; c++)
            if (!isfinite(sh[((int64_t)j * 3 + c) * N + g])) ok = 0;
    if (!ok) return;

    double fx = intr[0], fy = intr[1], cx = intr[2], cy = intr[3];
    double Wr[9] = {vm[0], vm[1], vm[2], vm[4], vm[5], vm[6], vm[8], vm[9], vm[10]};
    double tv[3] = {vm[3], vm[7], vm[11]};
    memcpy(P->Wr, Wr, sizeof Wr);

    /* camera-space mean, p = W mu + t */
    double p[3];
    for (int i = 0; i < 3; i++) p[i] = Wr[3 * i] * mu[0] + Wr[3 * i + 1] * mu[1] + Wr[3 * i + 2] * mu[2] + tv[i];
    P->x = p[0]; P->y = p[1]; P->z = p[2];
    double z = p[2];
    P->margin = fmin(P->margin, rel_margin(z, near_));
    P->margin_img = fmin(P->margin_img, rel_margin(z, near_));
    if (z <= near_ || z >= far_) return;

    /* opacity */
    P->sigma = 1.0 / (1.0 + exp(-o));
    P->margin = fmin(P->margin, rel_margin(P->sigma, OR_ALPHA_MIN));
    P->margin_img = fmin(P->margin_img, rel_margin(P->sigma, OR_ALPHA_MIN));
    if (P->sigma < OR_ALPHA_MIN) return;

    /* 3-D covariance Sigma = R S S^T R^T */
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(qn > 0.0)) return;
    P->qnorm = qn;
    for (int i = 0; i < 4; i++) P->qn[i] = q[i] / qn;
    quat_rot(P->qn, P->R);
    for (int i = 0; i < 3; i++) P->s[i] = exp(ls[i]);
    double M[9], Mt[9], Sig[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) M[3 * i + j] = P->R[3 * i + j] * P->s[j];
    mat_t(M, Mt, 3, 3);
    mat_mul(M, Mt, Sig, 3, 3, 3);

    /* camera-space covariance W Sigma W^T */
    double Wt[9], tmp[9];
    mat_t(Wr, Wt, 3, 3);
    mat_mul(Wr, Sig, tmp, 3, 3, 3);
    mat_mul(tmp, Wt, P->Sc, 3, 3, 3);

    /* Jacobian of the perspective projection at the (clamped) mean */
    double limx = OR_CLIP * (0.5 * W / fx), limy = OR_CLIP * (0.5 * H / fy);
    double rxz = p[0] / z, ryz = p[1] / z;
    P->margin = fmin(P->margin, rel_margin(fabs(rxz), limx));
    P->margin = fmin(P->margin, rel_margin(fabs(ryz), limy));
    P->clx = (rxz < -limx || rxz > limx);
    P->cly = (ryz < -limy || ryz > limy);
    if (rxz < -limx) rxz = -limx;
    if (rxz > limx) rxz = limx;
    if (ryz < -limy) ryz = -limy;
    if (ryz > limy) ryz = limy;
    P->rxz = rxz; P->ryz = ryz;
    double J[6] = {fx / z, 0.0, -fx * rxz / z, 0.0, fy / z, -fy * ryz / z};
    memcpy(P->J, J, sizeof J);
    double Jt[6], JS[6], S2[4];
    mat_t(J, Jt, 2, 3);
    mat_mul(J, P->Sc, JS, 2, 3, 3);
    mat_mul(JS, Jt, S2, 2, 3, 2);
    double a = S2[0] + eps2d, b = S2[1], c = S2[3] + eps2d;
    P->cov[0] = a; P->cov[1] = b; P->cov[2] = c;
    double det = a * c - b * b;
    if (!(det > 0.0)) return;
    P->conic[0] = c / det; P->conic[1] = -b / det; P->conic[2] = a / det;

    /* pixel-space mean */
    P->u = fx * p[0] / z + cx;
    P->v = fy * p[1] / z + cy;

    /* radii (half-widths of the screen box that selects tiles):
     *  0: 3-sigma box per axis, ceil(3 sqrt(a)), ceil(3 sqrt(c));
     *  1: opacity-aware, the smaller of the 3-sigma box and the box of the
     *     region alpha >= 1/255, i.e. d^T conic d <= tau = 2 ln(255 sigma),
     *     with tau widened to 1.001 tau + 0.01 and one pixel of padding so
     *     that float32 evaluation of alpha never reaches outside it;
     *  2: the square of 3D Gaussian Splatting, 3 sqrt(lambda_max) on both
     *     axes with lambda_max = m + sqrt(max(m^2 - det, 0.1)), m = (a + c) / 2. */
    double ex = 3.0 * sqrt(a), ey = 3.0 * sqrt(c);
    if (radius_mode == 2) {
        double m = 0.5 * (a + c);
        ex = ey = 3.0 * sqrt(m + sqrt(fmax(m * m - det, 0.1)));
    }
    P->margin = fmin(P->margin, int_margin(ex));
    P->margin_img = fmin(P->margin_img, int_margin(ex));
    P->margin = fmin(P->margin, int_margin(ey));
    P->margin_img = fmin(P->margin_img, int_margin(ey));
    P->rx = (int)fmin(ceil(ex), 1073741824.0);   /* radii saturate at 2^30 px */
    P->ry = (int)fmin(ceil(ey), 1073741824.0);
    if (radius_mode == 1) {
        double tau = 2.0 * log(255.0 * P->sigma);
        tau = (tau > 0.0 ? tau : 0.0) * 1.001 + 0.01;
        double ax = sqrt(tau * a), ay = sqrt(tau * c);
        P->margin = fmin(P->margin, int_margin(ax));
        P->margin_img = fmin(P->margin_img, int_margin(ax));
        P->margin = fmin(P->margin, int_margin(ay));
        P->margin_img = fmin(P->margin_img, int_margin(ay));
        int qx = (int)fmin(ceil(ax), 1073741823.0) + 1, qy = (int)fmin(ceil(ay), 1073741823.0) + 1;
        if (qx < P->rx) P->rx = qx;
        if (qy < P->ry) P->ry = qy;
    }

    /* tile rectangle, float32 arithmetic on float32-rounded values */
    /* a floor decision can change the rectangle only where it is not clamped */
    float uf = (float)P->u, vf = (float)P->v;
    double ts = (double)tile;
    double TXd = (double)((W + tile - 1) / tile), TYd = (double)((H + tile - 1) / tile);
    double edges[4] = {((double)uf - P->rx) / ts, ((double)uf + P->rx) / ts,
                       ((double)vf - P->ry) / ts, ((double)vf + P->ry) / ts};
    for (int e = 0; e < 4; e++) {
        double hi = e < 2 ? TXd : TYd;
        if (edges[e] > -1.0 && edges[e] < hi + 1.0) {
            /* distance to the tile boundary in pixels, relative to the size of
             * the coordinate (which sets its float32 rounding error) */
            double mag = e < 2 ? fabs((double)uf) : fabs((double)vf);
            double d = fabs(edges[e] - nearbyint(edges[e])) * ts;
            P->margin = fmin(P->margin, d / (mag > ts ? mag : ts));
            P->margin_img = fmin(P->margin_img, d / (mag > ts ? mag : ts));
        }
    }
    int r[4];
    tile_rect(uf, vf, P->rx, P->ry, tile, W, H, r);
    P->tiles = (r[2] - r[0]) * (r[3] - r[1]);
    if (P->tiles <= 0) { P->tiles = 0; return; }

    /* colour: SH along the unit ray from the camera centre, + 0.5, clamp >= 0 */
    double cam[3];
    for (int i = 0; i < 3; i++) cam[i] = -(Wr[i] * tv[0] + Wr[3 + i] * tv[1] + Wr[6 + i] * tv[2]);
    for (int i = 0; i < 3; i++) P->dirv[i] = mu[i] - cam[i];
    P->dnorm = sqrt(P->dirv[0] * P->dirv[0] + P->dirv[1] * P->dirv[1] + P->dirv[2] * P->dirv[2]);
    for (int i = 0; i < 3; i++) P->d[i] = P->dirv[i] / P->dnorm;
    double Y[16];
    sh_eval(K, P->d, Y, NULL);
    for (int ch = 0; ch < 3; ch++) {
        double acc = 0.0, mag = 0.0;
        for (int j = 0; j < K; j++) {
            double t = sh[((int64_t)j * 3 + ch) * N + g] * Y[j];
            acc += t;
            mag += fabs(t);
        }
        acc += 0.5;
        mag += 0.5;
        P->margin = fmin(P->margin, fabs(acc) / mag);
        P->clamp[ch] = acc < 0.0;
        P->rgb[ch] = acc < 0.0 ? 0.0 : acc;
    }
    P->visible = 1;
}

/*
 * Forward projection of N Gaussians into one view.  Outputs (N each unless
 * stated): u, v, depth, cov [3][N] (a, b, c of Sigma2), conic [3][N] (A, B, C),
 * sigma, rgb [3][N], radii [2][N], tiles, clamp (bit c = channel c clamped),
 * visible, margin (smallest relative distance of any decision to its
 * threshold) and, if not NULL, margin_img (the same over the decisions that
 * can change an image discontinuously: visibility, radii, tile rectangle).
 * Culled Gaussians have visible = 0, radii = 0, tiles = 0.
 */
int or_project(int64_t N, int sh_degree, const double* means, const double* log_scales,
               const double* quats, const double* opac, const double* sh,
               const double* viewmat, const double* intr, int W, int H,
               double near_, double far_, double eps2d, int tile, int radius_mode,
               double* u, double* v, double* depth, double* cov, double* conic,
               double* sigma, double* rgb, int32_t* radii, int32_t* tiles,
               uint8_t* clamp, uint8_t* visible, double* margin, double* margin_img)
{
    if (N < 0 || sh_degree < 0 || sh_degree > 3 || W <= 0 || H <= 0 || tile <= 0 || radius_mode < 0 ||
        radius_mode > 2)
        return -1;
    int K = (sh_degree + 1) * (sh_degree + 1);
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1)
    for (int64_t g = 0; g < N; g++) {
        proj_t P;
        project_one(g, N, K, means, log_scales, quats, opac, sh, viewmat, intr, W, H,
                    near_, far_, eps2d, tile, radius_mode, &P);
        u[g] = P.u; v[g] = P.v; depth[g] = P.z;
        for (int i = 0; i < 3; i++) {
            cov[i * N + g] = P.cov[i];
            conic[i * N + g] = P.conic[i];
            rgb[i * N + g] = P.rgb[i];
        }
        sigma[g] = P.sigma;
        radii[g] = P.visible ? P.rx : 0;
        radii[N + g] = P.visible ? P.ry : 0;
        tiles[g] = P.visible ? P.tiles : 0;
        clamp[g] = (uint8_t)(P.clamp[0] | (P.clamp[1] << 1) | (P.clamp[2] << 2));
        visible[g] = (uint8_t)P.visible;
        margin[g] = P.margin;
        if (margin_img) margin_img[g] = P.margin_img;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Binning: one (tile | depth) key per (Gaussian, tile), stable sort, ranges.  */
/* ------------------------------------------------------------------------- */

/*
 * Emit the intersections of one view.  Inputs are float32 (u, v, depth) and
 * int radii [2][N]; a Gaussian with radii (0, 0) is culled.  For each Gaussian
 * in index order, and for each tile of its rectangle in row-major order, write
 * key = ((tile_offset + ty*TX + tx) << 32) | bits(depth) and value g.
 * Returns the number of intersections (writes at most cap of them).
 */
int64_t or_bin_emit(int64_t N, const float* u, const float* v, const float* depth,
                    const int32_t* radii, int W, int H, int tile, int64_t tile_offset,
                    uint64_t* keys, int32_t* vals, int64_t cap)
{
    int TX = (W + tile - 1) / tile;
    int64_t m = 0;
    for (int64_t g = 0; g < N; g++) {
        int rx = radii[g], ry = radii[N + g];
        if (rx == 0 && ry == 0) continue;
        int r[4];
        tile_rect(u[g], v[g], rx, ry, tile, W, H, r);
        uint32_t zb;
        memcpy(&zb, &depth[g], 4);
        for (int ty = r[1]; ty < r[3]; ty++)
            for (int tx = r[0]; tx < r[2]; tx++) {
                if (m < cap) {
                    uint64_t t = (uint64_t)(tile_offset + (int64_t)ty * TX + tx);
                    keys[m] = (t << 32) | (uint64_t)zb;
                    vals[m] = (int32_t)g;
                }
                m++;
            }
    }
    return m;
}

typedef struct { uint64_t key; int64_t pos; int32_t val; } kv_t;

static int kv_cmp(const void* a, const void* b)
{
    const kv_t* x = (const kv_t*)a;
    const kv_t* y = (const kv_t*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->pos != y->pos) return x->pos < y->pos ? -1 : 1;
    return 0;
}

/* stable sort of (key, value) pairs by key: equal keys keep input order */
int or_sort_pairs(int64_t M, uint64_t* keys, int32_t* vals)
{
    kv_t* t = (kv_t*)malloc(sizeof(kv_t) * (size_t)(M > 0 ? M : 1));
    if (!t) return -1;
    for (int64_t i = 0; i < M; i++) { t[i].key = keys[i]; t[i].pos = i; t[i].val = vals[i]; }
    qsort(t, (size_t)M, sizeof(kv_t), kv_cmp);
    for (int64_t i = 0; i < M; i++) { keys[i] = t[i].key; vals[i] = t[i].val; }
    free(t);
    return 0;
}

/* ranges[2*t] = first, ranges[2*t+1] = one past last index of tile t in the
 * sorted keys (both 0 for an empty tile); n_tiles counts all views' tiles. */
int or_tile_ranges(int64_t M, const uint64_t* keys, int64_t n_tiles, int32_t* ranges)
{
    for (int64_t t = 0; t < 2 * n_tiles; t++) ranges[t] = 0;
    for (int64_t i = 0; i < M; i++) {
        int64_t t = (int64_t)(keys[i] >> 32);
        if (t < 0 || t >= n_tiles) return -1;
        if (i == 0 || (keys[i - 1] >> 32) != keys[i] >> 32) ranges[2 * t] = (int32_t)i;
        if (i == M - 1 || (keys[i + 1] >> 32) != keys[i] >> 32) ranges[2 * t + 1] = (int32_t)(i + 1);
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Compositing.                                                                */
/* ------------------------------------------------------------------------- */
typedef struct {
    double A, B, C, sig, dx, dy, G, a, alpha;
    int clamped, g;
} visit_t;

/*
 * Front-to-back compositing of one pixel over its tile's list.  Writes the
 * colour (without background), the final transmittance, the contributor count
 * (one past the list position of the last Gaussian composited) and the number
 * of list entries examined; returns the smallest relative distance of any
 * decision (alpha skip, alpha clamp, stop) to its threshold.  If `kept` is not
 * NULL the composited Gaussians are stored there in order and *nkept set.
 */
static double composite_pixel(double px, double py, int s, int e, const int32_t* vals,
                              const double* u, const double* v, const double* cA,
                              const double* cB, const double* cC, const double* sig,
                              const double* rgb, int64_t N, double C[3], double* Tout,
                              int* last, int* visits, visit_t* kept, int* nkept)
{
    double T = 1.0, margin = INFINITY;
    C[0] = C[1] = C[2] = 0.0;
    *last = 0;
    *visits = 0;
    int nk = 0;
    for (int k = s; k < e; k++) {
        int g = vals[k];
        (*visits)++;
        double dx = u[g] - px, dy = v[g] - py;
        double power = -0.5 * (cA[g] * dx * dx + cC[g] * dy * dy) - cB[g] * dx * dy;
        if (power > 0.0) continue;
        double G = exp(power);
        double a = sig[g] * G;
        margin = fmin(margin, rel_margin(a, OR_ALPHA_MAX));
        double alpha = a < OR_ALPHA_MAX ? a : OR_ALPHA_MAX;
        margin = fmin(margin, rel_margin(alpha, OR_ALPHA_MIN));
        if (alpha < OR_ALPHA_MIN) continue;
        double Tn = T * (1.0 - alpha);
        margin = fmin(margin, rel_margin(Tn, OR_T_MIN));
        if (Tn < OR_T_MIN) break;
        for (int c = 0; c < 3; c++) C[c] += alpha * T * rgb[c * N + g];
        if (kept) {
            visit_t* t = &kept[nk];
            t->A = cA[g]; t->B = cB[g]; t->C = cC[g]; t->sig = sig[g];
            t->dx = dx; t->dy = dy; t->G = G; t->a = a; t->alpha = alpha;
            t->clamped = !(a < OR_ALPHA_MAX); t->g = g;
        }
        nk++;
        T = Tn;
        *last = k - s + 1;
    }
    *Tout = T;
    if (nkept) *nkept = nk;
    return margin;
}

/*
 * Forward rasterisation of one view.  ranges holds [2] ints per tile of this
 * view (list positions into vals); img is [3][H][W] and includes T * bg.
 */
int or_raster_fwd(int W, int H, int tile, const int32_t* ranges, const int32_t* vals, int64_t N,
                  const double* u, const double* v, const double* cA, const double* cB,
                  const double* cC, const double* sig, const double* rgb, const double* bg,
                  double* img, double* Tfin, int32_t* last, int32_t* visits, double* margin)
{
    if (W <= 0 || H <= 0 || tile <= 0) return -1;
    int TX = (W + tile - 1) / tile;
#pragma omp parallel for schedule(dynamic, 1) num_threads(g_threads) if (g_threads > 1)
    for (int j = 0; j < H; j++)
        for (int i = 0; i < W; i++) {
            int t = (j / tile) * TX + i / tile;
            double C[3], T;
            int l, nv;
            double m = composite_pixel(i + 0.5, j + 0.5, ranges[2 * t], ranges[2 * t + 1], vals,
                                       u, v, cA, cB, cC, sig, rgb, N, C, &T, &l, &nv, NULL, NULL);
            int64_t p = (int64_t)j * W + i;
            for (int c = 0; c < 3; c++) img[(int64_t)c * W * H + p] = C[c] + T * bg[c];
            Tfin[p] = T;
            last[p] = l;
            visits[p] = nv;
            margin[p] = m;
        }
    return 0;
}

/*
 * Forward rasterisation of the pixel rectangle [x0, x1) x [y0, y1) of one view
 * (the same per-pixel compositing as or_raster_fwd), for local re-rendering.
 * img is [3][y1 - y0][x1 - x0] and includes T * bg; sig[(y1 - y0)(x1 - x0)]
 * receives each pixel's decision signature: a hash of the ordered list of the
 * Gaussians it composited, each with its 0.99-clamp flag, and of its stop
 * position, so two renders took the same discrete decisions at a pixel iff
 * (up to hash collisions) their signatures agree.
 */
int or_raster_fwd_rect(int W, int H, int tile, const int32_t* ranges, const int32_t* vals, int64_t N,
                       const double* u, const double* v, const double* cA, const double* cB,
                       const double* cC, const double* sig, const double* rgb, const double* bg,
                       int x0, int y0, int x1, int y1, double* img, uint64_t* sigout)
{
    if (W <= 0 || H <= 0 || tile <= 0 || x0 < 0 || y0 < 0 || x1 > W || y1 > H || x0 >= x1 || y0 >= y1)
        return -1;
    int TX = (W + tile - 1) / tile;
    int64_t maxlen = 0;
    for (int ty = y0 / tile; ty <= (y1 - 1) / tile; ty++)
        for (int tx = x0 / tile; tx <= (x1 - 1) / tile; tx++) {
            int64_t t = (int64_t)ty * TX + tx;
            if (ranges[2 * t + 1] - ranges[2 * t] > maxlen) maxlen = ranges[2 * t + 1] - ranges[2 * t];
        }
    visit_t* kept = (visit_t*)malloc(sizeof(visit_t) * (size_t)(maxlen + 1));
    if (!kept) return -2;
    const int w = x1 - x0, h = y1 - y0;
    for (int j = y0; j < y1; j++)
        for (int i = x0; i < x1; i++) {
            int t = (j / tile) * TX + i / tile;
            double C[3], T;
            int l, nv, nk;
            composite_pixel(i + 0.5, j + 0.5, ranges[2 * t], ranges[2 * t + 1], vals, u, v, cA, cB, cC, sig,
                            rgb, N, C, &T, &l, &nv, kept, &nk);
            int64_t q = (int64_t)(j - y0) * w + (i - x0);
            for (int c = 0; c < 3; c++) img[(int64_t)c * w * h + q] = C[c] + T * bg[c];
            /* FNV-1a over (g, clamped) of every composited entry, then the stop position */
            uint64_t hsh = 1469598103934665603ull;
            for (int k = 0; k < nk; k++) {
                uint64_t x = ((uint64_t)(uint32_t)kept[k].g << 1) | (uint64_t)(kept[k].clamped != 0);
                for (int b = 0; b < 8; b++) { hsh ^= (x >> (8 * b)) & 0xFFu; hsh *= 1099511628211ull; }
            }
            hsh ^= (uint64_t)(uint32_t)nv;
            hsh *= 1099511628211ull;
            sigout[q] = hsh;
        }
    free(kept);
    return 0;
}

/*
 * Backward rasterisation of one view: the exact derivative of the forward
 * with the pixel's decisions frozen.  For each pixel the composited Gaussians
 * are recomputed front to back with their transmittances T_k = prod_{j<k}
 * (1 - alpha_j), and
 *   dC/dc_k     = alpha_k T_k,
 *   dC/dalpha_k = T_k c_k - (sum_{j>k} alpha_j T_j c_j + T_N bg) / (1 - alpha_k),
 *   d(1-T_N)/dalpha_k = T_N / (1 - alpha_k);
 * alpha = sigma G with G = exp(power) unless clamped at 0.99 (then constant),
 * power = -(A dx^2 + C dy^2)/2 - B dx dy, dx = u - px, dy = v - py.
 * d_img is [3][H][W]; d_alpha ([H][W]) may be NULL.  Gradients are ADDED to
 * g_u, g_v, g_A, g_B, g_C, g_sig (N each) and g_rgb ([3][N]).
 */
/* one term added to a per-Gaussian sum (atomically when pixels run in parallel) */
#define ACC(dst, val)                           \
    do {                                        \
        const double acc_v_ = (val);            \
        if (par) {                              \
            _Pragma("omp atomic")               \
            (dst) += acc_v_;                    \
        } else {                                \
            (dst) += acc_v_;                    \
        }                                       \
    } while (0)

int or_raster_bwd(int W, int H, int tile, const int32_t* ranges, const int32_t* vals, int64_t N,
                  const double* u, const double* v, const double* cA, const double* cB,
                  const double* cC, const double* sig, const double* rgb, const double* bg,
                  const double* d_img, const double* d_alpha,
                  double* g_u, double* g_v, double* g_A, double* g_B, double* g_C,
                  double* g_sig, double* g_rgb)
{
    if (W <= 0 || H <= 0 || tile <= 0) return -1;
    int TX = (W + tile - 1) / tile;
    int64_t maxlen = 0;
    int64_t n_tiles = (int64_t)TX * ((H + tile - 1) / tile);
    for (int64_t t = 0; t < n_tiles; t++)
        if (ranges[2 * t + 1] - ranges[2 * t] > maxlen) maxlen = ranges[2 * t + 1] - ranges[2 * t];
    const int par = g_threads > 1;
    int failed = 0;
#pragma omp parallel num_threads(g_threads) if (par)
    {
    visit_t* kept = (visit_t*)malloc(sizeof(visit_t) * (size_t)(maxlen + 1));
    double* Tk = (double*)malloc(sizeof(double) * (size_t)(maxlen + 1));
    if (!kept || !Tk) {
#pragma omp atomic write
        failed = 1;
    }
#pragma omp for schedule(dynamic, 1)
    for (int j = 0; j < H; j++)
        for (int i = 0; i < W && kept && Tk; i++) {
            int t = (j / tile) * TX + i / tile;
            double C[3], TN;
            int l, nv, nk;
            composite_pixel(i + 0.5, j + 0.5, ranges[2 * t], ranges[2 * t + 1], vals, u, v, cA, cB,
                            cC, sig, rgb, N, C, &TN, &l, &nv, kept, &nk);
            int64_t p = (int64_t)j * W + i;
            double gC[3] = {d_img[p], d_img[(int64_t)W * H + p], d_img[2 * (int64_t)W * H + p]};
            double gA = d_alpha ? d_alpha[p] : 0.0;
            double T = 1.0;
            for (int k = 0; k < nk; k++) { Tk[k] = T; T *= 1.0 - kept[k].alpha; }
            /* behind[c] = sum_{j>k} alpha_j T_j c_j + T_N bg, built from the back */
            double behind[3] = {TN * bg[0], TN * bg[1], TN * bg[2]};
            for (int k = nk - 1; k >= 0; k--) {
                visit_t* q = &kept[k];
                int g = q->g;
                double c[3] = {rgb[g], rgb[N + g], rgb[2 * N + g]};
                double dalpha = 0.0;
                for (int ch = 0; ch < 3; ch++) {
                    ACC(g_rgb[ch * N + g], q->alpha * Tk[k] * gC[ch]);
                    dalpha += (Tk[k] * c[ch] - behind[ch] / (1.0 - q->alpha)) * gC[ch];
                }
                dalpha += gA * TN / (1.0 - q->alpha);
                for (int ch = 0; ch < 3; ch++) behind[ch] += q->alpha * Tk[k] * c[ch];
                if (q->clamped) continue;
                ACC(g_sig[g], q->G * dalpha);
                double gp = q->sig * q->G * dalpha;   /* d alpha / d power = alpha */
                ACC(g_A[g], -0.5 * q->dx * q->dx * gp);
                ACC(g_B[g], -q->dx * q->dy * gp);
                ACC(g_C[g], -0.5 * q->dy * q->dy * gp);
                ACC(g_u[g], -(q->A * q->dx + q->B * q->dy) * gp);
                ACC(g_v[g], -(q->B * q->dx + q->C * q->dy) * gp);
            }
        }
    free(kept);
    free(Tk);
    }
    return failed ? -2 : 0;
}

/* ------------------------------------------------------------------------- */
/* Projection + SH backward, one view, gradients ADDED into the outputs.       */
/* ------------------------------------------------------------------------- */

/* d R / d q for R = quat_rot(q), q = (w, x, y, z): dR[k][9] for k = w,x,y,z */
static void quat_rot_grad(const double q[4], double dR[4][9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double d[4][9] = {
        /* d/dw */ {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0},
        /* d/dx */ {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x},
        /* d/dy */ {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y},
        /* d/dz */ {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0},
    };
    memcpy(dR, d, sizeof d);
}

/*
 * Upstream gradients per Gaussian: g_uv [2][N] (u, v), g_conic [3][N] (A, B, C
 * of the conic [[A, B], [B, C]]), g_sig [N], g_rgb [3][N].  Culled Gaussians
 * receive nothing.  Gradients are added to d_means [3][N], d_log_scales [3][N],
 * d_quats [4][N], d_opac [N], d_sh [K][3][N].
 */
int or_project_bwd(int64_t N, int sh_degree, const double* means, const double* log_scales,
                   const double* quats, const double* opac, const double* sh,
                   const double* viewmat, const double* intr, int W, int H,
                   double near_, double far_, double eps2d, int tile, int radius_mode,
                   const double* g_uv, const double* g_conic, const double* g_sig,
                   const double* g_rgb, double* d_means, double* d_log_scales,
                   double* d_quats, double* d_opac, double* d_sh)
{
    if (N < 0 || sh_degree < 0 || sh_degree > 3) return -1;
    int K = (sh_degree + 1) * (sh_degree + 1);
    double fx = intr[0], fy = intr[1];
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1)
    for (int64_t g = 0; g < N; g++) {
        proj_t P;
        project_one(g, N, K, means, log_scales, quats, opac, sh, viewmat, intr, W, H,
                    near_, far_, eps2d, tile, radius_mode, &P);
        if (!P.visible) continue;
        double gmu[3] = {0, 0, 0};

        /* opacity: sigma = 1 / (1 + exp(-o)) */
        d_opac[g] += g_sig[g] * P.sigma * (1.0 - P.sigma);

        /* colour */
        double Y[16], dY[16][3];
        sh_eval(K, P.d, Y, dY);
        double gd[3] = {0, 0, 0};
        for (int ch = 0; ch < 3; ch++) {
            if (P.clamp[ch]) continue;
            double gc = g_rgb[ch * N + g];
            for (int j = 0; j < K; j++) {
                double k = sh[((int64_t)j * 3 + ch) * N + g];
                d_sh[((int64_t)j * 3 + ch) * N + g] += Y[j] * gc;
                for (int i = 0; i < 3; i++) gd[i] += k * dY[j][i] * gc;
            }
        }
        /* d = dirv / |dirv|, dirv = mu - cam */
        double dg = P.d[0] * gd[0] + P.d[1] * gd[1] + P.d[2] * gd[2];
        for (int i = 0; i < 3; i++) gmu[i] += (gd[i] - P.d[i] * dg) / P.dnorm;

        /* conic = Sigma2^{-1}:  dL/dSigma2 = -Q G Q, G = [[gA, gB/2], [gB/2, gC]] */
        double a = P.cov[0], b = P.cov[1], c = P.cov[2];
        double det = a * c - b * b;
        double Q[4] = {c / det, -b / det, -b / det, a / det};
        double Gq[4] = {g_conic[g], 0.5 * g_conic[N + g], 0.5 * g_conic[N + g], g_conic[2 * N + g]};
        double t1[4], GS[4];
        mat_mul(Q, Gq, t1, 2, 2, 2);
        mat_mul(t1, Q, GS, 2, 2, 2);
        for (int i = 0; i < 4; i++) GS[i] = -GS[i];

        /* Sigma2 = J Sc J^T + eps I:  dJ = 2 GS J Sc,  dSc = J^T GS J */
        double GJ[6], tJ[6], Jt[6], tmp[6], GSc[9];
        mat_mul(GS, P.J, tJ, 2, 2, 3);
        mat_mul(tJ, P.Sc, GJ, 2, 3, 3);
        for (int i = 0; i < 6; i++) GJ[i] *= 2.0;
        mat_t(P.J, Jt, 2, 3);
        mat_mul(Jt, GS, tmp, 3, 2, 2);
        mat_mul(tmp, P.J, GSc, 3, 2, 3);

        /* Sc = Wr Sigma Wr^T:  dSigma = Wr^T dSc Wr */
        double Wt[9], t3[9], GSig[9];
        mat_t(P.Wr, Wt, 3, 3);
        mat_mul(Wt, GSc, t3, 3, 3, 3);
        mat_mul(t3, P.Wr, GSig, 3, 3, 3);

        /* Sigma = M M^T, M = R diag(s):  dM = 2 dSigma M */
        double M[9], GM[9];
        for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) M[3 * i + j] = P.R[3 * i + j] * P.s[j];
        mat_mul(GSig, M, GM, 3, 3, 3);
        for (int i = 0; i < 9; i++) GM[i] *= 2.0;
        /* scales: s_j = exp(l_j) */
        for (int j = 0; j < 3; j++) {
            double gs = 0.0;
            for (int i = 0; i < 3; i++) gs += GM[3 * i + j] * P.R[3 * i + j];
            d_log_scales[j * N + g] += gs * P.s[j];
        }
        /* rotation: dR_ij = dM_ij s_j, then through q_hat = q / |q| */
        double dR[4][9], gqh[4] = {0, 0, 0, 0};
        quat_rot_grad(P.qn, dR);
        for (int k = 0; k < 4; k++)
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) gqh[k] += GM[3 * i + j] * P.s[j] * dR[k][3 * i + j];
        double qd = 0.0;
        for (int k = 0; k < 4; k++) qd += P.qn[k] * gqh[k];
        for (int k = 0; k < 4; k++) d_quats[k * N + g] += (gqh[k] - P.qn[k] * qd) / P.qnorm;

        /* J(p): J00 = fx/z, J02 = -fx rx/z, J11 = fy/z, J12 = -fy ry/z with
         * rx = clamp(x/z); u = fx x/z + cx, v = fy y/z + cy */
        double x = P.x, y = P.y, z = P.z;
        double gx = 0.0, gy = 0.0, gz = 0.0;
        gz += GJ[0] * (-fx / (z * z)) + GJ[4] * (-fy / (z * z));
        if (!P.clx) { gx += GJ[2] * (-fx / (z * z)); gz += GJ[2] * (2.0 * fx * x / (z * z * z)); }
        else gz += GJ[2] * (fx * P.rxz / (z * z));
        if (!P.cly) { gy += GJ[5] * (-fy / (z * z)); gz += GJ[5] * (2.0 * fy * y / (z * z * z)); }
        else gz += GJ[5] * (fy * P.ryz / (z * z));
        double gu = g_uv[g], gv = g_uv[N + g];
        gx += gu * fx / z;
        gz += -gu * fx * x / (z * z);
        gy += gv * fy / z;
        gz += -gv * fy * y / (z * z);
        /* p = Wr mu + t */
        double gp[3] = {gx, gy, gz};
        for (int i = 0; i < 3; i++) gmu[i] += P.Wr[i] * gp[0] + P.Wr[3 + i] * gp[1] + P.Wr[6 + i] * gp[2];
        for (int i = 0; i < 3; i++) d_means[i * N + g] += gmu[i];
    }
    return 0;
}
