/*
 * octmc oracle: a plain, slow FP64 CPU implementation of orthogonal-raster
 * OCT/OCTA 3-D motion correction (Ploner et al., "Efficient and high accuracy
 * 3-D OCT angiography motion correction in pathology", arXiv:2010.06931).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product path (the
 * HIP library under paper_2010_06931_amd/) shares no code, header, table or
 * helper with this file, and never calls it.
 *
 * Every quantity is computed in double precision with plain loops in the order
 * the definitions give them; there is no blocking, fusion or reordering beyond
 * what a definition states.  Per-A-scan partials are summed sequentially in
 * A-scan index order, so results are deterministic for any thread count.
 *
 * Conventions (Sec. 2.1, "definitions"):
 *   - voxel positions use 0-based pixel coordinates x_i = i, y_j = j, z_k = k;
 *   - a volume is stored [j][i][k] (depth contiguous), w = h (square, Sec. 5);
 *   - a displacement field D is [2][h][w][3]: scan V = 0 (X-fast) or 1
 *     (Y-fast), output A-scan (i, j), component (dx, dy, dz), in pixels of the
 *     current pyramid level.  Scan V's sample for output voxel (i, j, k) is
 *     taken at (i + dx, j + dy, k + dz) of its own volume ("pull" field).
 *
 * Readings of points the paper leaves open are stated where they are used.
 * Parity pins for every function live in tests/ (closed forms, invariants,
 * library routines and finite differences).  The stage-1 tilt normalisation
 * T (orc_tilt_term) has no formula in the paper, which leaves it to earlier
 * work; it is pinned to the properties its reading states (the energy of each
 * scan's common slope, zero for zero-sum tilts, independent per scan).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define EXPORT __attribute__((visibility("default")))

#ifdef _OPENMP
#include <omp.h>
#endif

/* Host threads the oracle's parallel loops use from now on (timing only:
 * every sum is formed per A-scan and combined in a fixed order, so results do
 * not depend on it).  Returns the count in effect. */
EXPORT int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Parameters of the objective and the solver.  Field meaning:
 *   alpha        weight of the scan-order regulariser R (Eq. 1)
 *   delta0       default angiography weight (Eq. 8)
 *   eps_h        pseudo-Huber parameter of the data term (Eq. 4)
 *   eps_r        pseudo-Huber parameter of R (reading: R uses a smoothed
 *                absolute difference, Sec. 2.1 "regularizers")
 *   flyback_frac flyback duration per B-scan as a fraction of the B-scan
 *                length, in A-scan periods (reading)
 *   mean_weight  gamma_M of the mean-displacement term M (reading)
 *   levels, iters, lbfgs_m, ls_max_evals, c1, c2: the L-BFGS solve
 *   merge_kappa, merge_tau: the density-based merge weights (Sec. 2.1,
 *                "merging"; reading)
 *   store        storage type of the structural volumes in the solve: 0 =
 *                exact, 1 = bfloat16, 2 = IEEE binary16; every pyramid level
 *                is built from the unrounded level above it and then rounded
 *                to nearest, ties to even (see orc_round_storage); the
 *                levels that are rounded are built in single precision
 *                (orc_pyr_down3_f32), the precision of the device pyramid,
 *                so that both sides take the same rounding decisions */
typedef struct {
    double alpha, delta0, eps_h, eps_r, flyback_frac, mean_weight;
    int levels, iters, lbfgs_m, ls_max_evals;
    double c1, c2;
    double merge_kappa, merge_tau;
    int store;
} orc_params;

/* Terms returned by orc_eval (indices). */
enum {
    T_F = 0,      /* full objective: data + alpha R + M                     */
    T_DATA = 1,   /* eta S_str + S_ang / eta (Eq. 9)                         */
    T_STR = 2,    /* S_str at the given delta0 (Eq. 6)                       */
    T_ANG = 3,    /* S_ang at the given delta0 (Eq. 7)                       */
    T_REG = 4,    /* R (without alpha)                                       */
    T_MEAN = 5,   /* M                                                       */
    T_STR05 = 6,  /* S_str at delta0 = 0.5, used for eta (Eq. 10)            */
    T_ANG05 = 7,  /* S_ang at delta0 = 0.5                                   */
    T_COUNT = 8
};

static inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* ------------------------------------------------------------------------ */
/* Interpolator I: "Hermitian" interpolation with continuous first
 * derivatives (Eq. 2 and the text after Eq. 5).  Reading: the cubic Hermite
 * spline whose knot tangents are central differences (Catmull-Rom).  On the
 * interval [p_n, p_{n+1}] with t in [0, 1):
 *   f(t) = h00(t) p_n + h10(t) m_n + h01(t) p_{n+1} + h11(t) m_{n+1},
 *   m_n = (p_{n+1} - p_{n-1}) / 2,
 * with the Hermite basis h00 = 2t^3 - 3t^2 + 1, h10 = t^3 - 2t^2 + t,
 * h01 = -2t^3 + 3t^2, h11 = t^3 - t^2.  Collecting the coefficients of the
 * four samples p_{n-1}, p_n, p_{n+1}, p_{n+2} gives the tap weights below, and
 * differentiating the basis gives the derivative weights. */
EXPORT void orc_hermite_taps(double t, double w[4], double dw[4])
{
    double h00 = 2 * t * t * t - 3 * t * t + 1;
    double h10 = t * t * t - 2 * t * t + t;
    double h01 = -2 * t * t * t + 3 * t * t;
    double h11 = t * t * t - t * t;
    double d00 = 6 * t * t - 6 * t;
    double d10 = 3 * t * t - 4 * t + 1;
    double d01 = -6 * t * t + 6 * t;
    double d11 = 3 * t * t - 2 * t;
    /* p_{n-1} enters only through m_n, p_{n+2} only through m_{n+1}. */
    w[0] = -0.5 * h10;
    w[1] = h00 - 0.5 * h11;
    w[2] = h01 + 0.5 * h10;
    w[3] = 0.5 * h11;
    dw[0] = -0.5 * d10;
    dw[1] = d00 - 0.5 * d11;
    dw[2] = d01 + 0.5 * d10;
    dw[3] = 0.5 * d11;
}

/* Boundary reading: tap indices are clamped to the volume (constant
 * extension), so that A-scans sampled beyond a gap replicate the edge
 * (Sec. 2.1, "merging", describes exactly that replication). */

/* 1-D sample and derivative at x of an array of n values. */
EXPORT void orc_sample1(const double* v, int n, double x, double out[2])
{
    double fx = floor(x);
    int nx = (int)fx;
    double w[4], dw[4];
    orc_hermite_taps(x - fx, w, dw);
    double val = 0, der = 0;
    for (int a = 0; a < 4; a++) {
        double s = v[clampi(nx - 1 + a, 0, n - 1)];
        val += w[a] * s;
        der += dw[a] * s;
    }
    out[0] = val;
    out[1] = der;
}

/* 2-D sample of an image stored [j][i] (w columns, h rows): value, d/dx, d/dy. */
EXPORT void orc_sample2(const double* img, int w, int h, double x, double y, double out[3])
{
    double fx = floor(x), fy = floor(y);
    int nx = (int)fx, ny = (int)fy;
    double wx[4], dwx[4], wy[4], dwy[4];
    orc_hermite_taps(x - fx, wx, dwx);
    orc_hermite_taps(y - fy, wy, dwy);
    double val = 0, gx = 0, gy = 0;
    for (int b = 0; b < 4; b++) {
        int yy = clampi(ny - 1 + b, 0, h - 1);
        for (int a = 0; a < 4; a++) {
            int xx = clampi(nx - 1 + a, 0, w - 1);
            double s = img[(size_t)yy * w + xx];
            val += wx[a] * wy[b] * s;
            gx += dwx[a] * wy[b] * s;
            gy += wx[a] * dwy[b] * s;
        }
    }
    out[0] = val;
    out[1] = gx;
    out[2] = gy;
}

/* 3-D sample of a volume stored [j][i][k]: value, d/dx, d/dy, d/dz.
 * Direct 64-tap tensor product. */
EXPORT void orc_sample3(const double* vol, int w, int h, int d,
                        double x, double y, double z, double out[4])
{
    double fx = floor(x), fy = floor(y), fz = floor(z);
    int nx = (int)fx, ny = (int)fy, nz = (int)fz;
    double wx[4], dwx[4], wy[4], dwy[4], wz[4], dwz[4];
    orc_hermite_taps(x - fx, wx, dwx);
    orc_hermite_taps(y - fy, wy, dwy);
    orc_hermite_taps(z - fz, wz, dwz);
    double val = 0, gx = 0, gy = 0, gz = 0;
    for (int b = 0; b < 4; b++) {
        int yy = clampi(ny - 1 + b, 0, h - 1);
        for (int a = 0; a < 4; a++) {
            int xx = clampi(nx - 1 + a, 0, w - 1);
            const double* col = vol + ((size_t)yy * w + xx) * (size_t)d;
            for (int c = 0; c < 4; c++) {
                double s = col[clampi(nz - 1 + c, 0, d - 1)];
                val += wx[a] * wy[b] * wz[c] * s;
                gx += dwx[a] * wy[b] * wz[c] * s;
                gy += wx[a] * dwy[b] * wz[c] * s;
                gz += wx[a] * wy[b] * dwz[c] * s;
            }
        }
    }
    out[0] = val;
    out[1] = gx;
    out[2] = gy;
    out[3] = gz;
}

/* Pseudo-Huber loss (Eq. 4): L(x) = eps (sqrt(1 + (x/eps)^2) - 1), written in
 * the algebraically identical form eps u^2 / (sqrt(1 + u^2) + 1), u = x/eps,
 * which does not cancel for small |x|.  dL/dx = u / sqrt(1 + u^2). */
EXPORT void orc_pseudo_huber(double x, double eps, double out[2])
{
    double u = x / eps;
    double s = sqrt(1.0 + u * u);
    out[0] = eps * u * u / (s + 1.0);
    out[1] = u / s;
}

/* ------------------------------------------------------------------------ */
/* Data term of one output A-scan (Eqs. 2-9).  Outputs:
 *   part[0] = contribution to eta S_str + S_ang / eta   (Eq. 9)
 *   part[1] = (1 - delta) Lambda                          (Eq. 6 summand)
 *   part[2] = delta d L(R^A)                              (Eq. 7 summand)
 *   part[3] = (1 - delta_0.5) Lambda,  part[4] = delta_0.5 d L(R^A)
 *   g[0..2] = d/d(d^X), g[3..5] = d/d(d^Y) of part[0].
 * Readings:
 *   - Eq. 7 writes the angiographic residual with a free depth index k while
 *     A is a 2-D en face image; the text says the depth sum is replaced by a
 *     multiplication with d.  So R^A_ij = I(A^X, i+dx^X, j+dy^X) -
 *     I(A^Y, i+dx^Y, j+dy^Y), weighted by d; dz does not enter it.
 *   - The resampled validity (Eq. 5) can over- or undershoot [0, 1] at a step
 *     of v, which would give a negative loss weight; it is clamped to [0, 1]
 *     and its derivative is 0 where clamped.
 *   - eta is a constant of the level; no derivative flows through it. */
static void data_ascan(const double* sx, const double* sy, const double* ax, const double* ay,
                       const double* vx, const double* vy, int w, int h, int d,
                       const double* dX, const double* dY, int i, int j,
                       double delta0, double eps_h, double eta,
                       double part[5], double g[6])
{
    double lam = 0, gam_x[3] = {0, 0, 0}, gam_y[3] = {0, 0, 0};
    for (int k = 0; k < d; k++) {
        double ix[4], iy[4], lh[2];
        orc_sample3(sx, w, h, d, i + dX[0], j + dX[1], k + dX[2], ix);
        orc_sample3(sy, w, h, d, i + dY[0], j + dY[1], k + dY[2], iy);
        double r = ix[0] - iy[0]; /* Eq. 2 */
        orc_pseudo_huber(r, eps_h, lh);
        lam += lh[0];
        for (int c = 0; c < 3; c++) {
            gam_x[c] += lh[1] * ix[1 + c];
            gam_y[c] += lh[1] * iy[1 + c];
        }
    }
    double jx[3], jy[3], la[2];
    orc_sample2(ax, w, h, i + dX[0], j + dX[1], jx);
    orc_sample2(ay, w, h, i + dY[0], j + dY[1], jy);
    orc_pseudo_huber(jx[0] - jy[0], eps_h, la);

    /* Eq. 5: X validity varies along y (X-fast B-scans are rows j), Y validity
     * along x (Y-fast B-scans are columns i). */
    double rx[2], ry[2];
    orc_sample1(vx, h, j + dX[1], rx);
    orc_sample1(vy, w, i + dY[0], ry);
    double tvx = rx[0] <= 0 ? 0 : (rx[0] >= 1 ? 1 : rx[0]);
    double dtvx = (rx[0] > 0 && rx[0] < 1) ? rx[1] : 0;
    double tvy = ry[0] <= 0 ? 0 : (ry[0] >= 1 ? 1 : ry[0]);
    double dtvy = (ry[0] > 0 && ry[0] < 1) ? ry[1] : 0;

    double delta = delta0 * tvx * tvy; /* Eq. 8 */
    double dd = (double)d;
    part[0] = eta * (1 - delta) * lam + (dd / eta) * delta * la[0];
    part[1] = (1 - delta) * lam;
    part[2] = delta * dd * la[0];
    part[3] = (1 - 0.5 * tvx * tvy) * lam;
    part[4] = 0.5 * tvx * tvy * dd * la[0];

    /* d part[0] / d delta */
    double dpd = -eta * lam + (dd / eta) * la[0];
    /* X scan: dR/d(d^X) = +grad I^X; Y scan: dR/d(d^Y) = -grad I^Y. */
    g[0] = eta * (1 - delta) * gam_x[0] + (dd / eta) * delta * la[1] * jx[1];
    g[1] = eta * (1 - delta) * gam_x[1] + (dd / eta) * delta * la[1] * jx[2] + dpd * delta0 * tvy * dtvx;
    g[2] = eta * (1 - delta) * gam_x[2];
    g[3] = -(eta * (1 - delta) * gam_y[0] + (dd / eta) * delta * la[1] * jy[1]) + dpd * delta0 * tvx * dtvy;
    g[4] = -(eta * (1 - delta) * gam_y[1] + (dd / eta) * delta * la[1] * jy[2]);
    g[5] = -(eta * (1 - delta) * gam_y[2]);
}

/* Scan-order regulariser R (Sec. 2.1, "regularizers").  The paper defers the
 * formula to earlier work; reading: pseudo-Huber (eps_r) of the per-component
 * difference between displacements of A-scans that are consecutive in the
 * scan's acquisition order, i.e. along the fast axis with weight 1, and one
 * link per B-scan boundary (last A-scan of a B-scan to the first of the next)
 * with the lower weight 1/sqrt(1 + f), f = round(flyback_frac * B-scan length)
 * A-scan periods of flyback.  The sum is multiplied by d, so the balance
 * between R and the per-A-scan data term does not depend on depth.
 * Acquisition order: X-fast visits (i, j) at t = j (w + f) + i, Y-fast at
 * t = i (h + f) + j.  Adds alpha dR/dD into grad (if grad != NULL) and
 * returns R. */
static double reg_term(const double* D, int w, int h, int d, double eps_r, double flyback_frac,
                       double alpha, double* grad)
{
    double total = 0;
    for (int V = 0; V < 2; V++) {
        int blen = (V == 0) ? w : h;   /* A-scans per B-scan */
        int nb = (V == 0) ? h : w;     /* number of B-scans */
        double f = floor(flyback_frac * blen + 0.5);
        double wfb = 1.0 / sqrt(1.0 + f);
        const double* DV = D + (size_t)V * w * h * 3;
        double* GV = grad ? grad + (size_t)V * w * h * 3 : NULL;
        long n = (long)nb * blen;
        for (long t = 0; t + 1 < n; t++) {
            long t1 = t + 1;
            int fa = (int)(t % blen), sa = (int)(t / blen);
            int fb = (int)(t1 % blen), sb = (int)(t1 / blen);
            /* (fast, slow) -> (i, j) */
            int ia = (V == 0) ? fa : sa, ja = (V == 0) ? sa : fa;
            int ib = (V == 0) ? fb : sb, jb = (V == 0) ? sb : fb;
            double om = (sa == sb) ? 1.0 : wfb;
            const double* da = DV + ((size_t)ja * w + ia) * 3;
            const double* db = DV + ((size_t)jb * w + ib) * 3;
            for (int c = 0; c < 3; c++) {
                double lh[2];
                orc_pseudo_huber(db[c] - da[c], eps_r, lh);
                total += om * d * lh[0];
                if (GV) {
                    GV[((size_t)jb * w + ib) * 3 + c] += alpha * om * d * lh[1];
                    GV[((size_t)ja * w + ia) * 3 + c] -= alpha * om * d * lh[1];
                }
            }
        }
    }
    return total;
}

/* Mean-displacement term M (Sec. 2.1): penalises the sum of displacements of
 * both scans, fixing the three translational degrees of freedom.  Reading:
 * M = gamma_M d / (2 N_A) * sum_c (sum_V sum_ij d^V_ij,c)^2, N_A = w h. */
static double mean_term(const double* D, int w, int h, int d, double gamma, double* grad)
{
    double sum[3] = {0, 0, 0};
    size_t na = (size_t)w * h;
    for (size_t q = 0; q < 2 * na; q++)
        for (int c = 0; c < 3; c++) sum[c] += D[q * 3 + c];
    double m = 0;
    for (int c = 0; c < 3; c++) m += sum[c] * sum[c];
    m *= gamma * d / (2.0 * (double)na);
    if (grad)
        for (size_t q = 0; q < 2 * na; q++)
            for (int c = 0; c < 3; c++) grad[q * 3 + c] += gamma * d * sum[c] / (double)na;
    return m;
}

/* Full objective (Eq. 1 without the stage-1 tilt term T) and its gradient at
 * displacement D, with the level constant eta.  terms[T_COUNT] receives the
 * pieces listed in the enum above; grad ([2][h][w][3]) may be NULL. */
EXPORT int orc_eval(const double* sx, const double* sy, const double* ax, const double* ay,
                    const double* vx, const double* vy, int w, int h, int d,
                    const double* D, const orc_params* p, double eta,
                    double* terms, double* grad)
{
    size_t na = (size_t)w * h;
    double* part = (double*)malloc(na * 5 * sizeof(double));
    double* g = (double*)malloc(na * 6 * sizeof(double));
    if (!part || !g) {
        free(part);
        free(g);
        return -1;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (long a = 0; a < (long)na; a++) {
        int i = (int)(a % w), j = (int)(a / w);
        data_ascan(sx, sy, ax, ay, vx, vy, w, h, d, D + (size_t)a * 3, D + (na + a) * 3, i, j,
                   p->delta0, p->eps_h, eta, part + a * 5, g + a * 6);
    }
    double s[5] = {0, 0, 0, 0, 0};
    for (size_t a = 0; a < na; a++)
        for (int q = 0; q < 5; q++) s[q] += part[a * 5 + q];
    if (grad) {
        for (size_t a = 0; a < na; a++)
            for (int c = 0; c < 3; c++) {
                grad[a * 3 + c] = g[a * 6 + c];
                grad[(na + a) * 3 + c] = g[a * 6 + 3 + c];
            }
    }
    double r = reg_term(D, w, h, d, p->eps_r, p->flyback_frac, p->alpha, grad);
    double m = mean_term(D, w, h, d, p->mean_weight, grad);
    terms[T_DATA] = s[0];
    terms[T_STR] = s[1];
    terms[T_ANG] = s[2];
    terms[T_STR05] = s[3];
    terms[T_ANG05] = s[4];
    terms[T_REG] = r;
    terms[T_MEAN] = m;
    terms[T_F] = s[0] + p->alpha * r + m;
    free(part);
    free(g);
    return 0;
}

/* The data term of Eqs. 2-9 and its gradient for a list of output A-scans
 * only (index a = j w + i), for checks at sizes where the full sum is too
 * slow: part[q*5 + 0..4] and g[q*6 + 0..5] as in data_ascan. */
EXPORT int orc_data_ascans(const double* sx, const double* sy, const double* ax, const double* ay,
                           const double* vx, const double* vy, int w, int h, int d, const double* D,
                           const orc_params* p, double eta, const int64_t* list, int nlist,
                           double* part, double* g)
{
    size_t na = (size_t)w * h;
#pragma omp parallel for schedule(dynamic, 1)
    for (int q = 0; q < nlist; q++) {
        int64_t a = list[q];
        int i = (int)(a % w), j = (int)(a / w);
        data_ascan(sx, sy, ax, ay, vx, vy, w, h, d, D + (size_t)a * 3, D + (na + a) * 3, i, j,
                   p->delta0, p->eps_h, eta, part + (size_t)q * 5, g + (size_t)q * 6);
    }
    return 0;
}

/* eta (Eq. 10): sqrt(S_ang_0.5 / S_str_0.5) at the level's initial field.
 * Reading: where either term is zero (e.g. identical inputs) eta = 1. */
EXPORT double orc_eta_from_terms(double s_str05, double s_ang05)
{
    if (!(s_str05 > 1e-300) || !(s_ang05 > 1e-300)) return 1.0;
    return sqrt(s_ang05 / s_str05);
}

/* ------------------------------------------------------------------------ */
/* Factor-2 pyramid (Sec. 2.1, "optimization").  Reading: all three axes are
 * halved with ceil(n/2); coarse sample I is the mean of fine samples 2I and
 * 2I+1, the latter clamped to the last sample for odd sizes.  The en face
 * images use the 2-D version and the validity vectors the 1-D version ("in the
 * same way", Sec. 2.2). */
EXPORT void orc_pyr_down3(const double* in, int w, int h, int d, double* out)
{
    int w2 = (w + 1) / 2, h2 = (h + 1) / 2, d2 = (d + 1) / 2;
    for (int J = 0; J < h2; J++)
        for (int I = 0; I < w2; I++)
            for (int K = 0; K < d2; K++) {
                double s = 0;
                for (int b = 0; b < 2; b++)
                    for (int a = 0; a < 2; a++)
                        for (int c = 0; c < 2; c++) {
                            int y = clampi(2 * J + b, 0, h - 1);
                            int x = clampi(2 * I + a, 0, w - 1);
                            int z = clampi(2 * K + c, 0, d - 1);
                            s += in[((size_t)y * w + x) * d + z];
                        }
                out[((size_t)J * w2 + I) * d2 + K] = s / 8.0;
            }
}

/* The same 2 x 2 x 2 box in single precision, for pyramids whose levels are
 * then rounded to a 16-bit storage type.  Rounding to the storage type
 * decides a quantised value, so it is taken from a level computed in the
 * precision the pyramid is built in on the device (single), from the
 * single-precision level above; the box is separable, summed along depth,
 * then x, then y, and scaled by 1/8 (exact).  `in` holds single-precision
 * values (the input volume, or a level this function wrote). */
EXPORT void orc_pyr_down3_f32(const double* in, int w, int h, int d, double* out)
{
    int w2 = (w + 1) / 2, h2 = (h + 1) / 2, d2 = (d + 1) / 2;
    for (int J = 0; J < h2; J++)
        for (int I = 0; I < w2; I++)
            for (int K = 0; K < d2; K++) {
                float sy[2];
                for (int b = 0; b < 2; b++) {
                    float sxz[2];
                    for (int a = 0; a < 2; a++) {
                        int y = clampi(2 * J + b, 0, h - 1);
                        int x = clampi(2 * I + a, 0, w - 1);
                        const double* col = in + ((size_t)y * w + x) * d;
                        sxz[a] = (float)col[clampi(2 * K, 0, d - 1)] + (float)col[clampi(2 * K + 1, 0, d - 1)];
                    }
                    sy[b] = sxz[0] + sxz[1];
                }
                const float s = sy[0] + sy[1];
                out[((size_t)J * w2 + I) * d2 + K] = (double)(0.125f * s);
            }
}

EXPORT void orc_pyr_down2(const double* in, int w, int h, double* out)
{
    int w2 = (w + 1) / 2, h2 = (h + 1) / 2;
    for (int J = 0; J < h2; J++)
        for (int I = 0; I < w2; I++) {
            double s = 0;
            for (int b = 0; b < 2; b++)
                for (int a = 0; a < 2; a++)
                    s += in[(size_t)clampi(2 * J + b, 0, h - 1) * w + clampi(2 * I + a, 0, w - 1)];
            out[(size_t)J * w2 + I] = s / 4.0;
        }
}

EXPORT void orc_pyr_down1(const double* in, int n, double* out)
{
    int n2 = (n + 1) / 2;
    for (int I = 0; I < n2; I++) out[I] = 0.5 * (in[2 * I] + in[clampi(2 * I + 1, 0, n - 1)]);
}

/* Level transition: the fine field is twice the bilinear interpolation of the
 * coarse field at the fine pixel's coarse position ((i - 0.5)/2, (j - 0.5)/2),
 * clamped to the coarse grid; all three components double because every axis
 * was halved.  coarse is [2][hc][wc][3], fine [2][hf][wf][3]. */
EXPORT void orc_upsample(const double* coarse, int wc, int hc, double* fine, int wf, int hf)
{
    for (int V = 0; V < 2; V++)
        for (int j = 0; j < hf; j++)
            for (int i = 0; i < wf; i++) {
                double x = (i - 0.5) / 2.0, y = (j - 0.5) / 2.0;
                if (x < 0) x = 0;
                if (x > wc - 1) x = wc - 1;
                if (y < 0) y = 0;
                if (y > hc - 1) y = hc - 1;
                int x0 = (int)floor(x), y0 = (int)floor(y);
                int x1 = x0 + 1 < wc ? x0 + 1 : wc - 1, y1 = y0 + 1 < hc ? y0 + 1 : hc - 1;
                double fx = x - x0, fy = y - y0;
                for (int c = 0; c < 3; c++) {
                    const double* C = coarse + (size_t)V * wc * hc * 3;
                    double v00 = C[((size_t)y0 * wc + x0) * 3 + c], v10 = C[((size_t)y0 * wc + x1) * 3 + c];
                    double v01 = C[((size_t)y1 * wc + x0) * 3 + c], v11 = C[((size_t)y1 * wc + x1) * 3 + c];
                    double v = (1 - fy) * ((1 - fx) * v00 + fx * v10) + fy * ((1 - fx) * v01 + fx * v11);
                    fine[(((size_t)V * hf + j) * wf + i) * 3 + c] = 2.0 * v;
                }
            }
}

/* ------------------------------------------------------------------------ */
/* L-BFGS (Sec. 2.1: "gradient-based L-BFGS solver").  The paper names only
 * the method; reading (textbook limited-memory BFGS, Nocedal & Wright,
 * "Numerical Optimization", Alg. 7.4 / 7.5 with the line search of
 * Alg. 3.5 / 3.6):
 *   - memory m pairs; initial inverse Hessian gamma I, gamma = s'y / y'y of
 *     the newest pair;
 *   - with an empty memory the direction is -g / max|g| (a step of at most one
 *     pixel at alpha = 1);
 *   - a pair is stored only if s'y > 1e-12 y'y;
 *   - strong Wolfe line search with c1, c2, first trial alpha = 1, doubling
 *     while bracketing, cubic interpolation in the zoom phase with the
 *     interpolant kept at least 10 % of the interval away from its ends
 *     (bisection otherwise), at most ls_max_evals evaluations;
 *   - the solve stops after max_iter accepted steps, when the line search
 *     fails, or when max|g| <= 1e-10 max(1, |f|). */
typedef int (*orc_fg_fn)(void* ctx, const double* x, double* f, double* g);

typedef struct {
    int iters, evals, ls_fail, converged;
    double f_start, f_end;
} orc_lbfgs_report;

typedef struct {
    int n;
    orc_fg_fn fg;
    void* ctx;
    const double* x;
    const double* p;
    double* xt;
    double* gt;
    int evals;
} ls_state;

static double dotn(int n, const double* a, const double* b)
{
    double s = 0;
    for (int q = 0; q < n; q++) s += a[q] * b[q];
    return s;
}

/* phi(alpha) = f(x + alpha p) and phi'(alpha) = g(x + alpha p)' p */
static int ls_eval(ls_state* st, double alpha, double* phi, double* dphi)
{
    for (int q = 0; q < st->n; q++) st->xt[q] = st->x[q] + alpha * st->p[q];
    if (st->fg(st->ctx, st->xt, phi, st->gt)) return -1;
    st->evals++;
    *dphi = dotn(st->n, st->gt, st->p);
    return 0;
}

/* Minimiser of the cubic that matches phi and phi' at a0 and a1
 * (Nocedal & Wright eq. 3.59), kept inside the bracket. */
static double cubic_step(double a0, double f0, double g0, double a1, double f1, double g1)
{
    double lo = a0 < a1 ? a0 : a1, hi = a0 < a1 ? a1 : a0, span = hi - lo;
    double mid = 0.5 * (a0 + a1);
    double d1 = g0 + g1 - 3.0 * (f0 - f1) / (a0 - a1);
    double disc = d1 * d1 - g0 * g1;
    if (!(disc >= 0)) return mid;
    double d2 = (a1 > a0 ? 1.0 : -1.0) * sqrt(disc);
    double den = g1 - g0 + 2.0 * d2;
    if (den == 0) return mid;
    double a = a1 - (a1 - a0) * (g1 + d2 - d1) / den;
    if (!isfinite(a) || a < lo + 0.1 * span || a > hi - 0.1 * span) return mid;
    return a;
}

/* Strong Wolfe line search.  On success xt/gt hold the accepted point. */
static int line_search(ls_state* st, double f0, double g0, double c1, double c2, int max_evals,
                       double* alpha_out, double* f_out)
{
    double a_prev = 0, f_prev = f0, g_prev = g0;
    double a = 1.0;
    double lo, flo, glo, hi, fhi, ghi;
    for (int i = 1;; i++) {
        if (st->evals >= max_evals) return -1;
        double fa, ga;
        if (ls_eval(st, a, &fa, &ga)) return -2;
        if (fa > f0 + c1 * a * g0 || (i > 1 && fa >= f_prev)) {
            lo = a_prev; flo = f_prev; glo = g_prev;
            hi = a; fhi = fa; ghi = ga;
            break;
        }
        if (fabs(ga) <= -c2 * g0) {
            *alpha_out = a;
            *f_out = fa;
            return 0;
        }
        if (ga >= 0) {
            lo = a; flo = fa; glo = ga;
            hi = a_prev; fhi = f_prev; ghi = g_prev;
            break;
        }
        a_prev = a; f_prev = fa; g_prev = ga;
        a = 2.0 * a;
    }
    /* zoom: lo satisfies sufficient decrease and has the lowest phi so far;
     * the minimiser lies between lo and hi. */
    for (;;) {
        if (st->evals >= max_evals) return -1;
        double aj = cubic_step(lo, flo, glo, hi, fhi, ghi);
        double fj, gj;
        if (ls_eval(st, aj, &fj, &gj)) return -2;
        if (fj > f0 + c1 * aj * g0 || fj >= flo) {
            hi = aj; fhi = fj; ghi = gj;
        } else {
            if (fabs(gj) <= -c2 * g0) {
                *alpha_out = aj;
                *f_out = fj;
                return 0;
            }
            if (gj * (hi - lo) >= 0) {
                hi = lo; fhi = flo; ghi = glo;
            }
            lo = aj; flo = fj; glo = gj;
        }
    }
}

/* Progress of long solves: every `every` accepted steps (0: never) orc_lbfgs
 * prints the step count, the evaluations and the objective to stderr.
 * Printing only; the arithmetic does not depend on it. */
static int g_progress_every = 0;
EXPORT void orc_set_progress(int every) { g_progress_every = every > 0 ? every : 0; }

EXPORT int orc_lbfgs(int n, double* x, orc_fg_fn fg, void* ctx, int m, int max_iter,
                     int ls_max_evals, double c1, double c2, orc_lbfgs_report* rep)
{
    double* g = (double*)calloc(n, sizeof(double));
    double* p = (double*)calloc(n, sizeof(double));
    double* q = (double*)calloc(n, sizeof(double));
    double* xt = (double*)calloc(n, sizeof(double));
    double* gt = (double*)calloc(n, sizeof(double));
    double* S = (double*)calloc((size_t)m * n, sizeof(double));
    double* Y = (double*)calloc((size_t)m * n, sizeof(double));
    double* rho = (double*)calloc(m, sizeof(double));
    double* al = (double*)calloc(m, sizeof(double));
    int rc = 0;
    memset(rep, 0, sizeof(*rep));
    if (!g || !p || !q || !xt || !gt || !S || !Y || !rho || !al) {
        rc = -1;
        goto done;
    }
    double f;
    if (fg(ctx, x, &f, g)) {
        rc = -2;
        goto done;
    }
    rep->evals = 1;
    rep->f_start = f;
    int count = 0, newest = -1; /* ring buffer of stored pairs */
    int it = 0;
    while (it < max_iter) {
        double gmax = 0;
        for (int k = 0; k < n; k++) gmax = fmax(gmax, fabs(g[k]));
        if (gmax <= 1e-10 * fmax(1.0, fabs(f))) {
            rep->converged = 1;
            break;
        }
        if (count == 0) {
            for (int k = 0; k < n; k++) p[k] = -g[k] / gmax;
        } else {
            /* two-loop recursion: q = H g */
            memcpy(q, g, n * sizeof(double));
            for (int c = 0; c < count; c++) {
                int s = (newest - c + m) % m;
                al[s] = rho[s] * dotn(n, S + (size_t)s * n, q);
                for (int k = 0; k < n; k++) q[k] -= al[s] * Y[(size_t)s * n + k];
            }
            double gamma = dotn(n, S + (size_t)newest * n, Y + (size_t)newest * n) /
                           dotn(n, Y + (size_t)newest * n, Y + (size_t)newest * n);
            for (int k = 0; k < n; k++) q[k] *= gamma;
            for (int c = count - 1; c >= 0; c--) {
                int s = (newest - c + m) % m;
                double b = rho[s] * dotn(n, Y + (size_t)s * n, q);
                for (int k = 0; k < n; k++) q[k] += (al[s] - b) * S[(size_t)s * n + k];
            }
            for (int k = 0; k < n; k++) p[k] = -q[k];
        }
        double g0 = dotn(n, g, p);
        if (!(g0 < 0)) {
            /* not a descent direction: drop the memory and restart */
            count = 0;
            for (int k = 0; k < n; k++) p[k] = -g[k] / gmax;
            g0 = dotn(n, g, p);
        }
        ls_state st = {n, fg, ctx, x, p, xt, gt, 0};
        double alpha, fn;
        int ls = line_search(&st, f, g0, c1, c2, ls_max_evals, &alpha, &fn);
        rep->evals += st.evals;
        if (ls == -2) {
            rc = -2;
            goto done;
        }
        if (ls != 0) {
            rep->ls_fail = 1;
            break;
        }
        /* new pair s = x_new - x, y = g_new - g; it replaces the oldest
         * stored pair only if it passes the curvature test */
        for (int k = 0; k < n; k++) {
            q[k] = xt[k] - x[k];   /* q is free here: reused as s */
            p[k] = gt[k] - g[k];   /* p is no longer needed: reused as y */
        }
        double sy = dotn(n, q, p), yy = dotn(n, p, p);
        if (sy > 1e-12 * yy && yy > 0) {
            int slot = (newest + 1) % m;
            memcpy(S + (size_t)slot * n, q, n * sizeof(double));
            memcpy(Y + (size_t)slot * n, p, n * sizeof(double));
            rho[slot] = 1.0 / sy;
            newest = slot;
            if (count < m) count++;
        }
        memcpy(x, xt, n * sizeof(double));
        memcpy(g, gt, n * sizeof(double));
        f = fn;
        it++;
        if (g_progress_every && it % g_progress_every == 0) {
            fprintf(stderr, "[oracle] lbfgs n=%d step %d evals %d f=%.10g\n", n, it, rep->evals, f);
            fflush(stderr);
        }
    }
    rep->iters = it;
    rep->f_end = f;
done:
    free(g); free(p); free(q); free(xt); free(gt); free(S); free(Y); free(rho); free(al);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Rounding to a narrower binary floating-point format, to nearest with ties
 * to even, from the definition: a format with p significant bits and
 * smallest normal exponent emin represents, near |x| = m 2^e (m in
 * [1/2, 1)), exactly the multiples of the quantum 2^max(e - p, emin - p + 1);
 * x is divided by the quantum (exact: a power of two), rounded to an integer
 * in the default rounding mode (nearest, ties to even) and scaled back.
 * Results beyond the largest finite value become infinite.
 *   bfloat16: p = 8,  emin = -126, largest finite (2 - 2^-7) 2^127
 *   binary16: p = 11, emin = -14,  largest finite 65504 */
static double round_format(double x, int p, int emin, double maxf)
{
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);
    int qe = e - p;
    if (qe < emin - p + 1) qe = emin - p + 1;
    const double r = ldexp(nearbyint(ldexp(x, -qe)), qe);
    if (fabs(r) > maxf) return r > 0 ? INFINITY : -INFINITY;
    return r;
}

EXPORT void orc_round_storage(double* v, size_t n, int store)
{
    if (store == 1) {
        const double maxf = ldexp(2.0 - ldexp(1.0, -7), 127);
        for (size_t i = 0; i < n; i++) v[i] = round_format(v[i], 8, -126, maxf);
    } else if (store == 2) {
        for (size_t i = 0; i < n; i++) v[i] = round_format(v[i], 11, -14, 65504.0);
    }
}

/* The pyramid filter of a solve: exact for float storage, single precision
 * (orc_pyr_down3_f32) when the levels are rounded to a 16-bit type. */
static void pyr_down3_for(int store, const double* in, int w, int h, int d, double* out)
{
    if (store)
        orc_pyr_down3_f32(in, w, h, d, out);
    else
        orc_pyr_down3(in, w, h, d, out);
}

/* ------------------------------------------------------------------------ */
/* Multi-resolution 3-D registration (Sec. 2.1, "optimization"): a factor-2
 * pyramid, zero displacement at the coarsest level, eta fixed per level at
 * the level's initial field (Eq. 10), L-BFGS per level, upsampling between
 * levels.  Volumes are the finest level; D_out is [2][h][w][3] at the finest
 * level.  levels_rep (may be NULL) receives per level, coarsest first:
 * eta, f_start, f_end, iters, evals. */
typedef struct {
    const double *sx, *sy, *ax, *ay, *vx, *vy;
    int w, h, d;
    const orc_params* p;
    double eta;
    double terms[T_COUNT];
} level_ctx;

static int level_fg(void* vctx, const double* x, double* f, double* g)
{
    level_ctx* c = (level_ctx*)vctx;
    if (orc_eval(c->sx, c->sy, c->ax, c->ay, c->vx, c->vy, c->w, c->h, c->d, x, c->p, c->eta,
                 c->terms, g))
        return -1;
    *f = c->terms[T_F];
    return 0;
}

EXPORT int orc_register(const double* sx, const double* sy, const double* ax, const double* ay,
                        const double* vx, const double* vy, int w, int h, int d,
                        const orc_params* p, double* D_out, double* levels_rep)
{
    int L = p->levels;
    if (L < 1 || L > 8) return -1;
    int W[8], H[8], Dd[8];
    double *SX[8], *SY[8], *AX[8], *AY[8], *VX[8], *VY[8];
    W[0] = w; H[0] = h; Dd[0] = d;
    SX[0] = (double*)sx; SY[0] = (double*)sy; AX[0] = (double*)ax; AY[0] = (double*)ay;
    VX[0] = (double*)vx; VY[0] = (double*)vy;
    for (int l = 1; l < L; l++) {
        W[l] = (W[l - 1] + 1) / 2; H[l] = (H[l - 1] + 1) / 2; Dd[l] = (Dd[l - 1] + 1) / 2;
        size_t nv = (size_t)W[l] * H[l] * Dd[l], ni = (size_t)W[l] * H[l];
        SX[l] = (double*)malloc(nv * sizeof(double));
        SY[l] = (double*)malloc(nv * sizeof(double));
        AX[l] = (double*)malloc(ni * sizeof(double));
        AY[l] = (double*)malloc(ni * sizeof(double));
        VX[l] = (double*)malloc(H[l] * sizeof(double));
        VY[l] = (double*)malloc(W[l] * sizeof(double));
        pyr_down3_for(p->store, SX[l - 1], W[l - 1], H[l - 1], Dd[l - 1], SX[l]);
        pyr_down3_for(p->store, SY[l - 1], W[l - 1], H[l - 1], Dd[l - 1], SY[l]);
        orc_pyr_down2(AX[l - 1], W[l - 1], H[l - 1], AX[l]);
        orc_pyr_down2(AY[l - 1], W[l - 1], H[l - 1], AY[l]);
        orc_pyr_down1(VX[l - 1], H[l - 1], VX[l]);
        orc_pyr_down1(VY[l - 1], W[l - 1], VY[l]);
    }
    /* storage rounding after the whole pyramid is built from exact values */
    double *sx0 = NULL, *sy0 = NULL;
    if (p->store) {
        const size_t nv0 = (size_t)w * h * d;
        sx0 = (double*)malloc(nv0 * sizeof(double));
        sy0 = (double*)malloc(nv0 * sizeof(double));
        memcpy(sx0, sx, nv0 * sizeof(double));
        memcpy(sy0, sy, nv0 * sizeof(double));
        SX[0] = sx0;
        SY[0] = sy0;
        for (int l = 0; l < L; l++) {
            const size_t nv = (size_t)W[l] * H[l] * Dd[l];
            orc_round_storage(SX[l], nv, p->store);
            orc_round_storage(SY[l], nv, p->store);
        }
    }
    int rc = 0;
    double* Dc = NULL;
    for (int l = L - 1; l >= 0; l--) {
        size_t n = (size_t)2 * W[l] * H[l] * 3;
        double* Dl = (double*)calloc(n, sizeof(double));
        if (Dc) {
            orc_upsample(Dc, W[l + 1], H[l + 1], Dl, W[l], H[l]);
            free(Dc);
        }
        level_ctx ctx = {SX[l], SY[l], AX[l], AY[l], VX[l], VY[l], W[l], H[l], Dd[l], p, 1.0, {0}};
        double terms[T_COUNT];
        orc_eval(SX[l], SY[l], AX[l], AY[l], VX[l], VY[l], W[l], H[l], Dd[l], Dl, p, 1.0, terms, NULL);
        ctx.eta = orc_eta_from_terms(terms[T_STR05], terms[T_ANG05]);
        orc_lbfgs_report rep;
        rc = orc_lbfgs((int)n, Dl, level_fg, &ctx, p->lbfgs_m, p->iters, p->ls_max_evals, p->c1, p->c2, &rep);
        if (levels_rep) {
            double* r = levels_rep + (size_t)(L - 1 - l) * 5;
            r[0] = ctx.eta; r[1] = rep.f_start; r[2] = rep.f_end; r[3] = rep.iters; r[4] = rep.evals;
        }
        Dc = Dl;
        if (rc) break;
    }
    if (rc == 0) memcpy(D_out, Dc, (size_t)2 * w * h * 3 * sizeof(double));
    free(Dc);
    for (int l = 1; l < L; l++) {
        free(SX[l]); free(SY[l]); free(AX[l]); free(AY[l]); free(VX[l]); free(VY[l]);
    }
    free(sx0);
    free(sy0);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Output (Sec. 2.1 "merging" and Sec. 2.5).  Each scan is resampled with its
 * final field; the two are fused by a weighted average whose weights decay
 * exponentially with the sampling density of the input.  Readings:
 *   - density rho^V_ij: every output A-scan splats its sample position
 *     (i+dx, j+dy), clamped to the image, bilinearly into an h x w grid; the
 *     grid is read back bilinearly at the same position.  Regular sampling
 *     gives rho = 1;
 *   - weight exp(-kappa max(0, rho - 1)), set to 0 below tau, then the two
 *     weights are normalised to sum 1;
 *   - if both weights are 0 the scan with the lower density is used (the data
 *     of the B-scan with less oversampling remains);
 *   - for OCTA (Sec. 2.5) the weights are further multiplied by the resampled
 *     validity of Eq. 5, and where both are 0 the output is 0 (a black gap).
 * rho_out ([2][h][w]) and weight_out ([2][h][w], OCT weights after
 * normalisation) may be NULL. */
EXPORT void orc_density(const double* D, int w, int h, double* rho)
{
    for (int V = 0; V < 2; V++) {
        double* grid = (double*)calloc((size_t)w * h, sizeof(double));
        const double* DV = D + (size_t)V * w * h * 3;
        for (int j = 0; j < h; j++)
            for (int i = 0; i < w; i++) {
                double x = i + DV[((size_t)j * w + i) * 3 + 0];
                double y = j + DV[((size_t)j * w + i) * 3 + 1];
                x = x < 0 ? 0 : (x > w - 1 ? w - 1 : x);
                y = y < 0 ? 0 : (y > h - 1 ? h - 1 : y);
                int x0 = (int)floor(x), y0 = (int)floor(y);
                int x1 = x0 + 1 < w ? x0 + 1 : w - 1, y1 = y0 + 1 < h ? y0 + 1 : h - 1;
                double fx = x - x0, fy = y - y0;
                grid[(size_t)y0 * w + x0] += (1 - fx) * (1 - fy);
                grid[(size_t)y0 * w + x1] += fx * (1 - fy);
                grid[(size_t)y1 * w + x0] += (1 - fx) * fy;
                grid[(size_t)y1 * w + x1] += fx * fy;
            }
        for (int j = 0; j < h; j++)
            for (int i = 0; i < w; i++) {
                double x = i + DV[((size_t)j * w + i) * 3 + 0];
                double y = j + DV[((size_t)j * w + i) * 3 + 1];
                x = x < 0 ? 0 : (x > w - 1 ? w - 1 : x);
                y = y < 0 ? 0 : (y > h - 1 ? h - 1 : y);
                int x0 = (int)floor(x), y0 = (int)floor(y);
                int x1 = x0 + 1 < w ? x0 + 1 : w - 1, y1 = y0 + 1 < h ? y0 + 1 : h - 1;
                double fx = x - x0, fy = y - y0;
                rho[((size_t)V * h + j) * w + i] =
                    (1 - fx) * (1 - fy) * grid[(size_t)y0 * w + x0] + fx * (1 - fy) * grid[(size_t)y0 * w + x1] +
                    (1 - fx) * fy * grid[(size_t)y1 * w + x0] + fx * fy * grid[(size_t)y1 * w + x1];
            }
        free(grid);
    }
}

EXPORT void orc_merge(const double* sx, const double* sy, const double* ox, const double* oy,
                      const double* vx, const double* vy, int w, int h, int d, const double* D,
                      double kappa, double tau, double* merged_oct, double* merged_octa,
                      double* rho_out, double* weight_out)
{
    size_t na = (size_t)w * h;
    double* rho = (double*)malloc(2 * na * sizeof(double));
    orc_density(D, w, h, rho);
    if (rho_out) memcpy(rho_out, rho, 2 * na * sizeof(double));
#pragma omp parallel for schedule(dynamic, 4)
    for (long a = 0; a < (long)na; a++) {
        int i = (int)(a % w), j = (int)(a / w);
        const double* dX = D + (size_t)a * 3;
        const double* dY = D + (na + a) * 3;
        double rx = rho[a], ry = rho[na + a];
        double wx = exp(-kappa * fmax(0.0, rx - 1.0)), wy = exp(-kappa * fmax(0.0, ry - 1.0));
        if (wx < tau) wx = 0;
        if (wy < tau) wy = 0;
        double ax_w, ay_w;
        if (wx + wy > 0) {
            ax_w = wx / (wx + wy);
            ay_w = wy / (wx + wy);
        } else if (rx <= ry) {
            ax_w = 1; ay_w = 0;
        } else {
            ax_w = 0; ay_w = 1;
        }
        if (weight_out) {
            weight_out[a] = ax_w;
            weight_out[na + a] = ay_w;
        }
        /* OCTA weights: density weights times the resampled validity (Eq. 5) */
        double ow_x = 0, ow_y = 0;
        if (merged_octa) {
            double r1[2], r2[2];
            orc_sample1(vx, h, j + dX[1], r1);
            orc_sample1(vy, w, i + dY[0], r2);
            double tvx = r1[0] <= 0 ? 0 : (r1[0] >= 1 ? 1 : r1[0]);
            double tvy = r2[0] <= 0 ? 0 : (r2[0] >= 1 ? 1 : r2[0]);
            ow_x = wx * tvx;
            ow_y = wy * tvy;
            double sum = ow_x + ow_y;
            if (sum > 0) {
                ow_x /= sum;
                ow_y /= sum;
            }
        }
        for (int k = 0; k < d; k++) {
            double s1[4], s2[4];
            orc_sample3(sx, w, h, d, i + dX[0], j + dX[1], k + dX[2], s1);
            orc_sample3(sy, w, h, d, i + dY[0], j + dY[1], k + dY[2], s2);
            merged_oct[(size_t)a * d + k] = ax_w * s1[0] + ay_w * s2[0];
            if (merged_octa) {
                double o1[4], o2[4];
                orc_sample3(ox, w, h, d, i + dX[0], j + dX[1], k + dX[2], o1);
                orc_sample3(oy, w, h, d, i + dY[0], j + dY[1], k + dY[2], o2);
                merged_octa[(size_t)a * d + k] = ow_x * o1[0] + ow_y * o2[0];
            }
        }
    }
    free(rho);
}

/* Plain depth mean of an OCTA volume: the simple en face image, used when
 * the segmentation-free projection of Sec. 2.3 (orc_enface_project) is not
 * asked for. */
EXPORT void orc_enface_mean(const double* vol, int w, int h, int d, double* out)
{
    for (size_t a = 0; a < (size_t)w * h; a++) {
        double s = 0;
        for (int k = 0; k < d; k++) s += vol[a * d + k];
        out[a] = s / d;
    }
}

/* Nearest-valid substitution of invalid B-scans (Sec. 2.3 and 2.5) for an
 * OCTA volume of scan V (V = 0: B-scans are rows j; V = 1: columns i).  An
 * invalid B-scan takes the data of the closest valid one (the lower index on
 * a tie); with no valid B-scan the volume is left unchanged. */
EXPORT void orc_substitute_invalid(double* vol, int w, int h, int d, const double* valid, int V)
{
    int nb = (V == 0) ? h : w;
    int* src = (int*)malloc(nb * sizeof(int));
    int any = 0;
    for (int b = 0; b < nb; b++) any |= valid[b] > 0.5;
    if (!any) {
        free(src);
        return;
    }
    for (int b = 0; b < nb; b++) {
        if (valid[b] > 0.5) {
            src[b] = b;
            continue;
        }
        int best = -1;
        for (int dist = 1; dist < nb && best < 0; dist++) {
            if (b - dist >= 0 && valid[b - dist] > 0.5) best = b - dist;
            else if (b + dist < nb && valid[b + dist] > 0.5) best = b + dist;
        }
        src[b] = best;
    }
    for (int b = 0; b < nb; b++) {
        if (src[b] == b) continue;
        for (int o = 0; o < ((V == 0) ? w : h); o++) {
            size_t dst = (V == 0) ? ((size_t)b * w + o) : ((size_t)o * w + b);
            size_t from = (V == 0) ? ((size_t)src[b] * w + o) : ((size_t)o * w + src[b]);
            memcpy(vol + dst * d, vol + from * d, d * sizeof(double));
        }
    }
    free(src);
}

/* ------------------------------------------------------------------------ */
/* Input validity of one OCTA volume (Sec. 2.2, "input validity").  A
 * saccade saturates the decorrelation of a whole B-scan; such B-scans are
 * found from their mean decorrelation and excluded together with two
 * neighbours on each side:
 *   m_b   mean of the OCTA volume over B-scan b (every A-scan and sample);
 *   flag  m_b > mu + 3 sigma, with mu and sigma the mean and standard
 *         deviation of m over all B-scans of the volume.  Reading: the
 *         population standard deviation (divisor = number of B-scans);
 *   v_b   1 if none of the B-scans b-2 .. b+2 (those inside the volume) is
 *         flagged, else 0.
 * B-scans of the X-fast scan are the rows j of the common-frame volume
 * [h][w][d] (nb = h); those of the Y-fast scan are the columns i (nb = w).
 * v receives nb values. */
EXPORT void orc_validity(const double* vol, int w, int h, int d, int V, double* v)
{
    const int nb = (V == 0) ? h : w;
    const int na = (V == 0) ? w : h; /* A-scans per B-scan */
    double* m = (double*)malloc(nb * sizeof(double));
    int* flag = (int*)malloc(nb * sizeof(int));
    for (int b = 0; b < nb; b++) {
        double s = 0.0;
        for (int o = 0; o < na; o++) {
            const size_t a = (V == 0) ? ((size_t)b * w + o) : ((size_t)o * w + b);
            for (int k = 0; k < d; k++) s += vol[a * d + k];
        }
        m[b] = s / ((double)na * d);
    }
    double mu = 0.0;
    for (int b = 0; b < nb; b++) mu += m[b];
    mu /= nb;
    double var = 0.0;
    for (int b = 0; b < nb; b++) var += (m[b] - mu) * (m[b] - mu);
    const double sigma = sqrt(var / nb);
    for (int b = 0; b < nb; b++) flag[b] = m[b] > mu + 3.0 * sigma;
    for (int b = 0; b < nb; b++) {
        int bad = 0;
        for (int q = b - 2; q <= b + 2; q++)
            if (q >= 0 && q < nb && flag[q]) bad = 1;
        v[b] = bad ? 0.0 : 1.0;
    }
    free(m);
    free(flag);
}

/* ------------------------------------------------------------------------ */
/* Segmentation-free en face OCTA projection (Sec. 2.3).  Volumes are
 * [h][w][d] in the common frame; the fast scan axis of scan V is x (i) for
 * the X-fast scan (V = 0) and y (j) for the Y-fast scan (V = 1).  Readings of
 * the points the paper leaves open are listed with each step. */

static int cmp_double(const void* a, const void* b)
{
    const double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

static size_t vidx(int i, int j, int k, int w, int h, int d)
{
    i = i < 0 ? 0 : (i >= w ? w - 1 : i);
    j = j < 0 ? 0 : (j >= h ? h - 1 : j);
    k = k < 0 ? 0 : (k >= d ? d - 1 : k);
    return ((size_t)j * w + i) * d + k;
}

/* 3-D median filter of radius 1: the 14th smallest of the 27 samples of the
 * 3 x 3 x 3 neighbourhood, indices clamped to the volume (reading). */
EXPORT void orc_median3(const double* in, int w, int h, int d, double* out)
{
#pragma omp parallel for schedule(static)
    for (int j = 0; j < h; j++)
        for (int i = 0; i < w; i++)
            for (int k = 0; k < d; k++) {
                double v[27];
                int n = 0;
                for (int dj = -1; dj <= 1; dj++)
                    for (int di = -1; di <= 1; di++)
                        for (int dk = -1; dk <= 1; dk++) v[n++] = in[vidx(i + di, j + dj, k + dk, w, h, d)];
                qsort(v, 27, sizeof(double), cmp_double);
                out[((size_t)j * w + i) * d + k] = v[13];
            }
}

/* 1-D rank filter along x (axis 0) or y (axis 1): the (rank + 1)-th smallest
 * of the 2 half + 1 samples centred on the voxel, indices clamped. */
EXPORT void orc_rank_line(const double* in, int w, int h, int d, int axis, int half, int rank, double* out)
{
    const int n = 2 * half + 1;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < h; j++) {
        double* v = (double*)malloc(n * sizeof(double));
        for (int i = 0; i < w; i++)
            for (int k = 0; k < d; k++) {
                for (int o = -half; o <= half; o++)
                    v[o + half] = axis == 0 ? in[vidx(i + o, j, k, w, h, d)] : in[vidx(i, j + o, k, w, h, d)];
                qsort(v, n, sizeof(double), cmp_double);
                out[((size_t)j * w + i) * d + k] = v[rank];
            }
        free(v);
    }
}

/* q-quantile (q in [0, 1]) of the voxels of the valid B-scans of scan V
 * (all voxels if no B-scan is valid), by linear interpolation between the
 * order statistics at position q (N - 1) (reading). */
EXPORT double orc_quantile_valid(const double* vol, int w, int h, int d, int V, const double* valid, double q)
{
    const int nb = V == 0 ? h : w;
    int any = 0;
    for (int b = 0; b < nb; b++) any |= valid[b] > 0.5;
    size_t n = 0;
    double* x = (double*)malloc((size_t)w * h * d * sizeof(double));
    for (int j = 0; j < h; j++)
        for (int i = 0; i < w; i++) {
            const int b = V == 0 ? j : i;
            if (any && !(valid[b] > 0.5)) continue;
            for (int k = 0; k < d; k++) x[n++] = vol[((size_t)j * w + i) * d + k];
        }
    qsort(x, n, sizeof(double), cmp_double);
    const double pos = q * (double)(n - 1);
    size_t lo = (size_t)floor(pos);
    if (lo >= n - 1) lo = n - 1;
    const double frac = pos - (double)lo;
    const double r = lo + 1 < n ? x[lo] + frac * (x[lo + 1] - x[lo]) : x[lo];
    free(x);
    return r;
}

/* The projection, step by step:
 *   1. M = 3-D median of radius 1 of the OCTA volume;
 *   2. R = rank filters of width 15 keeping the 3rd smallest value, first
 *      along the fast axis of the scan, then along its slow axis;
 *   3. p5, p95 = 5th and 95th percentile of R over the valid B-scans; the
 *      normalised value (R - p5) / (p95 - p5) is compared with 0.1, as
 *      R < p5 + 0.1 (p95 - p5) (reading: the mask keeps the low values, the
 *      retina between vessels, where the filtered volume is low);
 *   4. OCT mask (reading, the threshold is not given: a noise threshold as
 *      used for amplitude decorrelation): OCT intensity above mean + 2
 *      standard deviations (population) of the first nz = max(1,
 *      floor(0.05 d + 0.5)) samples of every A-scan;
 *   5. en face value = mean of the OCTA samples in both masks along depth
 *      (0 where none is);
 *   6. each B-scan's median (numpy convention: mean of the two middle values
 *      for an even count) is subtracted from it;
 *   7. invalid B-scans are replaced by their nearest valid neighbour.
 * fixed (NULL or {p5, p95}) replaces the percentiles of step 3 by a fixed
 * normalisation mapping, as the paper does for its wide-field runs.
 * out: [h][w]; count (NULL or [h][w]): number of voxels averaged in step 5,
 * before step 7; stats (NULL or 4 values): p5, p95, the threshold on the
 * filtered volume and the OCT threshold. */
EXPORT void orc_enface_project(const double* oct, const double* octa, int w, int h, int d, int V,
                               const double* valid, const double* fixed, double* out, double* count, double* stats)
{
    const size_t nv = (size_t)w * h * d;
    double* m = (double*)malloc(nv * sizeof(double));
    double* r = (double*)malloc(nv * sizeof(double));
    orc_median3(octa, w, h, d, m);
    orc_rank_line(m, w, h, d, V == 0 ? 0 : 1, 7, 2, r);
    orc_rank_line(r, w, h, d, V == 0 ? 1 : 0, 7, 2, m);
    const double p5 = fixed ? fixed[0] : orc_quantile_valid(m, w, h, d, V, valid, 0.05);
    const double p95 = fixed ? fixed[1] : orc_quantile_valid(m, w, h, d, V, valid, 0.95);
    const double thr_r = p5 + 0.1 * (p95 - p5);
    const int nz = (int)floor(0.05 * d + 0.5) < 1 ? 1 : (int)floor(0.05 * d + 0.5);
    double s = 0.0, s2 = 0.0;
    for (size_t a = 0; a < (size_t)w * h; a++)
        for (int k = 0; k < nz; k++) s += oct[a * d + k];
    const double cnt = (double)w * h * nz;
    const double mu = s / cnt;
    for (size_t a = 0; a < (size_t)w * h; a++)
        for (int k = 0; k < nz; k++) s2 += (oct[a * d + k] - mu) * (oct[a * d + k] - mu);
    const double thr_s = mu + 2.0 * sqrt(s2 / cnt);
    for (size_t a = 0; a < (size_t)w * h; a++) {
        double acc = 0.0;
        int c = 0;
        for (int k = 0; k < d; k++) {
            const size_t q = a * d + k;
            if (m[q] < thr_r && oct[q] > thr_s) {
                acc += octa[q];
                c++;
            }
        }
        out[a] = c ? acc / c : 0.0;
        if (count) count[a] = c;
    }
    if (stats) {
        stats[0] = p5;
        stats[1] = p95;
        stats[2] = thr_r;
        stats[3] = thr_s;
    }
    const int nb = V == 0 ? h : w, na = V == 0 ? w : h;
    double* line = (double*)malloc(na * sizeof(double));
    for (int b = 0; b < nb; b++) {
        for (int o = 0; o < na; o++) line[o] = V == 0 ? out[(size_t)b * w + o] : out[(size_t)o * w + b];
        qsort(line, na, sizeof(double), cmp_double);
        const double med = (na & 1) ? line[na / 2] : 0.5 * (line[na / 2 - 1] + line[na / 2]);
        for (int o = 0; o < na; o++) {
            if (V == 0) out[(size_t)b * w + o] -= med;
            else out[(size_t)o * w + b] -= med;
        }
    }
    free(line);
    orc_substitute_invalid(out, w, h, 1, valid, V);
    free(m);
    free(r);
}

/* ------------------------------------------------------------------------ */
/* Stage 1, rough axial prealignment (Fig. 1, Sec. 2.1 "optimization"): the
 * same objective, with displacements restricted to the axial direction at
 * B-scan granularity plus a tilt within each B-scan, on the factor-2 pyramid.
 * The en face OCTA term is not used (Sec. 2.4), so delta0 = 0 and eta = 1.
 *
 * Parameters theta: for the X-fast scan h B-scans (rows j, fast axis x, w
 * A-scans each), then for the Y-fast scan w B-scans (columns i, fast axis y,
 * h A-scans); per B-scan (z_b, t_b).  The field is
 *   dz(f, b) = z_b + t_b (f - (n_f - 1) / 2),  dx = dy = 0,
 * f the index along the fast axis, n_f the B-scan length.
 *
 * T, the tilt normalisation (Eq. 1), is defined only in earlier work that is
 * not available; reading: a quadratic penalty on the sum of each scan's
 * tilts, which fixes the two degrees of freedom the data term
 * cannot see (a common plane a x + b y added to both scans' fields), as M
 * fixes the translations:
 *   T = sum_V gamma_t d n_f (n_f^2 - 1) / (24 n_b) (sum_b t_b)^2,
 * i.e. gamma_t d / 2 times the squared norm of the common slope of each
 * scan's field along its fast axis, so that a uniform tilt tau costs
 * gamma_t d N_A var_f tau^2 / 2. */
static void tilt_dims(int V, int w, int h, int* nb, int* nf, int* off)
{
    *nb = V == 0 ? h : w;
    *nf = V == 0 ? w : h;
    *off = V == 0 ? 0 : 2 * h;
}

EXPORT void orc_tilt_expand(const double* th, int w, int h, double* D)
{
    memset(D, 0, (size_t)2 * w * h * 3 * sizeof(double));
    for (int V = 0; V < 2; V++) {
        int nb, nf, off;
        tilt_dims(V, w, h, &nb, &nf, &off);
        const double c = 0.5 * (nf - 1);
        for (int j = 0; j < h; j++)
            for (int i = 0; i < w; i++) {
                const int f = V == 0 ? i : j, b = V == 0 ? j : i;
                D[(((size_t)V * h + j) * w + i) * 3 + 2] = th[off + 2 * b] + th[off + 2 * b + 1] * (f - c);
            }
    }
}

/* Adjoint of orc_tilt_expand: gradient with respect to theta from the
 * gradient G ([2][h][w][3]) with respect to the field. */
EXPORT void orc_tilt_reduce(const double* G, int w, int h, double* gth)
{
    memset(gth, 0, (size_t)2 * (w + h) * sizeof(double));
    for (int V = 0; V < 2; V++) {
        int nb, nf, off;
        tilt_dims(V, w, h, &nb, &nf, &off);
        const double c = 0.5 * (nf - 1);
        for (int j = 0; j < h; j++)
            for (int i = 0; i < w; i++) {
                const int f = V == 0 ? i : j, b = V == 0 ? j : i;
                const double g = G[(((size_t)V * h + j) * w + i) * 3 + 2];
                gth[off + 2 * b] += g;
                gth[off + 2 * b + 1] += g * (f - c);
            }
    }
}

/* T and, if gth != NULL, its gradient added into gth. */
EXPORT double orc_tilt_term(const double* th, int w, int h, int d, double gamma_t, double* gth)
{
    double T = 0;
    for (int V = 0; V < 2; V++) {
        int nb, nf, off;
        tilt_dims(V, w, h, &nb, &nf, &off);
        double s = 0;
        for (int b = 0; b < nb; b++) s += th[off + 2 * b + 1];
        const double kap = gamma_t * d * (double)nf * ((double)nf * nf - 1.0) / (24.0 * nb);
        T += kap * s * s;
        if (gth)
            for (int b = 0; b < nb; b++) gth[off + 2 * b + 1] += 2.0 * kap * s;
    }
    return T;
}

/* Stage-1 objective at theta: terms[T_COUNT] as orc_eval (delta0 = 0, no en
 * face images) plus terms[T_COUNT] = T; returns F + T.  gth may be NULL. */
EXPORT double orc_prealign_eval(const double* sx, const double* sy, int w, int h, int d, const double* th,
                                const orc_params* p, double gamma_t, double* terms, double* gth)
{
    const size_t na = (size_t)w * h;
    double* D = (double*)malloc(2 * na * 3 * sizeof(double));
    double* G = gth ? (double*)calloc(2 * na * 3, sizeof(double)) : NULL;
    double* zero = (double*)calloc(na, sizeof(double));
    double* ones = (double*)malloc((size_t)(w > h ? w : h) * sizeof(double));
    for (int q = 0; q < (w > h ? w : h); q++) ones[q] = 1.0;
    orc_params p1 = *p;
    p1.delta0 = 0.0;
    orc_tilt_expand(th, w, h, D);
    orc_eval(sx, sy, zero, zero, ones, ones, w, h, d, D, &p1, 1.0, terms, G);
    if (gth) orc_tilt_reduce(G, w, h, gth);
    const double T = orc_tilt_term(th, w, h, d, gamma_t, gth);
    terms[T_COUNT] = T;
    free(D);
    free(G);
    free(zero);
    free(ones);
    return terms[T_F] + T;
}

/* Level transition of theta (reading): the fine field is twice the coarse
 * field at the coarse position ((f - 0.5)/2, (b - 0.5)/2), linear along the
 * fast axis as the field is, interpolated linearly between B-scans and
 * clamped to the first and last.  Per fine B-scan this gives
 *   t = t_c(u),  z = 2 z_c(u) + t (n_f - 2 n_fc) / 2,  u = (b - 0.5)/2. */
EXPORT void orc_tilt_upsample(const double* coarse, int wc, int hc, double* fine, int wf, int hf)
{
    for (int V = 0; V < 2; V++) {
        int nbc, nfc, offc, nbf, nff, offf;
        tilt_dims(V, wc, hc, &nbc, &nfc, &offc);
        tilt_dims(V, wf, hf, &nbf, &nff, &offf);
        for (int b = 0; b < nbf; b++) {
            double u = (b - 0.5) / 2.0;
            if (u < 0) u = 0;
            if (u > nbc - 1) u = nbc - 1;
            const int b0 = (int)floor(u), b1 = b0 + 1 < nbc ? b0 + 1 : nbc - 1;
            const double fr = u - b0;
            const double zc = (1 - fr) * coarse[offc + 2 * b0] + fr * coarse[offc + 2 * b1];
            const double tc = (1 - fr) * coarse[offc + 2 * b0 + 1] + fr * coarse[offc + 2 * b1 + 1];
            fine[offf + 2 * b + 1] = tc;
            fine[offf + 2 * b] = 2.0 * zc + tc * 0.5 * (nff - 2.0 * nfc);
        }
    }
}

typedef struct {
    const double *sx, *sy;
    int w, h, d;
    const orc_params* p;
    double gamma_t;
    double terms[T_COUNT + 1];
} pre_ctx;

static int pre_fg(void* vctx, const double* x, double* f, double* g)
{
    pre_ctx* c = (pre_ctx*)vctx;
    *f = orc_prealign_eval(c->sx, c->sy, c->w, c->h, c->d, x, c->p, c->gamma_t, c->terms, g);
    return 0;
}

/* The stage-1 solve: pyramid of the structural volumes (as orc_register,
 * with the same storage rounding), theta = 0 at the coarsest level, L-BFGS
 * with `iters` steps per level, orc_tilt_upsample between levels.  th_out:
 * 2 (h + w) values at the finest level; levels_rep (may be NULL): per level,
 * coarsest first, f_start, f_end, iters, evals. */
EXPORT int orc_prealign(const double* sx, const double* sy, int w, int h, int d, const orc_params* p,
                        double gamma_t, int iters, double* th_out, double* levels_rep)
{
    int L = p->levels;
    if (L < 1 || L > 8) return -1;
    int W[8], H[8], Dd[8];
    double *SX[8], *SY[8];
    W[0] = w; H[0] = h; Dd[0] = d;
    SX[0] = (double*)sx; SY[0] = (double*)sy;
    for (int l = 1; l < L; l++) {
        W[l] = (W[l - 1] + 1) / 2; H[l] = (H[l - 1] + 1) / 2; Dd[l] = (Dd[l - 1] + 1) / 2;
        const size_t nv = (size_t)W[l] * H[l] * Dd[l];
        SX[l] = (double*)malloc(nv * sizeof(double));
        SY[l] = (double*)malloc(nv * sizeof(double));
        pyr_down3_for(p->store, SX[l - 1], W[l - 1], H[l - 1], Dd[l - 1], SX[l]);
        pyr_down3_for(p->store, SY[l - 1], W[l - 1], H[l - 1], Dd[l - 1], SY[l]);
    }
    double *sx0 = NULL, *sy0 = NULL;
    if (p->store) {
        const size_t nv0 = (size_t)w * h * d;
        sx0 = (double*)malloc(nv0 * sizeof(double));
        sy0 = (double*)malloc(nv0 * sizeof(double));
        memcpy(sx0, sx, nv0 * sizeof(double));
        memcpy(sy0, sy, nv0 * sizeof(double));
        SX[0] = sx0;
        SY[0] = sy0;
        for (int l = 0; l < L; l++) {
            const size_t nv = (size_t)W[l] * H[l] * Dd[l];
            orc_round_storage(SX[l], nv, p->store);
            orc_round_storage(SY[l], nv, p->store);
        }
    }
    int rc = 0;
    double* tc = NULL;
    for (int l = L - 1; l >= 0; l--) {
        const int n = 2 * (W[l] + H[l]);
        double* tl = (double*)calloc(n, sizeof(double));
        if (tc) {
            orc_tilt_upsample(tc, W[l + 1], H[l + 1], tl, W[l], H[l]);
            free(tc);
        }
        pre_ctx ctx = {SX[l], SY[l], W[l], H[l], Dd[l], p, gamma_t, {0}};
        orc_lbfgs_report rep;
        rc = orc_lbfgs(n, tl, pre_fg, &ctx, p->lbfgs_m, iters, p->ls_max_evals, p->c1, p->c2, &rep);
        if (levels_rep) {
            double* r = levels_rep + (size_t)(L - 1 - l) * 4;
            r[0] = rep.f_start; r[1] = rep.f_end; r[2] = rep.iters; r[3] = rep.evals;
        }
        tc = tl;
        if (rc) break;
    }
    if (rc == 0) memcpy(th_out, tc, (size_t)2 * (w + h) * sizeof(double));
    free(tc);
    for (int l = 1; l < L; l++) {
        free(SX[l]);
        free(SY[l]);
    }
    free(sx0);
    free(sy0);
    return rc;
}

/* Axial resampling of a volume by a per-A-scan field (the prealigned volumes
 * of Fig. 1): out(i, j, k) = I(vol, i, j, k + dz(i, j)), the interpolator of
 * Eq. 2 at integer lateral positions, i.e. the 1-D Catmull-Rom spline along
 * depth with constant extension. */
EXPORT void orc_resample_z(const double* vol, int w, int h, int d, const double* dz, double* out)
{
#pragma omp parallel for schedule(static)
    for (long a = 0; a < (long)w * h; a++)
        for (int k = 0; k < d; k++) {
            double v[2];
            orc_sample1(vol + (size_t)a * d, d, k + dz[a], v);
            out[(size_t)a * d + k] = v[0];
        }
}

/* ------------------------------------------------------------------------ */
/* More than two volumes (Sec. 2.1 input: at least two raster scans, at least
 * one orthogonal to the others; the generalisation to more volumes is left
 * to earlier work).  Readings:
 *   - every volume V has an orientation o_V (0: X-fast, B-scans are rows j;
 *     1: Y-fast, columns i) and its own field d^V;
 *   - the data term is the two-volume data term (Eqs. 2-9) summed over all
 *     unordered pairs of volumes, each pair with its own eta (Eq. 10 at the
 *     level's initial field); the validity of Eq. 5 is resampled along each
 *     volume's own slow axis;
 *   - R is summed over the volumes, each with its own acquisition order;
 *   - M = gamma d / (n N_A) sum_c (sum_V sum_ij d^V_ij,c)^2 (n = 2: the
 *     two-volume term);
 *   - the merge weights of all volumes are normalised together; OCTA
 *     weights are multiplied by each volume's resampled validity; the
 *     lowest-density volume is used where every weight is 0 (OCT), a gap
 *     where every OCTA weight is 0.
 * With two volumes of orientations (0, 1) every function below equals its
 * two-volume counterpart. */
static void valid_sample(const double* v, int o, int w, int h, int i, int j, const double* dV, double* tv, double* dtv,
                         int* comp)
{
    double r[2];
    if (o == 0) {
        orc_sample1(v, h, j + dV[1], r);
        *comp = 1;
    } else {
        orc_sample1(v, w, i + dV[0], r);
        *comp = 0;
    }
    *tv = r[0] <= 0 ? 0 : (r[0] >= 1 ? 1 : r[0]);
    *dtv = (r[0] > 0 && r[0] < 1) ? r[1] : 0;
}

/* Data term of the pair (P, Q) at one output A-scan: part[5] as data_ascan,
 * g[0..2] = d/d(d^P), g[3..5] = d/d(d^Q) of part[0]. */
static void data_pair_ascan(const double* sp, const double* sq, const double* ap, const double* aq, const double* vp,
                            const double* vq, int op, int oq, int w, int h, int d, const double* dP, const double* dQ,
                            int i, int j, double delta0, double eps_h, double eta, double part[5], double g[6])
{
    double lam = 0, gp[3] = {0, 0, 0}, gq[3] = {0, 0, 0};
    for (int k = 0; k < d; k++) {
        double ip[4], iq[4], lh[2];
        orc_sample3(sp, w, h, d, i + dP[0], j + dP[1], k + dP[2], ip);
        orc_sample3(sq, w, h, d, i + dQ[0], j + dQ[1], k + dQ[2], iq);
        orc_pseudo_huber(ip[0] - iq[0], eps_h, lh);
        lam += lh[0];
        for (int c = 0; c < 3; c++) {
            gp[c] += lh[1] * ip[1 + c];
            gq[c] += lh[1] * iq[1 + c];
        }
    }
    double jp[3], jq[3], la[2];
    orc_sample2(ap, w, h, i + dP[0], j + dP[1], jp);
    orc_sample2(aq, w, h, i + dQ[0], j + dQ[1], jq);
    orc_pseudo_huber(jp[0] - jq[0], eps_h, la);
    double tvp, dtvp, tvq, dtvq;
    int cp, cq;
    valid_sample(vp, op, w, h, i, j, dP, &tvp, &dtvp, &cp);
    valid_sample(vq, oq, w, h, i, j, dQ, &tvq, &dtvq, &cq);
    const double delta = delta0 * tvp * tvq, dd = (double)d;
    part[0] = eta * (1 - delta) * lam + (dd / eta) * delta * la[0];
    part[1] = (1 - delta) * lam;
    part[2] = delta * dd * la[0];
    part[3] = (1 - 0.5 * tvp * tvq) * lam;
    part[4] = 0.5 * tvp * tvq * dd * la[0];
    const double dpd = -eta * lam + (dd / eta) * la[0];
    for (int c = 0; c < 2; c++) {
        g[c] = eta * (1 - delta) * gp[c] + (dd / eta) * delta * la[1] * jp[1 + c];
        g[3 + c] = -(eta * (1 - delta) * gq[c] + (dd / eta) * delta * la[1] * jq[1 + c]);
    }
    g[2] = eta * (1 - delta) * gp[2];
    g[5] = -(eta * (1 - delta) * gq[2]);
    g[cp] += dpd * delta0 * tvq * dtvp;
    g[3 + cq] += dpd * delta0 * tvp * dtvq;
}

/* R of one volume with orientation o (the acquisition order of reg_term),
 * added to `total` in link order. */
static double reg_volume(const double* DV, double* GV, int o, int w, int h, int d, double eps_r, double flyback_frac,
                         double alpha, double total)
{
    const int blen = o == 0 ? w : h, nb = o == 0 ? h : w;
    const double f = floor(flyback_frac * blen + 0.5), wfb = 1.0 / sqrt(1.0 + f);
    const long n = (long)nb * blen;
    for (long t = 0; t + 1 < n; t++) {
        const long t1 = t + 1;
        const int fa = (int)(t % blen), sa = (int)(t / blen), fb = (int)(t1 % blen), sb = (int)(t1 / blen);
        const int ia = o == 0 ? fa : sa, ja = o == 0 ? sa : fa, ib = o == 0 ? fb : sb, jb = o == 0 ? sb : fb;
        const double om = sa == sb ? 1.0 : wfb;
        const double* da = DV + ((size_t)ja * w + ia) * 3;
        const double* db = DV + ((size_t)jb * w + ib) * 3;
        for (int c = 0; c < 3; c++) {
            double lh[2];
            orc_pseudo_huber(db[c] - da[c], eps_r, lh);
            total += om * d * lh[0];
            if (GV) {
                GV[((size_t)jb * w + ib) * 3 + c] += alpha * om * d * lh[1];
                GV[((size_t)ja * w + ia) * 3 + c] -= alpha * om * d * lh[1];
            }
        }
    }
    return total;
}

static int pair_count(int n) { return n * (n - 1) / 2; }

/* The n-volume objective.  S, A, Vv: per volume the structural volume, the
 * en face image and the validity vector (h values for orientation 0, w for
 * 1); D: [n][h][w][3]; eta: [n (n - 1) / 2] per pair (P < Q, in the order
 * (0,1), (0,2), ..., (1,2), ...).  terms[T_COUNT] as orc_eval (sums over the
 * pairs; T_STR05 and T_ANG05 summed as well); pair05 (may be NULL):
 * [npairs][2] = the pairs' S_str and S_ang at delta0 = 0.5 (for eta);
 * grad: [n][h][w][3] or NULL. */
EXPORT int orc_eval_multi(int n, const double* const* S, const double* const* A, const double* const* Vv,
                          const int* orient, int w, int h, int d, const double* D, const orc_params* p,
                          const double* eta, double* terms, double* pair05, double* grad)
{
    if (n < 2 || n > 8) return -1;
    const size_t na = (size_t)w * h;
    const int np = pair_count(n);
    double* part = (double*)malloc(na * 5 * sizeof(double));
    double* g = (double*)malloc(na * 6 * sizeof(double));
    if (!part || !g) {
        free(part);
        free(g);
        return -1;
    }
    if (grad) memset(grad, 0, (size_t)n * na * 3 * sizeof(double));
    double s[5] = {0, 0, 0, 0, 0};
    int q = 0;
    for (int P = 0; P < n; P++)
        for (int Q = P + 1; Q < n; Q++, q++) {
#pragma omp parallel for schedule(dynamic, 4)
            for (long a = 0; a < (long)na; a++) {
                const int i = (int)(a % w), j = (int)(a / w);
                data_pair_ascan(S[P], S[Q], A[P], A[Q], Vv[P], Vv[Q], orient[P], orient[Q], w, h, d,
                                D + ((size_t)P * na + a) * 3, D + ((size_t)Q * na + a) * 3, i, j, p->delta0, p->eps_h,
                                eta[q], part + a * 5, g + a * 6);
            }
            double sp[5] = {0, 0, 0, 0, 0};
            for (size_t a = 0; a < na; a++)
                for (int c = 0; c < 5; c++) sp[c] += part[a * 5 + c];
            for (int c = 0; c < 5; c++) s[c] += sp[c];
            if (pair05) {
                pair05[2 * q] = sp[3];
                pair05[2 * q + 1] = sp[4];
            }
            if (grad)
                for (size_t a = 0; a < na; a++)
                    for (int c = 0; c < 3; c++) {
                        grad[((size_t)P * na + a) * 3 + c] += g[a * 6 + c];
                        grad[((size_t)Q * na + a) * 3 + c] += g[a * 6 + 3 + c];
                    }
        }
    double r = 0;
    for (int V = 0; V < n; V++)
        r = reg_volume(D + (size_t)V * na * 3, grad ? grad + (size_t)V * na * 3 : NULL, orient[V], w, h, d, p->eps_r,
                       p->flyback_frac, p->alpha, r);
    double sum[3] = {0, 0, 0};
    for (size_t e = 0; e < (size_t)n * na; e++)
        for (int c = 0; c < 3; c++) sum[c] += D[e * 3 + c];
    double m = 0;
    for (int c = 0; c < 3; c++) m += sum[c] * sum[c];
    m *= p->mean_weight * d / ((double)n * (double)na);
    if (grad)
        for (size_t e = 0; e < (size_t)n * na; e++)
            for (int c = 0; c < 3; c++) grad[e * 3 + c] += 2.0 * p->mean_weight * d * sum[c] / ((double)n * (double)na);
    terms[T_DATA] = s[0];
    terms[T_STR] = s[1];
    terms[T_ANG] = s[2];
    terms[T_STR05] = s[3];
    terms[T_ANG05] = s[4];
    terms[T_REG] = r;
    terms[T_MEAN] = m;
    terms[T_F] = s[0] + p->alpha * r + m;
    free(part);
    free(g);
    (void)np;
    return 0;
}

/* Level transition for n fields (orc_upsample per volume). */
EXPORT void orc_upsample_multi(int n, const double* coarse, int wc, int hc, double* fine, int wf, int hf)
{
    for (int V = 0; V < n; V++) {
        const double* C = coarse + (size_t)V * wc * hc * 3;
        double* Fo = fine + (size_t)V * wf * hf * 3;
        for (int j = 0; j < hf; j++)
            for (int i = 0; i < wf; i++) {
                double x = (i - 0.5) / 2.0, y = (j - 0.5) / 2.0;
                if (x < 0) x = 0;
                if (x > wc - 1) x = wc - 1;
                if (y < 0) y = 0;
                if (y > hc - 1) y = hc - 1;
                int x0 = (int)floor(x), y0 = (int)floor(y);
                int x1 = x0 + 1 < wc ? x0 + 1 : wc - 1, y1 = y0 + 1 < hc ? y0 + 1 : hc - 1;
                double fx = x - x0, fy = y - y0;
                for (int c = 0; c < 3; c++) {
                    double v00 = C[((size_t)y0 * wc + x0) * 3 + c], v10 = C[((size_t)y0 * wc + x1) * 3 + c];
                    double v01 = C[((size_t)y1 * wc + x0) * 3 + c], v11 = C[((size_t)y1 * wc + x1) * 3 + c];
                    double v = (1 - fy) * ((1 - fx) * v00 + fx * v10) + fy * ((1 - fx) * v01 + fx * v11);
                    Fo[((size_t)j * wf + i) * 3 + c] = 2.0 * v;
                }
            }
    }
}

typedef struct {
    int n;
    const double* const* S;
    const double* const* A;
    const double* const* Vv;
    const int* orient;
    int w, h, d;
    const orc_params* p;
    const double* eta;
    double terms[T_COUNT];
} multi_ctx;

static int multi_fg(void* vctx, const double* x, double* f, double* g)
{
    multi_ctx* c = (multi_ctx*)vctx;
    if (orc_eval_multi(c->n, c->S, c->A, c->Vv, c->orient, c->w, c->h, c->d, x, c->p, c->eta, c->terms, NULL, g))
        return -1;
    *f = c->terms[T_F];
    return 0;
}

/* The n-volume registration: per-volume pyramids (as orc_register, with the
 * same storage rounding), zero fields at the coarsest level, each pair's eta
 * at the level's initial field (Eq. 10), L-BFGS over all fields, upsampling
 * between levels.  D_out: [n][h][w][3]; levels_rep (may be NULL): per level,
 * coarsest first, f_start, f_end, iters, evals. */
EXPORT int orc_register_multi(int n, const double* const* S, const double* const* A, const double* const* Vv,
                              const int* orient, int w, int h, int d, const orc_params* p, double* D_out,
                              double* levels_rep)
{
    int L = p->levels;
    if (L < 1 || L > 8 || n < 2 || n > 8) return -1;
    int W[8], H[8], Dd[8];
    double* PS[8][8];
    double* PA[8][8];
    double* PV[8][8];
    W[0] = w; H[0] = h; Dd[0] = d;
    for (int V = 0; V < n; V++) {
        const size_t nv0 = (size_t)w * h * d;
        PS[0][V] = (double*)malloc(nv0 * sizeof(double));
        memcpy(PS[0][V], S[V], nv0 * sizeof(double));
        PA[0][V] = (double*)A[V];
        PV[0][V] = (double*)Vv[V];
    }
    for (int l = 1; l < L; l++) {
        W[l] = (W[l - 1] + 1) / 2; H[l] = (H[l - 1] + 1) / 2; Dd[l] = (Dd[l - 1] + 1) / 2;
        for (int V = 0; V < n; V++) {
            PS[l][V] = (double*)malloc((size_t)W[l] * H[l] * Dd[l] * sizeof(double));
            PA[l][V] = (double*)malloc((size_t)W[l] * H[l] * sizeof(double));
            const int nb = orient[V] == 0 ? H[l] : W[l];
            PV[l][V] = (double*)malloc((size_t)nb * sizeof(double));
            pyr_down3_for(p->store, PS[l - 1][V], W[l - 1], H[l - 1], Dd[l - 1], PS[l][V]);
            orc_pyr_down2(PA[l - 1][V], W[l - 1], H[l - 1], PA[l][V]);
            orc_pyr_down1(PV[l - 1][V], orient[V] == 0 ? H[l - 1] : W[l - 1], PV[l][V]);
        }
    }
    if (p->store)
        for (int l = 0; l < L; l++)
            for (int V = 0; V < n; V++) orc_round_storage(PS[l][V], (size_t)W[l] * H[l] * Dd[l], p->store);
    const int np = pair_count(n);
    double eta[28], p05[56];
    int rc = 0;
    double* Dc = NULL;
    for (int l = L - 1; l >= 0; l--) {
        const size_t nn = (size_t)n * W[l] * H[l] * 3;
        double* Dl = (double*)calloc(nn, sizeof(double));
        if (Dc) {
            orc_upsample_multi(n, Dc, W[l + 1], H[l + 1], Dl, W[l], H[l]);
            free(Dc);
        }
        for (int q = 0; q < np; q++) eta[q] = 1.0;
        double terms[T_COUNT];
        orc_eval_multi(n, (const double* const*)PS[l], (const double* const*)PA[l], (const double* const*)PV[l], orient,
                       W[l], H[l], Dd[l], Dl, p, eta, terms, p05, NULL);
        for (int q = 0; q < np; q++) eta[q] = orc_eta_from_terms(p05[2 * q], p05[2 * q + 1]);
        multi_ctx ctx = {n, (const double* const*)PS[l], (const double* const*)PA[l], (const double* const*)PV[l],
                         orient, W[l], H[l], Dd[l], p, eta, {0}};
        orc_lbfgs_report rep;
        rc = orc_lbfgs((int)nn, Dl, multi_fg, &ctx, p->lbfgs_m, p->iters, p->ls_max_evals, p->c1, p->c2, &rep);
        if (levels_rep) {
            double* r = levels_rep + (size_t)(L - 1 - l) * 4;
            r[0] = rep.f_start; r[1] = rep.f_end; r[2] = rep.iters; r[3] = rep.evals;
        }
        Dc = Dl;
        if (rc) break;
    }
    if (rc == 0) memcpy(D_out, Dc, (size_t)n * w * h * 3 * sizeof(double));
    free(Dc);
    for (int V = 0; V < n; V++) free(PS[0][V]);
    for (int l = 1; l < L; l++)
        for (int V = 0; V < n; V++) {
            free(PS[l][V]);
            free(PA[l][V]);
            free(PV[l][V]);
        }
    return rc;
}

/* Density of one field ([h][w][3]) as orc_density. */
static void density_one(const double* DV, int w, int h, double* rho)
{
    double* grid = (double*)calloc((size_t)w * h, sizeof(double));
    for (int pass = 0; pass < 2; pass++)
        for (int j = 0; j < h; j++)
            for (int i = 0; i < w; i++) {
                double x = i + DV[((size_t)j * w + i) * 3 + 0], y = j + DV[((size_t)j * w + i) * 3 + 1];
                x = x < 0 ? 0 : (x > w - 1 ? w - 1 : x);
                y = y < 0 ? 0 : (y > h - 1 ? h - 1 : y);
                const int x0 = (int)floor(x), y0 = (int)floor(y);
                const int x1 = x0 + 1 < w ? x0 + 1 : w - 1, y1 = y0 + 1 < h ? y0 + 1 : h - 1;
                const double fx = x - x0, fy = y - y0;
                if (pass == 0) {
                    grid[(size_t)y0 * w + x0] += (1 - fx) * (1 - fy);
                    grid[(size_t)y0 * w + x1] += fx * (1 - fy);
                    grid[(size_t)y1 * w + x0] += (1 - fx) * fy;
                    grid[(size_t)y1 * w + x1] += fx * fy;
                } else {
                    rho[(size_t)j * w + i] = (1 - fx) * (1 - fy) * grid[(size_t)y0 * w + x0] +
                                             fx * (1 - fy) * grid[(size_t)y0 * w + x1] +
                                             (1 - fx) * fy * grid[(size_t)y1 * w + x0] + fx * fy * grid[(size_t)y1 * w + x1];
                }
            }
    free(grid);
}

/* n-volume merge (readings above).  O (may be NULL) are the OCTA volumes with
 * invalid B-scans already replaced by their nearest valid neighbours. */
EXPORT void orc_merge_multi(int n, const double* const* S, const double* const* O, const double* const* Vv,
                            const int* orient, int w, int h, int d, const double* D, double kappa, double tau,
                            double* merged_oct, double* merged_octa)
{
    const size_t na = (size_t)w * h;
    double* rho = (double*)malloc((size_t)n * na * sizeof(double));
    for (int V = 0; V < n; V++) density_one(D + (size_t)V * na * 3, w, h, rho + (size_t)V * na);
#pragma omp parallel for schedule(dynamic, 4)
    for (long a = 0; a < (long)na; a++) {
        const int i = (int)(a % w), j = (int)(a / w);
        double wt[8], ow[8], sw = 0, so = 0;
        int lowest = 0;
        for (int V = 0; V < n; V++) {
            const double r = rho[(size_t)V * na + a];
            wt[V] = exp(-kappa * fmax(0.0, r - 1.0));
            if (wt[V] < tau) wt[V] = 0;
            sw += wt[V];
            if (r < rho[(size_t)lowest * na + a]) lowest = V;
        }
        for (int V = 0; V < n; V++) {
            double tv, dtv;
            int comp;
            valid_sample(Vv[V], orient[V], w, h, i, j, D + ((size_t)V * na + a) * 3, &tv, &dtv, &comp);
            ow[V] = wt[V] * tv;
            so += ow[V];
        }
        for (int V = 0; V < n; V++) {
            if (sw > 0) wt[V] /= sw;
            else wt[V] = V == lowest ? 1.0 : 0.0;
            if (so > 0) ow[V] /= so;
        }
        for (int k = 0; k < d; k++) {
            double mo = 0, ma = 0;
            for (int V = 0; V < n; V++) {
                const double* dV = D + ((size_t)V * na + a) * 3;
                double sv[4];
                orc_sample3(S[V], w, h, d, i + dV[0], j + dV[1], k + dV[2], sv);
                mo += wt[V] * sv[0];
                if (merged_octa) {
                    double ov[4];
                    orc_sample3(O[V], w, h, d, i + dV[0], j + dV[1], k + dV[2], ov);
                    ma += ow[V] * ov[0];
                }
            }
            merged_oct[a * d + k] = mo;
            if (merged_octa) merged_octa[a * d + k] = ma;
        }
    }
    free(rho);
}
