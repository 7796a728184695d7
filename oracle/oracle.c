/*
 * FP64 CPU oracle for explicit f-x poststack depth migration.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h): slow, plain, obviously correct.
 * Built with -O2 -ffp-contract=off so that every floating-point operation
 * written here is rounded on its own, in IEEE double precision.
 *
 * Paper references are to Shawahna, Salam & Al-Mouhamed (arXiv 1912.05529):
 * Eq. (1) is the f-x extrapolation sum, Algorithm 1 the explicit f-x
 * poststack depth migration loop, Sec. III the implementation notes
 * (predesigned filter bank accessed by cutoff, depth row = sum over
 * frequencies).
 */
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static const double PI = 3.14159265358979323846;

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int desc_ok(const orc_desc* d)
{
    if (!d) return 0;
    if (d->ntaps < 1 || (d->ntaps % 2) == 0) return 0;
    if (d->nk < 2) return 0;
    if (!(d->kmin > 0.0) || !(d->kmax > d->kmin)) return 0;
    if (!(d->dx > 0.0) || !(d->dz >= 0.0)) return 0;
    if (d->ngrid < 1 || d->ncheck < 1 || d->nreweight < 0) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Filter design (Sec. II: the design is an optimization trading filter      */
/* length against propagation angle; Eq. (1) is unstable unless the design  */
/* is accurate; Sec. III: filters designed in advance, looked up by cutoff). */
/*                                                                          */
/* Entry j targets the normalized wavenumber kappa = (kmin + j*dk)*dx with  */
/* dk = (kmax-kmin)/(nk-1).  On the midpoint grid theta_i = (i+1/2)pi/L of  */
/* normalized lateral wavenumber kx*dx, the desired response is the one-way */
/* phase shift over dz:                                                     */
/*   D = exp(+i zeta sqrt(kappa^2 - theta^2))   for theta <= kappa,         */
/*   D = exp(-zeta sqrt(theta^2 - kappa^2))     for theta >  kappa,         */
/* zeta = dz/dx.  With even taps h[-n] = h[n] the response is               */
/*   H(theta) = h0 + 2 sum_{n=1..M} h_n cos(n theta).                       */
/* The taps minimize sum_i w_i |H(theta_i) - D(theta_i)|^2 + lambda |h|^2,  */
/* then the weights of points with |H| > 1 are raised and the fit repeated  */
/* nreweight times; finally h is scaled so that |H| <= 1 - margin for every */
/* theta (bound from max on a check grid, see below).                       */
/* ------------------------------------------------------------------------ */

/* Solve (A^T W A + lambda I) h = A^T W D for complex h (two real right-hand
 * sides) by Cholesky.  A is [L][K] row-major. */
static int wls_solve(const double* A, int L, int K, const double* w,
                     const cplx* D, double lambda, cplx* h)
{
    double* G = (double*)calloc((size_t)K * K, sizeof(double));
    double* br = (double*)calloc((size_t)K, sizeof(double));
    double* bi = (double*)calloc((size_t)K, sizeof(double));
    if (!G || !br || !bi) { free(G); free(br); free(bi); return ORC_E_NOMEM; }

    for (int i = 0; i < L; ++i) {
        const double* a = A + (size_t)i * K;
        for (int p = 0; p < K; ++p) {
            for (int q = 0; q < K; ++q) G[p * K + q] += w[i] * a[p] * a[q];
            br[p] += w[i] * a[p] * creal(D[i]);
            bi[p] += w[i] * a[p] * cimag(D[i]);
        }
    }
    for (int p = 0; p < K; ++p) G[p * K + p] += lambda;

    /* G = C C^T, C lower triangular, stored in place. */
    for (int p = 0; p < K; ++p) {
        for (int q = 0; q <= p; ++q) {
            double s = G[p * K + q];
            for (int m = 0; m < q; ++m) s -= G[p * K + m] * G[q * K + m];
            if (p == q) {
                if (!(s > 0.0)) { free(G); free(br); free(bi); return ORC_E_NUMERIC; }
                G[p * K + p] = sqrt(s);
            } else {
                G[p * K + q] = s / G[q * K + q];
            }
        }
    }
    /* forward: C y = b */
    for (int p = 0; p < K; ++p) {
        double sr = br[p], si = bi[p];
        for (int m = 0; m < p; ++m) { sr -= G[p * K + m] * br[m]; si -= G[p * K + m] * bi[m]; }
        br[p] = sr / G[p * K + p];
        bi[p] = si / G[p * K + p];
    }
    /* backward: C^T h = y */
    for (int p = K - 1; p >= 0; --p) {
        double sr = br[p], si = bi[p];
        for (int m = p + 1; m < K; ++m) { sr -= G[m * K + p] * br[m]; si -= G[m * K + p] * bi[m]; }
        br[p] = sr / G[p * K + p];
        bi[p] = si / G[p * K + p];
    }
    for (int p = 0; p < K; ++p) h[p] = br[p] + I * bi[p];
    free(G); free(br); free(bi);
    return ORC_OK;
}

static int design_one(const orc_desc* d, int apply_scale, const double* A,
                      int j, double* tab_row, double* maxgain, double* passerr,
                      double* scale)
{
    const int M = (d->ntaps - 1) / 2, K = M + 1, L = d->ngrid, Lc = d->ncheck;
    const double dk = (d->kmax - d->kmin) / (double)(d->nk - 1);
    const double kappa = (d->kmin + (double)j * dk) * d->dx;
    const double zeta = d->dz / d->dx;
    const double edge = kappa * sin(d->theta_max_deg * PI / 180.0);

    double* w = (double*)malloc((size_t)L * sizeof(double));
    cplx* D = (cplx*)malloc((size_t)L * sizeof(cplx));
    cplx* h = (cplx*)malloc((size_t)K * sizeof(cplx));
    if (!w || !D || !h) { free(w); free(D); free(h); return ORC_E_NOMEM; }

    for (int i = 0; i < L; ++i) {
        double th = ((double)i + 0.5) * PI / (double)L;
        if (th <= kappa) D[i] = cexp(I * (zeta * sqrt(kappa * kappa - th * th)));
        else D[i] = exp(-zeta * sqrt(th * th - kappa * kappa));
        if (th <= edge) w[i] = d->w_pass;
        else if (th <= kappa) w[i] = d->w_trans;
        else w[i] = d->w_evan;
    }

    int rc = wls_solve(A, L, K, w, D, d->lambda, h);
    for (int it = 0; rc == ORC_OK && it < d->nreweight; ++it) {
        for (int i = 0; i < L; ++i) {
            cplx H = 0.0;
            for (int n = 0; n < K; ++n) H += A[(size_t)i * K + n] * h[n];
            double excess = cabs(H) - 1.0;
            if (excess > 0.0) w[i] = w[i] * (1.0 + d->beta * excess / d->tau);
        }
        rc = wls_solve(A, L, K, w, D, d->lambda, h);
    }
    if (rc != ORC_OK) { free(w); free(D); free(h); return rc; }

    /* Stability scale.  For a trigonometric polynomial T of degree M the
     * Szego form of Bernstein's inequality gives T(theta) >= |T|max
     * cos(M |theta - theta*|) near a maximum theta*, so on a midpoint grid
     * of spacing pi/Lc:  |H|max <= max_grid |H| / cos(M pi / (2 Lc)). */
    double g = 0.0;
    for (int c = 0; c < Lc; ++c) {
        double th = ((double)c + 0.5) * PI / (double)Lc;
        cplx H = h[0];
        for (int n = 1; n < K; ++n) H += 2.0 * cos((double)n * th) * h[n];
        double a = cabs(H);
        if (a > g) g = a;
    }
    double s = 1.0;
    if (apply_scale) {
        double lim = (1.0 - d->margin) * cos((double)M * PI / (2.0 * (double)Lc));
        if (g > lim) s = lim / g;
    }
    for (int n = 0; n < K; ++n) h[n] = s * h[n];

    double perr = 0.0;
    for (int i = 0; i < L; ++i) {
        double th = ((double)i + 0.5) * PI / (double)L;
        if (!(th <= edge)) continue;
        cplx H = 0.0;
        for (int n = 0; n < K; ++n) H += A[(size_t)i * K + n] * h[n];
        double e = cabs(H - D[i]);
        if (e > perr) perr = e;
    }

    for (int n = 0; n < K; ++n) {
        tab_row[2 * n] = creal(h[n]);
        tab_row[2 * n + 1] = cimag(h[n]);
    }
    if (maxgain) *maxgain = s * g;
    if (passerr) *passerr = perr;
    if (scale) *scale = s;
    free(w); free(D); free(h);
    return ORC_OK;
}

int orc_design_table(const orc_desc* d, int apply_scale, double* tab,
                     double* maxgain, double* passerr, double* scale)
{
    if (!desc_ok(d) || !tab) return ORC_E_ARG;
    const int M = (d->ntaps - 1) / 2, K = M + 1, L = d->ngrid;

    /* Design matrix on the midpoint grid: column 0 is 1, column n is
     * 2 cos(n theta_i). */
    double* A = (double*)malloc((size_t)L * K * sizeof(double));
    if (!A) return ORC_E_NOMEM;
    for (int i = 0; i < L; ++i) {
        double th = ((double)i + 0.5) * PI / (double)L;
        A[(size_t)i * K] = 1.0;
        for (int n = 1; n < K; ++n) A[(size_t)i * K + n] = 2.0 * cos((double)n * th);
    }

    int rc = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < d->nk; ++j) {
        int r = design_one(d, apply_scale, A, j, tab + (size_t)j * 2 * K,
                           maxgain ? maxgain + j : NULL,
                           passerr ? passerr + j : NULL,
                           scale ? scale + j : NULL);
        if (r != ORC_OK) {
#pragma omp critical
            rc = r;
        }
    }
    free(A);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Table look-up (the look-up inside the space loop of Algorithm 1;        */
/* Sec. III: the cutoff depends on the wavenumber omega/v, which varies     */
/* from point to point).  Nearest entry to k = omega/v on the uniform axis  */
/* k_j = kmin + j dk, rounding halves up, clamped to [0, nk-1]; a velocity  */
/* that is not > 0 (NaN, zero, negative) selects entry 0.  Each step is a   */
/* separately rounded IEEE double operation, in this order.                 */
/* ------------------------------------------------------------------------ */
static int index_of(double dk, double kmin, int nk, double omega, float v)
{
    if (!(v > 0.0f)) return 0;
    double a = omega / dk;
    double b = kmin / dk;
    double s = 1.0 / (double)v;
    double t = a * s;
    t = t - b;
    double u = t + 0.5;
    if (!(u >= 1.0)) return 0;
    if (u >= (double)nk) return nk - 1;
    return (int)floor(u);
}

int orc_table_index(const orc_desc* d, const double* omega, int32_t nw,
                    const float* vel, int32_t nx, int32_t nrows, int32_t* idx)
{
    if (!desc_ok(d) || !omega || !vel || !idx || nw < 1 || nx < 1 || nrows < 1)
        return ORC_E_ARG;
    const double dk = (d->kmax - d->kmin) / (double)(d->nk - 1);
    for (int k = 0; k < nrows; ++k)
        for (int x = 0; x < nx; ++x)
            for (int r = 0; r < nw; ++r)
                idx[((size_t)k * nx + x) * nw + r] =
                    index_of(dk, d->kmin, d->nk, omega[r], vel[(size_t)k * nx + x]);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Imaging (the depth-row step of Algorithm 1, a sum over frequencies;     */
/* Sec. III second kernel): row[x] = sum_r Re P[x][r], r in order.          */
/* ------------------------------------------------------------------------ */
int orc_image(const double* plane, int32_t nx, int32_t nw, double* row)
{
    if (!plane || !row || nx < 1 || nw < 1) return ORC_E_ARG;
    for (int x = 0; x < nx; ++x) {
        double s = 0.0;
        for (int r = 0; r < nw; ++r) s += plane[2 * ((size_t)x * nw + r)];
        row[x] = s;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Extrapolation, Eq. (1) written out:                                      */
/*   P_{k+1}[x][r] = sum_{n=-M..M} h_j[|n|] P_k[x-n][r],                    */
/* with P_k[x'] = 0 outside [0, nx) and j the table entry for               */
/* (omega_r, vel[k][x]) -- the filter of the output point.  Independent per */
/* frequency (Sec. II), so frequencies run in parallel; depth is serial.    */
/* ------------------------------------------------------------------------ */
int orc_extrapolate(const orc_desc* d, const double* tab, const double* omega,
                    int32_t nw, const float* vel, int32_t nx, int32_t nsteps,
                    const double* in, double* out, double* rows)
{
    if (!desc_ok(d) || !tab || !omega || !vel || !in || !out || nw < 1 ||
        nx < 1 || nsteps < 0)
        return ORC_E_ARG;
    const int M = (d->ntaps - 1) / 2, K = M + 1;
    const double dk = (d->kmax - d->kmin) / (double)(d->nk - 1);
    const cplx* T = (const cplx*)tab;
    size_t n_plane = (size_t)nx * nw;
    cplx* P = (cplx*)malloc(n_plane * sizeof(cplx));
    cplx* Q = (cplx*)malloc(n_plane * sizeof(cplx));
    if (!P || !Q) { free(P); free(Q); return ORC_E_NOMEM; }
    memcpy(P, in, n_plane * sizeof(cplx));

    for (int k = 0; k < nsteps; ++k) {
        const float* vrow = vel + (size_t)k * nx;
#pragma omp parallel for schedule(static)
        for (int r = 0; r < nw; ++r) {
            for (int x = 0; x < nx; ++x) {
                int j = index_of(dk, d->kmin, d->nk, omega[r], vrow[x]);
                const cplx* h = T + (size_t)j * K;
                cplx acc = 0.0;
                for (int n = -M; n <= M; ++n) {
                    int xs = x - n;
                    if (xs < 0 || xs >= nx) continue;
                    acc += h[n < 0 ? -n : n] * P[(size_t)xs * nw + r];
                }
                Q[(size_t)x * nw + r] = acc;
            }
        }
        cplx* t = P; P = Q; Q = t;
        if (rows) orc_image((const double*)P, nx, nw, rows + (size_t)k * nx);
    }
    memcpy(out, P, n_plane * sizeof(cplx));
    free(P); free(Q);
    return ORC_OK;
}

/* Algorithm 1 end to end on an f-x section (the t -> omega transform is
 * done by the caller).  Row 0 = image of the surface plane. */
int orc_migrate(const orc_desc* d, const double* tab, const double* omega,
                int32_t nw, const float* vel, int32_t nx, int32_t nz,
                const double* data, double* image)
{
    if (!data || !image || nz < 1 || nx < 1 || nw < 1) return ORC_E_ARG;
    int rc = orc_image(data, nx, nw, image);
    if (rc != ORC_OK || nz == 1) return rc;
    double* last = (double*)malloc((size_t)nx * nw * 2 * sizeof(double));
    if (!last) return ORC_E_NOMEM;
    rc = orc_extrapolate(d, tab, omega, nw, vel, nx, nz - 1, data, last,
                         image + nx);
    free(last);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Adjoint.  With <a,b> = Re sum conj(a) b, the image map                   */
/*   I_k = S E_{k-1} ... E_0 d,   (S P)[x] = sum_r Re P[x][r],              */
/* has adjoint d' = Q_0 where Q_{nz-1} = S* I'_{nz-1},                      */
/* Q_k = S* I'_k + E_k^H Q_{k+1}, (S* i)[x][r] = i[x], and                  */
/* (E_k^H q)[x] = sum_n conj(h_{j(x+n,k)}[|n|]) q[x+n] (filters of the      */
/* output points x+n that x fed in the forward step).                       */
/* ------------------------------------------------------------------------ */
int orc_demigrate(const orc_desc* d, const double* tab, const double* omega,
                  int32_t nw, const float* vel, int32_t nx, int32_t nz,
                  const double* image, double* data)
{
    if (!desc_ok(d) || !tab || !omega || !vel || !image || !data || nw < 1 ||
        nx < 1 || nz < 1)
        return ORC_E_ARG;
    const int M = (d->ntaps - 1) / 2, K = M + 1;
    const double dk = (d->kmax - d->kmin) / (double)(d->nk - 1);
    const cplx* T = (const cplx*)tab;
    size_t n_plane = (size_t)nx * nw;
    cplx* Q = (cplx*)malloc(n_plane * sizeof(cplx));
    cplx* R = (cplx*)malloc(n_plane * sizeof(cplx));
    if (!Q || !R) { free(Q); free(R); return ORC_E_NOMEM; }

    for (int x = 0; x < nx; ++x)
        for (int r = 0; r < nw; ++r)
            Q[(size_t)x * nw + r] = image[(size_t)(nz - 1) * nx + x];

    for (int k = nz - 2; k >= 0; --k) {
        const float* vrow = vel + (size_t)k * nx;
#pragma omp parallel for schedule(static)
        for (int r = 0; r < nw; ++r) {
            for (int x = 0; x < nx; ++x) {
                cplx acc = 0.0;
                for (int n = -M; n <= M; ++n) {
                    int xo = x + n;
                    if (xo < 0 || xo >= nx) continue;
                    int j = index_of(dk, d->kmin, d->nk, omega[r], vrow[xo]);
                    acc += conj(T[(size_t)j * K + (n < 0 ? -n : n)]) * Q[(size_t)xo * nw + r];
                }
                R[(size_t)x * nw + r] = acc + image[(size_t)k * nx + x];
            }
        }
        cplx* t = Q; Q = R; R = t;
    }
    memcpy(data, Q, n_plane * sizeof(cplx));
    free(Q); free(R);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Transform along t (first step of Algorithm 1; Sec. III), evaluated     */
/* directly at the requested frequencies with the forward sign             */
/* exp(-i omega t).                                                         */
/* ------------------------------------------------------------------------ */
int orc_transform_t(const float* p, int32_t nx, int32_t nt, double dt,
                    const double* omega, int32_t nw, double* out)
{
    if (!p || !omega || !out || nx < 1 || nt < 1 || nw < 1 || !(dt > 0.0)) return ORC_E_ARG;
#pragma omp parallel for schedule(static)
    for (int x = 0; x < nx; ++x) {
        for (int r = 0; r < nw; ++r) {
            cplx acc = 0.0;
            for (int n = 0; n < nt; ++n)
                acc += (double)p[(size_t)x * nt + n] * cexp(-I * (omega[r] * ((double)n * dt)));
            out[2 * ((size_t)x * nw + r)] = creal(acc);
            out[2 * ((size_t)x * nw + r) + 1] = cimag(acc);
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* 3-D extension (Sec. II: explicit f-x migration extends to 3-D with 2-D   */
/* filters; Eq. (1) becomes a 2-D convolution per frequency).               */
/*                                                                          */
/* Design: the 2-D analogue of design_one.  Target on the midpoint grid of  */
/* (theta_x, theta_y) in (0, pi)^2:                                         */
/*   D = exp(+i zeta sqrt(kappa^2 - r^2)) for r <= kappa, else              */
/*       exp(-zeta sqrt(r^2 - kappa^2)),   r^2 = theta_x^2 + theta_y^2,     */
/* weights by r as in 1-D.  Basis per unique coefficient (a, b): the sum of */
/* cos(n1 theta_x) cos(n2 theta_y) over the symmetry orbit of (a, b), i.e.  */
/*   1                                              a = b = 0               */
/*   2 (cos a tx + cos a ty)                        a > 0, b = 0            */
/*   4 cos a tx cos a ty                            a = b > 0               */
/*   4 (cos a tx cos b ty + cos b tx cos a ty)      a > b > 0               */
/* Stability: applying the 1-D Bernstein bound along each axis,             */
/* |H|max <= max_grid |H| / cos(M pi / (2 Lc))^2.                           */
/* ------------------------------------------------------------------------ */
static double basis2d(int a, int b, double tx, double ty)
{
    if (a == 0) return 1.0;
    if (b == 0) return 2.0 * (cos(a * tx) + cos(a * ty));
    if (a == b) return 4.0 * cos(a * tx) * cos(a * ty);
    return 4.0 * (cos(a * tx) * cos(b * ty) + cos(b * tx) * cos(a * ty));
}

static int design_one_2d(const orc_desc* d, int apply_scale, const double* A, int j,
                         double* tab_row, double* maxgain, double* passerr, double* scale)
{
    const int M = (d->ntaps - 1) / 2, NU = (M + 1) * (M + 2) / 2;
    const int L = d->ngrid, LL = L * L, Lc = d->ncheck;
    const double dk = (d->kmax - d->kmin) / (double)(d->nk - 1);
    const double kappa = (d->kmin + (double)j * dk) * d->dx;
    const double zeta = d->dz / d->dx;
    const double edge = kappa * sin(d->theta_max_deg * PI / 180.0);

    double* w = (double*)malloc((size_t)LL * sizeof(double));
    cplx* D = (cplx*)malloc((size_t)LL * sizeof(cplx));
    cplx* h = (cplx*)malloc((size_t)NU * sizeof(cplx));
    if (!w || !D || !h) { free(w); free(D); free(h); return ORC_E_NOMEM; }
    for (int i = 0; i < L; ++i) {
        for (int q = 0; q < L; ++q) {
            double tx = ((double)i + 0.5) * PI / (double)L;
            double ty = ((double)q + 0.5) * PI / (double)L;
            double r2 = tx * tx + ty * ty, k2 = kappa * kappa;
            double rr = sqrt(r2);
            size_t e = (size_t)i * L + q;
            if (r2 <= k2) D[e] = cexp(I * (zeta * sqrt(k2 - r2)));
            else D[e] = exp(-zeta * sqrt(r2 - k2));
            if (rr <= edge) w[e] = d->w_pass;
            else if (rr <= kappa) w[e] = d->w_trans;
            else w[e] = d->w_evan;
        }
    }
    int rc = wls_solve(A, LL, NU, w, D, d->lambda, h);
    for (int it = 0; rc == ORC_OK && it < d->nreweight; ++it) {
        for (int e = 0; e < LL; ++e) {
            cplx H = 0.0;
            for (int u = 0; u < NU; ++u) H += A[(size_t)e * NU + u] * h[u];
            double excess = cabs(H) - 1.0;
            if (excess > 0.0) w[e] = w[e] * (1.0 + d->beta * excess / d->tau);
        }
        rc = wls_solve(A, LL, NU, w, D, d->lambda, h);
    }
    if (rc != ORC_OK) { free(w); free(D); free(h); return rc; }

    /* Response on the Lc x Lc check grid, as the double sum over the
     * unexpanded (2M+1)^2 filter written with cosines: for each grid row the
     * inner sum over n2 of h[n1][n2] cos(n2 ty) is formed first. */
    double* cs = (double*)malloc((size_t)Lc * (M + 1) * sizeof(double));
    cplx* rowsum = (cplx*)malloc((size_t)(M + 1) * sizeof(cplx));
    if (!cs || !rowsum) { free(cs); free(rowsum); free(w); free(D); free(h); return ORC_E_NOMEM; }
    for (int i = 0; i < Lc; ++i)
        for (int n = 0; n <= M; ++n)
            cs[(size_t)i * (M + 1) + n] = cos((double)n * ((double)i + 0.5) * PI / (double)Lc);
    double g = 0.0;
    for (int q = 0; q < Lc; ++q) {
        const double* cy = cs + (size_t)q * (M + 1);
        for (int n1 = 0; n1 <= M; ++n1) {  /* |n1|; both signs of n2 folded */
            cplx acc = 0.0;
            for (int n2 = -M; n2 <= M; ++n2) {
                int a = n1 > abs(n2) ? n1 : abs(n2), b = n1 > abs(n2) ? abs(n2) : n1;
                acc += h[a * (a + 1) / 2 + b] * cy[abs(n2)];
            }
            rowsum[n1] = acc;
        }
        for (int i = 0; i < Lc; ++i) {
            const double* cx = cs + (size_t)i * (M + 1);
            cplx H = rowsum[0];
            for (int n1 = 1; n1 <= M; ++n1) H += 2.0 * cx[n1] * rowsum[n1];
            double v = cabs(H);
            if (v > g) g = v;
        }
    }
    free(cs);
    free(rowsum);
    double s = 1.0;
    if (apply_scale) {
        double c = cos((double)M * PI / (2.0 * (double)Lc));
        double lim = (1.0 - d->margin) * c * c;
        if (g > lim) s = lim / g;
    }
    for (int u = 0; u < NU; ++u) h[u] = s * h[u];
    double perr = 0.0;
    for (int e = 0; e < LL; ++e) {
        int i = e / L, q = e % L;
        double tx = ((double)i + 0.5) * PI / (double)L;
        double ty = ((double)q + 0.5) * PI / (double)L;
        if (!(sqrt(tx * tx + ty * ty) <= edge)) continue;
        cplx H = 0.0;
        for (int u = 0; u < NU; ++u) H += A[(size_t)e * NU + u] * h[u];
        double err = cabs(H - D[e]);
        if (err > perr) perr = err;
    }
    for (int u = 0; u < NU; ++u) {
        tab_row[2 * u] = creal(h[u]);
        tab_row[2 * u + 1] = cimag(h[u]);
    }
    if (maxgain) *maxgain = s * g;
    if (passerr) *passerr = perr;
    if (scale) *scale = s;
    free(w); free(D); free(h);
    return ORC_OK;
}

int orc_design_table_2d(const orc_desc* d, int apply_scale, double* tab,
                        double* maxgain, double* passerr, double* scale)
{
    if (!desc_ok(d) || !tab) return ORC_E_ARG;
    const int M = (d->ntaps - 1) / 2, NU = (M + 1) * (M + 2) / 2, L = d->ngrid;
    double* A = (double*)malloc((size_t)L * L * NU * sizeof(double));
    if (!A) return ORC_E_NOMEM;
    for (int i = 0; i < L; ++i)
        for (int q = 0; q < L; ++q) {
            double tx = ((double)i + 0.5) * PI / (double)L;
            double ty = ((double)q + 0.5) * PI / (double)L;
            for (int a = 0, u = 0; a <= M; ++a)
                for (int b = 0; b <= a; ++b, ++u)
                    A[((size_t)i * L + q) * NU + u] = basis2d(a, b, tx, ty);
        }
    int rc = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < d->nk; ++j) {
        int r = design_one_2d(d, apply_scale, A, j, tab + (size_t)j * 2 * NU,
                              maxgain ? maxgain + j : NULL, passerr ? passerr + j : NULL,
                              scale ? scale + j : NULL);
        if (r != ORC_OK) {
#pragma omp critical
            rc = r;
        }
    }
    free(A);
    return rc;
}

/* 3-D depth step, Eq. (1) with a 2-D sum over (n1, n2), literally. */
int orc_migrate3d(const orc_desc* d, const double* tab, const double* omega,
                  int32_t nw, const float* vel, int32_t nx, int32_t ny, int32_t nz,
                  const double* data, double* image, double* plane_out)
{
    if (!desc_ok(d) || !tab || !omega || !vel || !data || !image || nw < 1 || nx < 1 ||
        ny < 1 || nz < 1)
        return ORC_E_ARG;
    const int M = (d->ntaps - 1) / 2, NU = (M + 1) * (M + 2) / 2;
    const double dk = (d->kmax - d->kmin) / (double)(d->nk - 1);
    const cplx* T = (const cplx*)tab;
    const size_t np = (size_t)nx * ny * nw;
    cplx* P = (cplx*)malloc(np * sizeof(cplx));
    cplx* Q = (cplx*)malloc(np * sizeof(cplx));
    if (!P || !Q) { free(P); free(Q); return ORC_E_NOMEM; }
    memcpy(P, data, np * sizeof(cplx));
    for (int k = 0; k < nz; ++k) {
        if (k > 0) {
            const float* vrow = vel + (size_t)(k - 1) * nx * ny;
#pragma omp parallel for schedule(static)
            for (int r = 0; r < nw; ++r) {
                for (int x = 0; x < nx; ++x) {
                    for (int y = 0; y < ny; ++y) {
                        int j = index_of(dk, d->kmin, d->nk, omega[r], vrow[(size_t)x * ny + y]);
                        const cplx* c = T + (size_t)j * NU;
                        cplx acc = 0.0;
                        for (int n1 = -M; n1 <= M; ++n1) {
                            int xs = x - n1;
                            if (xs < 0 || xs >= nx) continue;
                            for (int n2 = -M; n2 <= M; ++n2) {
                                int ys = y - n2;
                                if (ys < 0 || ys >= ny) continue;
                                int a = abs(n1), b = abs(n2);
                                if (b > a) { int t = a; a = b; b = t; }
                                acc += c[a * (a + 1) / 2 + b] * P[((size_t)xs * ny + ys) * nw + r];
                            }
                        }
                        Q[((size_t)x * ny + y) * nw + r] = acc;
                    }
                }
            }
            cplx* t = P; P = Q; Q = t;
        }
        for (int x = 0; x < nx; ++x)
            for (int y = 0; y < ny; ++y) {
                double sum = 0.0;
                for (int r = 0; r < nw; ++r) sum += creal(P[((size_t)x * ny + y) * nw + r]);
                image[((size_t)k * nx + x) * ny + y] = sum;
            }
    }
    if (plane_out) memcpy(plane_out, P, np * sizeof(cplx));
    free(P); free(Q);
    return ORC_OK;
}
