// Extrapolator-table design in FP64 on the GPU (table row A0).
//
// The paper designs the 1-D FIR extrapolators in advance, as an optimization
// between filter length and propagation angle, and stresses that accurate
// designs are needed for the recursion of Eq. (1) to stay stable (Sec. II,
// Sec. III).  It does not give the method.  This file implements, per table
// entry, a weighted least-squares fit of even taps to the one-way phase shift
// over dz, with multiplicative reweighting of points whose gain exceeds one,
// and a final scale that bounds |H| below one for every wavenumber (Bernstein's
// inequality for trigonometric polynomials).  The formulas are in mig.h.
//
// Mapping: one workgroup per entry.  The grid quantities (weights, target) live
// in LDS; the basis matrices (design grid and check grid, shared by all
// entries) are computed once into the workspace and read through L2.  Each
// entry of the normal matrix is accumulated by one thread over the grid in
// increasing grid order, and the Cholesky solve runs on one thread: the design
// is a few thousand flops per entry per pass, far from any roofline, and a
// fixed sequential order keeps the result reproducible.
#include "common.hpp"

namespace mig {
namespace {

constexpr int kDesignThreads = 256;
constexpr int kMaxK = MIG_MAX_NTAPS / 2 + 1;  // 32

// A[i][n] = 1 (n = 0) or 2 cos(n theta_i) on the design midpoint grid;
// C[c][n] likewise on the check grid.
__global__ void k_design_basis(int L, int Lc, int K, double* A, double* C)
{
#pragma clang fp contract(off)
    int tid = blockIdx.x * blockDim.x + threadIdx.x;
    int total = (L + Lc) * K;
    for (int e = tid; e < total; e += gridDim.x * blockDim.x) {
        int i = e / K, n = e % K;
        if (i < L) {
            double th = ((double)i + 0.5) * kPi / (double)L;
            A[(size_t)i * K + n] = n == 0 ? 1.0 : 2.0 * cos((double)n * th);
        } else {
            int c = i - L;
            double th = ((double)c + 0.5) * kPi / (double)Lc;
            C[(size_t)c * K + n] = n == 0 ? 1.0 : 2.0 * cos((double)n * th);
        }
    }
}

struct DesignShared {
    double G[kMaxK * kMaxK];
    double br[kMaxK], bi[kMaxK];
    double hr[kMaxK], hi[kMaxK];
    double red[kDesignThreads];
    int fail;
};

// Normal equations (A^T W A + lambda I) h = A^T W D, Cholesky, two real RHS.
__device__ void wls_solve(const double* __restrict__ A, const double* w,
                          const double* Dr, const double* Di, int L, int K,
                          double lambda, DesignShared& sh)
{
#pragma clang fp contract(off)
    const int npair = K * (K + 1) / 2;
    for (int task = threadIdx.x; task < npair + K; task += blockDim.x) {
        if (task < npair) {
            // lower-triangle pair (p, q), q <= p
            int p = 0;
            while ((p + 1) * (p + 2) / 2 <= task) ++p;
            int q = task - p * (p + 1) / 2;
            // Loads of 8 grid points are issued ahead of their (sequential,
            // grid-ordered) accumulation, which keeps the oracle's order.
            double s = 0.0;
            int i = 0;
            for (; i + 8 <= L; i += 8) {
                double wv[8], ap[8], aq[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    wv[u] = w[i + u];
                    ap[u] = A[(size_t)(i + u) * K + p];
                    aq[u] = A[(size_t)(i + u) * K + q];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) s += wv[u] * ap[u] * aq[u];
            }
            for (; i < L; ++i) {
                const double* a = A + (size_t)i * K;
                s += w[i] * a[p] * a[q];
            }
            if (p == q) s += lambda;
            sh.G[p * K + q] = s;
        } else {
            int p = task - npair;
            double sr = 0.0, si = 0.0;
            int i = 0;
            for (; i + 8 <= L; i += 8) {
                double wv[8], ap[8], dr[8], di[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    wv[u] = w[i + u];
                    ap[u] = A[(size_t)(i + u) * K + p];
                    dr[u] = Dr[i + u];
                    di[u] = Di[i + u];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const double wa = wv[u] * ap[u];
                    sr += wa * dr[u];
                    si += wa * di[u];
                }
            }
            for (; i < L; ++i) {
                double wa = w[i] * A[(size_t)i * K + p];
                sr += wa * Dr[i];
                si += wa * Di[i];
            }
            sh.br[p] = sr;
            sh.bi[p] = si;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double* G = sh.G;
        for (int p = 0; p < K; ++p) {
            for (int q = 0; q <= p; ++q) {
                double s = G[p * K + q];
                for (int m = 0; m < q; ++m) s -= G[p * K + m] * G[q * K + m];
                if (p == q) {
                    if (!(s > 0.0)) { sh.fail = 1; s = 1.0; }
                    G[p * K + p] = sqrt(s);
                } else {
                    G[p * K + q] = s / G[q * K + q];
                }
            }
        }
        for (int p = 0; p < K; ++p) {
            double sr = sh.br[p], si = sh.bi[p];
            for (int m = 0; m < p; ++m) { sr -= G[p * K + m] * sh.br[m]; si -= G[p * K + m] * sh.bi[m]; }
            sh.br[p] = sr / G[p * K + p];
            sh.bi[p] = si / G[p * K + p];
        }
        for (int p = K - 1; p >= 0; --p) {
            double sr = sh.br[p], si = sh.bi[p];
            for (int m = p + 1; m < K; ++m) { sr -= G[m * K + p] * sh.br[m]; si -= G[m * K + p] * sh.bi[m]; }
            sh.br[p] = sr / G[p * K + p];
            sh.bi[p] = si / G[p * K + p];
        }
        for (int p = 0; p < K; ++p) { sh.hr[p] = sh.br[p]; sh.hi[p] = sh.bi[p]; }
    }
    __syncthreads();
}

__device__ double block_max(double v, DesignShared& sh)
{
    sh.red[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh.red[threadIdx.x] = fmax(sh.red[threadIdx.x], sh.red[threadIdx.x + s]);
        __syncthreads();
    }
    double r = sh.red[0];
    __syncthreads();
    return r;
}

struct DesignParams {
    int nk, K, L, Lc, nreweight, M;
    double kmin, dk, dx, zeta, edge_sin;
    double w_pass, w_trans, w_evan, lambda, beta, tau, margin;
};

DesignParams design_params(const mig_table_desc* d)
{
    DesignParams P;
    P.nk = d->nk;
    P.K = 0;
    P.M = (d->ntaps - 1) / 2;
    P.L = d->ngrid;
    P.Lc = d->ncheck;
    P.nreweight = d->nreweight;
    P.kmin = d->kmin;
    P.dk = (d->kmax - d->kmin) / (double)(d->nk - 1);
    P.dx = d->dx;
    P.zeta = d->dz / d->dx;
    P.edge_sin = sin(d->theta_max_deg * kPi / 180.0);
    P.w_pass = d->w_pass;
    P.w_trans = d->w_trans;
    P.w_evan = d->w_evan;
    P.lambda = d->lambda;
    P.beta = d->beta;
    P.tau = d->tau;
    P.margin = d->margin;
    return P;
}

__global__ void __launch_bounds__(kDesignThreads)
k_design(DesignParams P, const double* __restrict__ A, const double* __restrict__ C,
         mig_c128* tab64, mig_c64* tab32, double* maxgain, double* passerr,
         int* status)
{
#pragma clang fp contract(off)
    extern __shared__ double dyn[];
    __shared__ DesignShared sh;
    const int j = blockIdx.x, K = P.K, L = P.L, Lc = P.Lc;
    double* w = dyn;
    double* Dr = dyn + L;
    double* Di = dyn + 2 * L;

    const double kappa = (P.kmin + (double)j * P.dk) * P.dx;
    const double edge = kappa * P.edge_sin;
    if (threadIdx.x == 0) sh.fail = 0;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        double th = ((double)i + 0.5) * kPi / (double)L;
        if (th <= kappa) {
            double ph = P.zeta * sqrt(kappa * kappa - th * th);
            double sn, cs;
            sincos(ph, &sn, &cs);
            Dr[i] = cs;
            Di[i] = sn;
        } else {
            Dr[i] = exp(-P.zeta * sqrt(th * th - kappa * kappa));
            Di[i] = 0.0;
        }
        w[i] = th <= edge ? P.w_pass : (th <= kappa ? P.w_trans : P.w_evan);
    }
    __syncthreads();

    wls_solve(A, w, Dr, Di, L, K, P.lambda, sh);
    for (int it = 0; it < P.nreweight; ++it) {
        for (int i = threadIdx.x; i < L; i += blockDim.x) {
            double Hr = 0.0, Hi = 0.0;
            const double* a = A + (size_t)i * K;
            for (int n = 0; n < K; ++n) { Hr += a[n] * sh.hr[n]; Hi += a[n] * sh.hi[n]; }
            double excess = hypot(Hr, Hi) - 1.0;
            if (excess > 0.0) w[i] = w[i] * (1.0 + P.beta * excess / P.tau);
        }
        __syncthreads();
        wls_solve(A, w, Dr, Di, L, K, P.lambda, sh);
    }

    // Stability scale: |H|max <= max_grid |H| / cos(M pi / (2 Lc)).
    double g = 0.0;
    for (int c = threadIdx.x; c < Lc; c += blockDim.x) {
        const double* cc = C + (size_t)c * K;
        double Hr = sh.hr[0], Hi = sh.hi[0];
        for (int n = 1; n < K; ++n) { Hr += cc[n] * sh.hr[n]; Hi += cc[n] * sh.hi[n]; }
        g = fmax(g, hypot(Hr, Hi));
    }
    g = block_max(g, sh);
    double s = 1.0;
    double lim = (1.0 - P.margin) * cos((double)(K - 1) * kPi / (2.0 * (double)Lc));
    if (g > lim) s = lim / g;

    double perr = 0.0;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        double th = ((double)i + 0.5) * kPi / (double)L;
        if (!(th <= edge)) continue;
        const double* a = A + (size_t)i * K;
        double Hr = 0.0, Hi = 0.0;
        for (int n = 0; n < K; ++n) { Hr += a[n] * (s * sh.hr[n]); Hi += a[n] * (s * sh.hi[n]); }
        perr = fmax(perr, hypot(Hr - Dr[i], Hi - Di[i]));
    }
    perr = block_max(perr, sh);

    for (int n = threadIdx.x; n < K; n += blockDim.x) {
        double hr = s * sh.hr[n], hi = s * sh.hi[n];
        tab64[(size_t)j * K + n] = mig_c128{hr, hi};
        if (tab32) tab32[(size_t)j * K + n] = mig_c64{(float)hr, (float)hi};
    }
    if (threadIdx.x == 0) {
        double mg = s * g;
        if (maxgain) maxgain[j] = mg;
        if (passerr) passerr[j] = perr;
        status[j] = sh.fail ? 2 : (mg <= 1.0 ? 0 : 1);
    }
}

// ---- 2-D circularly symmetric extrapolators (3-D extension, Sec. II) ----
//
// Unique coefficient u = a (a + 1) / 2 + b, a >= b >= 0, stands for the taps
// (n1, n2) with max(|n1|,|n2|) = a and min = b.  Its basis function on
// (theta_x, theta_y) is the sum of cos(n1 tx) cos(n2 ty) over that orbit:
//   1;  2 (cos a tx + cos a ty);  4 cos a tx cos a ty;
//   4 (cos a tx cos b ty + cos b tx cos a ty)          (a = 0; b = 0; a = b; a > b).
__device__ __forceinline__ double orbit_basis(int a, int b, const double* cx, const double* cy)
{
#pragma clang fp contract(off)
    if (a == 0) return 1.0;
    if (b == 0) return 2.0 * (cx[a] + cy[a]);
    if (a == b) return 4.0 * cx[a] * cy[a];
    return 4.0 * (cx[a] * cy[b] + cx[b] * cy[a]);
}

// A[(i L + q)][u] on the L x L design midpoint grid; CS[c][n] = cos(n theta_c)
// on the Lc check grid (the check evaluates the basis from it).
__global__ void k_design2d_basis(int L, int Lc, int M, double* A, double* CS)
{
#pragma clang fp contract(off)
    const int NU = (M + 1) * (M + 2) / 2;
    const size_t nA = (size_t)L * L, total = nA + (size_t)Lc;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        if (e < nA) {
            const int i = (int)(e / L), q = (int)(e % L);
            double cx[kMaxK], cy[kMaxK];
            const double tx = ((double)i + 0.5) * kPi / (double)L;
            const double ty = ((double)q + 0.5) * kPi / (double)L;
            for (int n = 0; n <= M; ++n) { cx[n] = cos((double)n * tx); cy[n] = cos((double)n * ty); }
            for (int a = 0, u = 0; a <= M; ++a)
                for (int b = 0; b <= a; ++b, ++u) A[e * NU + u] = orbit_basis(a, b, cx, cy);
        } else {
            const int c = (int)(e - nA);
            const double th = ((double)c + 0.5) * kPi / (double)Lc;
            for (int n = 0; n <= M; ++n) CS[(size_t)c * (M + 1) + n] = cos((double)n * th);
        }
    }
}

__global__ void __launch_bounds__(kDesignThreads)
k_design2d(DesignParams P, const double* __restrict__ A, const double* __restrict__ CS,
           mig_c128* tab64, mig_c64* tab32, double* maxgain, double* passerr, int* status)
{
#pragma clang fp contract(off)
    extern __shared__ double dyn[];
    __shared__ DesignShared sh;
    const int j = blockIdx.x, NU = P.K, L = P.L, Lc = P.Lc, LL = L * L;
    const int M = P.M;
    double* w = dyn;
    double* Dr = dyn + LL;
    double* Di = dyn + 2 * LL;

    const double kappa = (P.kmin + (double)j * P.dk) * P.dx;
    const double k2 = kappa * kappa;
    const double edge = kappa * P.edge_sin;
    if (threadIdx.x == 0) sh.fail = 0;
    for (int e = threadIdx.x; e < LL; e += blockDim.x) {
        const double tx = ((double)(e / L) + 0.5) * kPi / (double)L;
        const double ty = ((double)(e % L) + 0.5) * kPi / (double)L;
        const double r2 = tx * tx + ty * ty;
        const double r = sqrt(r2);
        if (r2 <= k2) {
            double sn, cs;
            sincos(P.zeta * sqrt(k2 - r2), &sn, &cs);
            Dr[e] = cs;
            Di[e] = sn;
        } else {
            Dr[e] = exp(-P.zeta * sqrt(r2 - k2));
            Di[e] = 0.0;
        }
        w[e] = r <= edge ? P.w_pass : (r <= kappa ? P.w_trans : P.w_evan);
    }
    __syncthreads();

    wls_solve(A, w, Dr, Di, LL, NU, P.lambda, sh);
    for (int it = 0; it < P.nreweight; ++it) {
        for (int e = threadIdx.x; e < LL; e += blockDim.x) {
            double Hr = 0.0, Hi = 0.0;
            const double* a = A + (size_t)e * NU;
            for (int u = 0; u < NU; ++u) { Hr += a[u] * sh.hr[u]; Hi += a[u] * sh.hi[u]; }
            const double excess = hypot(Hr, Hi) - 1.0;
            if (excess > 0.0) w[e] = w[e] * (1.0 + P.beta * excess / P.tau);
        }
        __syncthreads();
        wls_solve(A, w, Dr, Di, LL, NU, P.lambda, sh);
    }

    // Stability scale: the per-axis Bernstein bound applied twice,
    // |H|max <= max_grid |H| / cos(M pi / (2 Lc))^2.
    double g = 0.0;
    for (int e = threadIdx.x; e < Lc * Lc; e += blockDim.x) {
        const double* cx = CS + (size_t)(e / Lc) * (M + 1);
        const double* cy = CS + (size_t)(e % Lc) * (M + 1);
        double Hr = 0.0, Hi = 0.0;
        for (int a = 0, u = 0; a <= M; ++a)
            for (int b = 0; b <= a; ++b, ++u) {
                const double f = orbit_basis(a, b, cx, cy);
                Hr += f * sh.hr[u];
                Hi += f * sh.hi[u];
            }
        g = fmax(g, hypot(Hr, Hi));
    }
    g = block_max(g, sh);
    const double c = cos((double)M * kPi / (2.0 * (double)Lc));
    const double lim = (1.0 - P.margin) * c * c;
    const double s = g > lim ? lim / g : 1.0;

    double perr = 0.0;
    for (int e = threadIdx.x; e < LL; e += blockDim.x) {
        const double tx = ((double)(e / L) + 0.5) * kPi / (double)L;
        const double ty = ((double)(e % L) + 0.5) * kPi / (double)L;
        if (!(sqrt(tx * tx + ty * ty) <= edge)) continue;
        const double* a = A + (size_t)e * NU;
        double Hr = 0.0, Hi = 0.0;
        for (int u = 0; u < NU; ++u) { Hr += a[u] * (s * sh.hr[u]); Hi += a[u] * (s * sh.hi[u]); }
        perr = fmax(perr, hypot(Hr - Dr[e], Hi - Di[e]));
    }
    perr = block_max(perr, sh);

    for (int u = threadIdx.x; u < NU; u += blockDim.x) {
        const double hr = s * sh.hr[u], hi = s * sh.hi[u];
        tab64[(size_t)j * NU + u] = mig_c128{hr, hi};
        if (tab32) tab32[(size_t)j * NU + u] = mig_c64{(float)hr, (float)hi};
    }
    if (threadIdx.x == 0) {
        const double mg = s * g;
        if (maxgain) maxgain[j] = mg;
        if (passerr) passerr[j] = perr;
        status[j] = sh.fail ? 2 : (mg <= 1.0 ? 0 : 1);
    }
}

}  // namespace

int launch_design2d_basis(const mig_table_desc* d, double* A, double* CS, hipStream_t s)
{
    const int M = (d->ntaps - 1) / 2;
    const size_t total = (size_t)d->ngrid * d->ngrid + d->ncheck;
    size_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_design2d_basis, dim3((unsigned)blocks), dim3(256), 0, s, d->ngrid,
                       d->ncheck, M, A, CS);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

int launch_design2d(const mig_table_desc* d, const double* A, const double* CS,
                    mig_c128* tab64, mig_c64* tab32, double* maxgain, double* passerr,
                    int* status, hipStream_t s)
{
    DesignParams P = design_params(d);
    P.M = (d->ntaps - 1) / 2;
    P.K = (P.M + 1) * (P.M + 2) / 2;
    const size_t lds = (size_t)3 * d->ngrid * d->ngrid * sizeof(double);
    if (lds > 65536 &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_design2d),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return MIG_E_DEVICE;
    hipLaunchKernelGGL(k_design2d, dim3(d->nk), dim3(kDesignThreads), lds, s, P, A, CS, tab64,
                       tab32, maxgain, passerr, status);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

int launch_design_basis(const mig_table_desc* d, double* A, double* C, hipStream_t s)
{
    const int K = (d->ntaps - 1) / 2 + 1;
    int total = (d->ngrid + d->ncheck) * K;
    int blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_design_basis, dim3(blocks), dim3(256), 0, s, d->ngrid,
                       d->ncheck, K, A, C);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

int launch_design(const mig_table_desc* d, const double* A, const double* C,
                  mig_c128* tab64, mig_c64* tab32, double* maxgain,
                  double* passerr, int* status, hipStream_t s)
{
    DesignParams P = design_params(d);
    P.K = (d->ntaps - 1) / 2 + 1;
    size_t lds = (size_t)3 * d->ngrid * sizeof(double);
    hipLaunchKernelGGL(k_design, dim3(d->nk), dim3(kDesignThreads), lds, s, P, A, C,
                       tab64, tab32, maxgain, passerr, status);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

}  // namespace mig
