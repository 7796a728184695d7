/*
 * FP64 CPU oracle for explicit f-x poststack depth migration.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path; it
 * is not part of the product.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the HIP library, and it includes nothing from it.
 *
 * What it computes (paper: Shawahna, Salam & Al-Mouhamed, arXiv 1912.05529):
 *   - orc_design_table : the predesigned 1-D complex FIR extrapolator bank
 *                        (Sec. II: the design is an optimization between two
 *                        trade-offs; Sec. III: designed in advance).  The paper gives no
 *                        design method; this is a weighted least-squares fit to
 *                        the phase-shift operator with multiplicative
 *                        reweighting and a rigorous stability scale.
 *   - orc_table_index  : the table look-up of Algorithm 1 (filter chosen by the
 *                        wavenumber omega/v, Sec. III).  Nearest entry.
 *   - orc_extrapolate  : Eq. (1), literally (unfolded sum over n), one depth
 *                        step after another (Algorithm 1 loops).
 *   - orc_image        : the depth row of Algorithm 1 (the second kernel of
 *                        Sec. III): real part of the sum over omega.
 *   - orc_migrate      : Algorithm 1 end to end on an f-x section.
 *   - orc_demigrate    : the exact adjoint of orc_migrate (real inner product).
 *
 * Layouts: complex numbers are interleaved (re, im) doubles.  A wavefield
 * plane is [nx][nw] (omega fastest).  Velocities are float32 [nrows][nx] and
 * are the propagation velocity.  Images are [nz][nx] doubles.
 *
 * Return codes: 0 on success, negative on bad arguments or numerical failure.
 */
#ifndef FXMIG_ORACLE_H
#define FXMIG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_NUMERIC (-2)
#define ORC_E_NOMEM (-3)

typedef struct {
    int32_t ntaps;          /* N, odd; M = (N-1)/2 half-length            */
    int32_t nk;             /* table entries, >= 2                          */
    double kmin, kmax;      /* wavenumber range omega/v of the table, rad/m */
    double dx, dz;          /* grid spacings, m                             */
    double theta_max_deg;   /* passband half-angle                          */
    double w_pass, w_trans, w_evan; /* initial LS weights per band          */
    int32_t ngrid;          /* design grid points on (0, pi)                */
    int32_t ncheck;         /* stability check grid points on (0, pi)       */
    int32_t nreweight;      /* reweighting passes                           */
    int32_t pad_;
    double lambda;          /* Tikhonov term added to the normal matrix     */
    double beta, tau;       /* reweighting gain and excess scale            */
    double margin;          /* stability margin: |H| <= 1 - margin          */
} orc_desc;

/* tab: [nk][M+1] complex (interleaved doubles).  maxgain, passerr, scale:
 * [nk] or NULL.  apply_scale = 0 skips the stability scale (used by the
 * textbook special-case check).  Returns ORC_E_NUMERIC if a normal matrix
 * is not positive definite. */
int orc_design_table(const orc_desc* d, int apply_scale, double* tab,
                     double* maxgain, double* passerr, double* scale);

/* idx: [nrows][nx][nw] table indices for velocity rows vel[nrows][nx]. */
int orc_table_index(const orc_desc* d, const double* omega, int32_t nw,
                    const float* vel, int32_t nx, int32_t nrows, int32_t* idx);

/* Advances plane in[nx][nw] by nsteps depth steps; step s uses vel[s][.].
 * out receives the last plane.  rows ([nsteps][nx]) or NULL receives the
 * image row of every new plane. */
int orc_extrapolate(const orc_desc* d, const double* tab, const double* omega,
                    int32_t nw, const float* vel, int32_t nx, int32_t nsteps,
                    const double* in, double* out, double* rows);

/* row[nx] = sum over omega of Re plane[x][omega]. */
int orc_image(const double* plane, int32_t nx, int32_t nw, double* row);

/* image[nz][nx]; row 0 is the image of data, row k the image after k steps
 * (step k-1 -> k uses vel[k-1][.]); vel is [nz][nx] (last row unused). */
int orc_migrate(const orc_desc* d, const double* tab, const double* omega,
                int32_t nw, const float* vel, int32_t nx, int32_t nz,
                const double* data, double* image);

/* Adjoint of orc_migrate for the real inner product Re sum conj(a) b:
 * image[nz][nx] -> data[nx][nw]. */
int orc_demigrate(const orc_desc* d, const double* tab, const double* omega,
                  int32_t nw, const float* vel, int32_t nx, int32_t nz,
                  const double* image, double* data);

/* Transform along t (Algorithm 1, first step; Sec. III): for a section
 * p[nx][nt] sampled at dt, out[x][r] = sum_n p[x][n] exp(-i omega_r n dt),
 * complex [nx][nw] (interleaved doubles), at arbitrary frequencies. */
int orc_transform_t(const float* p, int32_t nx, int32_t nt, double dt,
                    const double* omega, int32_t nw, double* out);

/* ---- 3-D extension (Sec. II: the f-x method extends to 3-D with 2-D
 * filters) --------------------------------------------------------------- */

/* Circularly symmetric (2M+1) x (2M+1) extrapolators: h[n1][n2] = c(a, b) with
 * a = max(|n1|,|n2|), b = min(|n1|,|n2|); coefficient (a, b), a >= b >= 0, is
 * stored at u = a (a + 1) / 2 + b, NU = (M+1)(M+2)/2 per entry.  Same
 * descriptor as the 1-D design; ngrid and ncheck are points per axis of the
 * 2-D midpoint grids on (0, pi)^2.  tab: [nk][NU] complex. */
int orc_design_table_2d(const orc_desc* d, int apply_scale, double* tab,
                        double* maxgain, double* passerr, double* scale);

/* 3-D migration: data [nx][ny][nw] complex, vel [nz][nx][ny] float32,
 * image [nz][nx][ny]; row 0 = image of data; step k -> k+1 applies the 2-D
 * filter of each output point (omega_r, vel[k][x][y]), zero outside the grid.
 * plane_out ([nx][ny][nw] complex) or NULL receives the last wavefield. */
int orc_migrate3d(const orc_desc* d, const double* tab, const double* omega,
                  int32_t nw, const float* vel, int32_t nx, int32_t ny, int32_t nz,
                  const double* data, double* image, double* plane_out);

/* Number of OpenMP threads the oracle will use. */
int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
