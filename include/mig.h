/*
 * mig.h -- C ABI of libmig.so: explicit f-x poststack depth migration on
 * AMD Instinct MI355X (gfx950), hand-written HIP kernels.
 *
 * The method (Shawahna, Salam & Al-Mouhamed, arXiv 1912.05529):
 *   - the zero-offset section is transformed along t to frequency (Algorithm 1,
 *     first step; done by the caller);
 *   - for every depth step z_k -> z_{k+1} = z_k + dz and every frequency
 *     omega_r, each lateral point x_i of the next plane is the spatial
 *     convolution of Eq. (1),
 *         P_{k+1}[x_i][r] = sum_{n=-M..M} h[n] P_k[x_{i-n}][r],  N = 2M+1,
 *     with a predesigned FIR extrapolator h chosen per point by the wavenumber
 *     omega_r / v(x_i, z_k) (the table look-up inside the loops of Algorithm 1;
 *     Sec. III: the cutoff varies from point to point);
 *   - the image row of depth z_k is the sum of the plane over frequencies
 *     (the imaging step of Algorithm 1; the second kernel of Sec. III), taken
 *     here as Re sum_r P_k[x][r] (zero-time imaging).
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer owned by the caller (e.g. torch
 *     tensor storage).  Descriptors are host memory, read during the call only.
 *     The library keeps no state between calls and allocates no memory: scratch
 *     comes from the caller's workspace `ws` (size from the *_workspace_size
 *     queries).  Calls are reentrant.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     work is enqueued on it; results are valid once the stream has completed.
 *     Only mig_design_table synchronizes (it reads back a stability flag).
 *   - Complex numbers are interleaved (re, im): mig_c64 / mig_c128 have the
 *     memory layout of torch.complex64 / torch.complex128.
 *   - Wavefield planes are [nx][nw] (frequency fastest), as produced by a
 *     transform along t of a [nx][nt] section.  Velocities are float32 [rows][nx]
 *     PROPAGATION velocities in m/s (for exploding-reflector zero-offset data
 *     pass half the medium velocity).  Frequencies omega are float64 [nw] in
 *     rad/s.  Images and rows are float64 [rows][nx].
 *   - Host-side validation (NULL pointers, non-positive sizes, even N, bad
 *     table range, aliasing, short workspace) returns a negative code before
 *     anything is launched.  A failed launch returns MIG_E_DEVICE.  No C++
 *     exception crosses this interface.
 *   - Velocities are not checked on the device: a velocity that is not > 0
 *     (zero, negative, NaN) selects table entry 0.
 */
#ifndef MIG_H
#define MIG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MIG_API __attribute__((visibility("default")))

typedef struct { float re, im; } mig_c64;
typedef struct { double re, im; } mig_c128;

enum {
    MIG_OK = 0,
    MIG_E_ARG = -1,        /* invalid argument (host-side check)            */
    MIG_E_UNSTABLE = -2,   /* designed table failed the |H| <= 1 check      */
    MIG_E_DEVICE = -3,     /* HIP launch or runtime error                   */
    MIG_E_WORKSPACE = -4   /* workspace missing or smaller than required    */
};

/* Largest supported sizes. */
#define MIG_MAX_NTAPS 63     /* N odd, 1..63 (M = (N-1)/2 <= 31)              */
#define MIG_MAX_NX 8192      /* lateral points per section                    */
#define MIG_MAX_NW 1048576   /* frequencies per call                          */
#define MIG_MAX_NT 4194304   /* time samples per trace (mig_transform_t)     */

/*
 * Extrapolator-table descriptor.  Entry j (0 <= j < nk) is designed for the
 * wavenumber k_j = kmin + j (kmax - kmin)/(nk - 1) (rad/m, k = omega/v).
 * The paper designs the filters in advance as an optimization (Sec. II,
 * Sec. III) but does not give the method; this library fits, per entry, the
 * one-way phase shift over dz,
 *     D(theta) = exp(+i zeta sqrt(kappa^2 - theta^2))    (theta <= kappa)
 *     D(theta) = exp(-zeta sqrt(theta^2 - kappa^2))      (theta >  kappa)
 * with kappa = k_j dx, zeta = dz/dx, theta = kx dx on a midpoint grid of
 * `ngrid` points in (0, pi), by weighted least squares over even taps
 * (H(theta) = h0 + 2 sum h_n cos(n theta)).  Initial weights: w_pass for
 * theta <= kappa sin(theta_max), w_trans up to kappa, w_evan beyond.  Then
 * `nreweight` passes multiply the weight of every point with |H| > 1 by
 * (1 + beta (|H| - 1)/tau) and refit.  Finally the taps are scaled so that
 * max |H| over an `ncheck`-point midpoint grid, divided by
 * cos(M pi / (2 ncheck)), is at most 1 - margin; by Bernstein's inequality this
 * bounds |H(theta)| for every theta.  `lambda` is added to the diagonal of the
 * normal matrix.
 */
typedef struct {
    int32_t ntaps;          /* N, odd, 1..MIG_MAX_NTAPS                       */
    int32_t nk;             /* table entries, >= 2                            */
    double kmin, kmax;      /* table axis, rad/m, 0 < kmin < kmax             */
    double dx, dz;          /* m, dx > 0, dz >= 0                             */
    double theta_max_deg;   /* passband half-angle (default 60)              */
    double w_pass, w_trans, w_evan; /* > 0 (defaults 1, 0.01, 0.01)            */
    int32_t ngrid;          /* design grid, 8..2048 (default 1024)            */
    int32_t ncheck;         /* check grid, >= 8 (default 8192)                */
    int32_t nreweight;      /* >= 0 (default 30)                              */
    int32_t reserved;       /* must be 0                                      */
    double lambda;          /* >= 0 (default 1e-9 * ngrid)                    */
    double beta, tau;       /* reweighting gain and scale (defaults 1, 5e-4)  */
    double margin;          /* stability margin in [0, 1) (default 1e-5)     */
} mig_table_desc;

/* Human-readable text for a status code (static storage). */
MIG_API const char* mig_strerror(int code);

/* Library version string (static storage). */
MIG_API const char* mig_version(void);

/* Bytes of workspace mig_design_table needs for this descriptor (0 on a bad
 * descriptor). */
MIG_API size_t mig_design_workspace_size(const mig_table_desc* d);

/*
 * A0 -- design the extrapolator table on the GPU in FP64 (the "predesigned
 * 1-D FIR filters" of Algorithm 1; Sec. II/III: design as an optimization,
 * accurate designs needed for stability; method as described above).
 *   tab64   [nk][M+1] complex128 half-taps h_0..h_M (h_{-n} = h_n)   (out)
 *   tab32   [nk][M+1] complex64, tab64 rounded to nearest, or NULL   (out)
 *   maxgain [nk] max |H| over the check grid after scaling, or NULL  (out)
 *   passerr [nk] max |H - D| over passband design-grid points, or NULL (out)
 *   ws      >= mig_design_workspace_size(d) bytes of device memory
 * Synchronizes `stream` and returns MIG_E_UNSTABLE if any entry's scaled
 * maxgain is not <= 1 (e.g. NaN), MIG_E_ARG if the normal matrix of an entry
 * is not positive definite.
 */
MIG_API int mig_design_table(const mig_table_desc* d, mig_c128* tab64,
                             mig_c64* tab32, double* maxgain, double* passerr,
                             void* ws, size_t ws_bytes, void* stream);

/*
 * A1 -- table look-up (the look-up step of Algorithm 1; Sec. III: the filter is
 * chosen by the wavenumber omega/v).  idx[row][x][r] = nearest entry j to
 * omega_r / vel[row][x], computed as the IEEE-double sequence
 *     a = omega/dk; b = kmin/dk; s = 1/(double)v; t = a*s; t = t - b;
 *     u = t + 0.5;  j = 0 if !(u >= 1), nk-1 if u >= nk, else floor(u),
 * (dk = (kmax-kmin)/(nk-1), every operation rounded separately; j = 0 when
 * v is not > 0).  The extrapolation kernels use exactly this rule.
 *   vel [nrows][nx] float32, omega [nw] float64, idx [nrows][nx][nw] int32.
 */
MIG_API int mig_table_index(const float* vel, const double* omega,
                            const mig_table_desc* d, int32_t nx, int32_t nw,
                            int32_t nrows, int32_t* idx, void* stream);

/* Bytes of workspace mig_extrapolate (with or without rows) and mig_migrate
 * need to run `nsteps` depth steps in one launch (for mig_migrate, nsteps =
 * nz - 1: the number of depth steps, not of image rows).  A smaller workspace
 * (at least mig_workspace_min_size) makes the library split the depth loop
 * into chunks of as many steps as fit; results are bit-identical. */
MIG_API size_t mig_workspace_size(int32_t nx, int32_t nsteps, int32_t nw,
                                  const mig_table_desc* d);
MIG_API size_t mig_workspace_min_size(int32_t nx, int32_t nw,
                                      const mig_table_desc* d);

/*
 * Status of the most recent call of mig_extrapolate, mig_migrate or
 * mig_migrate_batched that used the workspace `ws`.  The image rows are
 * summed over frequencies inside the depth-stepping launch by reducer
 * workgroups that wait for the frequency workgroups' published blocks; each
 * wait is bounded (20 s without any publish in the launch, or the limit of
 * mig_tuning), and a reducer that runs into the bound gives up for the
 * whole launch: the rows it and every later reducer task would have formed
 * are written as NaN and a status word at the head of the workspace is set.
 * Since calls are asynchronous, that status is read here: the call
 * synchronizes `stream` and returns MIG_OK, or MIG_E_DEVICE if a reduction
 * was abandoned (or the read failed).  MIG_E_ARG for ws == NULL.
 */
MIG_API int mig_workspace_status(const void* ws, void* stream);

/*
 * A2 + A3 + A4 -- advance a plane by `nsteps` depth steps with Eq. (1) in FP32
 * complex arithmetic, filters from `tab32` per output point (step s uses
 * vel[s][.]; zero wavefield outside [0, nx)), optionally forming the image row
 * of each new plane with FP64 accumulation over frequencies.
 *   wf_in  [nx][nw] complex64 plane at z_k0                          (in)
 *   wf_out [nx][nw] complex64 plane at z_k0+nsteps; must not overlap wf_in;
 *          may be NULL when rows is non-NULL                           (out)
 *   vel    [nsteps][nx] float32 propagation velocity                   (in)
 *   omega  [nw] float64                                               (in)
 *   tab32  [nk][M+1] complex64 half-taps (from mig_design_table)       (in)
 *   rows   [nsteps][nx] float64: rows[s][x] = sum_r Re P_{k0+s+1}[x][r], or
 *          NULL                                                        (out)
 *   ws     device workspace, >= mig_workspace_min_size bytes
 *          (mig_workspace_size(nx, nsteps, nw, d) for a single pass); it
 *          holds the slowness rows 1/v of the look-up, the partial image rows
 *          and, when the depth loop is split into chunks, the intermediate
 *          plane.  Must not overlap wf_in or wf_out.
 * nsteps = 0 copies wf_in to wf_out (ws unused).
 */
MIG_API int mig_extrapolate(const mig_c64* wf_in, mig_c64* wf_out,
                            const float* vel, const double* omega,
                            const mig_c64* tab32, const mig_table_desc* d,
                            int32_t nx, int32_t nw, int32_t nsteps,
                            double* rows, void* ws, size_t ws_bytes,
                            void* stream);

/*
 * A3 -- image row of one plane (Algorithm 1 "depth row by summing over
 * frequencies"): row[x] = sum_r Re wf[x][r], FP64 accumulation in a fixed
 * order (one wavefront per x, lane-strided partial sums combined by a
 * butterfly of cross-lane shuffles), so results are run-to-run identical.
 *   wf [nx][nw] complex64 (in), row [nx] float64 (out).
 */
MIG_API int mig_image(const mig_c64* wf, double* row, int32_t nx, int32_t nw,
                      void* stream);

/*
 * A0..A4 end to end -- Algorithm 1 on an f-x section: image row 0 is the
 * image of `data`; row k (1 <= k < nz) is the image after k depth steps, step
 * k-1 -> k using vel[k-1][.] (vel row nz-1 is not used).
 *   data  [nx][nw] complex64 surface plane (in), vel [nz][nx] float32 (in),
 *   omega [nw] float64 (in), tab32 [nk][M+1] complex64 (in),
 *   image [nz][nx] float64 (out), ws >= mig_workspace_min_size bytes
 *   (mig_workspace_size(nx, nz-1, nw, d) for a single pass).
 */
MIG_API int mig_migrate(const mig_c64* data, const float* vel,
                        const double* omega, const mig_c64* tab32,
                        const mig_table_desc* d, int32_t nx, int32_t nz,
                        int32_t nw, double* image, void* ws, size_t ws_bytes,
                        void* stream);

/*
 * Allocation-free form of mig_migrate, for callers that cannot allocate device
 * memory or hand over a workspace: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments and results
 * as mig_migrate without ws/ws_bytes: the scratch (status word, intermediate
 * plane, block counters, slowness rows, partial image rows) lives in a static
 * device array of MIG_STATIC_SCRATCH_BYTES per GPU, created with the library's
 * code object and held until the process ends.  The depth loop is split into
 * as many chunks as that array needs (images bit-identical to mig_migrate).
 * Calls nothing that allocates.
 *   Returns MIG_E_WORKSPACE when one depth step does not fit
 *   (mig_workspace_min_size(nx, nw, d) > MIG_STATIC_SCRATCH_BYTES, e.g.
 *   nx * nw beyond about 8e6 points), MIG_E_ARG as mig_migrate.
 *   Every call on a GPU uses that GPU's one array, which keeps the last call's
 *   contents (each call clears what must start at zero): calls that overlap
 *   on one GPU (other streams, other host threads) race and must be
 *   serialized by the caller.  The reduction status of mig_workspace_status
 *   is not reachable here: an abandoned reduction shows as NaN image rows.
 */
#define MIG_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
MIG_API int mig_migrate_noalloc(const mig_c64* data, const float* vel,
                                const double* omega, const mig_c64* tab32,
                                const mig_table_desc* d, int32_t nx,
                                int32_t nz, int32_t nw, double* image,
                                void* stream);

/*
 * The step before the depth loop (Algorithm 1: transform of the section along
 * t; Sec. III): out[x][r] = sum_n section[x][n] exp(-i omega_r n dt), directly
 * at the given frequencies (they need not be FFT bins), so that t-x sections
 * can be migrated.  A dense contraction section [nx][nt] x DFT matrix, run on
 * the matrix cores in FP32 (the DFT matrix is formed in FP64 and rounded).
 *   section [nx][nt] float32 (in), omega [nw] float64 (in),
 *   out [nx][nw] complex64 (out), ws >= mig_transform_workspace_size bytes.
 * nt <= MIG_MAX_NT (else MIG_E_ARG; the workspace query returns 0).
 */
MIG_API size_t mig_transform_workspace_size(int32_t nt, int32_t nw);
MIG_API int mig_transform_t(const float* section, int32_t nx, int32_t nt,
                            double dt, const double* omega, int32_t nw,
                            mig_c64* out, void* ws, size_t ws_bytes,
                            void* stream);

/*
 * Adjoint of mig_migrate (demigration / exploding-reflector modelling), for
 * least-squares migration and gradients.  With the real inner product
 * <a, b> = Re sum conj(a) b on planes and the ordinary one on images, it is the
 * exact transpose of the linear map data -> image of Algorithm 1 (same
 * filters, same look-up, same zero boundary):
 *     Q_{nz-1}[x][r] = image[nz-1][x],
 *     Q_k[x][r] = image[k][x] + sum_{n=-M..M} conj(h_{j(x+n,k)}[|n|]) Q_{k+1}[x+n][r],
 *     data = Q_0,
 * where j(x, k) is the table entry of (omega_r, vel[k][x]).  FP32 complex
 * arithmetic, one workgroup per frequency walking the depth steps backwards.
 * For nx <= 1024 and N <= 35 the step is the FIR with each point's own
 * conjugated taps plus exact corrections where the velocity changes along x
 * (at most 16 such points per row; otherwise, and for nk > 65536, a kernel
 * that forms every product conj(h_j(y)[m]) q[y] runs instead); results agree
 * to FP32 rounding either way and are run-to-run identical.
 *   image [nz][nx] float64 (in), vel [nz][nx] float32 (in; row nz-1 unused),
 *   omega [nw] float64 (in), tab32 [nk][M+1] complex64 (in),
 *   data  [nx][nw] complex64 (out), ws >= mig_demigrate_workspace_size bytes
 *   (slowness rows, the change points of every row and their table entries
 *   per frequency: about (nz-1)(8 ldp + 64 nw) bytes, ldp = nx rounded up to
 *   256).
 */
MIG_API size_t mig_demigrate_workspace_size(int32_t nx, int32_t nz, int32_t nw,
                                            const mig_table_desc* d);
MIG_API int mig_demigrate(const double* image, const float* vel,
                          const double* omega, const mig_c64* tab32,
                          const mig_table_desc* d, int32_t nx, int32_t nz,
                          int32_t nw, mig_c64* data, void* ws, size_t ws_bytes,
                          void* stream);

/*
 * Batched form: many independent 2-D sections (different nx, nz, nw, all
 * sharing one table) migrated in at most four launches -- one per kernel
 * variant -- instead of one per section.  Every section is Algorithm 1 end to
 * end exactly as mig_migrate computes it (bit-identical results for the same
 * tuning), so this is a scheduling form of the same method: frequency
 * workgroups of all sections are interleaved longest-first, and the image
 * reduction over frequencies of all sections runs in the same launches.
 *   secs   [nsec] host array of section descriptors (read during the call)
 *   tune   knobs chosen by an autotuner, or NULL for the library defaults
 *   ws     >= mig_batch_workspace_size(secs, nsec, d, tune) bytes of device
 *          memory (status word, slowness rows, partial image rows and the
 *          device copy of the launch descriptors; no chunking)
 * The launch descriptors are built on the host and copied into `ws` from a
 * buffer the call owns, so the call blocks until that copy (and the earlier
 * work of `stream`) has completed; the launches themselves are asynchronous.
 * It therefore cannot be captured into a HIP graph.
 */
typedef struct {
    const mig_c64* data;   /* [nx][nw] surface plane                        */
    const float* vel;      /* [nz][nx] propagation velocity                  */
    const double* omega;   /* [nw]                                           */
    double* image;         /* [nz][nx] output; row 0 = image of data         */
    int32_t nx, nz, nw;    /* nx <= MIG_MAX_NX, nz >= 1, nw >= 1             */
    int32_t reserved;      /* must be 0                                      */
} mig_section;

typedef struct {
    int32_t omegas_per_group; /* frequencies per workgroup in the two-output
                                 register-tap kernel (0 = as many as fit in
                                 512 threads); clamped to what fits          */
    int32_t reducers;         /* reducer workgroups per launch, 8..64
                                 (0 = the CUs the frequency workgroups leave
                                 idle, at least 8 and at most 32); never more
                                 than a quarter of the device's CUs          */
    int32_t stall_limit_us;   /* reducer stall limit in microseconds
                                 (0 = 20 s); see mig_workspace_status        */
    int32_t flags;            /* 0, or MIG_TUNE_FORCE_STALL                 */
    int32_t outputs_mid;      /* outputs per thread of the register-tap
                                 kernel for sections of 1025..1536 points:
                                 3 (6-8 waves per frequency) or 4 (5-6
                                 waves); 0 = library choice (3)              */
} mig_tuning;

/* Test hook for the failure path: reducers wait for one publish more than
 * the frequency workgroups make, so every wait runs into the stall limit and
 * the launch is abandoned (every kernel still ends normally). */
#define MIG_TUNE_FORCE_STALL 1

MIG_API size_t mig_batch_workspace_size(const mig_section* secs, int32_t nsec,
                                        const mig_table_desc* d,
                                        const mig_tuning* tune);
MIG_API int mig_migrate_batched(const mig_section* secs, int32_t nsec,
                                const mig_c64* tab32, const mig_table_desc* d,
                                const mig_tuning* tune, void* ws,
                                size_t ws_bytes, void* stream);

/* Diagnostic query: which extrapolation kernel a call with these sizes takes.
 * 1 = register-tap kernel, two outputs per thread (N <= 35, nx <= 1024);
 * 3 = register-tap kernel, three outputs per thread (N <= 35, nx <= 1536);
 * 2 = register-tap kernel, four outputs per thread (N <= 35, nx <= 2048);
 * 0 = general kernel (taps read from the table every step); -1 = bad
 * arguments.  All kernels compute the same sums; results agree to FP32
 * rounding. */
MIG_API int mig_kernel_kind(int32_t nx, int32_t ntaps);

/*
 * 3-D extension (Sec. II: the explicit f-x method carries over to 3-D, with
 * 2-D extrapolators in Eq. (1)).
 *
 * Circularly symmetric (2M+1) x (2M+1) filters: h[n1][n2] = c(a, b) with
 * a = max(|n1|,|n2|), b = min(|n1|,|n2|).  A 2-D table holds the unique
 * coefficients of each entry, u = a (a + 1) / 2 + b for 0 <= b <= a <= M,
 * NU = (M+1)(M+2)/2 complex values per entry: tab [nk][NU].
 *
 * Design (same descriptor; ngrid and ncheck count points per axis of the
 * midpoint grids on (0, pi)^2): per entry, the weighted least-squares fit of
 * sum_u c_u B_u(tx, ty) to the phase shift exp(+i zeta sqrt(kappa^2 - r^2))
 * (r^2 = tx^2 + ty^2; exp(-zeta sqrt(r^2 - kappa^2)) past kappa), with the
 * 1-D band weights and reweighting applied at radius r, where B_u is the sum
 * of cos(n1 tx) cos(n2 ty) over the taps of coefficient u.  The stability
 * scale applies the 1-D Bernstein bound along each axis:
 *   |H|max <= max over the Lc x Lc check grid / cos(M pi / (2 Lc))^2,
 * and scales the entry to (1 - margin) cos(M pi / (2 Lc))^2 when that is
 * exceeded.  Returns as mig_design_table (synchronizes the stream).
 */
#define MIG_MAX_NTAPS_2D 11     /* 2M+1 per axis, M <= 5 (NU <= 21)           */
#define MIG_MAX_NGRID_2D 64     /* design grid points per axis                */
#define MIG_MAX_NCHECK_2D 4096  /* check grid points per axis                 */
#define MIG_MAX_NXY 65536       /* lateral points per axis of a volume        */
#define MIG_MAX_PLANE_3D 134217728 /* nx * ny per volume (2^27: one frequency
                                      plane of complex64 within 1 GiB)        */

MIG_API size_t mig_design2d_workspace_size(const mig_table_desc* d);
MIG_API int mig_design_table_2d(const mig_table_desc* d, mig_c128* tab64,
                                mig_c64* tab32, double* maxgain,
                                double* passerr, void* ws, size_t ws_bytes,
                                void* stream);

/*
 * 3-D migration: Algorithm 1 on a volume.
 *   data  [nw][nx][ny] complex surface wavefield (one contiguous plane per
 *         frequency)
 *   vel   [nz][nx][ny] propagation velocity; step k-1 -> k uses vel[k-1]
 *         (last slice unused); v <= 0 or NaN selects entry 0
 *   image [nz][nx][ny] FP64 output; slice 0 = sum over omega of Re data,
 *         slice k = sum over omega of Re P_k
 *   plane_out  optional [nw][nx][ny] copy of the last wavefield P_{nz-1}
 *         (NULL = not wanted; for nz = 1 it is the data)
 * One step: P_k(x, y) = sum over |n1|,|n2| <= M of h_j[n1][n2]
 *   P_{k-1}(x - n1, y - n2), with P zero outside the volume and j the
 *   nearest entry for omega / vel[k-1][x][y] (the mig_table_index rule).
 * The image sums Re over frequencies in FP64: within groups of
 * omegas_per_group consecutive frequencies in order, then over groups in
 * order (0 = library choice, see mig_omegas_per_group_3d); results are
 * deterministic for a given grouping.  ntaps <= MIG_MAX_NTAPS_2D.
 * ws >= mig_migrate3d_workspace_size(...) bytes of device memory, disjoint
 * from data, image and plane_out.  Asynchronous on `stream`.
 */
MIG_API int mig_omegas_per_group_3d(int32_t nx, int32_t ny, int32_t nw,
                                    int32_t want);
MIG_API size_t mig_migrate3d_workspace_size(int32_t nx, int32_t ny, int32_t nw,
                                            int32_t nz,
                                            int32_t omegas_per_group);
MIG_API int mig_migrate3d(const mig_c64* data, const float* vel,
                          const double* omega, const mig_c64* tab32,
                          const mig_table_desc* d, int32_t nx, int32_t ny,
                          int32_t nw, int32_t nz, int32_t omegas_per_group,
                          double* image, mig_c64* plane_out, void* ws,
                          size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MIG_H */
