// C ABI of libmig.so (declarations and contracts in include/mig.h).
//
// Host code here only validates arguments, lays out the caller's workspace and
// launches kernels; every arithmetic step of the method runs on the GPU.
#include <string.h>

#include "common.hpp"

using namespace mig;

namespace {

constexpr size_t kAlign = 256;

bool desc_valid(const mig_table_desc* d)
{
    if (!d) return false;
    if (d->ntaps < 1 || d->ntaps > MIG_MAX_NTAPS || (d->ntaps % 2) == 0) return false;
    if (d->nk < 2) return false;
    if (!(d->kmin > 0.0) || !(d->kmax > d->kmin)) return false;
    if (!(d->dx > 0.0) || !(d->dz >= 0.0)) return false;
    if (d->reserved != 0) return false;
    return true;
}

bool design_desc_valid(const mig_table_desc* d)
{
    if (!desc_valid(d)) return false;
    if (d->ngrid < 8 || d->ngrid > 2048 || d->ncheck < 8 || d->ncheck > (1 << 20)) return false;
    if (d->nreweight < 0 || d->nreweight > 1000) return false;
    if (!(d->w_pass > 0.0) || !(d->w_trans > 0.0) || !(d->w_evan > 0.0)) return false;
    if (!(d->lambda >= 0.0) || !(d->beta >= 0.0) || !(d->tau > 0.0)) return false;
    if (!(d->margin >= 0.0) || !(d->margin < 1.0)) return false;
    if (!(d->theta_max_deg > 0.0) || !(d->theta_max_deg <= 90.0)) return false;
    return true;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb)
{
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + nb && pb < pa + na;
}

size_t plane_bytes(int nx, int nw) { return align_up((size_t)nx * nw * sizeof(float2), kAlign); }

// Workspace per depth step: one slowness row (+ one partial-row plane when
// image rows are formed).
size_t step_bytes(int nx, int nw, bool rows)
{
    size_t b = (size_t)row_stride(nx) * sizeof(double);
    if (rows) b += (size_t)nw * row_stride(nx) * sizeof(float);
    return b;
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// Depth loop, split into chunks that fit the workspace.  Workspace layout:
// [scratch plane][slowness chunk x ldp doubles][partials chunk x nw x ldp floats].
int run_extrap(const float2* src, float2* dst, const float* vel, const double* omega,
               const float2* tab, const mig_table_desc* d, int nx, int nw, int nsteps,
               double* rows, void* ws, size_t ws_bytes, hipStream_t s)
{
    const size_t pb = plane_bytes(nx, nw);
    const size_t sb = step_bytes(nx, nw, rows != nullptr);
    if (!ws || ws_bytes < pb + sb) return MIG_E_WORKSPACE;
    size_t fit = (ws_bytes - pb) / sb;
    const int chunk = fit >= (size_t)nsteps ? nsteps : (int)fit;
    const int ldp = row_stride(nx);
    // ldp is a multiple of 256, so every region below starts 2 KB-aligned.
    float2* scratch = static_cast<float2*>(ws);
    double* slow = reinterpret_cast<double*>(static_cast<char*>(ws) + pb);
    float* part = reinterpret_cast<float*>(static_cast<char*>(ws) + pb +
                                           (size_t)chunk * ldp * sizeof(double));

    ExtrapArgs a;
    a.omega = omega;
    a.tab = tab;
    a.slow = slow;
    a.part = rows ? part : nullptr;
    a.nx = nx;
    a.nw = nw;
    a.nk = d->nk;
    a.M = (d->ntaps - 1) / 2;
    a.ldp = ldp;
    a.dk = (d->kmax - d->kmin) / (double)(d->nk - 1);
    a.b = d->kmin / a.dk;

    const float2* cur = src;
    for (int c0 = 0; c0 < nsteps; c0 += chunk) {
        int cs = nsteps - c0 < chunk ? nsteps - c0 : chunk;
        bool last = c0 + cs == nsteps;
        int rc = launch_slowness(vel + (size_t)c0 * nx, nx, cs, ldp, slow, s);
        if (rc != MIG_OK) return rc;
        a.win = cur;
        // Intermediate planes go to the scratch plane, in place: each workgroup
        // reads its whole frequency column before writing it back.
        a.wout = last ? dst : scratch;
        a.nsteps = cs;
        rc = launch_extrap(a, s);
        if (rc != MIG_OK) return rc;
        if (rows) {
            rc = launch_rows_reduce(part, ldp, nx, nw, cs, rows + (size_t)c0 * nx, s);
            if (rc != MIG_OK) return rc;
        }
        cur = scratch;
    }
    return MIG_OK;
}

bool sizes_ok(int nx, int nw) { return nx >= 1 && nx <= MIG_MAX_NX && nw >= 1 && nw <= MIG_MAX_NW; }

}  // namespace

extern "C" {

MIG_API const char* mig_strerror(int code)
{
    switch (code) {
    case MIG_OK: return "success";
    case MIG_E_ARG: return "invalid argument";
    case MIG_E_UNSTABLE: return "designed table failed the |H| <= 1 check";
    case MIG_E_DEVICE: return "HIP launch or runtime error";
    case MIG_E_WORKSPACE: return "workspace missing or too small";
    default: return "unknown status";
    }
}

MIG_API const char* mig_version(void) { return "libmig 0.1 (gfx950)"; }

MIG_API size_t mig_design_workspace_size(const mig_table_desc* d)
{
    if (!design_desc_valid(d)) return 0;
    const size_t K = (size_t)(d->ntaps - 1) / 2 + 1;
    return align_up((size_t)d->ngrid * K * sizeof(double), kAlign) +
           align_up((size_t)d->ncheck * K * sizeof(double), kAlign) +
           align_up((size_t)d->nk * sizeof(int), kAlign);
}

MIG_API int mig_design_table(const mig_table_desc* d, mig_c128* tab64, mig_c64* tab32,
                             double* maxgain, double* passerr, void* ws, size_t ws_bytes,
                             void* stream)
{
    if (!design_desc_valid(d) || !tab64) return MIG_E_ARG;
    const size_t need = mig_design_workspace_size(d);
    if (!ws || ws_bytes < need) return MIG_E_WORKSPACE;
    const size_t K = (size_t)(d->ntaps - 1) / 2 + 1;
    if (tab32 && overlap(tab64, d->nk * K * sizeof(mig_c128), tab32, d->nk * K * sizeof(mig_c64)))
        return MIG_E_ARG;
    hipStream_t s = as_stream(stream);
    char* p = static_cast<char*>(ws);
    double* A = reinterpret_cast<double*>(p);
    p += align_up((size_t)d->ngrid * K * sizeof(double), kAlign);
    double* C = reinterpret_cast<double*>(p);
    p += align_up((size_t)d->ncheck * K * sizeof(double), kAlign);
    int* status = reinterpret_cast<int*>(p);

    int rc = launch_design_basis(d, A, C, s);
    if (rc == MIG_OK) rc = launch_design(d, A, C, tab64, tab32, maxgain, passerr, status, s);
    if (rc != MIG_OK) return rc;
    if (hipStreamSynchronize(s) != hipSuccess) return MIG_E_DEVICE;
    int worst = 0;
    const int chunk = 1024;
    int buf[chunk];
    for (int j0 = 0; j0 < d->nk; j0 += chunk) {
        int n = d->nk - j0 < chunk ? d->nk - j0 : chunk;
        if (hipMemcpy(buf, status + j0, n * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
            return MIG_E_DEVICE;
        for (int i = 0; i < n; ++i) worst = buf[i] > worst ? buf[i] : worst;
    }
    if (worst == 2) return MIG_E_ARG;
    if (worst == 1) return MIG_E_UNSTABLE;
    return MIG_OK;
}

MIG_API int mig_table_index(const float* vel, const double* omega, const mig_table_desc* d,
                            int32_t nx, int32_t nw, int32_t nrows, int32_t* idx, void* stream)
{
    if (!desc_valid(d) || !vel || !omega || !idx || !sizes_ok(nx, nw) || nrows < 1)
        return MIG_E_ARG;
    const double dk = (d->kmax - d->kmin) / (double)(d->nk - 1);
    const double b = d->kmin / dk;
    return launch_index(vel, omega, nx, nw, nrows, d->nk, dk, b, idx, as_stream(stream));
}

MIG_API size_t mig_workspace_size(int32_t nx, int32_t nsteps, int32_t nw, const mig_table_desc* d)
{
    if (!desc_valid(d) || !sizes_ok(nx, nw) || nsteps < 0) return 0;
    size_t steps = nsteps > 0 ? (size_t)nsteps : 1;
    return plane_bytes(nx, nw) + steps * step_bytes(nx, nw, true);
}

MIG_API size_t mig_workspace_min_size(int32_t nx, int32_t nw, const mig_table_desc* d)
{
    if (!desc_valid(d) || !sizes_ok(nx, nw)) return 0;
    return plane_bytes(nx, nw) + step_bytes(nx, nw, true);
}

MIG_API int mig_extrapolate(const mig_c64* wf_in, mig_c64* wf_out, const float* vel,
                            const double* omega, const mig_c64* tab32, const mig_table_desc* d,
                            int32_t nx, int32_t nw, int32_t nsteps, double* rows, void* ws,
                            size_t ws_bytes, void* stream)
{
    if (!desc_valid(d) || !wf_in || !vel || !omega || !tab32 || !sizes_ok(nx, nw) || nsteps < 0)
        return MIG_E_ARG;
    if (!wf_out && !rows) return MIG_E_ARG;
    const size_t pl = (size_t)nx * nw * sizeof(mig_c64);
    if (wf_out && overlap(wf_in, pl, wf_out, pl)) return MIG_E_ARG;
    hipStream_t s = as_stream(stream);
    const float2* src = reinterpret_cast<const float2*>(wf_in);
    float2* dst = reinterpret_cast<float2*>(wf_out);
    if (nsteps == 0) {
        if (wf_out && hipMemcpyAsync(dst, src, pl, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return MIG_E_DEVICE;
        return MIG_OK;
    }
    if (ws && (overlap(ws, ws_bytes, wf_in, pl) || (wf_out && overlap(ws, ws_bytes, wf_out, pl))))
        return MIG_E_ARG;
    return run_extrap(src, dst, vel, omega, reinterpret_cast<const float2*>(tab32), d, nx, nw,
                      nsteps, rows, ws, ws_bytes, s);
}

MIG_API int mig_image(const mig_c64* wf, double* row, int32_t nx, int32_t nw, void* stream)
{
    if (!wf || !row || !sizes_ok(nx, nw)) return MIG_E_ARG;
    return launch_image(reinterpret_cast<const float2*>(wf), row, nx, nw, as_stream(stream));
}

MIG_API int mig_migrate(const mig_c64* data, const float* vel, const double* omega,
                        const mig_c64* tab32, const mig_table_desc* d, int32_t nx, int32_t nz,
                        int32_t nw, double* image, void* ws, size_t ws_bytes, void* stream)
{
    if (!desc_valid(d) || !data || !vel || !omega || !tab32 || !image || !sizes_ok(nx, nw) ||
        nz < 1)
        return MIG_E_ARG;
    hipStream_t s = as_stream(stream);
    int rc = launch_image(reinterpret_cast<const float2*>(data), image, nx, nw, s);
    if (rc != MIG_OK || nz == 1) return rc;
    const size_t pl = (size_t)nx * nw * sizeof(mig_c64);
    if (ws && overlap(ws, ws_bytes, data, pl)) return MIG_E_ARG;
    return run_extrap(reinterpret_cast<const float2*>(data), nullptr, vel, omega,
                      reinterpret_cast<const float2*>(tab32), d, nx, nw, nz - 1, image + nx, ws,
                      ws_bytes, s);
}

// Internal query used by tests and the benchmark: which extrapolation kernel
// a call with these sizes takes (1 = register-tap kernel, 0 = general).
MIG_API int mig_kernel_kind(int32_t nx, int32_t ntaps)
{
    if (ntaps < 1 || ntaps > MIG_MAX_NTAPS || (ntaps % 2) == 0 || nx < 1) return -1;
    return extrap_kernel_kind(nx, (ntaps - 1) / 2);
}

}  // extern "C"
