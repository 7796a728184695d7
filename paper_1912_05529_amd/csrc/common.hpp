// Internal declarations shared by the HIP translation units of libmig.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "mig.h"

namespace mig {

constexpr double kPi = 3.14159265358979323846;

// Arguments of the depth-stepping kernels (one workgroup per frequency).
struct ExtrapArgs {
    const float2* win;     // [nx][nw] plane at the first depth of the launch
    float2* wout;          // [nx][nw] plane after nsteps, or nullptr
    const double* slow;    // [nsteps][ldp] slowness rows (see slowness_of)
    const double* omega;   // [nw]
    const float2* tab;     // [nk][M+1] complex64 half-taps
    float* part;           // [nsteps][nw][ldp] Re of each new plane, or nullptr
    int nx, nw, nsteps, nk, M, ldp;
    double dk;             // table spacing (kmax-kmin)/(nk-1)
    double b;              // kmin / dk
};

// Slowness used by the table look-up: 1/v as an IEEE double division, or NaN
// when v is not > 0 (which selects entry 0).
__device__ __forceinline__ double slowness_of(float v)
{
    return v > 0.0f ? 1.0 / (double)v : __builtin_nan("");
}

// Table look-up of Algorithm 1: nearest entry to omega/v, as the IEEE-double
// sequence documented for mig_table_index (no contraction, every operation
// rounded on its own), from s = slowness_of(v).  a = omega/dk and
// b = kmin/dk are computed with IEEE division.
__device__ __forceinline__ int index_of_slowness(double a, double b, int nk, double s)
{
#pragma clang fp contract(off)
    double t = a * s;
    t = t - b;
    double u = t + 0.5;
    if (!(u >= 1.0)) return 0;
    if (u >= (double)nk) return nk - 1;
    return (int)floor(u);
}

__device__ __forceinline__ int table_index(double a, double b, int nk, float v)
{
    return index_of_slowness(a, b, nk, slowness_of(v));
}

// Row stride of the slowness and partial-row buffers: nx rounded up so that
// every thread of the register-tap kernels can load and store whole vectors.
inline int row_stride(int nx) { return (nx + 255) / 256 * 256; }

// Host launchers (return MIG_OK or MIG_E_DEVICE).
int launch_design_basis(const mig_table_desc* d, double* A, double* C, hipStream_t s);
int launch_design(const mig_table_desc* d, const double* A, const double* C,
                  mig_c128* tab64, mig_c64* tab32, double* maxgain,
                  double* passerr, int* status, hipStream_t s);
int launch_index(const float* vel, const double* omega, int nx, int nw,
                 int nrows, int nk, double dk, double b, int32_t* idx,
                 hipStream_t s);
int launch_slowness(const float* vel, int nx, int nrows, int ldp, double* slow, hipStream_t s);
int launch_extrap(const ExtrapArgs& a, hipStream_t s);
int launch_rows_reduce(const float* part, int ldp, int nx, int nw, int nsteps,
                       double* rows, hipStream_t s);
int launch_image(const float2* wf, double* row, int nx, int nw, hipStream_t s);

// Which extrapolation kernel a launch with these sizes takes (for tests and
// the benchmark): 1 = register-tap kernel (two outputs per thread, two tap
// sets), 2 = register-tap kernel (four outputs per thread, one tap set),
// 0 = general kernel.
int extrap_kernel_kind(int nx, int M);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace mig
