// Internal declarations shared by the HIP translation units of libmig.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "mig.h"

namespace mig {

constexpr double kPi = 3.14159265358979323846;

// Frequency workgroups publish their partial rows every kPublish depth steps.
constexpr int kPublish = 32;
// Reducers poll a block counter with this s_sleep argument (x 64 cycles).
constexpr int kPollSleep = 127;
// Default reducer stall limit: a reducer that sees no publish anywhere in the
// launch for this long gives up for the whole launch (NaN rows, status set).
constexpr unsigned long long kStallTicks = 20ull * 100000000ull;  // 20 s at 100 MHz
// The device clock read by wall_clock64() runs at 100 MHz.
constexpr unsigned long long kWallTicksPerUs = 100ull;

// Sticky status word at the head of a workspace (kStatusBytes reserved):
// 0, or kStatusAbandoned once a reducer gave up waiting for a block.
constexpr size_t kStatusBytes = 256;
constexpr int kStatusAbandoned = 1;

// One section as the depth-stepping kernels see it (device pointers).
struct SecDev {
    const float2* win;     // [nx][nw] plane at the first depth of the launch
    float2* wout;          // [nx][nw] plane after nsteps, or nullptr
    const float* vel;      // [nsteps][nx] propagation velocity rows
    const double* slow;    // [nsteps][ldp] slowness rows (see slowness_of)
    const double* omega;   // [nw]
    float* part;           // [nsteps][nw][ldp] Re of each new plane, or nullptr
    double* rows;          // [nsteps][nx] image rows, or nullptr
    int* cnt;              // [ceil(nsteps/kPublish)] published-block counters
    int nx, nw, nsteps, ldp;
    int nprod;             // frequency workgroups of this section in the launch
    int G;                 // frequencies per workgroup (sub-groups of tsub threads)
};

// A frequency workgroup: section and first frequency (it owns G of them).
struct ItemDev {
    int sec, r0;
};

// A reducer task: image rows of the published block `block` (steps
// block*kPublish ... +kPublish-1) of section `sec`, points [x0, x1).
struct TaskDev {
    int sec, block, x0, x1;
};

// Arguments of one depth-stepping launch.  With nsec == 1 the section lives
// in `one`, workgroup i owns frequencies [i*G, i*G+G) (G = one.G) and reducer
// task i is part i % parts of block i / parts; otherwise the three arrays
// (device memory) describe the batch.
struct BatchArgs {
    SecDev one;
    const SecDev* secs;
    const ItemDev* items;
    const TaskDev* tasks;
    const float2* tab;     // [nk][M+1] complex64 half-taps
    float* trash;          // [ldp_max] sink for partial rows of idle sub-groups
    // progress[0]: publishes of the whole launch (restarts the reducers'
    // stall clock); progress[1]: abandon word, set by the first reducer that
    // runs into the stall limit, after which no reducer of the launch waits
    int* progress;
    int* status;           // sticky status of the call (workspace head), or nullptr
    unsigned long long stall_ticks;  // reducer stall limit (wall_clock64 ticks)
    int reset_status;      // the slowness launch zeroes *status (first launch of a call)
    int extra_wait;        // test hook: reducers wait for nprod + extra_wait publishes
    int nsec, nitems, ntasks, nred;
    int rows;              // frequency workgroups write and publish partial rows
    int parts;             // x-parts per block (nsec == 1)
    int nk, M;
    double dk;             // table spacing (kmax-kmin)/(nk-1)
    double b;              // kmin / dk
};

// Lateral change points of one depth row (x where the slowness differs from
// x-1), as the folded adjoint kernel reads them: at most kAdjKmax per row.
constexpr int kAdjKmax = 16;
struct AdjRow {
    int cnt;               // change points in the row (may exceed kAdjKmax)
    int pos[kAdjKmax];     // the first min(cnt, kAdjKmax), increasing
    int pad[3];
};

// Arguments of the demigration (adjoint) launch: one workgroup per frequency.
struct AdjArgs {
    const double* image;   // [nz][nx] image rows (input)
    const double* slow;    // [nz-1][ldp] slowness rows of the depth steps
    const double* omega;   // [nw]
    const float2* tab;     // [nk][M+1]
    float2* out;           // [nx][nw] surface plane (output)
    // folded kernel: change points per row, their table entries per
    // frequency [nz-1][nw][kAdjKmax] (left | right << 16; nk <= 65536), and
    // the flag set when some row has more than kmax change points (then the
    // product kernel runs instead); dense == nullptr: only the product (or
    // general) kernel is launched
    AdjRow* chg;
    int* jpair;
    int* dense;
    int kmax;
    int nx, nz, nw, ldp, nk, M;
    int chunk;             // filter taps handled per LDS pass
    double dk, b;
};

// A pointer that the compiler cannot see to be global (one read from a struct
// of arguments) makes flat instructions, which also count against the LDS wait
// counter: a barrier's LDS wait would then wait for them too.  Casting to the
// global address space makes them global instructions.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* as_global(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}

// Loads of the HIP vector structs through a global pointer, as native vectors.
__device__ __forceinline__ float2 load_global(const float2* p)
{
    typedef float v2f __attribute__((ext_vector_type(2)));
    const v2f v = *as_global(reinterpret_cast<const v2f*>(p));
    return make_float2(v.x, v.y);
}

__device__ __forceinline__ double2 load_global(const double2* p)
{
    typedef double v2d __attribute__((ext_vector_type(2)));
    const v2d v = *as_global(reinterpret_cast<const v2d*>(p));
    return make_double2(v.x, v.y);
}

// Slowness used by the table look-up: 1/v as an IEEE double division, or NaN
// when v is not > 0 (which selects entry 0).
__device__ __forceinline__ double slowness_of(float v)
{
    return v > 0.0f ? 1.0 / (double)v : __builtin_nan("");
}

// The slowness rows handed to the depth-stepping kernels carry one flag in the
// sign bit (slowness itself is never negative): set when the value differs
// from the one `dist` rows earlier, i.e. when a tap set last loaded for that
// row must be refilled.
constexpr unsigned long long kSignBit = 0x8000000000000000ull;

__device__ __forceinline__ bool slowness_changed(double s)
{
    return (__double_as_longlong(s) & (long long)kSignBit) != 0;
}

__device__ __forceinline__ double slowness_value(double s)
{
    return __longlong_as_double(__double_as_longlong(s) & (long long)~kSignBit);
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

// Kernel variants (tests and the benchmark can query which one runs):
// 1 = register taps, two outputs per thread, two tap sets (nx <= 1024);
// 3 = register taps, three outputs per thread, one tap set (nx <= 1536);
// 2 = register taps, four outputs per thread, one tap set (nx <= 2048);
// 0 = general kernel, taps read from the table every step.
int extrap_kernel_kind(int nx, int M);
// Threads one frequency needs in kernel `kind` for nx points.
int threads_per_omega(int kind, int nx);

// Host launchers (return MIG_OK or MIG_E_DEVICE).
int launch_design_basis(const mig_table_desc* d, double* A, double* C, hipStream_t s);
int launch_design(const mig_table_desc* d, const double* A, const double* C,
                  mig_c128* tab64, mig_c64* tab32, double* maxgain,
                  double* passerr, int* status, hipStream_t s);
int launch_index(const float* vel, const double* omega, int nx, int nw,
                 int nrows, int nk, double dk, double b, int32_t* idx,
                 hipStream_t s);
// Slowness rows of every section of the launch (one launch for all), with the
// change flag taken against the row `dist` steps earlier (negative: -dist
// steps later; 0 = no flags).
int launch_slowness(const BatchArgs& a, int max_rows, int max_ldp, int dist, hipStream_t s);
// Row distance of the change flag a kernel variant reads.
inline int flag_distance(int kind) { return kind == 1 ? 2 : (kind == 0 ? 0 : 1); }
// Depth stepping for every workgroup item (+ reducers when sections want rows).
// `kind` and `threads` (workgroup size) are the same for all items.
int launch_extrap(const BatchArgs& a, int kind, int threads, hipStream_t s);
int launch_general(const BatchArgs& a, int max_nx, hipStream_t s);
// Taps per LDS pass of the demigration kernel for an LDS budget (0 = too big).
int adjoint_chunk(int nx, int M, size_t lds_limit);
int launch_demigrate(const AdjArgs& a, hipStream_t s);
// Register-tap adjoint kernel: usable for these sizes within an LDS budget?
bool adjoint_uses_registers(int nx, int M, size_t lds_limit);
int launch_demigrate_reg(const AdjArgs& a, hipStream_t s);
// Folded adjoint kernel (own-filter FIR + corrections at lateral change
// points): usable for these sizes?  Change points it handles per row.
bool adjoint_uses_fold(int nx, int M);
int adjoint_fold_kmax(int nx, int M);
// Change-point pre-pass (after the slowness rows), then the folded kernel.
int launch_adj_changes(const AdjArgs& a, hipStream_t s);
int launch_demigrate_fold(const AdjArgs& a, hipStream_t s);
// Transform along t: builds the FP32 DFT matrix B [nt][2 nw] and computes the
// plane out [nx][nw] = section [nx][nt] . B on the matrix cores.
int launch_transform(const float* section, int nx, int nt, double dt, const double* omega,
                     int nw, float2* out, float* B, hipStream_t s);
int launch_image(const float2* wf, double* row, int nx, int nw, hipStream_t s);
// Zeroes a workspace's status word (calls that run no depth-stepping launch).
int launch_clear_status(int* status, hipStream_t s);
// Image rows of depth steps [s0, s1) of one section from its partial rows
// ([step][nw][ldp] floats), after the depth-stepping launch.
int launch_rows(const float* part, double* rows, int s0, int s1, int nx, int nw, int ldp,
                hipStream_t s);

// One 3-D depth step (device pointers; planes are [nw][nx][ny]).
struct Step3dArgs {
    const float2* in;       // plane before the step
    float2* out;            // plane after the step
    const float* vel;       // [nx][ny] velocity of this step
    const float2* tab;      // [nk][NU] 2-D table
    const double* omega;    // [nw]
    double* part;           // [ngroups][nx][ny] partial image of the new plane
    const double* prev;     // partials of the previous step, or nullptr
    double* prev_row;       // image row receiving the previous step's sum
    int nx, ny, nw, nk;
    int wpg, ngroups;       // frequencies per group, groups
    int tiles_x, tiles_y;
    double dk, b;           // table spacing, kmin / dk
};
int step3d_tiles_x(int nx);
int step3d_tiles_y(int ny);
int launch_step3d(const Step3dArgs& a, int M, hipStream_t s);
int launch_image3d(const float2* wf, double* row, size_t plane, int nw, hipStream_t s);
int launch_reduce3d(const double* part, double* row, size_t plane, int ngroups, hipStream_t s);
int launch_design2d_basis(const mig_table_desc* d, double* A, double* CS, hipStream_t s);
int launch_design2d(const mig_table_desc* d, const double* A, const double* CS,
                    mig_c128* tab64, mig_c64* tab32, double* maxgain, double* passerr,
                    int* status, hipStream_t s);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace mig
