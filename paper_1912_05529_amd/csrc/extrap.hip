// Depth stepping (Eq. 1 with per-point filters), imaging and table look-up.
//
// Design (MI355X / gfx950):
//   * Frequencies never interact during extrapolation (Sec. II: the process
//     runs independently for each frequency), only through the image sum.  So
//     one workgroup owns one frequency for the whole depth range: its plane
//     (nx complex64, a few KB) stays in LDS, depth steps are separated by a
//     workgroup barrier instead of a kernel exit (the "block level
//     synchronization" the paper names as future work, Sec. V), and there is no
//     inter-workgroup traffic at all.
//   * Lanes run along x (coalesced, conflict-free LDS windows); each thread
//     owns two (or four) adjacent outputs and reads its window with 16-byte LDS
//     loads.  Even taps are folded: h_n (u[x-n] + u[x+n]).
//   * Taps live in registers.  The filter of an output only changes when the
//     velocity under it changes (omega is fixed per workgroup), which in layered
//     media is a few times per column.  Two register sets alternate between
//     even and odd steps; the set for step k+1 is refilled during step k only
//     for outputs whose slowness changed, so table reads (L2-resident) are rare
//     and their latency is hidden behind a full step of arithmetic.
//   * The look-up needs 1/v in FP64; it is computed once per (depth, x) by a
//     small pre-pass (shared by all frequencies) instead of once per refill.
//   * The image row needs a sum over frequencies, i.e. across workgroups.
//     Each workgroup writes Re of its new plane (float32, exact) to a partial
//     buffer [step][omega][x]; a second kernel sums over omega in a fixed order
//     in FP64, so images are run-to-run identical.
#include "common.hpp"

namespace mig {
namespace {

// s_waitcnt vmcnt(N) with the other counters left alone (GFX9 encoding:
// vmcnt[3:0] | expcnt[6:4] | lgkmcnt[11:8] | vmcnt[5:4] in bits 15:14).
template <int N>
__device__ __forceinline__ void wait_vmem()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

__device__ __forceinline__ float2 cmulf(float2 h, float2 u)
{
    return make_float2(fmaf(-h.y, u.y, h.x * u.x), fmaf(h.y, u.x, h.x * u.y));
}

__device__ __forceinline__ float2 cfmaf(float2 h, float2 s, float2 acc)
{
    acc.x = fmaf(h.x, s.x, acc.x);
    acc.x = fmaf(-h.y, s.y, acc.x);
    acc.y = fmaf(h.x, s.y, acc.y);
    acc.y = fmaf(h.y, s.x, acc.y);
    return acc;
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b)
{
    return make_float2(a.x + b.x, a.y + b.y);
}

__device__ __forceinline__ unsigned long long dbits(double d)
{
    return (unsigned long long)__double_as_longlong(d);
}

template <int M>
__device__ __forceinline__ void load_taps(float2 (&h)[M + 1], const float2* __restrict__ row)
{
#pragma unroll
    for (int n = 0; n <= M; ++n) h[n] = row[n];
}

// Two outputs x0, x0+1 from the window w[i] = P[x0 - M + i], i = 0..2M+1.
template <int M>
__device__ __forceinline__ void fir2(const float2* __restrict__ win, const float2 (&h0)[M + 1],
                                     const float2 (&h1)[M + 1], float2& o0, float2& o1)
{
    float2 w[2 * M + 2];
    const float4* w4 = reinterpret_cast<const float4*>(win);
#pragma unroll
    for (int i = 0; i <= M; ++i) {
        float4 q = w4[i];
        w[2 * i] = make_float2(q.x, q.y);
        w[2 * i + 1] = make_float2(q.z, q.w);
    }
    float2 a0 = cmulf(h0[0], w[M]);
    float2 a1 = cmulf(h1[0], w[M + 1]);
#pragma unroll
    for (int n = 1; n <= M; ++n) {
        a0 = cfmaf(h0[n], cadd(w[M - n], w[M + n]), a0);
        a1 = cfmaf(h1[n], cadd(w[M + 1 - n], w[M + 1 + n]), a1);
    }
    o0 = a0;
    o1 = a1;
}

// Four outputs x0..x0+3 from the window w[i] = P[x0 - M + i], i = 0..2M+3.
template <int M>
__device__ __forceinline__ void fir4(const float2* __restrict__ win, const float2 (&h)[4][M + 1],
                                     float2 (&o)[4])
{
    float2 w[2 * M + 4];
    const float4* w4 = reinterpret_cast<const float4*>(win);
#pragma unroll
    for (int i = 0; i < M + 2; ++i) {
        float4 q = w4[i];
        w[2 * i] = make_float2(q.x, q.y);
        w[2 * i + 1] = make_float2(q.z, q.w);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = cmulf(h[q][0], w[M + q]);
#pragma unroll
    for (int n = 1; n <= M; ++n) {
#pragma unroll
        for (int q = 0; q < 4; ++q) o[q] = cfmaf(h[q][n], cadd(w[M + q - n], w[M + q + n]), o[q]);
    }
}

// slow[k][x] = slowness_of(vel[k][min(x, nx-1)]) for x < ldp.
__global__ void k_slowness(const float* __restrict__ vel, int nx, int nrows, int ldp,
                           double* __restrict__ slow)
{
    const size_t total = (size_t)nrows * ldp;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        size_t k = e / ldp;
        int x = (int)(e % ldp);
        slow[e] = slowness_of(vel[k * nx + (x < nx ? x : nx - 1)]);
    }
}

struct Lane {
    int t, x0, LB, r;
    bool ok0, ok1;
    double ar;
};

// One depth step k: wait for this step's taps (issued during step k-1),
// refill the other set for step k+1 where the slowness changed, prefetch the
// slowness of step k+2, then the folded FIR, LDS write and partial row.
// VMEM operations of a step are issued in a fixed order -- [refills], one
// slowness load, [one partial-row store] -- so the wait at the top of the
// next step has a static count that never includes that step's refills.
template <int M, bool ROWS>
__device__ __forceinline__ void step_fast(const ExtrapArgs& a, float2* sm, const Lane& L, int k,
                                          float2 (&hc)[2][M + 1], float2 (&ho)[2][M + 1],
                                          unsigned long long (&bo)[2], double2& sn, float2& o0,
                                          float2& o1)
{
    wait_vmem<ROWS ? 1 : 0>();
    if (k >= 1 && k + 1 < a.nsteps) {
        unsigned long long u0 = dbits(sn.x), u1 = dbits(sn.y);
        if (u0 != bo[0]) {
            bo[0] = u0;
            load_taps<M>(ho[0], a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk, sn.x) * (M + 1));
        }
        if (u1 != bo[1]) {
            bo[1] = u1;
            load_taps<M>(ho[1], a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk, sn.y) * (M + 1));
        }
    }
    const int kp = k + 2 < a.nsteps ? k + 2 : a.nsteps - 1;
    const double2 p = *reinterpret_cast<const double2*>(a.slow + (size_t)kp * a.ldp + L.x0);
    fir2<M>(sm + (k & 1) * L.LB + 2 * L.t, hc[0], hc[1], o0, o1);
    float2* dst = sm + ((k + 1) & 1) * L.LB + M + L.x0;
    if (L.ok0) dst[0] = o0;
    if (L.ok1) dst[1] = o1;
    if (ROWS) {
        float* pr = a.part + ((size_t)k * a.nw + L.r) * a.ldp + L.x0;
        *reinterpret_cast<float2*>(pr) = make_float2(o0.x, o1.x);
    }
    sn = p;
    __syncthreads();
}

// Register-tap kernel.  Block = ceil(nx/2) threads rounded up to a wavefront;
// LDS = two planes of 2*blockDim + 2M + 2 points, P[x] at offset M + x, zero
// elsewhere (the zero boundary of Eq. 1).
template <int M, bool ROWS>
__global__ void __launch_bounds__(512) k_extrap_fast(ExtrapArgs a)
{
    extern __shared__ float4 smem4[];
    float2* sm = reinterpret_cast<float2*>(smem4);
    Lane L;
    L.t = threadIdx.x;
    L.r = blockIdx.x;
    L.LB = 2 * blockDim.x + 2 * M + 2;
    L.x0 = 2 * L.t;
    L.ok0 = L.x0 < a.nx;
    L.ok1 = L.x0 + 1 < a.nx;
    L.ar = a.omega[L.r] / a.dk;

    for (int i = L.t; i < 2 * L.LB; i += blockDim.x) sm[i] = make_float2(0.0f, 0.0f);
    __syncthreads();
    if (L.ok0) sm[M + L.x0] = a.win[(size_t)L.x0 * a.nw + L.r];
    if (L.ok1) sm[M + L.x0 + 1] = a.win[(size_t)(L.x0 + 1) * a.nw + L.r];

    float2 hA[2][M + 1], hB[2][M + 1];
    unsigned long long bA[2], bB[2];
    {
        const double2 s0 = *reinterpret_cast<const double2*>(a.slow + L.x0);
        bA[0] = dbits(s0.x);
        bA[1] = dbits(s0.y);
        load_taps<M>(hA[0], a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk, s0.x) * (M + 1));
        load_taps<M>(hA[1], a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk, s0.y) * (M + 1));
        const int k1 = a.nsteps > 1 ? 1 : 0;
        const double2 s1 = *reinterpret_cast<const double2*>(a.slow + (size_t)k1 * a.ldp + L.x0);
        bB[0] = dbits(s1.x);
        bB[1] = dbits(s1.y);
        load_taps<M>(hB[0], a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk, s1.x) * (M + 1));
        load_taps<M>(hB[1], a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk, s1.y) * (M + 1));
    }
    double2 sn = make_double2(0.0, 0.0);
    wait_vmem<0>();
    __syncthreads();

    float2 o0 = make_float2(0.0f, 0.0f), o1 = o0;
    for (int k = 0; k < a.nsteps; k += 2) {
        step_fast<M, ROWS>(a, sm, L, k, hA, hB, bB, sn, o0, o1);
        if (k + 1 >= a.nsteps) break;
        step_fast<M, ROWS>(a, sm, L, k + 1, hB, hA, bA, sn, o0, o1);
    }
    if (a.wout) {
        if (L.ok0) a.wout[(size_t)L.x0 * a.nw + L.r] = o0;
        if (L.ok1) a.wout[(size_t)(L.x0 + 1) * a.nw + L.r] = o1;
    }
}

// Register-tap kernel for wider sections (nx <= 4 * 512): four outputs per
// thread and one tap set (two do not fit in 256 VGPRs), refilled at the end of
// a step for outputs whose slowness changes at the next step.  A workgroup
// touches only the table rows of its own frequency, so refills mostly hit in
// L1 and the barrier covers part of their latency.
template <int M, bool ROWS>
__global__ void __launch_bounds__(512) k_extrap_wide(ExtrapArgs a)
{
    extern __shared__ float4 smem4[];
    float2* sm = reinterpret_cast<float2*>(smem4);
    const int t = threadIdx.x, r = blockIdx.x;
    const int LB = 4 * blockDim.x + 2 * M + 4;
    const int x0 = 4 * t;
    bool ok[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) ok[q] = x0 + q < a.nx;
    const double ar = a.omega[r] / a.dk;

    for (int i = t; i < 2 * LB; i += blockDim.x) sm[i] = make_float2(0.0f, 0.0f);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (ok[q]) sm[M + x0 + q] = a.win[(size_t)(x0 + q) * a.nw + r];

    float2 h[4][M + 1];
    unsigned long long bits[4];
    double sn[4];
    {
        const double2* s0 = reinterpret_cast<const double2*>(a.slow + x0);
        const int k1 = a.nsteps > 1 ? 1 : 0;
        const double2* s1 = reinterpret_cast<const double2*>(a.slow + (size_t)k1 * a.ldp + x0);
        double c[4] = {s0[0].x, s0[0].y, s0[1].x, s0[1].y};
        double n1[4] = {s1[0].x, s1[0].y, s1[1].x, s1[1].y};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            bits[q] = dbits(c[q]);
            load_taps<M>(h[q], a.tab + (size_t)index_of_slowness(ar, a.b, a.nk, c[q]) * (M + 1));
            sn[q] = n1[q];
        }
    }
    wait_vmem<0>();
    __syncthreads();

    float2 o[4];
    for (int k = 0; k < a.nsteps; ++k) {
        const int kp = k + 2 < a.nsteps ? k + 2 : a.nsteps - 1;
        const double2* sp = reinterpret_cast<const double2*>(a.slow + (size_t)kp * a.ldp + x0);
        const double2 p01 = sp[0], p23 = sp[1];
        fir4<M>(sm + (k & 1) * LB + x0, h, o);
        float2* dst = sm + ((k + 1) & 1) * LB + M + x0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (ok[q]) dst[q] = o[q];
        if (ROWS) {
            float* pr = a.part + ((size_t)k * a.nw + r) * a.ldp + x0;
            *reinterpret_cast<float4*>(pr) = make_float4(o[0].x, o[1].x, o[2].x, o[3].x);
        }
        if (k + 1 < a.nsteps) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                unsigned long long u = dbits(sn[q]);
                if (u != bits[q]) {
                    bits[q] = u;
                    load_taps<M>(h[q], a.tab + (size_t)index_of_slowness(ar, a.b, a.nk, sn[q]) * (M + 1));
                }
            }
        }
        sn[0] = p01.x;
        sn[1] = p01.y;
        sn[2] = p23.x;
        sn[3] = p23.y;
        __syncthreads();
    }
    if (a.wout) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (ok[q]) a.wout[(size_t)(x0 + q) * a.nw + r] = o[q];
    }
}

// General kernel: any M <= 31 and nx up to MIG_MAX_NX.  Same ownership (one
// workgroup per frequency, plane in LDS), taps read from the table every step.
__global__ void __launch_bounds__(256) k_extrap_general(ExtrapArgs a)
{
    extern __shared__ float4 smem4[];
    float2* sm = reinterpret_cast<float2*>(smem4);
    const int M = a.M, nx = a.nx, r = blockIdx.x;
    const int LB = nx + 2 * M;
    const double ar = a.omega[r] / a.dk;
    for (int i = threadIdx.x; i < 2 * LB; i += blockDim.x) sm[i] = make_float2(0.0f, 0.0f);
    __syncthreads();
    for (int x = threadIdx.x; x < nx; x += blockDim.x) sm[M + x] = a.win[(size_t)x * a.nw + r];
    __syncthreads();
    for (int k = 0; k < a.nsteps; ++k) {
        const float2* src = sm + (k & 1) * LB + M;
        float2* dst = sm + ((k + 1) & 1) * LB + M;
        const double* sr = a.slow + (size_t)k * a.ldp;
        for (int x = threadIdx.x; x < nx; x += blockDim.x) {
            const float2* h = a.tab + (size_t)index_of_slowness(ar, a.b, a.nk, sr[x]) * (M + 1);
            float2 acc = cmulf(h[0], src[x]);
            for (int n = 1; n <= M; ++n) acc = cfmaf(h[n], cadd(src[x - n], src[x + n]), acc);
            dst[x] = acc;
            if (a.part) a.part[((size_t)k * a.nw + r) * a.ldp + x] = acc.x;
        }
        __syncthreads();
    }
    if (a.wout) {
        const float2* src = sm + (a.nsteps & 1) * LB + M;
        for (int x = threadIdx.x; x < nx; x += blockDim.x) a.wout[(size_t)x * a.nw + r] = src[x];
    }
}

// rows[s][x] = sum_{r=0..nw-1} part[s][r][x], FP64, r in increasing order.
__global__ void __launch_bounds__(256) k_rows_reduce(const float* __restrict__ part, int ldp,
                                                     int nx, int nw, int nsteps,
                                                     double* __restrict__ rows)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    for (int s = blockIdx.y; s < nsteps; s += gridDim.y) {
        const float* p = part + (size_t)s * nw * ldp + x;
        double acc = 0.0;
        for (int r = 0; r < nw; ++r) acc += (double)p[(size_t)r * ldp];
        rows[(size_t)s * nx + x] = acc;
    }
}

// row[x] = sum_r Re wf[x][r]: one wavefront per x, lane-strided FP64 partial
// sums, then a xor-butterfly of cross-lane shuffles (fixed order).
__global__ void __launch_bounds__(256) k_image(const float2* __restrict__ wf,
                                               double* __restrict__ row, int nx, int nw)
{
    const int lane = threadIdx.x & 63;
    const int x = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (x >= nx) return;
    const float2* p = wf + (size_t)x * nw;
    double acc = 0.0;
    for (int r = lane; r < nw; r += 64) acc += (double)p[r].x;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) row[x] = acc;
}

__global__ void k_index(const float* __restrict__ vel, const double* __restrict__ omega,
                        int nx, int nw, int nrows, int nk, double dk, double b,
                        int32_t* __restrict__ idx)
{
#pragma clang fp contract(off)
    const size_t total = (size_t)nrows * nx * nw;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        int r = (int)(e % nw);
        size_t kx = e / nw;
        double a = omega[r] / dk;
        idx[e] = table_index(a, b, nk, vel[kx]);
    }
}

template <int M>
int launch_fast(const ExtrapArgs& a, hipStream_t s)
{
    int threads = ((a.nx + 1) / 2 + 63) / 64 * 64;
    size_t lds = (size_t)2 * (2 * threads + 2 * M + 2) * sizeof(float2);
    if (a.part)
        hipLaunchKernelGGL((k_extrap_fast<M, true>), dim3(a.nw), dim3(threads), lds, s, a);
    else
        hipLaunchKernelGGL((k_extrap_fast<M, false>), dim3(a.nw), dim3(threads), lds, s, a);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

template <int M>
int launch_wide(const ExtrapArgs& a, hipStream_t s)
{
    int threads = ((a.nx + 3) / 4 + 63) / 64 * 64;
    size_t lds = (size_t)2 * (4 * threads + 2 * M + 4) * sizeof(float2);
    if (a.part)
        hipLaunchKernelGGL((k_extrap_wide<M, true>), dim3(a.nw), dim3(threads), lds, s, a);
    else
        hipLaunchKernelGGL((k_extrap_wide<M, false>), dim3(a.nw), dim3(threads), lds, s, a);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

typedef int (*launch_fn)(const ExtrapArgs&, hipStream_t);

// Register-tap kernels are instantiated for N = 1..35 (M = 0..17); beyond
// that two tap sets no longer fit in 256 VGPRs without spilling.
#define MIG_INST(f)                                                                   \
    {&f<0>, &f<1>, &f<2>, &f<3>, &f<4>, &f<5>, &f<6>, &f<7>, &f<8>, &f<9>, &f<10>,     \
     &f<11>, &f<12>, &f<13>, &f<14>, &f<15>, &f<16>, &f<17>}
const launch_fn kFast[] = MIG_INST(launch_fast);
const launch_fn kWide[] = MIG_INST(launch_wide);
constexpr int kRegMaxM = 17;
constexpr int kFastMaxNx = 2 * 512;
constexpr int kWideMaxNx = 4 * 512;

}  // namespace

int extrap_kernel_kind(int nx, int M)
{
    if (M > kRegMaxM) return 0;
    if (nx <= kFastMaxNx) return 1;
    if (nx <= kWideMaxNx) return 2;
    return 0;
}

int launch_slowness(const float* vel, int nx, int nrows, int ldp, double* slow, hipStream_t s)
{
    size_t total = (size_t)nrows * ldp;
    size_t blocks = (total + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_slowness, dim3((unsigned)blocks), dim3(256), 0, s, vel, nx, nrows, ldp,
                       slow);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

int launch_extrap(const ExtrapArgs& a, hipStream_t s)
{
    int kind = extrap_kernel_kind(a.nx, a.M);
    if (kind == 1) return kFast[a.M](a, s);
    if (kind == 2) return kWide[a.M](a, s);
    size_t lds = (size_t)2 * (a.nx + 2 * a.M) * sizeof(float2);
    if (lds > 65536) {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_extrap_general),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds) != hipSuccess)
            return MIG_E_DEVICE;
    }
    hipLaunchKernelGGL(k_extrap_general, dim3(a.nw), dim3(256), lds, s, a);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

int launch_rows_reduce(const float* part, int ldp, int nx, int nw, int nsteps,
                       double* rows, hipStream_t s)
{
    dim3 grid((nx + 255) / 256, nsteps < 65535 ? nsteps : 65535);
    hipLaunchKernelGGL(k_rows_reduce, grid, dim3(256), 0, s, part, ldp, nx, nw, nsteps, rows);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

int launch_image(const float2* wf, double* row, int nx, int nw, hipStream_t s)
{
    dim3 grid((nx + 3) / 4);
    hipLaunchKernelGGL(k_image, grid, dim3(256), 0, s, wf, row, nx, nw);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

int launch_index(const float* vel, const double* omega, int nx, int nw, int nrows,
                 int nk, double dk, double b, int32_t* idx, hipStream_t s)
{
    size_t total = (size_t)nrows * nx * nw;
    size_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_index, dim3((unsigned)blocks), dim3(256), 0, s, vel, omega, nx, nw,
                       nrows, nk, dk, b, idx);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

}  // namespace mig
