// Adjoint of the migration (demigration): image rows -> surface plane.
//
// With the real inner product <a, b> = Re sum conj(a) b, the image map of
// Algorithm 1, I_k = S E_{k-1} ... E_0 d with (S P)[x] = sum_r Re P[x][r] and
// E_k the Eq. (1) step with output-indexed filters, has the adjoint
//     Q_{nz-1} = S* I'_{nz-1},   Q_k = S* I'_k + E_k^H Q_{k+1},   d' = Q_0,
// where (S* i)[x][r] = i[x] and
//     (E_k^H q)[x] = sum_{n=-M..M} conj(h_{j(x+n,k)}[|n|]) q[x+n]:
// every point x+n contributes through the filter of that point.  A workgroup
// owns one frequency for all depths (walking them backwards); per step it
// forms g_m[y] = conj(h_{j(y)}[m]) q[y] for its points in LDS and gathers
// out[x] = g_0[x] + sum_m (g_m[x-m] + g_m[x+m]).  The register-tap kernel
// (nx <= 1024, N <= 35) does all taps in one LDS pass; the general kernel
// handles any size a chunk of taps at a time.
#include "common.hpp"

namespace mig {
namespace {

__device__ __forceinline__ float2 cmul_conj(float2 h, float2 q)
{
    // conj(h) * q
    return make_float2(fmaf(h.y, q.y, h.x * q.x), fmaf(-h.y, q.x, h.x * q.y));
}

__global__ void __launch_bounds__(512) k_demigrate(AdjArgs a)
{
    extern __shared__ float4 smem4[];
    float2* Q = reinterpret_cast<float2*>(smem4);          // [nx]
    float2* acc = Q + a.nx;                                 // [nx]
    float2* Gm = acc + a.nx;                                // [C][nx + 2M], zero borders
    const int M = a.M, nx = a.nx, nw = a.nw, C = a.chunk;
    const int LG = nx + 2 * M;
    const int r = blockIdx.x;
    const double ar = a.omega[r] / a.dk;

    for (int i = threadIdx.x; i < C * LG; i += blockDim.x) Gm[i] = make_float2(0.0f, 0.0f);
    for (int x = threadIdx.x; x < nx; x += blockDim.x)
        Q[x] = make_float2((float)a.image[(size_t)(a.nz - 1) * nx + x], 0.0f);
    __syncthreads();

    for (int k = a.nz - 2; k >= 0; --k) {
        const double* srow = a.slow + (size_t)k * a.ldp;
        for (int x = threadIdx.x; x < nx; x += blockDim.x)
            acc[x] = make_float2((float)a.image[(size_t)k * nx + x], 0.0f);
        for (int m0 = 0; m0 <= M; m0 += C) {
            const int m1 = m0 + C <= M + 1 ? m0 + C : M + 1;
            for (int y = threadIdx.x; y < nx; y += blockDim.x) {
                const float2* h = a.tab + (size_t)index_of_slowness(ar, a.b, a.nk,
                                                                    slowness_value(srow[y])) * (M + 1);
                const float2 q = Q[y];
                for (int m = m0; m < m1; ++m) Gm[(m - m0) * LG + M + y] = cmul_conj(h[m], q);
            }
            __syncthreads();
            for (int x = threadIdx.x; x < nx; x += blockDim.x) {
                float2 s = acc[x];
                for (int m = m0; m < m1; ++m) {
                    const float2* g = Gm + (m - m0) * LG + M + x;
                    if (m == 0) {
                        s.x += g[0].x;
                        s.y += g[0].y;
                    } else {
                        s.x += g[-m].x + g[m].x;
                        s.y += g[-m].y + g[m].y;
                    }
                }
                acc[x] = s;
            }
            __syncthreads();
        }
        for (int x = threadIdx.x; x < nx; x += blockDim.x) Q[x] = acc[x];
        __syncthreads();
    }
    for (int x = threadIdx.x; x < nx; x += blockDim.x) a.out[(size_t)x * nw + r] = Q[x];
}

// Register-tap form (nx <= 2 * kAdjThreads, M <= kAdjMaxM): each thread owns
// two adjacent points y, y+1 of the frequency, keeps their Q values and their
// (M+1) taps in registers, writes the products conj(h_y[m]) q[y] of every tap
// m to LDS in one pass, and after one barrier gathers its two outputs from
// them.  The plane Q never leaves registers; two barriers per depth step.
// Taps come in two sets that alternate between steps: while a step runs on
// one set, the other is refilled for the next step (only where the slowness
// differs from the row two steps away, flag in the slowness sign bit), so the
// L2 latency of a refill hides behind a whole step.
constexpr int kAdjThreads = 512;
constexpr int kAdjMaxM = 17;

__device__ __forceinline__ void wait_vmem()
{
    __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));  // vmcnt(0) only
}

template <int M>
__device__ __forceinline__ void load_taps_adj(float2 (&h)[M + 1], const float2* __restrict__ row)
{
#pragma unroll
    for (int m = 0; m <= M; ++m) h[m] = row[m];
}

// Per-thread state of the register-tap kernel.
struct AdjLane {
    int y0, c0, c1;
    bool live0, live1;
    double ar;
    double fl0, fl1;  // slowness of row k+1 (its flag: differs from row k-1)
    double sv0, sv1;  // slowness of row k-1 (taps of step k-1)
    double i0, i1;    // image row k
};

template <int M>
__device__ __forceinline__ void adj_step(const AdjArgs& a, float2* G, int LG, AdjLane& L, int k,
                                         float2 (&hc0)[M + 1], float2 (&hc1)[M + 1],
                                         float2 (&ho0)[M + 1], float2 (&ho1)[M + 1], float2& q0,
                                         float2& q1, bool first)
{
    // everything issued during the previous step has arrived: the taps of
    // this step and the values prefetched for it
    wait_vmem();
    if (!first && k >= 1) {
        if (slowness_changed(L.fl0))
            load_taps_adj<M>(ho0, a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk,
                                                                    slowness_value(L.sv0)) * (M + 1));
        if (slowness_changed(L.fl1))
            load_taps_adj<M>(ho1, a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk,
                                                                    slowness_value(L.sv1)) * (M + 1));
    }
    const double ci0 = L.i0, ci1 = L.i1;
    // prefetch for step k-1, branch-free (rows clamped; values past the top
    // are never used), so that nothing consumes them before the next step
    const int ks = k >= 2 ? k - 2 : 0, ki = k >= 1 ? k - 1 : 0;
    L.fl0 = a.slow[(size_t)k * a.ldp + L.c0];
    L.fl1 = a.slow[(size_t)k * a.ldp + L.c1];
    L.sv0 = a.slow[(size_t)ks * a.ldp + L.c0];
    L.sv1 = a.slow[(size_t)ks * a.ldp + L.c1];
    L.i0 = a.image[(size_t)ki * a.nx + L.c0];
    L.i1 = a.image[(size_t)ki * a.nx + L.c1];
    if (L.live0) {
        // q1 = 0 when y0 + 1 is past the end: the store keeps that border zero
        float2* g = G + M + L.y0;
#pragma unroll
        for (int m = 0; m <= M; ++m) {
            g[(size_t)m * LG] = cmul_conj(hc0[m], q0);
            g[(size_t)m * LG + 1] = cmul_conj(hc1[m], q1);
        }
    }
    __syncthreads();
    // Two partial sums per output (taps m odd / m even) halve the chain of
    // dependent additions.
    float2 a0 = make_float2((float)ci0, 0.0f), a1 = make_float2((float)ci1, 0.0f);
    if (L.live0) {
        const float2* g = G + M + L.y0;
        float2 e = g[0], o = make_float2(0.0f, 0.0f);
#pragma unroll
        for (int m = 1; m <= M; ++m) {
            const float2* gm = g + (size_t)m * LG;
            float2& t = (m & 1) ? o : e;
            t.x += gm[-m].x + gm[m].x;
            t.y += gm[-m].y + gm[m].y;
        }
        a0.x += e.x + o.x;
        a0.y += e.y + o.y;
    }
    if (L.live1) {
        const float2* g = G + M + L.y0 + 1;
        float2 e = g[0], o = make_float2(0.0f, 0.0f);
#pragma unroll
        for (int m = 1; m <= M; ++m) {
            const float2* gm = g + (size_t)m * LG;
            float2& t = (m & 1) ? o : e;
            t.x += gm[-m].x + gm[m].x;
            t.y += gm[-m].y + gm[m].y;
        }
        a1.x += e.x + o.x;
        a1.y += e.y + o.y;
    }
    __syncthreads();
    q0 = L.live0 ? a0 : make_float2(0.0f, 0.0f);
    q1 = L.live1 ? a1 : make_float2(0.0f, 0.0f);
}

template <int M>
__global__ void __launch_bounds__(kAdjThreads) k_demigrate_reg(AdjArgs a)
{
    extern __shared__ float4 smem4[];
    float2* G = reinterpret_cast<float2*>(smem4);  // [M+1][nx + 2M], zero outside [M, M + nx)
    const int nx = a.nx, LG = nx + 2 * M, r = blockIdx.x;
    AdjLane L;
    L.ar = a.omega[r] / a.dk;
    L.y0 = 2 * threadIdx.x;
    L.live0 = L.y0 < nx;
    L.live1 = L.y0 + 1 < nx;
    L.c0 = L.live0 ? L.y0 : 0;
    L.c1 = L.live1 ? L.y0 + 1 : 0;

    for (int i = threadIdx.x; i < (M + 1) * LG; i += blockDim.x) G[i] = make_float2(0.0f, 0.0f);
    float2 q0 = make_float2(L.live0 ? (float)a.image[(size_t)(a.nz - 1) * nx + L.y0] : 0.0f, 0.0f);
    float2 q1 = make_float2(L.live1 ? (float)a.image[(size_t)(a.nz - 1) * nx + L.y0 + 1] : 0.0f, 0.0f);
    // set A: taps of the first step (row nz-2); set B: of the second (row nz-3)
    float2 hA0[M + 1], hA1[M + 1], hB0[M + 1], hB1[M + 1];
    int k = a.nz - 2;
    if (k >= 0) {
        const double* s0 = a.slow + (size_t)k * a.ldp;
        load_taps_adj<M>(hA0, a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk, slowness_value(s0[L.c0])) * (M + 1));
        load_taps_adj<M>(hA1, a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk, slowness_value(s0[L.c1])) * (M + 1));
        const double* s1 = a.slow + (size_t)(k >= 1 ? k - 1 : k) * a.ldp;
        load_taps_adj<M>(hB0, a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk, slowness_value(s1[L.c0])) * (M + 1));
        load_taps_adj<M>(hB1, a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk, slowness_value(s1[L.c1])) * (M + 1));
        L.i0 = L.live0 ? a.image[(size_t)k * nx + L.c0] : 0.0;
        L.i1 = L.live1 ? a.image[(size_t)k * nx + L.c1] : 0.0;
    }
    L.fl0 = L.fl1 = L.sv0 = L.sv1 = 0.0;
    __syncthreads();

    bool first = true;
    for (; k >= 0; k -= 2) {
        adj_step<M>(a, G, LG, L, k, hA0, hA1, hB0, hB1, q0, q1, first);
        first = false;
        if (k == 0) break;
        adj_step<M>(a, G, LG, L, k - 1, hB0, hB1, hA0, hA1, q0, q1, false);
    }
    if (L.live0) a.out[(size_t)L.y0 * a.nw + r] = q0;
    if (L.live1) a.out[(size_t)(L.y0 + 1) * a.nw + r] = q1;
}

template <int M>
int launch_reg(const AdjArgs& a, size_t lds, hipStream_t s)
{
    if (lds > 65536 &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_demigrate_reg<M>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return MIG_E_DEVICE;
    const int threads = ((a.nx + 1) / 2 + 63) / 64 * 64;
    hipLaunchKernelGGL(k_demigrate_reg<M>, dim3(a.nw), dim3(threads), lds, s, a);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

}  // namespace

bool adjoint_uses_registers(int nx, int M, size_t lds_limit)
{
    // M >= 1: the pair store of the last point of an odd nx lands on the
    // right border, which then exists
    return nx <= 2 * kAdjThreads && M >= 1 && M <= kAdjMaxM &&
           (size_t)(M + 1) * (nx + 2 * M) * sizeof(float2) <= lds_limit;
}

int launch_demigrate_reg(const AdjArgs& a, hipStream_t s)
{
    const size_t lds = (size_t)(a.M + 1) * (a.nx + 2 * a.M) * sizeof(float2);
    switch (a.M) {
#define MIG_ADJ_CASE(m) \
    case m: return launch_reg<m>(a, lds, s);
    MIG_ADJ_CASE(1) MIG_ADJ_CASE(2) MIG_ADJ_CASE(3) MIG_ADJ_CASE(4)
    MIG_ADJ_CASE(5) MIG_ADJ_CASE(6) MIG_ADJ_CASE(7) MIG_ADJ_CASE(8) MIG_ADJ_CASE(9)
    MIG_ADJ_CASE(10) MIG_ADJ_CASE(11) MIG_ADJ_CASE(12) MIG_ADJ_CASE(13) MIG_ADJ_CASE(14)
    MIG_ADJ_CASE(15) MIG_ADJ_CASE(16) MIG_ADJ_CASE(17)
#undef MIG_ADJ_CASE
    default: return MIG_E_ARG;
    }
}

int adjoint_chunk(int nx, int M, size_t lds_limit)
{
    // LDS = (2 nx + C (nx + 2M)) complex64
    long long room = (long long)(lds_limit / sizeof(float2)) - 2LL * nx;
    long long c = room / (nx + 2 * M);
    if (c > M + 1) c = M + 1;
    return (int)(c < 1 ? 0 : c);
}

int launch_demigrate(const AdjArgs& a, hipStream_t s)
{
    size_t lds = (size_t)(2 * a.nx + a.chunk * (a.nx + 2 * a.M)) * sizeof(float2);
    if (lds > 65536) {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_demigrate),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return MIG_E_DEVICE;
    }
    hipLaunchKernelGGL(k_demigrate, dim3(a.nw), dim3(512), lds, s, a);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

}  // namespace mig
