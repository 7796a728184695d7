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
// L2 latency of a refill hides behind a whole step.  The products live in
// two LDS arrays, one for even and one for odd points, so that every LDS
// access of a wave -- the stores of a thread's two points and each gather of
// a neighbour at any shift -- touches consecutive 8-byte words across the
// lanes: free of bank conflicts, which with the points interleaved took half
// of the LDS cycles.
constexpr int kAdjThreads = 512;
constexpr int kAdjMaxM = 17;

// Halo, in point pairs, on each side of the product arrays: the gather reaches
// (M+1)/2 pairs away.
__host__ __device__ constexpr int adj_halo(int M) { return (M + 2) / 2; }

// LDS bytes of the register-tap kernel: products at even and odd points.
__host__ __device__ constexpr size_t adj_reg_lds(int nx, int M)
{
    return (size_t)2 * (M + 1) * ((nx + 1) / 2 + 2 * adj_halo(M)) * sizeof(float2);
}

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
__device__ __forceinline__ void adj_step(const AdjArgs& a, float2* G, int LP, AdjLane& L, int k,
                                         float2 (&hc0)[M + 1], float2 (&hc1)[M + 1],
                                         float2 (&ho0)[M + 1], float2 (&ho1)[M + 1], float2& q0,
                                         float2& q1, bool first)
{
    constexpr int kH = adj_halo(M);
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
    // E[m][H + p] = g_m[2p], O[m][H + p] = g_m[2p + 1]: thread t owns pair t.
    // q1 = 0 when y0 + 1 is past the end: the store keeps that point zero
    float2* E = G;
    float2* O = G + (size_t)(M + 1) * LP;
    const int t = threadIdx.x;
    if (L.live0) {
#pragma unroll
        for (int m = 0; m <= M; ++m) {
            E[(size_t)m * LP + kH + t] = cmul_conj(hc0[m], q0);
            O[(size_t)m * LP + kH + t] = cmul_conj(hc1[m], q1);
        }
    }
    __syncthreads();
    // out[2t] and out[2t+1] = g_0 + sum_m g_m[x - m] + g_m[x + m]: for m = 2s the
    // neighbours of 2t are even points (pairs t -+ s) and those of 2t+1 odd
    // ones; for m = 2s+1 they swap (pairs t-s-1, t+s and t-s, t+s+1).  Two
    // partial sums per output (taps m odd / m even) halve the chain of
    // dependent additions.
    float2 a0 = make_float2((float)ci0, 0.0f), a1 = make_float2((float)ci1, 0.0f);
    if (L.live0) {
        const float2* e = E + kH + t;
        const float2* o = O + kH + t;
        float2 se0 = e[0], so0 = make_float2(0.0f, 0.0f);
        float2 se1 = o[0], so1 = make_float2(0.0f, 0.0f);
#pragma unroll
        for (int m = 1; m <= M; ++m) {
            const int sh = m >> 1;
            const float2* em = e + (size_t)m * LP;
            const float2* om = o + (size_t)m * LP;
            float2 l0, r0, l1, r1;
            if (m & 1) {
                l0 = om[-sh - 1];
                r0 = om[sh];
                l1 = em[-sh];
                r1 = em[sh + 1];
            } else {
                l0 = em[-sh];
                r0 = em[sh];
                l1 = om[-sh];
                r1 = om[sh];
            }
            float2& u0 = (m & 1) ? so0 : se0;
            float2& u1 = (m & 1) ? so1 : se1;
            u0.x += l0.x + r0.x;
            u0.y += l0.y + r0.y;
            u1.x += l1.x + r1.x;
            u1.y += l1.y + r1.y;
        }
        a0.x += se0.x + so0.x;
        a0.y += se0.y + so0.y;
        a1.x += se1.x + so1.x;
        a1.y += se1.y + so1.y;
    }
    __syncthreads();
    q0 = L.live0 ? a0 : make_float2(0.0f, 0.0f);
    q1 = L.live1 ? a1 : make_float2(0.0f, 0.0f);
}

template <int M>
__global__ void __launch_bounds__(kAdjThreads) k_demigrate_reg(AdjArgs a)
{
    extern __shared__ float4 smem4[];
    // [2][M+1][LP]: products at even and odd points, LP = pairs + 2 kH, zero
    // outside the points of the section
    constexpr int kH = adj_halo(M);
    float2* G = reinterpret_cast<float2*>(smem4);
    const int nx = a.nx, LP = (nx + 1) / 2 + 2 * kH, r = blockIdx.x;
    AdjLane L;
    L.ar = a.omega[r] / a.dk;
    L.y0 = 2 * threadIdx.x;
    L.live0 = L.y0 < nx;
    L.live1 = L.y0 + 1 < nx;
    L.c0 = L.live0 ? L.y0 : 0;
    L.c1 = L.live1 ? L.y0 + 1 : 0;

    for (int i = threadIdx.x; i < 2 * (M + 1) * LP; i += blockDim.x) G[i] = make_float2(0.0f, 0.0f);
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
        adj_step<M>(a, G, LP, L, k, hA0, hA1, hB0, hB1, q0, q1, first);
        first = false;
        if (k == 0) break;
        adj_step<M>(a, G, LP, L, k - 1, hB0, hB1, hA0, hA1, q0, q1, false);
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
    return nx <= 2 * kAdjThreads && M >= 1 && M <= kAdjMaxM && adj_reg_lds(nx, M) <= lds_limit;
}

int launch_demigrate_reg(const AdjArgs& a, hipStream_t s)
{
    const size_t lds = adj_reg_lds(a.nx, a.M);
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
