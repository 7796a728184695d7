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
// forms g_m[y] = conj(h_{j(y)}[m]) q[y] for its points in LDS, a chunk of m
// at a time, and gathers out[x] = g_0[x] + sum_m (g_m[x-m] + g_m[x+m]).
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

}  // namespace

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
