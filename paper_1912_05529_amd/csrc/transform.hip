// Transform along t of a zero-offset section (Algorithm 1, first step:
// "Fourier transform ... along t-axis"), evaluated directly at the requested
// frequencies:  P[x][r] = sum_n p[x][n] exp(-i omega_r n dt).
//
// The frequencies need not be FFT bins, so this is a dense contraction
//     C[nx][2 nw] = A[nx][nt] . B[nt][2 nw],
//     B[n][2r] = cos(omega_r n dt),  B[n][2r+1] = -sin(omega_r n dt),
// whose row-major result is exactly the interleaved complex64 plane [nx][nw].
// B is built once per call in FP64 (phases up to thousands of radians) and
// rounded to FP32; the product runs on the matrix cores with
// v_mfma_f32_16x16x4f32 (FP32 in, FP32 accumulate): 64 x 64 output tiles per
// 256-thread workgroup, each wavefront a 32 x 32 quadrant (2 x 2 MFMA tiles),
// K staged through LDS 16 at a time with zero padding at the ragged edges.
#include "common.hpp"

namespace mig {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;
constexpr int kK = 16;

__global__ void k_dft_matrix(const double* __restrict__ omega, int nw, int nt, double dt,
                             float* __restrict__ B)
{
    const size_t total = (size_t)nt * nw;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int n = (int)(e / nw), r = (int)(e % nw);
        double s, c;
        sincos(omega[r] * ((double)n * dt), &s, &c);
        B[(size_t)n * 2 * nw + 2 * r] = (float)c;
        B[(size_t)n * 2 * nw + 2 * r + 1] = (float)-s;
    }
}

// MFMA 16x16x4 operand layout (lane l of a wavefront): A element
// (row l % 16, k l / 16), B element (k l / 16, column l % 16); result lane l
// holds D[4 (l / 16) + v][l % 16], v = 0..3.
__global__ void __launch_bounds__(256) k_gemm_mfma(const float* __restrict__ A,
                                                   const float* __restrict__ B,
                                                   float* __restrict__ C, int M, int N, int K)
{
    __shared__ float As[kTile][kK + 1];
    __shared__ float Bs[kK][kTile + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int row0 = blockIdx.y * kTile, col0 = blockIdx.x * kTile;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    for (int k0 = 0; k0 < K; k0 += kK) {
        for (int e = threadIdx.x; e < kTile * kK; e += blockDim.x) {
            const int r = e / kK, c = e % kK;
            const int gr = row0 + r, gc = k0 + c;
            As[r][c] = (gr < M && gc < K) ? A[(size_t)gr * K + gc] : 0.0f;
        }
        for (int e = threadIdx.x; e < kK * kTile; e += blockDim.x) {
            const int r = e / kTile, c = e % kTile;
            const int gr = k0 + r, gc = col0 + c;
            Bs[r][c] = (gr < K && gc < N) ? B[(size_t)gr * N + gc] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kK; kk += 4) {
            const int k = kk + (lane >> 4);
            float a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[wr * 32 + i * 16 + (lane & 15)][k];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[k][wc * 32 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = row0 + wr * 32 + i * 16 + 4 * (lane >> 4) + v;
                const int c = col0 + wc * 32 + j * 16 + (lane & 15);
                if (r < M && c < N) C[(size_t)r * N + c] = acc[i][j][v];
            }
}

}  // namespace

int launch_transform(const float* section, int nx, int nt, double dt, const double* omega,
                     int nw, float2* out, float* B, hipStream_t s)
{
    size_t total = (size_t)nt * nw;
    size_t blocks = (total + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_dft_matrix, dim3((unsigned)blocks), dim3(256), 0, s, omega, nw, nt, dt, B);
    if (hipGetLastError() != hipSuccess) return MIG_E_DEVICE;
    const int N = 2 * nw;
    dim3 grid((N + kTile - 1) / kTile, (nx + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_gemm_mfma, grid, dim3(256), 0, s, section, B,
                       reinterpret_cast<float*>(out), nx, N, nt);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

}  // namespace mig
