// Transform along t of a zero-offset section (the first step of Algorithm 1),
// evaluated directly at the requested frequencies:
//     P[x][r] = sum_n p[x][n] exp(-i omega_r n dt).
//
// The frequencies need not be FFT bins, so this is a dense contraction
//     C[nx][2 nw] = A[nx][nt] . B[nt][2 nw],
//     B[n][2r] = cos(omega_r n dt),  B[n][2r+1] = -sin(omega_r n dt),
// whose row-major result is exactly the interleaved complex64 plane [nx][nw].
// B is built once per call in FP64 (phases up to thousands of radians) and
// rounded to FP32; the product runs on the matrix cores with
// v_mfma_f32_16x16x4f32 (FP32 in, FP32 accumulate).
#include "common.hpp"

namespace mig {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// B in runs of kDftRun consecutive n per thread: sincos in FP64 at the run's
// first n and for one step of omega dt, then the run by FP64 rotation (error
// ~1e-16 per step, far below the FP32 rounding of the entries).  Consecutive
// threads take consecutive frequencies, so each row of B is written coalesced.
constexpr int kDftRun = 16;

__global__ void k_dft_matrix(const double* __restrict__ omega, int nw, int nt, double dt,
                             float* __restrict__ B)
{
    const int nrun = (nt + kDftRun - 1) / kDftRun;
    const size_t total = (size_t)nrun * nw;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e % nw), n0 = (int)(e / nw) * kDftRun;
        double s, c, sd, cd;
        sincos(omega[r] * ((double)n0 * dt), &s, &c);
        sincos(omega[r] * dt, &sd, &cd);
        const int n1 = n0 + kDftRun < nt ? n0 + kDftRun : nt;
        for (int n = n0; n < n1; ++n) {
            B[(size_t)n * 2 * nw + 2 * r] = (float)c;
            B[(size_t)n * 2 * nw + 2 * r + 1] = (float)-s;
            const double c2 = c * cd - s * sd;
            s = s * cd + c * sd;
            c = c2;
        }
    }
}

// Main kernel: 64 x 32 output block per 256-thread workgroup, each wave a
// 16 x 32 strip (1 x 2 MFMA tiles), so that the grid spreads over every CU;
// k in chunks of 64 copied global -> LDS by buffer-to-LDS loads (no registers
// on the way), four chunk buffers in flight: chunk c+3 is requested while
// chunk c is multiplied.  Elements past the ragged edges (rows >= M, columns
// >= N, k >= K) are read at an offset pushed out of the buffer's range and
// arrive as zeros.  The buffer resources are rebased for every chunk at the
// workgroup's first row and the chunk's first k, so offsets stay below 2^30
// for nt <= MIG_MAX_NT and any nw <= MIG_MAX_NW.
//
// LDS: A chunk [64 rows][64 k], the 16-byte k-groups of row r stored at slot
// group ^ (r & 7), so that the eight rows a 16-byte MFMA-operand read touches
// per cycle land on different banks; B chunk [64 k][32 columns], column c of
// k row kr stored at c ^ 16 ((kr >> 2) & 1), so that the 32 lanes of a B-operand
// read (k rows 4 apart) cover all 32 banks.
constexpr int kGM = 64;          // output rows per workgroup
constexpr int kGN = 32;          // output columns per workgroup
constexpr int kGK = 64;          // k per chunk
constexpr int kGChunkF = kGM * kGK + kGK * kGN;   // floats per chunk buffer (A then B)
constexpr int kGBuf = 4;         // chunk buffers
constexpr int kOOR = 0x40000000; // byte offset past any buffer this kernel reads

typedef __attribute__((address_space(3))) void* lds_ptr_t;
constexpr int kRawWord3 = 0x00020000;

// Copy instructions per wave per chunk: 16-byte copies (X4, K and N multiples of
// 4: every 4-float group wholly inside or wholly past the edges) or 4-byte ones.
template <bool X4>
constexpr int gemm_copies() { return X4 ? 6 : 24; }

// Resources for the chunk at k0: A from row row0, column k0; B from row k0,
// column col0 (64-bit bases, so the 32-bit offsets stay small).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t chunk_rsrc(const float* base, size_t first,
                                                             size_t total)
{
    const size_t left = total > first ? (total - first) * 4 : 0;
    const int nrec = left < (size_t)kOOR ? (int)left : kOOR;
    return __builtin_amdgcn_make_buffer_rsrc((void*)(base + first), 0, nrec, kRawWord3);
}

template <bool X4>
__device__ __forceinline__ void gemm_copy_chunk(float* buf, const float* __restrict__ A,
                                                const float* __restrict__ B, int M, int N, int K,
                                                int row0, int col0, int k0, int wave, int lane)
{
    static_assert(kGK == 64 && kGM == 64 && kGN == 32, "copy pattern");
    const __amdgpu_buffer_rsrc_t ra = chunk_rsrc(A, (size_t)row0 * K + k0, (size_t)M * K);
    const __amdgpu_buffer_rsrc_t rb = chunk_rsrc(B, (size_t)k0 * N + col0, (size_t)K * N);
    float* bb = buf + kGM * kGK;
    if constexpr (X4) {
        // A: wave w copies rows 16w .. 16w+15, four rows (16 groups each) per
        // instruction
        const int s16 = lane & 15, r4 = lane >> 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 16 * wave + 4 * q + r4;
            const int k = k0 + 4 * (s16 ^ (r & 7));
            const int gr = row0 + r;
            const int off = (gr < M && k < K) ? (r * K + (k - k0)) * 4 : kOOR;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_ptr_t)(buf + (16 * wave + 4 * q) * kGK),
                                                     16, off, 0, 0, 0);
        }
        // B: wave w copies k rows 16w .. 16w+15, eight rows per instruction
        const int s8 = lane & 7, r8 = lane >> 3;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int kr = 16 * wave + 8 * q + r8;
            const int k = k0 + kr, c = col0 + 4 * (s8 ^ (((kr >> 2) & 1) << 2));
            const int off = (k < K && c < N) ? (kr * N + (c - col0)) * 4 : kOOR;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_ptr_t)(bb + (16 * wave + 8 * q) * kGN),
                                                     16, off, 0, 0, 0);
        }
        return;
    }
    // A: wave w copies rows 16w .. 16w+15, one row per instruction
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int r = 16 * wave + q;
        const int k = k0 + 4 * ((lane >> 2) ^ (r & 7)) + (lane & 3);
        const int gr = row0 + r;
        const int off = (gr < M && k < K) ? (r * K + (k - k0)) * 4 : kOOR;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_ptr_t)(buf + r * kGK), 4, off, 0, 0, 0);
    }
    // B: wave w copies k rows 16w .. 16w+15, two rows of 32 columns per
    // instruction
    const int half = lane >> 5, p = lane & 31;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int kr = 16 * wave + 2 * q + half;
        const int k = k0 + kr, c = col0 + (p ^ (((kr >> 2) & 1) << 4));
        const int off = (k < K && c < N) ? (kr * N + (c - col0)) * 4 : kOOR;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_ptr_t)(bb + (16 * wave + 2 * q) * kGN), 4,
                                                 off, 0, 0, 0);
    }
}

// vmcnt(2 copies): all but this wave's copies of the two newest chunks are
// complete (vmcnt[3:0] | vmcnt[5:4] in bits 15:14).
template <bool X4>
__device__ __forceinline__ void wait_all_but_two_chunks()
{
    constexpr int n = 2 * gemm_copies<X4>();
    static_assert(n < 64, "vmcnt field");
    __builtin_amdgcn_s_waitcnt((n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14));
}

__device__ __forceinline__ void barrier_lds()
{
    __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (0 << 8) | (3 << 14));  // lgkmcnt(0)
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <bool X4>
__global__ void __launch_bounds__(256) k_gemm_lds(const float* __restrict__ A,
                                                  const float* __restrict__ B,
                                                  float* __restrict__ C, int M, int N, int K)
{
    __shared__ float buf[kGBuf][kGChunkF];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int row0 = blockIdx.y * kGM, col0 = blockIdx.x * kGN;
    const int g = lane >> 4, l16 = lane & 15;
    f32x4 acc[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    // Chunk copies are issued unconditionally (chunks past the end read only
    // out-of-range offsets, i.e. zeros, into a buffer nobody reads), so that
    // exactly two chunks' copies are always newer than those of the chunk in
    // use.
    const int nch = (K + kGK - 1) / kGK;
#pragma unroll
    for (int q = 0; q < kGBuf - 1; ++q)
        gemm_copy_chunk<X4>(buf[q], A, B, M, N, K, row0, col0, q * kGK, wave, lane);
    const int r = 16 * wave + l16;   // this lane's A row in the block
    for (int c = 0; c < nch; ++c) {
        // this wave's copies of chunk c are in; after the barrier every wave's
        // are, and every wave is done with chunk c-1, whose buffer takes
        // chunk c+3
        wait_all_but_two_chunks<X4>();
        barrier_lds();
        gemm_copy_chunk<X4>(buf[(c + kGBuf - 1) % kGBuf], A, B, M, N, K, row0, col0,
                        (c + kGBuf - 1) * kGK, wave, lane);
        const float* a = buf[c % kGBuf];
        const float* b = a + kGM * kGK;
#pragma unroll
        for (int h = 0; h < kGK / 16; ++h) {
            const f32x4 av = *reinterpret_cast<const f32x4*>(a + r * kGK + 4 * ((4 * h + g) ^ (r & 7)));
            float bv[2][4];
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    bv[t][j] = b[(16 * h + 4 * g + j) * kGN + ((16 * t + l16) ^ ((g & 1) << 4))];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int t = 0; t < 2; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[j], bv[t][j], acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rr = row0 + 16 * wave + 4 * g + v;
            const int cc = col0 + 16 * t + l16;
            if (rr < M && cc < N) C[(size_t)rr * N + cc] = acc[t][v];
        }
}

}  // namespace

int launch_transform(const float* section, int nx, int nt, double dt, const double* omega,
                     int nw, float2* out, float* B, hipStream_t s)
{
    size_t total = (size_t)((nt + kDftRun - 1) / kDftRun) * nw;
    size_t blocks = (total + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_dft_matrix, dim3((unsigned)blocks), dim3(256), 0, s, omega, nw, nt, dt, B);
    if (hipGetLastError() != hipSuccess) return MIG_E_DEVICE;
    const int N = 2 * nw;
    dim3 grid((N + kGN - 1) / kGN, (nx + kGM - 1) / kGM);
    if ((nt & 3) == 0 && (N & 3) == 0)  // every 4-float group wholly in or past the edges
        hipLaunchKernelGGL(k_gemm_lds<true>, grid, dim3(256), 0, s, section, B,
                           reinterpret_cast<float*>(out), nx, N, nt);
    else
        hipLaunchKernelGGL(k_gemm_lds<false>, grid, dim3(256), 0, s, section, B,
                           reinterpret_cast<float*>(out), nx, N, nt);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

}  // namespace mig
