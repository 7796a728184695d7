// Adjoint of the migration (demigration): image rows -> surface plane.
//
// With the real inner product <a, b> = Re sum conj(a) b, the image map of
// Algorithm 1, I_k = S E_{k-1} ... E_0 d with (S P)[x] = sum_r Re P[x][r] and
// E_k the Eq. (1) step with output-indexed filters, has the adjoint
//     Q_{nz-1} = S* I'_{nz-1},   Q_k = S* I'_k + E_k^H Q_{k+1},   d' = Q_0,
// where (S* i)[x][r] = i[x] and
//     (E_k^H q)[x] = sum_{n=-M..M} conj(h_{j(x+n,k)}[|n|]) q[x+n]:
// every point x+n contributes through the filter of that point.  A workgroup
// owns one frequency for all depths (walking them backwards).  Three kernels:
//   * folded (nx <= 1024, N <= 35, at most 16 lateral velocity changes per
//     row): the Eq. (1) FIR with each point's own conjugated taps plus exact
//     corrections around the points where the filter changes along x (see
//     the derivation before k_demigrate_fold);
//   * product (same sizes, any velocity; runs when some row has more change
//     points): per step it forms g_m[y] = conj(h_{j(y)}[m]) q[y] for its
//     points in LDS and gathers out[x] = g_0[x] + sum_m (g_m[x-m] + g_m[x+m]);
//   * general (any size): the product form a chunk of taps at a time.
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
// of a row differs from the row below, flag in the slowness sign bit), so the
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
    double sn0, sn1;  // slowness of row k-1, flagged where it differs from row k
    double sp0, sp1;  // the row before (k), flagged where it differs from row k+1
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
    // the other set was last loaded for step k+1: refill it for step k-1
    // where row k-1 may differ from row k+1, i.e. where row k-1 differs from
    // row k or row k from row k+1
    if (!first && k >= 1) {
        if (slowness_changed(L.sn0) || slowness_changed(L.sp0))
            load_taps_adj<M>(ho0, a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk,
                                                                    slowness_value(L.sn0)) * (M + 1));
        if (slowness_changed(L.sn1) || slowness_changed(L.sp1))
            load_taps_adj<M>(ho1, a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk,
                                                                    slowness_value(L.sn1)) * (M + 1));
    }
    const double ci0 = L.i0, ci1 = L.i1;
    // prefetch for step k-1, branch-free (rows clamped; values past the top
    // are never used), so that nothing consumes them before the next step
    const int ks = k >= 2 ? k - 2 : 0, ki = k >= 1 ? k - 1 : 0;
    L.sp0 = L.sn0;
    L.sp1 = L.sn1;
    L.sn0 = a.slow[(size_t)ks * a.ldp + L.c0];
    L.sn1 = a.slow[(size_t)ks * a.ldp + L.c1];
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
    // launched beside the folded kernel: runs only when some row has more
    // change points than that kernel handles (the flag is uniform)
    if (a.dense && *as_global(a.dense) == 0) return;
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
    // the first refill (step nz-3, for step nz-4) compares with row nz-3,
    // whose flag (against row nz-2) is never loaded: the first step moves
    // this flagged placeholder into sp, which makes that refill unconditional
    L.sn0 = L.sn1 = -0.0;
    L.sp0 = L.sp1 = -0.0;
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


// ---------------------------------------------------------------------------
// Folded form.  Write j(y) for the table entry of point y (this frequency,
// row k).  Where j is constant over x-M..x+M, E^H at x is the Eq. (1) FIR
// with the conjugated taps of x itself, folded like the forward step.  In
// general, telescoping h_j(y) - h_j(x) over the points between x and y gives
//   (E^H q)[x] = sum_n conj(h_j(x)[|n|]) q[x+n]                 (own filter)
//     + sum over change points c (j(c) != j(c-1)), with D_c = h_j(c) - h_j(c-1):
//         x = c-d, d = 1..M:     + sum_{e=0..M-d}   conj(D_c[d+e])   q[c+e]
//         x = c+d, d = 0..M-1:   - sum_{e=0..M-d-1} conj(D_c[d+1+e]) q[c-1-e]
// so each change point adds a triangle of M(M+1) products to the 2M outputs
// around it.  In layered media a row has a few change points (they sit where
// an interface or a body crosses it), so the step costs about what the
// forward step costs.  Change points are those of the slowness (a velocity
// change that keeps the entry adds exact zeros).
//
// Mapping: as the forward register-tap kernel (two outputs per thread, plane
// ping-pong in LDS, one barrier per step), with one tap set per output,
// refilled at the end of a step where the row changes.  A wave owns 128
// consecutive outputs and computes the corrections of its own outputs at the
// start of a step: the triangle of a change point is cut into at most 64
// chunks of at most T terms (a fixed table, one chunk per lane, the chunks of
// one output in consecutive lanes); each lane sums its chunk, the chunk sums
// of an output are added at its first chunk's lane (DPP lane shifts) and that
// lane adds the total to the wave's correction row in LDS; each lane adds its
// two entries of the row to its FIR results and clears them.  All of it stays
// within the wave (LDS keeps one wave's accesses in order), so no extra
// barrier is needed, and every sum is formed in a fixed order, so the result
// is run-to-run identical.
// The differences D_c of the next step are built during a step: the entry
// pairs (from the change-point pre-pass) are loaded two steps ahead, the two
// table rows one step ahead, and the differences go to an LDS cache before
// the step's barrier.
// ---------------------------------------------------------------------------
constexpr int adj_chunk_count(int M, int T)
{
    int n = 0;
    for (int d = 1; d <= M; ++d) n += (M - d + 1 + T - 1) / T;
    for (int d = 0; d < M; ++d) n += (M - d + T - 1) / T;
    return n;
}

constexpr int adj_chunk_len(int M)
{
    int T = 1;
    while (adj_chunk_count(M, T) > 64) ++T;
    return T;
}

// Chunk of the triangle that lane `lane` sums: side 0 = outputs left of the
// change point (x = c-d), 1 = right (x = c+d); terms [e0, e0+len); rank =
// position of the chunk among those of its output.  len = 0: no chunk.
struct AdjChunk {
    int side, d, e0, len, rank;
};

__device__ AdjChunk adj_lane_chunk(int lane, int M, int T)
{
    AdjChunk c = {0, 0, 0, 0, 0};
    int idx = 0;
    for (int s = 0; s < 2; ++s) {
        const int d0 = s == 0 ? 1 : 0, d1 = s == 0 ? M + 1 : M;
        for (int d = d0; d < d1; ++d) {
            const int t = s == 0 ? M - d + 1 : M - d;
            for (int e = 0, q = 0; e < t; e += T, ++q, ++idx)
                if (idx == lane) c = AdjChunk{s, d, e, t - e < T ? t - e : T, q};
        }
    }
    return c;
}

// Two outputs x0, x0+1 of the folded FIR with conjugated taps,
// sum_n conj(h[n]) (w[M-n] + w[M+n]), from the window w[i] = P[x0 - M + i]
// (16-byte LDS reads); the conjugation is a sign in the multiply-adds.  Two
// passes (taps 0..P, then P+1..M), each reading only the window part it uses,
// with a scheduling barrier between them: the whole window would take 72
// registers next to the two tap sets.
template <int M, int LO, int HI>
__device__ __forceinline__ void fold2_pass(const float4* __restrict__ w4, const float2 (&h0)[M + 1],
                                           const float2 (&h1)[M + 1], float2& a0, float2& a1)
{
    // window indices this pass reads: out0 uses M-n, M+n; out1 M+1-n, M+1+n
    constexpr int lo = M - HI, hi = M + 1 + HI;                 // outer bounds
    constexpr int ilo = lo / 2, ihi = hi / 2;
    float2 w[2 * M + 2];
#pragma unroll
    for (int i = ilo; i <= ihi; ++i) {
        const bool inner_gap = LO > 0 && 2 * i > M - LO + 1 && 2 * i + 1 < M + LO;
        if (inner_gap) continue;
        // a native 4-float vector keeps the read one 16-byte LDS access (the
        // HIP float4 struct is copied field by field, and 8-byte reads at a
        // 16-byte lane stride conflict on the banks)
        typedef float v4f __attribute__((ext_vector_type(4)));
        const v4f q = *reinterpret_cast<const v4f*>(w4 + i);
        w[2 * i] = make_float2(q.x, q.y);
        w[2 * i + 1] = make_float2(q.z, q.w);
    }
#pragma unroll
    for (int n = LO; n <= HI; ++n) {
        if (n == 0) {
            a0.x = fmaf(h0[0].x, w[M].x, a0.x);
            a0.x = fmaf(h0[0].y, w[M].y, a0.x);
            a0.y = fmaf(h0[0].x, w[M].y, a0.y);
            a0.y = fmaf(-h0[0].y, w[M].x, a0.y);
            a1.x = fmaf(h1[0].x, w[M + 1].x, a1.x);
            a1.x = fmaf(h1[0].y, w[M + 1].y, a1.x);
            a1.y = fmaf(h1[0].x, w[M + 1].y, a1.y);
            a1.y = fmaf(-h1[0].y, w[M + 1].x, a1.y);
            continue;
        }
        const float2 s0 = make_float2(w[M - n].x + w[M + n].x, w[M - n].y + w[M + n].y);
        const float2 s1 = make_float2(w[M + 1 - n].x + w[M + 1 + n].x, w[M + 1 - n].y + w[M + 1 + n].y);
        a0.x = fmaf(h0[n].x, s0.x, a0.x);
        a0.x = fmaf(h0[n].y, s0.y, a0.x);
        a0.y = fmaf(h0[n].x, s0.y, a0.y);
        a0.y = fmaf(-h0[n].y, s0.x, a0.y);
        a1.x = fmaf(h1[n].x, s1.x, a1.x);
        a1.x = fmaf(h1[n].y, s1.y, a1.x);
        a1.y = fmaf(h1[n].x, s1.y, a1.y);
        a1.y = fmaf(-h1[n].y, s1.x, a1.y);
    }
}

template <int M>
__device__ __forceinline__ void fold2(const float2* __restrict__ win, const float2 (&h0)[M + 1],
                                      const float2 (&h1)[M + 1], float2& o0, float2& o1)
{
    constexpr int P = M / 2;
    const float4* w4 = reinterpret_cast<const float4*>(win);
    float2 a0 = make_float2(0.0f, 0.0f), a1 = a0;
    fold2_pass<M, 0, P>(w4, h0, h1, a0, a1);
    __builtin_amdgcn_sched_barrier(0);
    fold2_pass<M, P + 1, M>(w4, h0, h1, a0, a1);
    o0 = a0;
    o1 = a1;
}

// LDS of the folded kernel: two planes, a row of corrections per wave (its
// 128 outputs), then per parity the differences D_c[1..M] of each change
// point followed by a zero.
__host__ __device__ constexpr int fold_plane_len(int tsub, int M) { return 2 * tsub + 2 * M + 2; }
__host__ __device__ constexpr int fold_lds_len(int tsub, int M)
{
    return 2 * fold_plane_len(tsub, M) + 2 * tsub + 2 * kAdjKmax * (M + 1);
}
__host__ __device__ constexpr size_t fold_lds(int tsub, int M)
{
    return (size_t)fold_lds_len(tsub, M) * sizeof(float2);
}

// A lane's part in the correction of a change point c: its chunk's terms read
// the differences D_c[1 + dofs[e]] (index M is the zero after them) and the
// values q[c + qofs[e]]; `info` packs side (bit 0), d (bits 1-6), whether the
// lane leads its output's chunks (bit 7) and how many chunks that output has
// (bits 8-15).
template <int T>
struct FoldLane {
    int dofs[T], qofs[T];
    int info;
};

template <int M, int T>
__device__ FoldLane<T> fold_lane(int lane)
{
    const AdjChunk c = adj_lane_chunk(lane, M, T);
    FoldLane<T> L;
    const int terms = c.side ? M - c.d : M - c.d + 1;
    const int nr = (terms + T - 1) / T;
    const int d0 = (c.side ? c.d : c.d - 1) + c.e0;
#pragma unroll
    for (int e = 0; e < T; ++e) {
        const bool in = e < c.len;
        L.dofs[e] = in ? d0 + e : M;
        L.qofs[e] = in ? (c.side ? -(1 + c.e0 + e) : c.e0 + e) : 0;
    }
    L.info = c.side | (c.d << 1) | ((c.len > 0 && c.rank == 0) << 7) | (nr << 8);
    return L;
}

// v of lane l + 1 at lane l (0 at the last lane): a DPP wave shift
__device__ __forceinline__ float lane_next(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}

struct FoldState {
    int t, x0, lane, xw, LB;
    bool ok0, ok1;
    int c0, c1;        // image columns (clamped into the section)
    double ar;
    // loader: thread t builds D_c[m] of change point i, t = i*M + m-1
    bool on;
    int i_ld, m_ld;    // loader role: change point i_ld, tap m_ld
};

// What a step hands to the next one, formed after its FIR from values it
// loaded before the FIR: nothing a step starts with waits for a load (loads
// complete in order, so a wait at the start of a step, or at the end of the
// step before, would also wait for the tap refills issued last).
struct FoldCarry {
    unsigned long long mask;  // the row's change points that reach the wave's outputs (uniform)
    int mp;                   // positions of all the row's change points (lane i: the i-th)
    int nb;                   // change count of the row after (uniform)
    int jp;                   // (left | right << 16) entries of its change point i_ld
    double2 img;              // image row
};

template <int M>
__device__ __forceinline__ void fold_step(const AdjArgs& a, float2* sm, float4* cw, float2* dh,
                                          const FoldState& F, const FoldLane<adj_chunk_len(M)>& CL,
                                          int k_in, float2 (&h)[2][M + 1], FoldCarry& C)
{
    constexpr int T = adj_chunk_len(M);
    constexpr int R = (M + T - 1) / T;
    // the depth index is wave-uniform: keeping it scalar keeps every row
    // address computation on the scalar unit
    const int k = __builtin_amdgcn_readfirstlane(k_in);
    const int nx = a.nx;
    const double2 cimg = C.img;
    // change points of row k that reach this wave's outputs, and row k-1's
    // change count (both formed during the step before)
    const unsigned long long mask0 = C.mask;
    const int mypos = C.mp;
    const int n_build = C.nb;
    const int i_ld = F.i_ld, m_ld = F.m_ld;
    const bool build = k >= 1 && F.on && i_ld < n_build;
    const int LB = F.LB;
    const float2* Pin = sm + ((k + 1) & 1) * LB;
    float2* Pout = sm + (k & 1) * LB + M;
    float4* cwv = cw + (F.t >> 6) * 64;  // this wave's outputs, by pair
    // corrections of this wave's outputs around the change points of row k
    // (Q_{k+1} is complete since the barrier): per change point every lane
    // sums its chunk's T terms (terms past the chunk read the zero after the
    // differences), the chunks of one output (in consecutive lanes) are added
    // at its leading lane and that sum goes to the wave's correction row,
    // change points in increasing order.  They come first in the step, even
    // before the loads are issued, so that their LDS reads go ahead of the
    // other waves' FIR window reads: a wave with corrections is the step's
    // slowest, and behind those reads its own waited for most of a step.
    if (mask0) {
        const float2* dk = dh + (k & 1) * kAdjKmax * (M + 1);
        float* cwf = reinterpret_cast<float*>(cwv);
        const int side = CL.info & 1, d = (CL.info >> 1) & 63, lead = (CL.info >> 7) & 1;
        const int nr = CL.info >> 8;
        unsigned long long mask = mask0;
        while (mask) {
            const int i = __builtin_ctzll(mask);
            mask &= mask - 1;
            const int c = __builtin_amdgcn_readlane(mypos, i);
            const float2* qb = Pin + M + c;
            const float2* db = dk + i * (M + 1);
            float2 hd[T], qv[T];
#pragma unroll
            for (int e = 0; e < T; ++e) {
                hd[e] = db[CL.dofs[e]];
                qv[e] = qb[CL.qofs[e]];
            }
            float2 acc = make_float2(0.0f, 0.0f);
#pragma unroll
            for (int e = 0; e < T; ++e) {
                acc.x = fmaf(hd[e].x, qv[e].x, acc.x);
                acc.x = fmaf(hd[e].y, qv[e].y, acc.x);
                acc.y = fmaf(hd[e].x, qv[e].y, acc.y);
                acc.y = fmaf(-hd[e].y, qv[e].x, acc.y);
            }
            float2 tot = acc, s = acc;
#pragma unroll
            for (int q = 1; q < R; ++q) {
                s = make_float2(lane_next(s.x), lane_next(s.y));
                if (nr > q) {
                    tot.x += s.x;
                    tot.y += s.y;
                }
            }
            if (side) tot = make_float2(-tot.x, -tot.y);
            const int xi = (side ? c + d : c - d) - F.xw;
            if (lead && xi >= 0 && xi < 128) {
                __hip_atomic_fetch_add(cwf + 2 * xi, tot.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                __hip_atomic_fetch_add(cwf + 2 * xi + 1, tot.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            }
        }
    }
    // loader: table rows of row k-1's change points
    float2 hr = make_float2(0.0f, 0.0f), hl = hr;
    if (build) {
        hr = load_global(a.tab + (size_t)((unsigned)C.jp >> 16) * (M + 1) + m_ld);
        hl = load_global(a.tab + (size_t)((unsigned)C.jp & 0xffffu) * (M + 1) + m_ld);
    }
    // loads for this step's end and the next step, branch-free (rows clamped;
    // values past the top are unused): slowness row k-1 (flagged where it
    // differs from row k) for the refill at the end of this step, image row
    // k-1 and its change points, the change count and entries of row k-2
    double2 sn, img_n;
    int cnt_n, mp_n, jp_n;
    {
        const int ks = k >= 1 ? k - 1 : 0, kn = k >= 2 ? k - 2 : 0;
        sn = load_global(reinterpret_cast<const double2*>(a.slow + (size_t)ks * a.ldp + F.x0));
        img_n = make_double2(a.image[(size_t)ks * nx + F.c0], a.image[(size_t)ks * nx + F.c1]);
        // vector loads: as scalar loads their completion would be tracked by
        // the counter the FIR's LDS waits use, and they would wait for them
        int zero = 0;
        asm volatile("" : "+v"(zero));
        cnt_n = *as_global(&a.chg[kn].cnt + zero);
        mp_n = *as_global(&a.chg[ks].pos[F.lane < kAdjKmax ? F.lane : 0]);
        const int il = F.on ? i_ld : 0;
        jp_n = *as_global(a.jpair + ((size_t)kn * a.nw + blockIdx.x) * kAdjKmax + il);
    }
    // own-filter FIR on Q_{k+1} (plane (k+1)&1), plus the image row and the
    // corrections (read back and cleared: LDS keeps one wave's accesses in
    // order, the fence keeps the compiler from moving the read up)
    float2 o0, o1;
    fold2<M>(Pin + F.x0, h[0], h[1], o0, o1);
    o0.x += (float)cimg.x;
    o1.x += (float)cimg.y;
    if (mask0) {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        const float4 c4 = cwv[F.lane];
        o0.x += c4.x;
        o0.y += c4.y;
        o1.x += c4.z;
        o1.y += c4.w;
        cwv[F.lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    }
    if (F.ok0) Pout[F.x0] = o0;
    if (F.ok1) Pout[F.x0 + 1] = o1;
    // the next step's values, formed here (the loads have had the FIR's time);
    // the empty asm statements make each value exist at this point
    __builtin_amdgcn_sched_barrier(0);
    {
        const bool rel = F.lane < n_build && mp_n >= F.xw - M + 1 && mp_n <= F.xw + 127 + M;
        C.mask = __ballot(rel);
        const int c = __builtin_amdgcn_readfirstlane(cnt_n);
        C.nb = c < a.kmax ? c : a.kmax;
        asm volatile("" : "+v"(mp_n), "+v"(jp_n), "+v"(img_n.x), "+v"(img_n.y));
        C.mp = mp_n;
        C.jp = jp_n;
        C.img = img_n;
    }
    if (k >= 1) {
        // differences of row k-1 into the other cache (read from step k-1 on)
        if (build) {
            const int kp = (k - 1) & 1;
            dh[(kp * kAdjKmax + i_ld) * (M + 1) + m_ld - 1] = make_float2(hr.x - hl.x, hr.y - hl.y);
        }
        // taps of step k-1 where row k-1 differs from row k; the FIR of the
        // next step waits for them (mostly L1 hits: the rows of one frequency)
        if (slowness_changed(sn.x))
            load_taps_adj<M>(h[0], a.tab + (size_t)index_of_slowness(F.ar, a.b, a.nk, slowness_value(sn.x)) * (M + 1));
        if (slowness_changed(sn.y))
            load_taps_adj<M>(h[1], a.tab + (size_t)index_of_slowness(F.ar, a.b, a.nk, slowness_value(sn.y)) * (M + 1));
    }
    __syncthreads();
}

template <int M>
__global__ void __launch_bounds__(512) k_demigrate_fold(AdjArgs a)
{
    if (*as_global(a.dense) != 0) return;  // uniform: the product kernel runs
    extern __shared__ float4 smem4[];
    constexpr int T = adj_chunk_len(M);
    const int tsub = blockDim.x, nx = a.nx, nz = a.nz, r = blockIdx.x;
    FoldState F;
    F.LB = fold_plane_len(tsub, M);
    float2* sm = reinterpret_cast<float2*>(smem4);
    float4* cw = reinterpret_cast<float4*>(sm + 2 * F.LB);         // [tsub] (a pair per thread)
    float2* dh = sm + 2 * F.LB + 2 * tsub;                          // [2][kAdjKmax][M+1]
    F.t = threadIdx.x;
    F.x0 = 2 * F.t;
    F.lane = F.t & 63;
    F.xw = (F.t >> 6) * 128;
    F.ok0 = F.x0 < nx;
    F.ok1 = F.x0 + 1 < nx;
    F.c0 = F.ok0 ? F.x0 : 0;
    F.c1 = F.ok1 ? F.x0 + 1 : 0;
    F.ar = a.omega[r] / a.dk;
    const FoldLane<T> CL = fold_lane<M, T>(F.lane);
    const int i_ld = F.t / M, m_ld = F.t - i_ld * M + 1;
    F.i_ld = i_ld;
    F.m_ld = m_ld;
    F.on = i_ld < a.kmax;

    for (int i = F.t; i < fold_lds_len(tsub, M); i += tsub) sm[i] = make_float2(0.0f, 0.0f);
    __syncthreads();
    // Q_{nz-1} = image row nz-1, in plane (nz-1)&1
    {
        float2* P = sm + ((nz - 1) & 1) * F.LB + M;
        if (F.ok0) P[F.x0] = make_float2((float)a.image[(size_t)(nz - 1) * nx + F.x0], 0.0f);
        if (F.ok1) P[F.x0 + 1] = make_float2((float)a.image[(size_t)(nz - 1) * nx + F.x0 + 1], 0.0f);
    }
    // prologue: differences of the first step (row nz-2) into cache
    // (nz-2)&1, its change points for the corrections; entries of row nz-3
    // loaded for the first step's loader
    int k = nz - 2;
    FoldCarry C;
    {
        const int c = a.chg[k].cnt;
        const int n = c < a.kmax ? c : a.kmax;
        if (F.on && i_ld < n) {
            const int jp = a.jpair[((size_t)k * a.nw + r) * kAdjKmax + i_ld];
            const float2 hr = a.tab[(size_t)((unsigned)jp >> 16) * (M + 1) + m_ld];
            const float2 hl = a.tab[(size_t)((unsigned)jp & 0xffffu) * (M + 1) + m_ld];
            dh[((k & 1) * kAdjKmax + i_ld) * (M + 1) + m_ld - 1] = make_float2(hr.x - hl.x, hr.y - hl.y);
        }
        C.mp = a.chg[k].pos[F.lane < kAdjKmax ? F.lane : 0];
        C.mask = __ballot(F.lane < n && C.mp >= F.xw - M + 1 && C.mp <= F.xw + 127 + M);
        const int kn = k >= 1 ? k - 1 : k;
        const int cn = a.chg[kn].cnt;
        C.nb = cn < a.kmax ? cn : a.kmax;
        C.jp = F.on ? a.jpair[((size_t)kn * a.nw + r) * kAdjKmax + i_ld] : 0;
    }
    // taps of the first step (row nz-2)
    float2 h[2][M + 1];
    {
        const double2 s0 = *reinterpret_cast<const double2*>(a.slow + (size_t)k * a.ldp + F.x0);
        load_taps_adj<M>(h[0], a.tab + (size_t)index_of_slowness(F.ar, a.b, a.nk, slowness_value(s0.x)) * (M + 1));
        load_taps_adj<M>(h[1], a.tab + (size_t)index_of_slowness(F.ar, a.b, a.nk, slowness_value(s0.y)) * (M + 1));
    }
    C.img = make_double2(a.image[(size_t)k * nx + F.c0], a.image[(size_t)k * nx + F.c1]);
    __syncthreads();

    for (; k >= 0; --k) fold_step<M>(a, sm, cw, dh, F, CL, k, h, C);
    const float2* P0 = sm + M;  // Q_0 is in plane 0
    if (F.ok0) a.out[(size_t)F.x0 * a.nw + r] = P0[F.x0];
    if (F.ok1) a.out[(size_t)(F.x0 + 1) * a.nw + r] = P0[F.x0 + 1];
}

template <int M>
int launch_fold(const AdjArgs& a, hipStream_t s)
{
    const int tsub = ((a.nx + 1) / 2 + 63) / 64 * 64;
    const size_t lds = fold_lds(tsub, M);
    if (lds > 65536 &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_demigrate_fold<M>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return MIG_E_DEVICE;
    hipLaunchKernelGGL(k_demigrate_fold<M>, dim3(a.nw), dim3(tsub), lds, s, a);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

// Change-point pre-pass, one workgroup per depth row: the first wave lists the
// points where the slowness changes (ballot compaction, increasing x) and
// flags the launch dense past kmax; then every thread forms (left, right)
// table entries of the listed points for its frequencies, with the look-up
// of the depth-stepping kernels.
__global__ void __launch_bounds__(256) k_adj_changes(AdjArgs a)
{
    __shared__ double s_l[kAdjKmax], s_r[kAdjKmax];
    __shared__ int s_n;
    const int k = blockIdx.x;
    const double* srow = a.slow + (size_t)k * a.ldp;
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        int count = 0;
        for (int x0 = 1; x0 < a.nx; x0 += 64) {
            const int x = x0 + lane;
            double sl = 0.0, sr = 0.0;
            bool chg = false;
            if (x < a.nx) {
                sl = slowness_value(srow[x - 1]);
                sr = slowness_value(srow[x]);
                chg = __double_as_longlong(sl) != __double_as_longlong(sr);
            }
            const unsigned long long m = __ballot(chg);
            const int slot = count + __popcll(m & ((1ull << lane) - 1ull));
            if (chg && slot < kAdjKmax) {
                a.chg[k].pos[slot] = x;
                s_l[slot] = sl;
                s_r[slot] = sr;
            }
            count += __popcll(m);
        }
        if (lane == 0) {
            a.chg[k].cnt = count;
            s_n = count < a.kmax ? count : a.kmax;
            if (count > a.kmax)
                __hip_atomic_fetch_or(as_global(a.dense), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    const int n = s_n;
    for (int e = threadIdx.x; e < a.nw * n; e += blockDim.x) {
        const int r = e / n, i = e - r * n;
        const double ar = a.omega[r] / a.dk;
        a.jpair[((size_t)k * a.nw + r) * kAdjKmax + i] =
            (int)((unsigned)index_of_slowness(ar, a.b, a.nk, s_l[i]) |
                  ((unsigned)index_of_slowness(ar, a.b, a.nk, s_r[i]) << 16));
    }
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

bool adjoint_uses_fold(int nx, int M)
{
    return nx <= 2 * kAdjThreads && M >= 1 && M <= kAdjMaxM && adjoint_fold_kmax(nx, M) >= 1;
}

int adjoint_fold_kmax(int nx, int M)
{
    // one loader thread per (change point, tap 1..M)
    const int tsub = ((nx + 1) / 2 + 63) / 64 * 64;
    const int k = M >= 1 ? tsub / M : 0;
    return k < kAdjKmax ? k : kAdjKmax;
}

int launch_adj_changes(const AdjArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_changes, dim3(a.nz - 1), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

int launch_demigrate_fold(const AdjArgs& a, hipStream_t s)
{
    switch (a.M) {
#define MIG_FOLD_CASE(m) \
    case m: return launch_fold<m>(a, s);
    MIG_FOLD_CASE(1) MIG_FOLD_CASE(2) MIG_FOLD_CASE(3) MIG_FOLD_CASE(4)
    MIG_FOLD_CASE(5) MIG_FOLD_CASE(6) MIG_FOLD_CASE(7) MIG_FOLD_CASE(8) MIG_FOLD_CASE(9)
    MIG_FOLD_CASE(10) MIG_FOLD_CASE(11) MIG_FOLD_CASE(12) MIG_FOLD_CASE(13) MIG_FOLD_CASE(14)
    MIG_FOLD_CASE(15) MIG_FOLD_CASE(16) MIG_FOLD_CASE(17)
#undef MIG_FOLD_CASE
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
