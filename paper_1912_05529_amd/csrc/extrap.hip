// Depth stepping (Eq. 1 with per-point filters), imaging and table look-up.
//
// Design (MI355X / gfx950):
//   * Frequencies never interact during extrapolation (Sec. II: the process
//     runs independently for each frequency), only through the image sum.  So
//     a frequency is owned by one workgroup for the whole depth range: its
//     plane (nx complex64, a few KB) stays in LDS, depth steps are separated by
//     a workgroup barrier instead of a kernel exit (the "block level
//     synchronization" the paper names as future work, Sec. V), and there is
//     no traffic between frequency workgroups.
//   * A workgroup item owns G frequencies of one section (G sub-groups of
//     `tsub` threads; G > 1 fills a workgroup when nx is small).  Items of many
//     sections of different nx, nz and nw run in one launch (the batched form).
//   * Lanes run along x (coalesced, conflict-free LDS windows); each thread
//     owns two (or four) adjacent outputs and reads its window with 16-byte LDS
//     loads.  Even taps are folded: h_n (u[x-n] + u[x+n]).
//   * Taps live in registers.  The filter of an output only changes when the
//     velocity under it changes (omega is fixed per sub-group), which in
//     layered media is a few times per column.  Two register sets alternate
//     between even and odd steps; the set for step k+1 is refilled during step
//     k only for outputs whose slowness changed, so table reads (L2-resident)
//     are rare and their latency is hidden behind a full step of arithmetic.
//     All vector-memory operations of a step are issued at its start (last
//     step's partial row, refills, slowness prefetch), so one wait at the top
//     of the next step finds them long complete.
//   * The look-up needs 1/v in FP64; it is computed once per (depth, x) by a
//     small pre-pass (shared by all frequencies) instead of once per refill.
//   * The image row needs a sum over frequencies, i.e. across workgroups.
//     Each frequency sub-group writes Re of its new plane (float32, exact) to a
//     partial buffer [step][omega][x], write-through; every kPublish steps the
//     workgroup publishes its progress (its stores complete, then a counter
//     increment).  Reducer workgroups in the same launch -- the first
//     workgroups of the grid, so they run beside the frequency workgroups from
//     the start even when items outnumber the CUs -- take blocks in the order
//     they are expected to be published, wait for a block of steps to be
//     published by every workgroup of the section, acquire, and sum it over
//     omega in increasing order in FP64, so images are run-to-run identical
//     and the reduction overlaps the extrapolation; the last block of a plain
//     launch is summed after it (k_rows) by the whole GPU.  Frequency
//     workgroups never wait on anyone; reducer waits are bounded: after
//     kStallTicks (or the caller's limit) without any publish in the launch,
//     the launch is abandoned as a whole -- every remaining task writes NaN
//     rows without waiting -- and the call's status word says so.
#include "common.hpp"

namespace mig {
namespace {

// s_waitcnt vmcnt(0), other counters left alone (GFX9 encoding:
// vmcnt[3:0] | expcnt[6:4] | lgkmcnt[11:8] | vmcnt[5:4] in bits 15:14).
__device__ __forceinline__ void wait_vmem_all()
{
    __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));
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

// Partial image rows are stored write-through (agent-scope relaxed atomic
// stores): reducers on other XCDs read them once their block is counted, and
// nothing of them is left in this XCD's L2 to write back first.
__device__ __forceinline__ void store_partial2(float* p, float a, float b)
{
    const unsigned long long u =
        (unsigned long long)__float_as_uint(a) | ((unsigned long long)__float_as_uint(b) << 32);
    __hip_atomic_store(as_global(reinterpret_cast<unsigned long long*>(p)), u, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
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

// Q adjacent outputs x0..x0+Q-1 from the window w[i] = P[x0 - M + i],
// i = 0..2M+Q-1.  Even Q: x0 is even, so the window is read with 16-byte LDS
// loads; odd Q (x0 of either parity): 8-byte loads.
template <int M, int Q>
__device__ __forceinline__ void firq(const float2* __restrict__ win, const float2 (&h)[Q][M + 1],
                                     float2 (&o)[Q])
{
    float2 w[2 * M + Q];
    if constexpr (Q % 2 == 0) {
        const float4* w4 = reinterpret_cast<const float4*>(win);
#pragma unroll
        for (int i = 0; i < M + Q / 2; ++i) {
            float4 q = w4[i];
            w[2 * i] = make_float2(q.x, q.y);
            w[2 * i + 1] = make_float2(q.z, q.w);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 2 * M + Q; ++i) w[i] = win[i];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) o[q] = cmulf(h[q][0], w[M + q]);
#pragma unroll
    for (int n = 1; n <= M; ++n) {
#pragma unroll
        for (int q = 0; q < Q; ++q) o[q] = cfmaf(h[q][n], cadd(w[M + q - n], w[M + q + n]), o[q]);
    }
}

__device__ __forceinline__ SecDev sec_of(const BatchArgs& a, int i)
{
    return a.nsec == 1 ? a.one : a.secs[i];
}

__device__ __forceinline__ ItemDev item_of(const BatchArgs& a, int i)
{
    return a.nsec == 1 ? ItemDev{0, i * a.one.G} : a.items[i];
}

__device__ __forceinline__ TaskDev task_of(const BatchArgs& a, int i)
{
    if (a.nsec != 1) return a.tasks[i];
    const int p = i % a.parts;
    const int span = ((a.one.nx + a.parts - 1) / a.parts + 1) & ~1;  // even part width
    const int x0 = p * span;
    return TaskDev{0, i / a.parts, x0, x0 + span < a.one.nx ? x0 + span : a.one.nx};
}

// Per-workgroup constants: frequencies per workgroup and sub-group size.
__device__ __forceinline__ void group_shape(const SecDev& S, int kind, int& G, int& tsub)
{
    const int q = kind == 1 ? 2 : (kind == 2 ? 4 : 3);  // outputs per thread
    tsub = ((S.nx + q - 1) / q + 63) / 64 * 64;
    G = S.G;
}

// slow[k][x] = slowness_of(vel[k][min(x, nx-1)]) for x < ldp, every section,
// with the sign bit set where it differs (bitwise) from row k - dist (when
// that row exists); also
// zeroes each section's block counters (one launch fewer before the depth
// stepping).
__global__ void k_slowness(BatchArgs a, int dist)
{
    const SecDev S = sec_of(a, blockIdx.y);
    // the section's published-block counters start the coming launch at zero
    if (S.cnt && blockIdx.x == 0)
        for (int i = threadIdx.x; i < (S.nsteps + kPublish - 1) / kPublish; i += blockDim.x)
            S.cnt[i] = 0;
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        if (a.progress) {
            a.progress[0] = 0;
            a.progress[1] = 0;
        }
        if (a.status && a.reset_status) *a.status = 0;
    }
    double* slow = const_cast<double*>(S.slow);
    const size_t total = (size_t)S.nsteps * S.ldp;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        size_t k = e / S.ldp;
        int x = (int)(e % S.ldp);
        const int xc = x < S.nx ? x : S.nx - 1;
        double v = slowness_of(S.vel[k * S.nx + xc]);
        long long bits = __double_as_longlong(v);
        // dist > 0: flag against the row dist steps earlier (depth stepping
        // downward); dist < 0: against the row -dist steps later (the adjoint
        // walks upward)
        const long long kr = (long long)k - dist;
        if (dist != 0 && kr >= 0 && kr < S.nsteps) {
            long long prev = __double_as_longlong(slowness_of(S.vel[(size_t)kr * S.nx + xc]));
            if (bits != prev) bits |= (long long)kSignBit;
        }
        slow[e] = __longlong_as_double(bits);
    }
}

// Thread 0 of a frequency workgroup, after a barrier that follows the stores of
// the partial rows of block c: count the block (and the launch's publishes).  The partial rows are stored
// write-through (agent-scope atomic stores) and every wave waits for its own
// stores to complete before that barrier (wait_vmem_all), so when the counter
// moves the rows are already where other XCDs read them.  No release fence:
// at agent scope it would write back the whole L2 of the XCD, which the
// barrier after the next step would make every wave of the workgroup wait for.
__device__ __forceinline__ void publish_block(const BatchArgs& a, const SecDev& S, int c)
{
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(as_global(S.cnt + c), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(as_global(a.progress), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Block b (steps 32b .. 32b+31) is published at the end of step 32b+33: its
// last partial row was stored at the start of step 32b+32, the wait for all
// memory operations at the start of step 32b+33 covers it, and the barrier
// ending that step means every wave of the workgroup has passed that wait.
// So no extra wait stands in the loop.  Blocks whose publishing step lies
// past the last step are published after the loop.
__device__ __forceinline__ bool publishes_at(int k) { return k >= kPublish + 1 && k % kPublish == 1; }
__device__ __forceinline__ int published_in_loop(int nsteps)
{
    return nsteps - 1 >= kPublish + 1 ? (nsteps - 1 - (kPublish + 1)) / kPublish + 1 : 0;
}

__device__ __forceinline__ int load_relaxed(int* p)
{
    return __hip_atomic_load(as_global(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0 of a reducer: wait until block T.block of section S is published
// by all its frequency workgroups.  Returns false when the launch has been
// abandoned: by this reducer, after kStallTicks (or the caller's limit)
// without any publish in the launch, or by another reducer before.  The
// first reducer to give up sets the launch's abandon word and the call's
// status word; every later wait of the launch returns at once.
__device__ bool wait_block(const BatchArgs& a, const SecDev& S, int block)
{
    int* const abandon = a.progress + 1;
    const int need = S.nprod + a.extra_wait;
    int v, last = -1, seen = -1;
    unsigned long long t0 = wall_clock64();
    while ((v = load_relaxed(S.cnt + block)) < need) {
        if (load_relaxed(abandon) != 0) return false;
        // the stall clock restarts whenever the block's counter or the
        // launch's publish count moves: a section whose items start late in
        // a long batch is waited for, a launch that stops is not
        const int g = load_relaxed(a.progress);
        const unsigned long long now = wall_clock64();
        if (v != last || g != seen) {
            last = v;
            seen = g;
            t0 = now;
        } else if (now - t0 > a.stall_ticks) {
            __hip_atomic_store(as_global(abandon), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (a.status)
                __hip_atomic_store(as_global(a.status), kStatusAbandoned, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(kPollSleep);
    }
    return true;
}

// Reducer workgroup q of a.nred: tasks q, q + nred, ... (ordered block-major
// across sections, i.e. in production order).  One wait and one acquire per
// task: an acquire invalidates the L2 of the reducer's XCD, which the
// frequency workgroups there pay for in table refills, so tasks are whole
// published blocks (split along x only when there are few blocks).
constexpr int kRedDepth = 32;

__device__ void reduce_role(const BatchArgs& a, int q, int* flag)
{
    for (int i = q; i < a.ntasks; i += a.nred) {
        const TaskDev T = task_of(a, i);
        const SecDev S = sec_of(a, T.sec);
        if (T.block * kPublish >= S.nsteps) continue;  // no such block (uniform)
        if (threadIdx.x == 0) {
            const bool ok = wait_block(a, S, T.block);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            *flag = ok ? 1 : 0;
        }
        __syncthreads();
        const bool ok = *flag != 0;
        __syncthreads();
        const int s0 = T.block * kPublish;
        const int s1 = s0 + kPublish < S.nsteps ? s0 + kPublish : S.nsteps;
        const int npair = (T.x1 - T.x0 + 1) / 2;
        const int items = (s1 - s0) * npair;
        for (int it = threadIdx.x; it < items; it += blockDim.x) {
            const int st = s0 + it / npair;
            const int x0 = T.x0 + 2 * (it % npair);
            const float* p = S.part + (size_t)st * S.nw * S.ldp;
            __attribute__((address_space(1))) double* row = as_global(S.rows + (size_t)st * S.nx);
            // kRedDepth loads in flight per thread (the reads are latency-bound);
            // rows past nw are clamped loads that are not added, so the sum
            // runs over r in increasing order like k_rows
            double a0 = 0.0, a1 = 0.0;
            for (int r = 0; r < S.nw; r += kRedDepth) {
                float2 v[kRedDepth];
#pragma unroll
                for (int j = 0; j < kRedDepth; ++j) {
                    const int rr = r + j < S.nw ? r + j : S.nw - 1;
                    v[j] = load_global(reinterpret_cast<const float2*>(p + (size_t)rr * S.ldp + x0));
                }
                __builtin_amdgcn_sched_barrier(0);  // every load issued before the first add
#pragma unroll
                for (int j = 0; j < kRedDepth; ++j)
                    if (r + j < S.nw) {
                        a0 += (double)v[j].x;
                        a1 += (double)v[j].y;
                    }
            }
            const double nan = __builtin_nan("");
            row[x0] = ok ? a0 : nan;
            if (x0 + 1 < T.x1) row[x0 + 1] = ok ? a1 : nan;
        }
        __syncthreads();  // *flag is reused by the next task
    }
}

// Threads of a workgroup beyond its G sub-groups take no part in the work but
// must meet every barrier of the active threads.
__device__ __forceinline__ void idle_barriers(int n)
{
    for (int i = 0; i < n; ++i) __syncthreads();
}

struct Lane {
    int t, x0, LB, r;
    bool live, ok0, ok1;
    double ar;
};

// One depth step k with the current tap set.  All vector-memory operations
// are issued first: the partial row of step k-1, refills of the other set for
// step k+1 where the slowness changed, and the slowness prefetch for step
// k+2; then the FIR.  The single wait at the top of the next step therefore
// only covers operations issued a whole step earlier.
template <int M, bool ROWS>
__device__ __forceinline__ void step_fast(const BatchArgs& a, const SecDev& S, float2* sm,
                                          const Lane& L, int k, float2 (&hc)[2][M + 1],
                                          float2 (&ho)[2][M + 1], double2& sn, float2& o0,
                                          float2& o1)
{
    wait_vmem_all();
    if (ROWS && k >= 1) {
        float* pr = L.live ? S.part + ((size_t)(k - 1) * S.nw + L.r) * S.ldp + L.x0
                           : a.trash + L.x0;
        store_partial2(pr, o0.x, o1.x);
    }
    // sn = slowness of step k+1, flagged where it differs from step k-1 (the
    // step the other set was last loaded for)
    if (k >= 1 && k + 1 < S.nsteps) {
        if (slowness_changed(sn.x))
            load_taps<M>(ho[0], a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk,
                                                                  slowness_value(sn.x)) * (M + 1));
        if (slowness_changed(sn.y))
            load_taps<M>(ho[1], a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk,
                                                                  slowness_value(sn.y)) * (M + 1));
    }
    const int kp = k + 2 < S.nsteps ? k + 2 : S.nsteps - 1;
    const double2 p = load_global(reinterpret_cast<const double2*>(S.slow + (size_t)kp * S.ldp + L.x0));
    fir2<M>(sm + (k & 1) * L.LB + 2 * L.t, hc[0], hc[1], o0, o1);
    float2* dst = sm + ((k + 1) & 1) * L.LB + M + L.x0;
    if (L.ok0) dst[0] = o0;
    if (L.ok1) dst[1] = o1;
    sn = p;
    __syncthreads();
    if (ROWS && publishes_at(k)) publish_block(a, S, k / kPublish - 1);
}

// Register-tap kernel, two outputs per thread.  Sub-group of tsub threads per
// frequency; LDS per sub-group = two planes of 2*tsub + 2M + 2 points, P[x] at
// offset M + x, zero elsewhere (the zero boundary of Eq. 1).
template <int M, bool ROWS>
__global__ void __launch_bounds__(512) k_extrap_fast(BatchArgs a)
{
    extern __shared__ float4 smem4[];
    if (ROWS && (int)blockIdx.x < a.nred) {
        reduce_role(a, blockIdx.x, reinterpret_cast<int*>(smem4));
        return;
    }
    const ItemDev it = item_of(a, blockIdx.x - (ROWS ? a.nred : 0));
    const SecDev S = sec_of(a, it.sec);
    int G, tsub;
    group_shape(S, 1, G, tsub);
    const int g = threadIdx.x / tsub;
    Lane L;
    L.LB = 2 * tsub + 2 * M + 2;
    if (g >= G) {
        idle_barriers(2 + S.nsteps + (ROWS ? 1 : 0));
        return;
    }
    float2* sm = reinterpret_cast<float2*>(smem4) + (size_t)g * 2 * L.LB;
    L.t = threadIdx.x - g * tsub;
    L.live = it.r0 + g < S.nw;
    L.r = L.live ? it.r0 + g : S.nw - 1;
    L.x0 = 2 * L.t;
    L.ok0 = L.live && L.x0 < S.nx;
    L.ok1 = L.live && L.x0 + 1 < S.nx;
    L.ar = S.omega[L.r] / a.dk;

    for (int i = L.t; i < 2 * L.LB; i += tsub) sm[i] = make_float2(0.0f, 0.0f);
    __syncthreads();
    if (L.ok0) sm[M + L.x0] = S.win[(size_t)L.x0 * S.nw + L.r];
    if (L.ok1) sm[M + L.x0 + 1] = S.win[(size_t)(L.x0 + 1) * S.nw + L.r];

    float2 hA[2][M + 1], hB[2][M + 1];
    {
        const double2 s0 = *reinterpret_cast<const double2*>(S.slow + L.x0);
        load_taps<M>(hA[0], a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk, slowness_value(s0.x)) * (M + 1));
        load_taps<M>(hA[1], a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk, slowness_value(s0.y)) * (M + 1));
        const int k1 = S.nsteps > 1 ? 1 : 0;
        const double2 s1 = *reinterpret_cast<const double2*>(S.slow + (size_t)k1 * S.ldp + L.x0);
        load_taps<M>(hB[0], a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk, slowness_value(s1.x)) * (M + 1));
        load_taps<M>(hB[1], a.tab + (size_t)index_of_slowness(L.ar, a.b, a.nk, slowness_value(s1.y)) * (M + 1));
    }
    double2 sn = make_double2(0.0, 0.0);
    __syncthreads();

    float2 o0 = make_float2(0.0f, 0.0f), o1 = o0;
    for (int k = 0; k < S.nsteps; k += 2) {
        step_fast<M, ROWS>(a, S, sm, L, k, hA, hB, sn, o0, o1);
        if (k + 1 >= S.nsteps) break;
        step_fast<M, ROWS>(a, S, sm, L, k + 1, hB, hA, sn, o0, o1);
    }
    if (ROWS) {
        float* pr = L.live ? S.part + ((size_t)(S.nsteps - 1) * S.nw + L.r) * S.ldp + L.x0
                           : a.trash + L.x0;
        store_partial2(pr, o0.x, o1.x);
        wait_vmem_all();
        __syncthreads();
        for (int b = published_in_loop(S.nsteps); b * kPublish < S.nsteps; ++b) publish_block(a, S, b);
    }
    if (S.wout) {
        if (L.ok0) S.wout[(size_t)L.x0 * S.nw + L.r] = o0;
        if (L.ok1) S.wout[(size_t)(L.x0 + 1) * S.nw + L.r] = o1;
    }
}

// Write-through store of one partial-row value (see store_partial2).
__device__ __forceinline__ void store_partial1(float* p, float a)
{
    __hip_atomic_store(as_global(p), a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Partial row of Q outputs.  Q = 4: x0 is a multiple of 4 and 4 * tsub is
// the row stride, so every lane stores (lanes past nx into the padding).
// Q = 3: 3 * tsub can pass the row stride, so only outputs inside the section
// are stored.
template <int Q>
__device__ __forceinline__ void store_partial_q(float* pr, const float2 (&o)[Q], const bool (&ok)[Q])
{
    if constexpr (Q == 4) {
        store_partial2(pr, o[0].x, o[1].x);
        store_partial2(pr + 2, o[2].x, o[3].x);
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (ok[q]) store_partial1(pr + q, o[q].x);
    }
}

// Register-tap kernel for wider sections (nx <= Q * 512): Q = 3 or 4 outputs
// per thread and one tap set (two do not fit in 256 VGPRs), refilled at the
// end of a step for outputs whose slowness changes at the next step.  A
// workgroup touches only the table rows of its own frequency, so refills
// mostly hit in L1 and the barrier covers part of their latency.  One
// frequency per workgroup.  Q = 3 serves 1024 < nx <= 1536: there Q = 4 would
// leave 5 or 6 waves for 4 SIMDs (the SIMD with two waves sets the pace),
// while Q = 3 gives 6 to 8 waves and three quarters of the work per wave.
template <int M, int Q, bool ROWS>
__global__ void __launch_bounds__(512) k_extrap_wide(BatchArgs a)
{
    extern __shared__ float4 smem4[];
    if (ROWS && (int)blockIdx.x < a.nred) {
        reduce_role(a, blockIdx.x, reinterpret_cast<int*>(smem4));
        return;
    }
    const ItemDev it = item_of(a, blockIdx.x - (ROWS ? a.nred : 0));
    const SecDev S = sec_of(a, it.sec);
    int G, tsub;
    group_shape(S, Q == 4 ? 2 : 3, G, tsub);
    if ((int)threadIdx.x >= tsub) {
        idle_barriers(2 + S.nsteps + (ROWS ? 1 : 0));
        return;
    }
    float2* sm = reinterpret_cast<float2*>(smem4);
    const int t = threadIdx.x;
    const int LB = Q * tsub + 2 * M + 4;
    const int x0 = Q * t;
    const bool live = it.r0 < S.nw;
    const int r = live ? it.r0 : S.nw - 1;
    bool ok[Q];
    int xs[Q];  // slowness columns, clamped into the section
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        ok[q] = live && x0 + q < S.nx;
        xs[q] = x0 + q < S.nx ? x0 + q : S.nx - 1;
    }
    const double ar = S.omega[r] / a.dk;

    for (int i = t; i < 2 * LB; i += tsub) sm[i] = make_float2(0.0f, 0.0f);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q)
        if (ok[q]) sm[M + x0 + q] = S.win[(size_t)(x0 + q) * S.nw + r];

    float2 h[Q][M + 1];
#pragma unroll
    for (int q = 0; q < Q; ++q)
        load_taps<M>(h[q], a.tab + (size_t)index_of_slowness(ar, a.b, a.nk, slowness_value(S.slow[xs[q]])) * (M + 1));
    __syncthreads();

    float2 o[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) o[q] = make_float2(0.0f, 0.0f);
    for (int k = 0; k < S.nsteps; ++k) {
        wait_vmem_all();
        if (ROWS && k >= 1) {
            float* pr = live ? S.part + ((size_t)(k - 1) * S.nw + r) * S.ldp + x0 : a.trash + x0;
            store_partial_q<Q>(pr, o, ok);
        }
        // slowness of step k+1 (flagged where it differs from step k), used
        // after the FIR to refill taps
        const int kp = k + 1 < S.nsteps ? k + 1 : S.nsteps - 1;
        const double* sp = S.slow + (size_t)kp * S.ldp;
        double sn[Q];
        if constexpr (Q == 4) {
            const double2 p01 = load_global(reinterpret_cast<const double2*>(sp + x0));
            const double2 p23 = load_global(reinterpret_cast<const double2*>(sp + x0 + 2));
            sn[0] = p01.x;
            sn[1] = p01.y;
            sn[2] = p23.x;
            sn[3] = p23.y;
        } else {
#pragma unroll
            for (int q = 0; q < Q; ++q) sn[q] = *as_global(sp + xs[q]);
        }
        firq<M, Q>(sm + (k & 1) * LB + x0, h, o);
        float2* dst = sm + ((k + 1) & 1) * LB + M + x0;
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (ok[q]) dst[q] = o[q];
        if (k + 1 < S.nsteps) {
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (slowness_changed(sn[q]))
                    load_taps<M>(h[q], a.tab + (size_t)index_of_slowness(ar, a.b, a.nk,
                                                                         slowness_value(sn[q])) * (M + 1));
        }
        __syncthreads();
        if (ROWS && publishes_at(k)) publish_block(a, S, k / kPublish - 1);
    }
    if (ROWS) {
        float* pr = live ? S.part + ((size_t)(S.nsteps - 1) * S.nw + r) * S.ldp + x0 : a.trash + x0;
        store_partial_q<Q>(pr, o, ok);
        wait_vmem_all();
        __syncthreads();
        for (int b = published_in_loop(S.nsteps); b * kPublish < S.nsteps; ++b) publish_block(a, S, b);
    }
    if (S.wout) {
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (ok[q]) S.wout[(size_t)(x0 + q) * S.nw + r] = o[q];
    }
}

// General kernel: any M <= 31 and nx up to MIG_MAX_NX.  One frequency per
// workgroup, plane in LDS, taps read from the table every step.
__global__ void __launch_bounds__(256) k_extrap_general(BatchArgs a)
{
    extern __shared__ float4 smem4[];
    const bool rows_on = a.rows != 0;
    if (rows_on && (int)blockIdx.x < a.nred) {
        reduce_role(a, blockIdx.x, reinterpret_cast<int*>(smem4));
        return;
    }
    const ItemDev it = item_of(a, blockIdx.x - (rows_on ? a.nred : 0));
    const SecDev S = sec_of(a, it.sec);
    float2* sm = reinterpret_cast<float2*>(smem4);
    const int M = a.M, nx = S.nx;
    const bool live = it.r0 < S.nw;
    const int r = live ? it.r0 : S.nw - 1;
    const int LB = nx + 2 * M;
    const double ar = S.omega[r] / a.dk;
    for (int i = threadIdx.x; i < 2 * LB; i += blockDim.x) sm[i] = make_float2(0.0f, 0.0f);
    __syncthreads();
    for (int x = threadIdx.x; x < nx; x += blockDim.x) sm[M + x] = S.win[(size_t)x * S.nw + r];
    __syncthreads();
    for (int k = 0; k < S.nsteps; ++k) {
        const float2* src = sm + (k & 1) * LB + M;
        float2* dst = sm + ((k + 1) & 1) * LB + M;
        const auto* sr = as_global(S.slow + (size_t)k * S.ldp);
        for (int x = threadIdx.x; x < nx; x += blockDim.x) {
            const float2* h = a.tab + (size_t)index_of_slowness(ar, a.b, a.nk, slowness_value(sr[x])) * (M + 1);
            float2 acc = cmulf(h[0], src[x]);
            for (int n = 1; n <= M; ++n) acc = cfmaf(h[n], cadd(src[x - n], src[x + n]), acc);
            dst[x] = acc;
            if (rows_on && live)  // write-through, as store_partial2
                __hip_atomic_store(as_global(S.part + ((size_t)k * S.nw + r) * S.ldp + x), acc.x,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const bool publish = rows_on && ((k + 1) % kPublish == 0 || k + 1 == S.nsteps);
        if (publish) wait_vmem_all();
        __syncthreads();
        if (publish) publish_block(a, S, k / kPublish);
    }
    if (S.wout && live) {
        const float2* src = sm + (S.nsteps & 1) * LB + M;
        for (int x = threadIdx.x; x < nx; x += blockDim.x) S.wout[(size_t)x * S.nw + r] = src[x];
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


// Image rows of depth steps [s0, s1) from their partial rows, once the
// depth-stepping launch is over: one thread per point, the frequencies added in
// increasing order in FP64, the order of the reducer workgroups, so a row is the
// same whichever of the two forms it.  Small workgroups spread the rows over
// every CU; 16 loads in flight per thread.
__global__ void __launch_bounds__(64) k_rows(const float* __restrict__ part,
                                             double* __restrict__ rows, int s0, int nx, int nw,
                                             int ldp)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const int st = s0 + blockIdx.y;
    const float* p = part + (size_t)st * nw * ldp + x;
    double acc = 0.0;
    int r = 0;
    for (; r + 16 <= nw; r += 16) {
        float v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) v[j] = p[(size_t)(r + j) * ldp];
#pragma unroll
        for (int j = 0; j < 16; ++j) acc += (double)v[j];
    }
    for (; r < nw; ++r) acc += (double)p[(size_t)r * ldp];
    rows[(size_t)st * nx + x] = acc;
}

template <int M>
int launch_fast(const BatchArgs& a, int threads, size_t lds, hipStream_t s)
{
    if (a.rows)
        hipLaunchKernelGGL((k_extrap_fast<M, true>), dim3(a.nitems + a.nred), dim3(threads), lds,
                           s, a);
    else
        hipLaunchKernelGGL((k_extrap_fast<M, false>), dim3(a.nitems), dim3(threads), lds, s, a);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

template <int M, int Q>
int launch_wide(const BatchArgs& a, int threads, size_t lds, hipStream_t s)
{
    if (a.rows)
        hipLaunchKernelGGL((k_extrap_wide<M, Q, true>), dim3(a.nitems + a.nred), dim3(threads),
                           lds, s, a);
    else
        hipLaunchKernelGGL((k_extrap_wide<M, Q, false>), dim3(a.nitems), dim3(threads), lds, s, a);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

template <int M>
int launch_wide4(const BatchArgs& a, int threads, size_t lds, hipStream_t s)
{
    return launch_wide<M, 4>(a, threads, lds, s);
}

template <int M>
int launch_wide3(const BatchArgs& a, int threads, size_t lds, hipStream_t s)
{
    return launch_wide<M, 3>(a, threads, lds, s);
}

typedef int (*launch_fn)(const BatchArgs&, int, size_t, hipStream_t);

// Register-tap kernels are instantiated for N = 1..35 (M = 0..17); beyond
// that two tap sets no longer fit in 256 VGPRs without spilling.
#define MIG_INST(f)                                                                   \
    {&f<0>, &f<1>, &f<2>, &f<3>, &f<4>, &f<5>, &f<6>, &f<7>, &f<8>, &f<9>, &f<10>,     \
     &f<11>, &f<12>, &f<13>, &f<14>, &f<15>, &f<16>, &f<17>}
const launch_fn kFast[] = MIG_INST(launch_fast);
const launch_fn kWide[] = MIG_INST(launch_wide4);
const launch_fn kMid[] = MIG_INST(launch_wide3);
constexpr int kRegMaxM = 17;
constexpr int kFastMaxNx = 2 * 512;
constexpr int kMidMaxNx = 3 * 512;
constexpr int kWideMaxNx = 4 * 512;

}  // namespace

int extrap_kernel_kind(int nx, int M)
{
    if (M > kRegMaxM) return 0;
    if (nx <= kFastMaxNx) return 1;
    if (nx <= kMidMaxNx) return 3;
    if (nx <= kWideMaxNx) return 2;
    return 0;
}

int threads_per_omega(int kind, int nx)
{
    if (kind == 1) return ((nx + 1) / 2 + 63) / 64 * 64;
    if (kind == 2) return ((nx + 3) / 4 + 63) / 64 * 64;
    if (kind == 3) return ((nx + 2) / 3 + 63) / 64 * 64;
    return 256;
}

int launch_slowness(const BatchArgs& a, int max_rows, int max_ldp, int dist, hipStream_t s)
{
    size_t per = (size_t)max_rows * max_ldp;
    size_t blocks = (per + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_slowness, dim3((unsigned)blocks, a.nsec), dim3(256), 0, s, a, dist);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

int launch_extrap(const BatchArgs& a, int kind, int threads, hipStream_t s)
{
    // LDS: G sub-groups x two planes; the host picks threads = G * tsub.
    if (kind == 1) {
        int tsub_min = 64;
        size_t lds = (size_t)2 * (2 * threads + (threads / tsub_min) * (2 * a.M + 2)) * sizeof(float2);
        return kFast[a.M](a, threads, lds, s);
    }
    if (kind == 2 || kind == 3) {
        const int Q = kind == 2 ? 4 : 3;
        size_t lds = (size_t)2 * (Q * threads + 2 * a.M + 4) * sizeof(float2);
        return (kind == 2 ? kWide : kMid)[a.M](a, threads, lds, s);
    }
    return MIG_E_ARG;
}

int launch_general(const BatchArgs& a, int max_nx, hipStream_t s)
{
    size_t lds = (size_t)2 * (max_nx + 2 * a.M) * sizeof(float2);
    if (lds > 65536) {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_extrap_general),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds) != hipSuccess)
            return MIG_E_DEVICE;
    }
    hipLaunchKernelGGL(k_extrap_general, dim3(a.nitems + a.nred), dim3(256), lds, s, a);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

int launch_rows(const float* part, double* rows, int s0, int s1, int nx, int nw, int ldp,
                hipStream_t s)
{
    if (s1 <= s0) return MIG_OK;
    dim3 grid((nx + 63) / 64, s1 - s0);
    hipLaunchKernelGGL(k_rows, grid, dim3(64), 0, s, part, rows, s0, nx, nw, ldp);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

namespace {
__global__ void k_clear_status(int* status) { *status = 0; }
}  // namespace

int launch_clear_status(int* status, hipStream_t s)
{
    hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(1), 0, s, status);
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
