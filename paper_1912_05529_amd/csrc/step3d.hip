// 3-D extension (Sec. II): the depth step of Eq. (1) with circularly
// symmetric (2M+1) x (2M+1) extrapolators, and the image of each new plane
// (real part summed over frequencies, Algorithm 1) accumulated in FP64.
//
// Filter of output (x, y) at frequency omega: h[n1][n2] = c(a, b) with
// a = max(|n1|,|n2|), b = min; the unique coefficients (a >= b >= 0) are stored
// at u = a (a + 1) / 2 + b.  Folding the symmetric taps, one output is
//   out = sum_u c_u S_u,   S_u = sum of P(x + n1, y + n2) over the orbit of u,
// formed from pair sums along y, Y_b(x') = P(x', y + b) + P(x', y - b):
//   S(0,0) = Y_0(x)
//   S(a,0) = Y_a(x) + Y_0(x + a) + Y_0(x - a)
//   S(a,a) = Y_a(x + a) + Y_a(x - a)
//   S(a,b) = Y_b(x + a) + Y_b(x - a) + Y_a(x + b) + Y_a(x - b)     (a > b > 0)
// i.e. M + 3M + 3M(M-1)/2 complex additions (50 for M = 5) and (M+1)(M+2)/2
// complex multiply-adds (21) per output instead of (2M+1)^2 (121).
//
// Layout: wavefield planes [nw][nx][ny] complex64 (y fastest), so one
// frequency's plane is a contiguous 2-D array.
//
// Mapping: a workgroup owns a tile of 32 x-rows by 64 y-columns and a group of
// consecutive frequencies.  For each frequency it stages the tile and its halo
// of M points in LDS (one coalesced row per wave load), then each of its four
// waves walks 8 x-rows with one y-column per lane, keeping the pair sums of the
// 2M + 1 rows around the current output in registers (one new LDS row of
// 2M + 1 values per output).  Taps stay in registers and are reloaded only when
// the table entry of some lane changes.  The tile's slowness lives in LDS.
//
// Image: each workgroup sums Re over its frequencies in FP64 (frequency order)
// and writes a partial row for its group; the kernel of the next depth step
// adds the groups' partials in group order (so no atomics and no waiting), and
// a last small kernel closes the final step.  Results are deterministic for a
// given frequency grouping.
#include <cstddef>
#include <type_traits>

#include "common.hpp"

namespace mig {
namespace {

constexpr int kLanes3 = 64;                  // y columns per tile (one per lane)
constexpr int kWaves3 = 4;                   // waves per workgroup
constexpr int kRows3 = 8;                    // x rows walked by each wave
constexpr int kTileX3 = kWaves3 * kRows3;    // x rows per tile
constexpr int kThreads3 = kWaves3 * 64;
constexpr int kSlots3 = 4;                   // LDS tap slots per wave (see k_step3d)
constexpr int kSlotF2 = 32;                  // complex values per slot (>= unique taps)
constexpr int kNoSlot = 7;                   // 3-bit slot code of a point without a slot

// Buffer resource word 3 for raw (unformatted, unswizzled) buffers on the
// gfx9 family; loads beyond num_records return zero.
constexpr int kRawBufferWord3 = 0x00020000;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float2 buf_load_c64(__amdgpu_buffer_rsrc_t r, int byte_off)
{
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0);
    return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
}

__device__ __forceinline__ void buf_store_c64(__amdgpu_buffer_rsrc_t r, int byte_off, float2 v)
{
    const u32x2 u = {__float_as_uint(v.x), __float_as_uint(v.y)};
    __builtin_amdgcn_raw_buffer_store_b64(u, r, byte_off, 0, 0);
}

// s_waitcnt vmcnt(0), other counters left alone (GFX9 encoding:
// vmcnt[3:0] | expcnt[6:4] | lgkmcnt[11:8] | vmcnt[5:4] in bits 15:14).
__device__ __forceinline__ void wait_vmem_all()
{
    __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));
}

// Workgroup barrier for the staged tiles: this wave's LDS stores complete
// (lgkmcnt(0); its buffer-to-LDS copies were waited for by the caller), then
// s_barrier, with compiler-only fences so no LDS access moves across it.  A
// __syncthreads() would also wait for every global store in flight, which
// here are the last pass's output stores.
__device__ __forceinline__ void barrier_lds()
{
    __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (0 << 8) | (3 << 14));  // lgkmcnt(0)
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// s_waitcnt vmcnt(kRows3): all but the last kRows3 vector-memory operations of
// this wave complete (they complete in issue order).
__device__ __forceinline__ void wait_vmem_but_rows()
{
    static_assert(kRows3 < 16, "vmcnt low field");
    __builtin_amdgcn_s_waitcnt(kRows3 | (7 << 4) | (15 << 8));
}

__device__ __forceinline__ float2 c_add(float2 a, float2 b)
{
    return make_float2(a.x + b.x, a.y + b.y);
}

// Workgroup index -> (frequency group, tile).  Consecutive workgroup indices
// are dealt round-robin to the 8 XCDs; when the grid is a multiple of 8 the
// index is remapped so that each XCD receives a contiguous run of tiles of
// the same frequencies, whose halos then meet in that XCD's L2.
__device__ __forceinline__ int logical_block()
{
    const int nb = gridDim.x, b = blockIdx.x;
    return (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
}

// Coefficient index of the orbit (a, b), a >= b.
constexpr int cidx(int a, int b) { return a * (a + 1) / 2 + b; }
constexpr bool in_set(int p, int lo, int hi) { return p >= lo && p < hi; }

// Position of orbit (a, b) among the coefficients a pass over planes [lo, hi)
// multiplies (the orbits with a part in one of those planes), in (a, b) order.
constexpr int pass_slot(int M, int lo, int hi, int a0, int b0)
{
    int n = 0;
    for (int a = 0; a <= M; ++a)
        for (int b = 0; b <= a; ++b) {
            if (a == a0 && b == b0) return n;
            if (in_set(a, lo, hi) || in_set(b, lo, hi)) ++n;
        }
    return n;
}

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// One pass of a wave over its kRows3 output rows using only the pair-sum
// planes b in [LO, HI).  out = sum over orbits (a, b) of c(a,b) S(a,b) is
// linear in the planes, so every orbit sum splits into a plane-a part and a
// plane-b part:
//   (0,0): Y_0(x)                      plane 0
//   (a,0): Y_a(x)  | Y_0(x+a)+Y_0(x-a) planes a | 0
//   (a,a): Y_a(x+a)+Y_a(x-a)           plane a
//   (a,b): Y_a(x+b)+Y_a(x-b) | Y_b(x+a)+Y_b(x-a)   planes a | b
// A pass adds the parts whose plane it holds (both parts under one
// multiply when both planes are in the pass).  Two passes over halves of the
// planes hold half the pair-sum window in registers, at the price of one
// extra multiply-add for each orbit whose planes fall in different halves.
// The last pass also finishes each output at once: Re into the image
// partial, and a buffer store whose offset is pushed out of range for
// points outside the volume (so no output waits behind a branch).
template <int M, int LO, int HI>
__device__ __forceinline__ void load_pass_taps(float2 (&h)[pass_slot(M, LO, HI, M + 1, 0)],
                                               __amdgpu_buffer_rsrc_t rt, int j)
{
    constexpr int NU = (M + 1) * (M + 2) / 2;
    const int toff = j * (NU * 8);
    static_for<0, M + 1>([&](auto AA) {
        constexpr int a = decltype(AA)::value;
        static_for<0, a + 1>([&](auto BB) {
            constexpr int b = decltype(BB)::value;
            if constexpr (in_set(a, LO, HI) || in_set(b, LO, HI))
                h[pass_slot(M, LO, HI, a, b)] = buf_load_c64(rt, toff + cidx(a, b) * 8);
        });
    });
}

typedef float v2f3 __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(3))) v2f3* lds_cf2;

__device__ __forceinline__ float2 lds_c64(lds_cf2 p)
{
    const v2f3 v = *p;
    return make_float2(v.x, v.y);
}

// An LDS address the compiler cannot split into a constant and a variable
// part: reads from it then put their small offsets in the instructions'
// offset fields instead of one address add per read.
__device__ __forceinline__ lds_cf2 opaque_lds(const float2* p)
{
    const unsigned a = (unsigned)(size_t)(const __attribute__((address_space(3))) void*)p;
    return (lds_cf2)(size_t)(unsigned)__builtin_amdgcn_readfirstlane((int)a);
}

// The same taps from an LDS slot holding the NU unique coefficients of one
// table entry (in coefficient order).
template <int M, int LO, int HI>
__device__ __forceinline__ void lds_pass_taps(float2 (&h)[pass_slot(M, LO, HI, M + 1, 0)],
                                              lds_cf2 slot)
{
    static_for<0, M + 1>([&](auto AA) {
        constexpr int a = decltype(AA)::value;
        static_for<0, a + 1>([&](auto BB) {
            constexpr int b = decltype(BB)::value;
            if constexpr (in_set(a, LO, HI) || in_set(b, LO, HI))
                h[pass_slot(M, LO, HI, a, b)] = lds_c64(slot + cidx(a, b));
        });
    });
}

__device__ __forceinline__ int slot_of(unsigned slots, int r) { return (slots >> (3 * r)) & 7u; }

// Where taps come from.  With SLOTS, a row's key is the point's slot and its
// taps come from the wave's LDS slots (TSw); otherwise the key is the table
// entry and the taps come from the table.  The two forms are separate code
// paths (a workgroup takes one for all its frequencies), so that the slot
// path issues no tap load to memory: the compiler's waits after a load that
// may or may not have been issued are conservative and would also wait for
// the tile copy in flight.
struct TapSrc {
    lds_cf2 TSw;
    __amdgpu_buffer_rsrc_t rt;
};

template <int M, int LO, int HI, bool SLOTS>
__device__ __forceinline__ void row_taps(float2 (&h)[pass_slot(M, LO, HI, M + 1, 0)],
                                         const TapSrc& ts, int key)
{
    if constexpr (SLOTS)
        lds_pass_taps<M, LO, HI>(h, ts.TSw + key * kSlotF2);
    else
        load_pass_taps<M, LO, HI>(h, ts.rt, key);
}

// Partial output of a pass: Re = re1 - re2 with re1 = sum Re h Re s and
// re2 = sum Im h Im s kept apart (no negated operands), Im = sum of the
// cross products.
struct Acc3 {
    float re1, re2, im;
};

// The last pass also finishes each output at once: Re into the image
// partial, and a buffer store whose offset is pushed out of range for
// points outside the volume (so no output waits behind a branch).
// `issue(i)` runs at the start of row i of the pass (the last pass uses it
// to copy the next frequency's tile a few rows at a time).
// Taps are reloaded at a row where some lane's key (slot or table entry,
// keys[r]) differs from the one its registers hold (kcur).  With LDS_TAPS
// (slots only) no taps are held: each output row reads its slot's taps from
// LDS as it multiplies, which frees the registers of a tap set, enough for one
// pass over all planes (no split, so the unique multiply-adds only).
template <int M, int LO, int HI, bool LAST, bool PRELOADED, bool SLOTS, bool LDS_TAPS,
          typename Issue>
__device__ __forceinline__ void fir_pass(const float2* __restrict__ Tw, const TapSrc& ts,
                                         const int (&keys)[kRows3],
                                         float2 (&h)[pass_slot(M, LO, HI, M + 1, 0)], int& kcur,
                                         float2 (&acc)[kRows3], double (&img)[kRows3],
                                         __amdgpu_buffer_rsrc_t rq, int qbase, int ny8, int Wr,
                                         Issue&& issue)
{
    constexpr int NP = HI - LO;
    constexpr int NR = kRows3 + 2 * M;
    float2 Y[NR][NP];
    // The LDS values of row i+1 are requested before row i's arithmetic, so
    // their latency hides behind it (v[i & 1] holds row i: index 2q for
    // column +b, 2q+1 for column -b of plane b = LO + q).
    float2 v[2][2 * NP];
    auto fetch = [&](auto I) {
        constexpr int i = decltype(I)::value;
        // The row stride is a run-time value (Wr == W): one register then
        // holds the row's first column (y - M) and the reads take their
        // columns from the instructions' small offset fields, instead of an
        // address add per read pair (paired reads reach only 255 values past
        // their base).
        const float2* row = Tw + i * Wr - M;
        static_for<0, NP>([&](auto Q) {
            constexpr int q = decltype(Q)::value;
            constexpr int b = LO + q;
            v[i & 1][2 * q] = row[M + b];
            if constexpr (b != 0) v[i & 1][2 * q + 1] = row[M - b];
        });
    };
    // Taps of the first output row (unless the caller has them), requested
    // before the 2M rows of pair sums that precede it, so their latency hides
    // behind those rows.
    if constexpr (!PRELOADED && !LDS_TAPS) {
        row_taps<M, LO, HI, SLOTS>(h, ts, keys[0]);
        kcur = keys[0];
    }
    fetch(std::integral_constant<int, 0>{});
    static_for<0, NR>([&](auto I) {
        constexpr int i = decltype(I)::value;
        issue(I);
        if constexpr (i + 1 < NR) fetch(std::integral_constant<int, i + 1>{});
        static_for<0, NP>([&](auto Q) {
            constexpr int q = decltype(Q)::value;
            constexpr int b = LO + q;
            if constexpr (b == 0) {
                Y[i][0] = v[i & 1][0];
            } else {
                Y[i][q] = c_add(v[i & 1][2 * q], v[i & 1][2 * q + 1]);
                // Keep the pair sum (not its two operands) alive across rows.
                __asm__ volatile("" : "+v"(Y[i][q].x), "+v"(Y[i][q].y));
            }
        });
        if constexpr (i >= 2 * M) {
            constexpr int r = i - 2 * M;  // output row x0 + r0 + r
            constexpr int c = r + M;      // its pair sums
            if constexpr (!LDS_TAPS) {
                if (__builtin_amdgcn_ballot_w64(keys[r] != kcur) != 0) {
                    row_taps<M, LO, HI, SLOTS>(h, ts, keys[r]);
                    kcur = keys[r];
                }
            }
            const lds_cf2 tp = ts.TSw + (LDS_TAPS ? keys[r] : 0) * kSlotF2;
            Acc3 o{acc[r].x, 0.0f, acc[r].y};
            static_for<0, M + 1>([&](auto AA) {
                constexpr int a = decltype(AA)::value;
                static_for<0, a + 1>([&](auto BB) {
                    constexpr int b = decltype(BB)::value;
                    constexpr bool ha = in_set(a, LO, HI), hb = in_set(b, LO, HI);
                    if constexpr (ha || hb) {
                        constexpr int n = pass_slot(M, LO, HI, a, b);
                        float2 sum;
                        if constexpr (a == 0) {
                            sum = Y[c][0];
                        } else if constexpr (a == b) {
                            sum = c_add(Y[c + a][a - LO], Y[c - a][a - LO]);
                        } else if constexpr (b == 0) {
                            if constexpr (ha && hb)
                                sum = c_add(Y[c][a - LO], c_add(Y[c + a][0], Y[c - a][0]));
                            else if constexpr (ha)
                                sum = Y[c][a - LO];
                            else
                                sum = c_add(Y[c + a][0], Y[c - a][0]);
                        } else {
                            if constexpr (ha && hb)
                                sum = c_add(c_add(Y[c + b][a - LO], Y[c - b][a - LO]),
                                            c_add(Y[c + a][b - LO], Y[c - a][b - LO]));
                            else if constexpr (ha)
                                sum = c_add(Y[c + b][a - LO], Y[c - b][a - LO]);
                            else
                                sum = c_add(Y[c + a][b - LO], Y[c - a][b - LO]);
                        }
                        float2 hv;
                        if constexpr (LDS_TAPS)
                            hv = lds_c64(tp + cidx(a, b));
                        else
                            hv = h[n];
                        o.re1 = fmaf(hv.x, sum.x, o.re1);
                        o.re2 = fmaf(hv.y, sum.y, o.re2);
                        o.im = fmaf(hv.x, sum.y, o.im);
                        o.im = fmaf(hv.y, sum.x, o.im);
                    }
                });
            });
            float2 out = make_float2(o.re1 - o.re2, o.im);
            if constexpr (LAST) {
                img[r] += (double)out.x;
                buf_store_c64(rq, qbase + r * ny8, out);
            } else {
                // Pin the partial sum here: otherwise the compiler sinks this
                // pass's arithmetic to its use in the next pass and keeps the
                // whole pair-sum window of every row alive until then.
                __asm__ volatile("" : "+v"(out.x), "+v"(out.y));
                acc[r] = out;
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    });
}

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Stage the tile of one frequency plane into LDS by direct buffer-to-LDS
// loads (no registers on the way): each wave copies its rows, a row being
// the 2 (64 + 2M) dwords of columns y0 - M .. y0 + 63 + M, 64 dwords per
// instruction.  Rows outside [0, nx) lie outside the buffer and arrive as
// zeros; so do columns outside [0, ny), whose lanes read at an offset pushed
// out of range (the same for every row).  A call copies this wave's rows
// q in [Q0, Q1), q-th row of the wave being tile row q * 4 + wave.
template <int M>
constexpr int stage_chunks() { return (2 * (kLanes3 + 2 * M) + 63) / 64; }

// Per-lane offset bias of each 64-dword chunk of a row (columns outside the
// volume pushed out of range); the same for every row and frequency.
template <int M>
__device__ __forceinline__ void stage_bias(int (&bias)[stage_chunks<M>()], int y0, int ny, int lane)
{
    static_for<0, stage_chunks<M>()>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const int yc = y0 - M + (i * 64 + lane) / 2;  // column of this lane's dword
        bias[i] = (unsigned)yc < (unsigned)ny ? 0 : 0x40000000;
    });
}

template <int M, int Q0, int Q1>
__device__ __forceinline__ void stage_rows(float2* Tb, __amdgpu_buffer_rsrc_t rp,
                                           const int (&bias)[stage_chunks<M>()], int x0, int y0,
                                           int ny, int wave, int lane)
{
    constexpr int W = kLanes3 + 2 * M;
    constexpr int DW = 2 * W;  // dwords per row
    // wave, x0, y0 and ny are wave-uniform: row offsets and LDS destinations
    // are scalar; one vector add per row, chunks of 64 dwords by the
    // instruction's immediate offset, which applies to the global and the LDS
    // address alike (so the LDS base stays at the row start).
    const int lane4 = lane * 4;
    constexpr int NCH = stage_chunks<M>();
#pragma unroll
    for (int q = Q0; q < Q1; ++q) {
        const int r = q * kWaves3 + wave;
        const int voff = ((x0 - M + r) * ny + (y0 - M)) * 8 + lane4;
        char* dst = reinterpret_cast<char*>(Tb + r * W);
        static_for<0, NCH>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if (i * 64 + lane < DW)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rp, (lds_ptr_t)dst, 4, voff + bias[i], 0,
                                                         i * 256, 0);
        });
    }
}

template <int M>
__global__ void __launch_bounds__(kThreads3) __attribute__((amdgpu_waves_per_eu(2)))
k_step3d(Step3dArgs A)
{
    constexpr int W = kLanes3 + 2 * M;       // LDS tile row length (with halo)
    constexpr int H = kTileX3 + 2 * M;       // LDS tile rows (with halo)
    constexpr int HP = (H + kWaves3 - 1) / kWaves3 * kWaves3;  // padded to whole wave rounds
    constexpr int SPLIT = M >= 3 ? (M + 1) / 2 : M + 1;  // planes of the first pass
    constexpr int NC1 = pass_slot(M, 0, SPLIT, M + 1, 0);
    constexpr int NC2 = pass_slot(M, SPLIT, M + 1, M + 1, 0);
    constexpr int QW = HP / kWaves3;       // tile rows copied by each wave
    // LDS in one block, in this order: the targets of buffer-to-LDS copies
    // (tiles, tap slots) come first and stay within the low 64 KiB; the tiles
    // start at address 0, so a row address plus a column offset fits the
    // offset field of the paired reads.
    struct Lds {
        float2 T[2][HP * W];                        // double-buffered frequency tiles
        float2 TS[2][kWaves3 * kSlots3 * kSlotF2];  // tap slots, by frequency parity
        double S[kTileX3 * kLanes3];                // slowness of the tile
        double SL[kWaves3 * kSlots3];               // slowness of each slot
        int FB[kWaves3];                            // wave has points without a slot
    };
    static_assert(offsetof(Lds, S) <= 65536 && offsetof(Lds, T) == 0, "copy targets below 64 KiB");
    __shared__ Lds L;
    auto& TS = L.TS;
    auto& T = L.T;
    auto& S = L.S;
    auto& SL = L.SL;
    auto& FB = L.FB;
    constexpr int NU = (M + 1) * (M + 2) / 2;
    static_assert(NU <= kSlotF2, "tap slot size");

    const int ntiles = A.tiles_x * A.tiles_y;
    const int bid = logical_block();
    const int g = bid / ntiles, t = bid % ntiles;
    const int x0 = (t / A.tiles_y) * kTileX3, y0 = (t % A.tiles_y) * kLanes3;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const size_t plane = (size_t)A.nx * A.ny;
    const int y = y0 + lane;
    const int r0 = wave * kRows3;

    const int wbeg = g * A.wpg;
    const int wend = wbeg + A.wpg < A.nw ? wbeg + A.wpg : A.nw;
    const int pbytes = (int)(plane * sizeof(float2));
    const __amdgpu_buffer_rsrc_t rt = __builtin_amdgcn_make_buffer_rsrc(
        (void*)A.tab, 0, A.nk * NU * (int)sizeof(float2), kRawBufferWord3);
    // The first tile's copy goes out first; the velocity and previous-image
    // loads below are all issued before any of them is waited for, so the
    // prologue costs about one memory latency, not one per load.
    int bias[stage_chunks<M>()];
    stage_bias<M>(bias, y0, A.ny, lane);
    stage_rows<M, 0, QW>(T[0], __builtin_amdgcn_make_buffer_rsrc((void*)(A.in + (size_t)wbeg * plane),
                                                                0, pbytes, kRawBufferWord3),
                         bias, x0, y0, A.ny, wave, lane);

    constexpr int kPer3 = kTileX3 * kLanes3 / kThreads3;  // tile points per thread
    float vv[kPer3];
#pragma unroll
    for (int i = 0; i < kPer3; ++i) {
        const int e = threadIdx.x + i * kThreads3;
        const int x = x0 + e / kLanes3, yy = y0 + e % kLanes3;
        vv[i] = (x < A.nx && yy < A.ny) ? A.vel[(size_t)x * A.ny + yy] : 0.0f;
    }

    // Image row of the previous depth step: this workgroup's share of the
    // tile, groups added in group order (the partials of the previous launch
    // are complete when this one starts).
    if (A.prev) {
        constexpr int pts = kTileX3 * kLanes3;
        constexpr int kBatch = 8;  // partial loads in flight per thread
        const int share = (pts + A.ngroups - 1) / A.ngroups;
        const int e1 = (g + 1) * share < pts ? (g + 1) * share : pts;
        for (int e = g * share + threadIdx.x; e < e1; e += kThreads3) {
            const int x = x0 + e / kLanes3, yy = y0 + e % kLanes3;
            if (x < A.nx && yy < A.ny) {
                const size_t p = (size_t)x * A.ny + yy;
                double s = 0.0;
                for (int q0 = 0; q0 < A.ngroups; q0 += kBatch) {
                    double pv[kBatch];
#pragma unroll
                    for (int i = 0; i < kBatch; ++i)
                        pv[i] = q0 + i < A.ngroups ? A.prev[(size_t)(q0 + i) * plane + p] : 0.0;
#pragma unroll
                    for (int i = 0; i < kBatch; ++i)
                        if (q0 + i < A.ngroups) s += pv[i];
                }
                A.prev_row[p] = s;
            }
        }
    }

#pragma unroll
    for (int i = 0; i < kPer3; ++i) {
        const int e = threadIdx.x + i * kThreads3;
        const int x = x0 + e / kLanes3, yy = y0 + e % kLanes3;
        S[e] = (x < A.nx && yy < A.ny) ? slowness_of(vv[i]) : __builtin_nan("");
    }

    barrier_lds();  // the wave's slowness rows were written by other waves

    // Tap slots.  A point's table entry is a function of its slowness, so
    // points of equal slowness share the entry at every frequency, and a wave
    // of a layered volume sees only a few distinct slowness values (a layer,
    // two across an interface).  Each of the first kSlots3 distinct values of
    // the wave's 8 x 64 points gets a slot in LDS holding its entry's taps;
    // per frequency the slots are refilled by buffer-to-LDS copies issued one
    // frequency ahead, so a change of entry between rows reads LDS instead of
    // waiting for L2 (and, vector-memory operations completing in order, for
    // every copy in flight).  A workgroup with a point beyond the slots
    // loads every tap from the table instead.  Values are compared by bit
    // pattern (one NaN for every point without a velocity).
    unsigned slots = 0xFFFFFFu;  // 3 bits per row, kNoSlot = none
    int nsl = 0;
    {
        unsigned long long pat[kRows3];
#pragma unroll
        for (int r = 0; r < kRows3; ++r)
            pat[r] = (unsigned long long)__double_as_longlong(S[(r0 + r) * kLanes3 + lane]);
        for (int k = 0; k < kSlots3; ++k) {
            unsigned long long key = 0;
            bool found = false;
#pragma unroll
            for (int r = 0; r < kRows3; ++r) {
                const unsigned long long m =
                    __builtin_amdgcn_ballot_w64(slot_of(slots, r) == kNoSlot);
                if (!found && m != 0) {
                    const int l = __builtin_ctzll(m);
                    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(pat[r] >> 32), l);
                    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)pat[r], l);
                    key = ((unsigned long long)hi << 32) | lo;
                    found = true;
                }
            }
            if (!found) break;
#pragma unroll
            for (int r = 0; r < kRows3; ++r)
                if (slot_of(slots, r) == kNoSlot && pat[r] == key)
                    slots = (slots & ~(7u << (3 * r))) | ((unsigned)k << (3 * r));
            if (lane == 0) SL[wave * kSlots3 + k] = __longlong_as_double((long long)key);
            nsl = k + 1;
        }
    }
    // Whether all the wave's points share slot 0 (then nothing is reloaded).
    const bool one_slot = nsl == 1;
    // One path per workgroup: slots when every point of every wave has one.
    bool none = false;
#pragma unroll
    for (int r = 0; r < kRows3; ++r) none = none || slot_of(slots, r) == kNoSlot;
    const bool wave_none = __builtin_amdgcn_ballot_w64(none) != 0;  // all lanes vote
    if (lane == 0) FB[wave] = wave_none ? 1 : 0;
    barrier_lds();
    const bool use_slots = (FB[0] | FB[1] | FB[2] | FB[3]) == 0;
    // Copies of the slots' taps for frequency omega = a * dk into `dst`
    // (64 dwords per slot: the entry's 2 NU dwords and what follows it).
    auto copy_slots = [&](float2* dst, double a) {
        const int js = index_of_slowness(a, A.b, A.nk, SL[wave * kSlots3 + (lane & (kSlots3 - 1))]);
        for (int k = 0; k < nsl; ++k) {
            const int j = __builtin_amdgcn_readlane(js, k);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rt, (lds_ptr_t)(dst + k * kSlotF2), 4, lane * 4,
                                                     j * NU * (int)sizeof(float2), 0, 0);
        }
    };

    double img[kRows3];
#pragma unroll
    for (int r = 0; r < kRows3; ++r) img[r] = 0.0;
    const int ny8 = A.ny * 8;
    const int Wr = __builtin_amdgcn_readfirstlane(A.nx > 0 ? W : W + 1);  // == W
    // Byte offset of this lane's first output within a plane.  Rows at or
    // past nx land past the plane's end by themselves; a column past ny is
    // moved out of range as a whole (stores out of range are dropped).
    const int qbase = y < A.ny ? (x0 + r0) * ny8 + y * 8 : 0x40000000;

    // Frequencies are read through the constant address space: uniform loads
    // of read-only data become scalar loads, so waiting for one never waits for
    // the vector-memory operations in flight (tile copies, output stores).
    typedef const __attribute__((address_space(4))) double* const_f64_ptr;
    const const_f64_ptr omc = (const_f64_ptr)A.omega;

    auto frequencies = [&](auto SLOTS_) {
        constexpr bool SLOTS = decltype(SLOTS_)::value;
        double om = omc[wbeg];  // frequency of the coming iteration, loaded one ahead
        if constexpr (SLOTS) copy_slots(TS[0] + wave * kSlots3 * kSlotF2, om / A.dk);
        for (int w = wbeg; w < wend; ++w) {
            const int cur = (w - wbeg) & 1;
            float2* Tb = T[cur];
            // This wave's copies into Tb (and its slot copies) are complete;
            // after the barrier so are every wave's, and nobody reads the other
            // buffers any more.  After the first frequency, the copies were
            // followed by the kRows3 output stores of the last pass (one per
            // row, unconditional), which need not have completed.
            if (w == wbeg)
                wait_vmem_all();
            else
                wait_vmem_but_rows();
            barrier_lds();
            const double ar = om / A.dk;
            if (w + 1 < wend) om = omc[w + 1];
            // Row keys: slots, or table entries.
            int keys[kRows3];
#pragma unroll
            for (int r = 0; r < kRows3; ++r)
                keys[r] = SLOTS ? slot_of(slots, r)
                                : index_of_slowness(ar, A.b, A.nk, S[(r0 + r) * kLanes3 + lane]);
            TapSrc ts;
            ts.TSw = opaque_lds(TS[cur] + wave * kSlots3 * kSlotF2);
            ts.rt = rt;
            // First taps of the first pass.  Vector-memory operations complete
            // in issue order, so a tap load issued after the next tile's copy
            // would wait for that copy: the copy is issued during the last pass
            // instead, one tile row per row of that pass's first 2M rows (the
            // rows of pair sums before its first output), and only tap loads
            // in the last pass's output rows can wait for it (none with slots).
            float2 h1[NC1];
            int k1 = keys[0];
            if constexpr (!SLOTS) row_taps<M, 0, SPLIT, SLOTS>(h1, ts, k1);
            const bool more = w + 1 < wend;
            const __amdgpu_buffer_rsrc_t rn = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(A.in + (size_t)(more ? w + 1 : w) * plane), 0, pbytes, kRawBufferWord3);
            float2* Tn = T[cur ^ 1];
            // Column biases of the copy, formed again in the last pass (from a
            // lane index the compiler cannot see through, so they are not kept
            // in registers across the whole loop).
            int biasn[stage_chunks<M>()];
            auto copy_next = [&](auto I) {
                constexpr int i = decltype(I)::value;
                if constexpr (i == 0) {
                    int ln = lane;
                    __asm__ volatile("" : "+v"(ln));
                    stage_bias<M>(biasn, y0, A.ny, ln);
                    // the next frequency's slots (om was loaded one ahead)
                    if constexpr (SLOTS)
                        if (more) copy_slots(TS[cur ^ 1] + wave * kSlots3 * kSlotF2, om / A.dk);
                }
                constexpr int PRE = 2 * M > 0 ? 2 * M : 1;  // rows of the pass carrying the copy
                constexpr int q0 = i < PRE ? i : QW;
                constexpr int q1 = i + 1 < PRE ? (i + 1 < QW ? i + 1 : QW) : (i < PRE ? QW : 0);
                if constexpr (q0 < q1) {
                    if (more) stage_rows<M, q0, q1>(Tn, rn, biasn, x0, y0, A.ny, wave, lane);
                }
            };
            auto no_copy = [](auto) {};

            const float2* Tw = Tb + r0 * W + lane + M;  // tile row of x0 + r0 - M, column y
            const __amdgpu_buffer_rsrc_t rq =
                __builtin_amdgcn_make_buffer_rsrc((void*)(A.out + (size_t)w * plane), 0, pbytes,
                                                  kRawBufferWord3);
            float2 acc[kRows3];
#pragma unroll
            for (int r = 0; r < kRows3; ++r) acc[r] = make_float2(0.0f, 0.0f);
            if constexpr (SLOTS) {
                // A wave whose points all share one slot keeps its taps in
                // registers (loaded once per pass, no reload), and takes the
                // plane split; the others read taps from LDS row by row in one
                // pass.  Passes hold no barrier, so waves may differ.
                auto lds_pass = [&]() {
                    float2 hu[NU];  // unused: taps come from LDS
                    int ku = 0;
                    fir_pass<M, 0, M + 1, true, true, true, true>(Tw, ts, keys, hu, ku, acc, img,
                                                                  rq, qbase, ny8, Wr, copy_next);
                };
                if constexpr (SPLIT <= M) {
                    if (one_slot) {
                        row_taps<M, 0, SPLIT, true>(h1, ts, k1);
                        fir_pass<M, 0, SPLIT, false, true, true, false>(Tw, ts, keys, h1, k1, acc,
                                                                        img, rq, qbase, ny8, Wr,
                                                                        no_copy);
                        float2 h2[NC2];
                        int k2 = -1;
                        fir_pass<M, SPLIT, M + 1, true, false, true, false>(Tw, ts, keys, h2, k2,
                                                                            acc, img, rq, qbase,
                                                                            ny8, Wr, copy_next);
                    } else {
                        lds_pass();
                    }
                } else {
                    lds_pass();
                }
            } else if constexpr (SPLIT <= M) {
                fir_pass<M, 0, SPLIT, false, true, false, false>(Tw, ts, keys, h1, k1, acc, img,
                                                                 rq, qbase, ny8, Wr, no_copy);
                float2 h2[NC2];
                int k2 = -1;
                fir_pass<M, SPLIT, M + 1, true, false, false, false>(Tw, ts, keys, h2, k2, acc,
                                                                     img, rq, qbase, ny8, Wr,
                                                                     copy_next);
            } else {
                fir_pass<M, 0, M + 1, true, true, false, false>(Tw, ts, keys, h1, k1, acc, img, rq,
                                                                qbase, ny8, Wr, copy_next);
            }
        }
    };
    if (use_slots)
        frequencies(std::true_type{});
    else
        frequencies(std::false_type{});

#pragma unroll
    for (int r = 0; r < kRows3; ++r) {
        const int x = x0 + r0 + r;
        if (x < A.nx && y < A.ny) A.part[(size_t)g * plane + (size_t)x * A.ny + y] = img[r];
    }
}

// Image of a plane: row[p] = sum over frequencies, in order, of Re wf[w][p].
__global__ void k_image3d(const float2* __restrict__ wf, double* __restrict__ row, size_t plane,
                          int nw)
{
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < plane;
         p += (size_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int w0 = 0; w0 < nw; w0 += 16) {
            float v[16];  // loads in flight, summed in frequency order
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i] = w0 + i < nw ? wf[(size_t)(w0 + i) * plane + p].x : 0.0f;
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (w0 + i < nw) s += (double)v[i];
        }
        row[p] = s;
    }
}

// row[p] = sum over groups, in order, of part[g][p].
__global__ void k_reduce3d(const double* __restrict__ part, double* __restrict__ row, size_t plane,
                           int ngroups)
{
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < plane;
         p += (size_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int q0 = 0; q0 < ngroups; q0 += 16) {
            double v[16];  // loads in flight, summed in group order
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i] = q0 + i < ngroups ? part[(size_t)(q0 + i) * plane + p] : 0.0;
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (q0 + i < ngroups) s += v[i];
        }
        row[p] = s;
    }
}

unsigned grid_for(size_t n)
{
    size_t b = (n + 255) / 256;
    return (unsigned)(b > 65535 ? 65535 : (b < 1 ? 1 : b));
}

}  // namespace

int step3d_tiles_x(int nx) { return (nx + kTileX3 - 1) / kTileX3; }
int step3d_tiles_y(int ny) { return (ny + kLanes3 - 1) / kLanes3; }

int launch_step3d(const Step3dArgs& a, int M, hipStream_t s)
{
    const unsigned nb = (unsigned)(a.tiles_x * a.tiles_y * a.ngroups);
    switch (M) {
    case 0: hipLaunchKernelGGL(k_step3d<0>, dim3(nb), dim3(kThreads3), 0, s, a); break;
    case 1: hipLaunchKernelGGL(k_step3d<1>, dim3(nb), dim3(kThreads3), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_step3d<2>, dim3(nb), dim3(kThreads3), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_step3d<3>, dim3(nb), dim3(kThreads3), 0, s, a); break;
    case 4: hipLaunchKernelGGL(k_step3d<4>, dim3(nb), dim3(kThreads3), 0, s, a); break;
    case 5: hipLaunchKernelGGL(k_step3d<5>, dim3(nb), dim3(kThreads3), 0, s, a); break;
    default: return MIG_E_ARG;
    }
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

int launch_image3d(const float2* wf, double* row, size_t plane, int nw, hipStream_t s)
{
    hipLaunchKernelGGL(k_image3d, dim3(grid_for(plane)), dim3(256), 0, s, wf, row, plane, nw);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

int launch_reduce3d(const double* part, double* row, size_t plane, int ngroups, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce3d, dim3(grid_for(plane)), dim3(256), 0, s, part, row, plane,
                       ngroups);
    return hipGetLastError() == hipSuccess ? MIG_OK : MIG_E_DEVICE;
}

}  // namespace mig
