// C ABI of libmig.so (declarations and contracts in include/mig.h).
//
// Host code here only validates arguments, lays out the caller's workspace and
// launches kernels; every arithmetic step of the method runs on the GPU.
#include <string.h>

#include <algorithm>
#include <functional>
#include <mutex>
#include <queue>
#include <vector>

#include "common.hpp"

using namespace mig;

namespace {

constexpr size_t kAlign = 256;

bool desc_valid(const mig_table_desc* d)
{
    if (!d) return false;
    if (d->ntaps < 1 || d->ntaps > MIG_MAX_NTAPS || (d->ntaps % 2) == 0) return false;
    if (d->nk < 2) return false;
    if (!(d->kmin > 0.0) || !(d->kmax > d->kmin)) return false;
    if (!(d->dx > 0.0) || !(d->dz >= 0.0)) return false;
    if (d->reserved != 0) return false;
    return true;
}

bool design_desc_valid(const mig_table_desc* d)
{
    if (!desc_valid(d)) return false;
    if (d->ngrid < 8 || d->ngrid > 2048 || d->ncheck < 8 || d->ncheck > (1 << 20)) return false;
    if (d->nreweight < 0 || d->nreweight > 1000) return false;
    if (!(d->w_pass > 0.0) || !(d->w_trans > 0.0) || !(d->w_evan > 0.0)) return false;
    if (!(d->lambda >= 0.0) || !(d->beta >= 0.0) || !(d->tau > 0.0)) return false;
    if (!(d->margin >= 0.0) || !(d->margin < 1.0)) return false;
    if (!(d->theta_max_deg > 0.0) || !(d->theta_max_deg <= 90.0)) return false;
    return true;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb)
{
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + nb && pb < pa + na;
}

size_t plane_bytes(int nx, int nw) { return align_up((size_t)nx * nw * sizeof(float2), kAlign); }

// Workspace per depth step: one slowness row (+ one partial-row plane when
// image rows are formed).
size_t step_bytes(int nx, int nw, bool rows)
{
    size_t b = (size_t)row_stride(nx) * sizeof(double);
    if (rows) b += (size_t)nw * row_stride(nx) * sizeof(float);
    return b;
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// Fixed workspace region for the published-block counters of one launch.
constexpr size_t kCounterBytes = 16384;
// the last two words are the launch's publish count (reducers' stall clock)
// and its abandon word
constexpr int kMaxBlocks = (int)(kCounterBytes / sizeof(int)) - 2;
constexpr int kMaxChunk = kMaxBlocks * kPublish;
constexpr int kMaxThreads = 512;

int device_cus()
{
    int dev = 0, ncu = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        ncu = 256;
    return ncu;
}

// Reducer workgroups beside `nprod` frequency workgroups: by default the CUs
// they leave idle, at most 32 (more reducers than keep pace only add memory
// traffic beside the frequency workgroups: configuration 2 runs 3 % slower
// with 56 than with 24-32); at least 8, at most 64 when asked for (before
// capping by the number of tasks), and never more than a quarter of the
// device's CUs, so that frequency workgroups always find CUs to run on while
// reducers wait for them.
int reducer_count(int nprod, int want)
{
    const int cus = device_cus();
    const int cap = cus / 4 > 1 ? cus / 4 : 1;
    int n = want > 0 ? want : (cus - nprod < 32 ? cus - nprod : 32);
    if (n < 8) n = 8;
    if (n > 64) n = 64;
    return n < cap ? n : cap;
}

int blocks_of(int nsteps) { return (nsteps + kPublish - 1) / kPublish; }

// x-parts per published block of a section: parts 32 points wide, so
// that a task is one pair of points per thread of a 512-thread workgroup for
// the 32 steps of a block.  A task then takes about half a block period, and
// the reducers keep up with the frequency workgroups instead of trailing them
// by a task's length at the end of the launch.
int parts_of(int nx) { return (nx + 31) / 32; }

// Frequencies per workgroup for one section in the register-tap kernel with two
// outputs per thread: `want` if given (clamped to what fits), else 1.
int omegas_per_group(int kind, int nx, int want)
{
    if (kind != 1) return 1;
    int fit = kMaxThreads / threads_per_omega(1, nx);
    if (fit < 1) fit = 1;
    int g = want > 0 ? want : 1;
    return g < fit ? g : fit;
}

struct Tuning {
    int G = 0;              // frequencies per workgroup (0 = default)
    int nred = 0;           // reducer workgroups (0 = default)
    int stall_us = 0;       // reducer stall limit in microseconds (0 = default)
    int flags = 0;          // MIG_TUNE_* bits
    int q_mid = 0;          // outputs per thread for 1025..1536 points (0 = 3)
};

Tuning tuning_of(const mig_tuning* t)
{
    Tuning tn;
    if (t) {
        tn.G = t->omegas_per_group;
        tn.nred = t->reducers;
        tn.stall_us = t->stall_limit_us;
        tn.flags = t->flags;
        tn.q_mid = t->outputs_mid;
    }
    return tn;
}

bool tuning_valid(const mig_tuning* t)
{
    return !t || (t->omegas_per_group >= 0 && t->reducers >= 0 && t->stall_limit_us >= 0 &&
                  (t->flags & ~MIG_TUNE_FORCE_STALL) == 0 &&
                  (t->outputs_mid == 0 || t->outputs_mid == 3 || t->outputs_mid == 4));
}

// Kernel variant of a batched section: the library's choice, except that
// sections of 1025..1536 points take the four-output kernel when tuned so.
int batch_kernel_kind(int nx, int M, const Tuning& tn)
{
    const int kind = extrap_kernel_kind(nx, M);
    return (kind == 3 && tn.q_mid == 4) ? 2 : kind;
}

// Calls that run no depth step still leave a defined status in a workspace
// they were given.
int clear_status(void* ws, size_t ws_bytes, hipStream_t s)
{
    if (!ws || ws_bytes < kStatusBytes) return MIG_OK;
    return launch_clear_status(static_cast<int*>(ws), s);
}

void set_reducer_limits(BatchArgs& a, const Tuning& tn)
{
    a.stall_ticks = tn.stall_us > 0 ? (unsigned long long)tn.stall_us * kWallTicksPerUs : kStallTicks;
    a.extra_wait = (tn.flags & MIG_TUNE_FORCE_STALL) ? 1 : 0;
}

// Bytes of the depth-loop workspace before the per-step regions.
size_t extrap_head_bytes(int nx, int nw)
{
    return kStatusBytes + plane_bytes(nx, nw) + kCounterBytes + (size_t)row_stride(nx) * sizeof(float);
}

// Depth loop of one section, split into chunks that fit the workspace.
// Workspace layout: [status word][scratch plane][counters][trash row]
// [slowness chunk x ldp doubles][partials chunk x nw x ldp floats].
int run_extrap(const float2* src, float2* dst, const float* vel, const double* omega,
               const float2* tab, const mig_table_desc* d, int nx, int nw, int nsteps,
               double* rows, void* ws, size_t ws_bytes, hipStream_t s, const Tuning& tn)
{
    const int ldp = row_stride(nx);
    const size_t head = extrap_head_bytes(nx, nw);
    const size_t sb = step_bytes(nx, nw, rows != nullptr);
    if (!ws || ws_bytes < head + sb) return MIG_E_WORKSPACE;
    size_t fit = (ws_bytes - head) / sb;
    int chunk = fit >= (size_t)nsteps ? nsteps : (int)fit;
    if (chunk > kMaxChunk) chunk = kMaxChunk;
    // ldp is a multiple of 256, so every region below stays 1 KB-aligned.
    char* base = static_cast<char*>(ws);
    int* status = reinterpret_cast<int*>(base);
    base += kStatusBytes;
    float2* mid = reinterpret_cast<float2*>(base);
    int* cnt = reinterpret_cast<int*>(base + plane_bytes(nx, nw));
    float* trash = reinterpret_cast<float*>(base + plane_bytes(nx, nw) + kCounterBytes);
    double* slow = reinterpret_cast<double*>(static_cast<char*>(ws) + head);
    float* part = reinterpret_cast<float*>(static_cast<char*>(ws) + head +
                                           (size_t)chunk * ldp * sizeof(double));

    const int M = (d->ntaps - 1) / 2;
    const int kind = extrap_kernel_kind(nx, M);
    const int G = omegas_per_group(kind, nx, tn.G);
    const int nitems = (nw + G - 1) / G;

    BatchArgs a = {};
    a.one.omega = omega;
    a.one.slow = slow;
    a.one.part = rows ? part : nullptr;
    a.one.cnt = cnt;
    a.one.nx = nx;
    a.one.nw = nw;
    a.one.ldp = ldp;
    a.one.nprod = nitems;
    a.one.G = G;
    a.tab = tab;
    a.trash = trash;
    a.progress = cnt + kMaxBlocks;
    a.status = status;
    set_reducer_limits(a, tn);
    a.nsec = 1;
    a.nitems = nitems;
    a.nk = d->nk;
    a.M = M;
    a.dk = (d->kmax - d->kmin) / (double)(d->nk - 1);
    a.b = d->kmin / a.dk;

    const float2* cur = src;
    for (int c0 = 0; c0 < nsteps; c0 += chunk) {
        int cs = nsteps - c0 < chunk ? nsteps - c0 : chunk;
        bool last = c0 + cs == nsteps;
        a.one.win = cur;
        // Intermediate planes go to the scratch plane, in place: each workgroup
        // reads its whole frequency columns before writing them back.
        a.one.wout = last ? dst : mid;
        a.one.vel = vel + (size_t)c0 * nx;
        a.one.nsteps = cs;
        a.one.rows = rows ? rows + (size_t)c0 * nx : nullptr;
        // Reducer workgroups form the rows of every published block but the
        // last, overlapped with the depth stepping; the last block, which
        // nothing is left to overlap with, is reduced after the launch by the
        // whole GPU (launch_rows).
        const int nb = blocks_of(cs);
        a.rows = rows ? 1 : 0;
        if (rows && nb > 1) {
            const int nred = reducer_count(nitems, tn.nred);
            a.parts = parts_of(nx);
            a.ntasks = (nb - 1) * a.parts;
            a.nred = nred < a.ntasks ? nred : a.ntasks;
        } else {
            a.parts = 1;
            a.ntasks = 0;
            a.nred = 0;
        }
        // the slowness launch also zeroes the block counters, and the status
        // word at the first chunk of the call
        a.reset_status = c0 == 0 ? 1 : 0;
        int rc = launch_slowness(a, cs, ldp, flag_distance(kind), s);
        if (rc == MIG_OK) {
            if (kind == 0) rc = launch_general(a, nx, s);
            else rc = launch_extrap(a, kind, G * threads_per_omega(kind, nx), s);
        }
        if (rc == MIG_OK && rows) rc = launch_rows(part, a.one.rows, (nb - 1) * kPublish, cs, nx, nw, ldp, s);
        if (rc != MIG_OK) return rc;
        cur = mid;
    }
    return MIG_OK;
}

bool sizes_ok(int nx, int nw) { return nx >= 1 && nx <= MIG_MAX_NX && nw >= 1 && nw <= MIG_MAX_NW; }

// ---------------------------------------------------------------------------
// Batched form: many independent sections in at most four launches (one per
// kernel variant).  The layout of the workspace is computed by one planner,
// used both by the size query (base == nullptr) and by the run.
// ---------------------------------------------------------------------------
struct BatchPlan {
    size_t bytes = 0;
    struct Group {
        int kind = 0, threads = 0, max_nx = 0, max_rows = 0, max_ldp = 0, nred = 0, parts = 1;
        std::vector<SecDev> secs;
        std::vector<ItemDev> items;
        std::vector<TaskDev> tasks;
        size_t desc_off = 0, desc_bytes = 0;  // SecDev + ItemDev + TaskDev arrays
        size_t cnt_off = 0;
        int ncnt = 0;
    } group[4];
    size_t trash_off = 0;
};

size_t bump(size_t& off, size_t n)
{
    size_t at = align_up(off, kAlign);
    off = at + n;
    return at;
}

bool sections_ok(const mig_section* secs, int nsec)
{
    if (!secs || nsec < 1) return false;
    for (int i = 0; i < nsec; ++i) {
        const mig_section& q = secs[i];
        if (!q.data || !q.vel || !q.omega || !q.image || !sizes_ok(q.nx, q.nw) || q.nz < 1 ||
            q.reserved != 0)
            return false;
    }
    return true;
}

// Relative time of one depth step of a workgroup item in kernel `kind`: the
// busiest SIMD runs ceil(waves / 4) waves, each with q outputs per thread
// (the general kernel: 4 waves, ceil(nx / 256) outputs per thread).  Only
// used to order reducer tasks.
double step_cost(int kind, const SecDev& S)
{
    if (kind == 0) return (double)((S.nx + 255) / 256);
    const int q = kind == 1 ? 2 : (kind == 2 ? 4 : 3);
    const int waves = S.G * threads_per_omega(kind, S.nx) / 64;
    return (double)((waves + 3) / 4 * q);
}

void plan_batch(const mig_section* secs, int nsec, const mig_table_desc* d, const Tuning& tn,
                char* base, BatchPlan& P)
{
    const int M = (d->ntaps - 1) / 2;
    size_t off = kStatusBytes;  // [status word] first, as for a single section
    int max_ldp = 0;
    for (int i = 0; i < nsec; ++i) max_ldp = row_stride(secs[i].nx) > max_ldp ? row_stride(secs[i].nx) : max_ldp;
    P.trash_off = bump(off, (size_t)max_ldp * sizeof(float));
    for (int i = 0; i < nsec; ++i) {
        const mig_section& q = secs[i];
        if (q.nz < 2) continue;
        const int kind = batch_kernel_kind(q.nx, M, tn);
        BatchPlan::Group& g = P.group[kind];
        g.kind = kind;
        SecDev S = {};
        S.win = reinterpret_cast<const float2*>(q.data);
        S.wout = nullptr;
        S.vel = q.vel;
        S.omega = q.omega;
        S.rows = q.image + q.nx;
        S.nx = q.nx;
        S.nw = q.nw;
        S.nsteps = q.nz - 1;
        S.ldp = row_stride(q.nx);
        S.G = omegas_per_group(kind, q.nx, tn.G > 0 ? tn.G : kMaxThreads);
        S.nprod = (q.nw + S.G - 1) / S.G;
        size_t so = bump(off, (size_t)S.nsteps * S.ldp * sizeof(double));
        size_t po = bump(off, (size_t)S.nsteps * S.nw * S.ldp * sizeof(float));
        S.slow = reinterpret_cast<const double*>(base ? base + so : nullptr);
        S.part = reinterpret_cast<float*>(base ? base + po : nullptr);
        S.cnt = reinterpret_cast<int*>((size_t)g.ncnt);  // offset, fixed up below
        g.ncnt += (S.nsteps + kPublish - 1) / kPublish;
        const int tpo = threads_per_omega(kind, q.nx);
        const int th = kind == 0 ? 256 : S.G * tpo;
        g.threads = th > g.threads ? th : g.threads;
        g.max_nx = q.nx > g.max_nx ? q.nx : g.max_nx;
        g.max_rows = S.nsteps > g.max_rows ? S.nsteps : g.max_rows;
        g.max_ldp = S.ldp > g.max_ldp ? S.ldp : g.max_ldp;
        g.secs.push_back(S);
    }
    for (int k = 0; k < 4; ++k) {
        BatchPlan::Group& g = P.group[k];
        if (g.secs.empty()) continue;
        g.cnt_off = bump(off, (size_t)(g.ncnt + 2) * sizeof(int));  // + publish count, abandon
        for (SecDev& S : g.secs)
            S.cnt = reinterpret_cast<int*>(base ? base + g.cnt_off + (size_t)S.cnt * sizeof(int) : nullptr);
        // Items: longest first (depth steps x points), so the tail of the
        // launch is made of short items.
        std::vector<int> order(g.secs.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            return (long long)g.secs[x].nsteps * g.secs[x].nx > (long long)g.secs[y].nsteps * g.secs[y].nx;
        });
        for (int si : order)
            for (int r0 = 0; r0 < g.secs[si].nw; r0 += g.secs[si].G) g.items.push_back(ItemDev{si, r0});
        g.nred = reducer_count((int)g.items.size(), tn.nred);
        g.parts = parts_of(g.secs[0].nx);  // read by a batch of one section only
        // Reducer tasks in the order their blocks are expected to be published
        // (reducers take tasks round-robin and wait for each in turn).  Items
        // start in launch order on the CUs the reducers leave free; block c of
        // a section is published when its last-starting item has done
        // (c + 1) * kPublish steps.
        const int slots = device_cus() - g.nred > 1 ? device_cus() - g.nred : 1;
        std::vector<double> last_start(g.secs.size(), 0.0);
        std::priority_queue<double, std::vector<double>, std::greater<double>> free_at;
        for (int i = 0; i < slots; ++i) free_at.push(0.0);
        for (const ItemDev& it : g.items) {
            const double t0 = free_at.top();
            free_at.pop();
            free_at.push(t0 + g.secs[it.sec].nsteps * step_cost(k, g.secs[it.sec]));
            last_start[it.sec] = t0 > last_start[it.sec] ? t0 : last_start[it.sec];
        }
        struct Blk {
            double t;
            int sec, c;
        };
        std::vector<Blk> blks;
        for (int c = 0; c < blocks_of(g.max_rows); ++c)
            for (int si : order) {
                const SecDev& S = g.secs[si];
                if (c >= blocks_of(S.nsteps)) continue;
                const int done = (c + 1) * kPublish < S.nsteps ? (c + 1) * kPublish : S.nsteps;
                blks.push_back(Blk{last_start[si] + done * step_cost(k, S), si, c});
            }
        std::stable_sort(blks.begin(), blks.end(), [](const Blk& x, const Blk& y) { return x.t < y.t; });
        for (const Blk& b : blks) {
            const int nx = g.secs[b.sec].nx;
            const int parts = parts_of(nx);
            const int span = ((nx + parts - 1) / parts + 1) & ~1;
            // exactly `parts` tasks per block (trailing ones may be empty), as
            // task_of derives them for a batch of one section
            for (int p = 0; p < parts; ++p) {
                const int x0 = p * span < nx ? p * span : nx;
                g.tasks.push_back(TaskDev{b.sec, b.c, x0, x0 + span < nx ? x0 + span : nx});
            }
        }
        g.desc_bytes = g.secs.size() * sizeof(SecDev) + g.items.size() * sizeof(ItemDev) +
                       g.tasks.size() * sizeof(TaskDev);
        g.desc_off = bump(off, g.desc_bytes);
    }
    P.bytes = align_up(off, kAlign);
}

int run_batch(const mig_section* secs, int nsec, const float2* tab, const mig_table_desc* d,
              const Tuning& tn, void* ws, size_t ws_bytes, hipStream_t s)
{
    BatchPlan P;
    char* base = static_cast<char*>(ws);
    plan_batch(secs, nsec, d, tn, base, P);
    if (!ws || ws_bytes < P.bytes) return MIG_E_WORKSPACE;
    // The descriptors of every kernel variant go to the workspace in one copy
    // from a host buffer owned by this call; the call waits for that copy
    // (and so for the stream's earlier work) before the buffer goes away.
    size_t lo = 0, hi = 0;
    for (const BatchPlan::Group& g : P.group)
        if (!g.secs.empty()) {
            lo = lo == 0 && hi == 0 ? g.desc_off : (g.desc_off < lo ? g.desc_off : lo);
            hi = g.desc_off + g.desc_bytes > hi ? g.desc_off + g.desc_bytes : hi;
        }
    if (hi > lo) {
        std::vector<char> host(hi - lo, 0);
        for (const BatchPlan::Group& g : P.group) {
            if (g.secs.empty()) continue;
            char* o = host.data() + (g.desc_off - lo);
            memcpy(o, g.secs.data(), g.secs.size() * sizeof(SecDev));
            o += g.secs.size() * sizeof(SecDev);
            memcpy(o, g.items.data(), g.items.size() * sizeof(ItemDev));
            o += g.items.size() * sizeof(ItemDev);
            memcpy(o, g.tasks.data(), g.tasks.size() * sizeof(TaskDev));
        }
        if (hipMemcpyAsync(base + lo, host.data(), hi - lo, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return MIG_E_DEVICE;
    }
    for (int i = 0; i < nsec; ++i) {
        int rc = launch_image(reinterpret_cast<const float2*>(secs[i].data), secs[i].image,
                              secs[i].nx, secs[i].nw, s);
        if (rc != MIG_OK) return rc;
    }
    const int M = (d->ntaps - 1) / 2;
    // wide sections first: their items are the longest
    const int kinds[4] = {2, 3, 1, 0};
    bool first = true;
    for (int kk = 0; kk < 4; ++kk) {
        BatchPlan::Group& g = P.group[kinds[kk]];
        if (g.secs.empty()) continue;
        char* dev = base + g.desc_off;
        BatchArgs a = {};
        a.secs = reinterpret_cast<const SecDev*>(dev);
        a.items = reinterpret_cast<const ItemDev*>(dev + g.secs.size() * sizeof(SecDev));
        a.tasks = reinterpret_cast<const TaskDev*>(dev + g.secs.size() * sizeof(SecDev) +
                                                   g.items.size() * sizeof(ItemDev));
        a.tab = tab;
        a.trash = reinterpret_cast<float*>(base + P.trash_off);
        a.progress = reinterpret_cast<int*>(base + g.cnt_off) + g.ncnt;
        a.status = reinterpret_cast<int*>(base);
        a.reset_status = first ? 1 : 0;
        first = false;
        set_reducer_limits(a, tn);
        a.nsec = (int)g.secs.size();
        a.nitems = (int)g.items.size();
        a.ntasks = (int)g.tasks.size();
        a.nred = g.nred < a.ntasks ? g.nred : a.ntasks;
        a.rows = a.nred > 0 ? 1 : 0;
        // a batch of one section derives its tasks from `parts` (task_of) with
        // the same split as the task list built by the planner
        a.parts = g.parts;
        a.nk = d->nk;
        a.M = M;
        a.dk = (d->kmax - d->kmin) / (double)(d->nk - 1);
        a.b = d->kmin / a.dk;
        if (a.nsec == 1) {
            // a batch of one section uses the argument-resident descriptor
            a.one = g.secs[0];
            a.secs = nullptr;
            a.items = nullptr;
            a.tasks = nullptr;
        }
        // the slowness launch also zeroes every section's block counters
        int rc = launch_slowness(a, g.max_rows, g.max_ldp, flag_distance(g.kind), s);
        if (rc == MIG_OK) {
            if (g.kind == 0) rc = launch_general(a, g.max_nx, s);
            else rc = launch_extrap(a, g.kind, g.threads, s);
        }
        if (rc != MIG_OK) return rc;
    }
    return MIG_OK;
}

// Allocation-free form of mig_migrate: the workspace is a static device array,
// one per GPU (the loader creates it with the code object), held until the
// process ends.  In host code `scratch` names a host-side stand-in, not device
// memory: its device address is looked up once per device with
// hipGetSymbolAddress and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[MIG_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's static workspace, or nullptr.
void* static_scratch()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

MIG_API const char* mig_strerror(int code)
{
    switch (code) {
    case MIG_OK: return "success";
    case MIG_E_ARG: return "invalid argument";
    case MIG_E_UNSTABLE: return "designed table failed the |H| <= 1 check";
    case MIG_E_DEVICE: return "HIP launch or runtime error";
    case MIG_E_WORKSPACE: return "workspace missing or too small";
    default: return "unknown status";
    }
}

MIG_API const char* mig_version(void) { return "libmig 0.1 (gfx950)"; }

MIG_API size_t mig_design_workspace_size(const mig_table_desc* d)
{
    if (!design_desc_valid(d)) return 0;
    const size_t K = (size_t)(d->ntaps - 1) / 2 + 1;
    return align_up((size_t)d->ngrid * K * sizeof(double), kAlign) +
           align_up((size_t)d->ncheck * K * sizeof(double), kAlign) +
           align_up((size_t)d->nk * sizeof(int), kAlign);
}

MIG_API int mig_design_table(const mig_table_desc* d, mig_c128* tab64, mig_c64* tab32,
                             double* maxgain, double* passerr, void* ws, size_t ws_bytes,
                             void* stream)
{
    if (!design_desc_valid(d) || !tab64) return MIG_E_ARG;
    const size_t need = mig_design_workspace_size(d);
    if (!ws || ws_bytes < need) return MIG_E_WORKSPACE;
    const size_t K = (size_t)(d->ntaps - 1) / 2 + 1;
    if (tab32 && overlap(tab64, d->nk * K * sizeof(mig_c128), tab32, d->nk * K * sizeof(mig_c64)))
        return MIG_E_ARG;
    hipStream_t s = as_stream(stream);
    char* p = static_cast<char*>(ws);
    double* A = reinterpret_cast<double*>(p);
    p += align_up((size_t)d->ngrid * K * sizeof(double), kAlign);
    double* C = reinterpret_cast<double*>(p);
    p += align_up((size_t)d->ncheck * K * sizeof(double), kAlign);
    int* status = reinterpret_cast<int*>(p);

    int rc = launch_design_basis(d, A, C, s);
    if (rc == MIG_OK) rc = launch_design(d, A, C, tab64, tab32, maxgain, passerr, status, s);
    if (rc != MIG_OK) return rc;
    if (hipStreamSynchronize(s) != hipSuccess) return MIG_E_DEVICE;
    int worst = 0;
    const int chunk = 1024;
    int buf[chunk];
    for (int j0 = 0; j0 < d->nk; j0 += chunk) {
        int n = d->nk - j0 < chunk ? d->nk - j0 : chunk;
        if (hipMemcpy(buf, status + j0, n * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
            return MIG_E_DEVICE;
        for (int i = 0; i < n; ++i) worst = buf[i] > worst ? buf[i] : worst;
    }
    if (worst == 2) return MIG_E_ARG;
    if (worst == 1) return MIG_E_UNSTABLE;
    return MIG_OK;
}

MIG_API int mig_table_index(const float* vel, const double* omega, const mig_table_desc* d,
                            int32_t nx, int32_t nw, int32_t nrows, int32_t* idx, void* stream)
{
    if (!desc_valid(d) || !vel || !omega || !idx || !sizes_ok(nx, nw) || nrows < 1)
        return MIG_E_ARG;
    const double dk = (d->kmax - d->kmin) / (double)(d->nk - 1);
    const double b = d->kmin / dk;
    return launch_index(vel, omega, nx, nw, nrows, d->nk, dk, b, idx, as_stream(stream));
}

MIG_API size_t mig_workspace_size(int32_t nx, int32_t nsteps, int32_t nw, const mig_table_desc* d)
{
    if (!desc_valid(d) || !sizes_ok(nx, nw) || nsteps < 0) return 0;
    size_t steps = nsteps > 0 ? (size_t)nsteps : 1;
    return extrap_head_bytes(nx, nw) + steps * step_bytes(nx, nw, true);
}

MIG_API size_t mig_workspace_min_size(int32_t nx, int32_t nw, const mig_table_desc* d)
{
    if (!desc_valid(d) || !sizes_ok(nx, nw)) return 0;
    return extrap_head_bytes(nx, nw) + step_bytes(nx, nw, true);
}

MIG_API int mig_workspace_status(const void* ws, void* stream)
{
    if (!ws) return MIG_E_ARG;
    hipStream_t s = as_stream(stream);
    int st = 0;
    if (hipStreamSynchronize(s) != hipSuccess ||
        hipMemcpy(&st, ws, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return MIG_E_DEVICE;
    return st == 0 ? MIG_OK : MIG_E_DEVICE;
}

MIG_API int mig_extrapolate(const mig_c64* wf_in, mig_c64* wf_out, const float* vel,
                            const double* omega, const mig_c64* tab32, const mig_table_desc* d,
                            int32_t nx, int32_t nw, int32_t nsteps, double* rows, void* ws,
                            size_t ws_bytes, void* stream)
{
    if (!desc_valid(d) || !wf_in || !vel || !omega || !tab32 || !sizes_ok(nx, nw) || nsteps < 0)
        return MIG_E_ARG;
    if (!wf_out && !rows) return MIG_E_ARG;
    const size_t pl = (size_t)nx * nw * sizeof(mig_c64);
    if (wf_out && overlap(wf_in, pl, wf_out, pl)) return MIG_E_ARG;
    hipStream_t s = as_stream(stream);
    const float2* src = reinterpret_cast<const float2*>(wf_in);
    float2* dst = reinterpret_cast<float2*>(wf_out);
    if (nsteps == 0) {
        if (wf_out && hipMemcpyAsync(dst, src, pl, hipMemcpyDeviceToDevice, s) != hipSuccess)
            return MIG_E_DEVICE;
        return clear_status(ws, ws_bytes, s);
    }
    if (ws && (overlap(ws, ws_bytes, wf_in, pl) || (wf_out && overlap(ws, ws_bytes, wf_out, pl))))
        return MIG_E_ARG;
    return run_extrap(src, dst, vel, omega, reinterpret_cast<const float2*>(tab32), d, nx, nw,
                      nsteps, rows, ws, ws_bytes, s, Tuning{});
}

MIG_API int mig_image(const mig_c64* wf, double* row, int32_t nx, int32_t nw, void* stream)
{
    if (!wf || !row || !sizes_ok(nx, nw)) return MIG_E_ARG;
    return launch_image(reinterpret_cast<const float2*>(wf), row, nx, nw, as_stream(stream));
}

MIG_API int mig_migrate(const mig_c64* data, const float* vel, const double* omega,
                        const mig_c64* tab32, const mig_table_desc* d, int32_t nx, int32_t nz,
                        int32_t nw, double* image, void* ws, size_t ws_bytes, void* stream)
{
    if (!desc_valid(d) || !data || !vel || !omega || !tab32 || !image || !sizes_ok(nx, nw) ||
        nz < 1)
        return MIG_E_ARG;
    hipStream_t s = as_stream(stream);
    int rc = launch_image(reinterpret_cast<const float2*>(data), image, nx, nw, s);
    if (rc != MIG_OK) return rc;
    if (nz == 1) return clear_status(ws, ws_bytes, s);
    const size_t pl = (size_t)nx * nw * sizeof(mig_c64);
    if (ws && overlap(ws, ws_bytes, data, pl)) return MIG_E_ARG;
    return run_extrap(reinterpret_cast<const float2*>(data), nullptr, vel, omega,
                      reinterpret_cast<const float2*>(tab32), d, nx, nw, nz - 1, image + nx, ws,
                      ws_bytes, s, Tuning{});
}

MIG_API int mig_migrate_noalloc(const mig_c64* data, const float* vel, const double* omega,
                                const mig_c64* tab32, const mig_table_desc* d, int32_t nx,
                                int32_t nz, int32_t nw, double* image, void* stream)
{
    if (!desc_valid(d) || !data || !vel || !omega || !tab32 || !image || !sizes_ok(nx, nw) ||
        nz < 1)
        return MIG_E_ARG;
    // at least one depth step (plus the plane between chunks) must fit
    if (mig_workspace_min_size(nx, nw, d) > (size_t)MIG_STATIC_SCRATCH_BYTES) return MIG_E_WORKSPACE;
    void* ws = static_scratch();
    if (!ws) return MIG_E_DEVICE;
    return mig_migrate(data, vel, omega, tab32, d, nx, nz, nw, image, ws,
                       (size_t)MIG_STATIC_SCRATCH_BYTES, stream);
}

MIG_API size_t mig_batch_workspace_size(const mig_section* secs, int32_t nsec,
                                        const mig_table_desc* d, const mig_tuning* tune)
{
    if (!desc_valid(d) || !sections_ok(secs, nsec) || !tuning_valid(tune)) return 0;
    Tuning tn = tuning_of(tune);
    BatchPlan P;
    plan_batch(secs, nsec, d, tn, nullptr, P);
    return P.bytes;
}

MIG_API int mig_migrate_batched(const mig_section* secs, int32_t nsec, const mig_c64* tab32,
                                const mig_table_desc* d, const mig_tuning* tune, void* ws,
                                size_t ws_bytes, void* stream)
{
    if (!desc_valid(d) || !tab32 || !sections_ok(secs, nsec) || !tuning_valid(tune))
        return MIG_E_ARG;
    for (int i = 0; i < nsec; ++i) {
        const size_t pl = (size_t)secs[i].nx * secs[i].nw * sizeof(mig_c64);
        if (ws && overlap(ws, ws_bytes, secs[i].data, pl)) return MIG_E_ARG;
    }
    Tuning tn = tuning_of(tune);
    return run_batch(secs, nsec, reinterpret_cast<const float2*>(tab32), d, tn, ws, ws_bytes,
                     as_stream(stream));
}

// Demigration workspace: [slowness rows][dense flag][change points per row]
// [(left, right) entries per row, frequency and change point].
static size_t demig_slow_bytes(int32_t nx, int32_t nz)
{
    const size_t rows = nz > 1 ? (size_t)(nz - 1) : 1;
    return align_up(rows * row_stride(nx) * sizeof(double), kAlign);
}

MIG_API size_t mig_demigrate_workspace_size(int32_t nx, int32_t nz, int32_t nw,
                                            const mig_table_desc* d)
{
    if (!desc_valid(d) || !sizes_ok(nx, nw) || nz < 1) return 0;
    const size_t rows = nz > 1 ? (size_t)(nz - 1) : 1;
    return demig_slow_bytes(nx, nz) + kAlign + align_up(rows * sizeof(AdjRow), kAlign) +
           align_up(rows * nw * kAdjKmax * sizeof(int), kAlign);
}

MIG_API int mig_demigrate(const double* image, const float* vel, const double* omega,
                          const mig_c64* tab32, const mig_table_desc* d, int32_t nx, int32_t nz,
                          int32_t nw, mig_c64* data, void* ws, size_t ws_bytes, void* stream)
{
    if (!desc_valid(d) || !image || !vel || !omega || !tab32 || !data || !sizes_ok(nx, nw) ||
        nz < 1)
        return MIG_E_ARG;
    const size_t need = mig_demigrate_workspace_size(nx, nz, nw, d);
    if (!ws || ws_bytes < need) return MIG_E_WORKSPACE;
    if (overlap(ws, ws_bytes, data, (size_t)nx * nw * sizeof(mig_c64))) return MIG_E_ARG;
    int dev = 0, lds_max = 65536;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        lds_max = 65536;
    const int M = (d->ntaps - 1) / 2;
    AdjArgs a = {};
    const bool reg = adjoint_uses_registers(nx, M, (size_t)lds_max);
    const bool fold = reg && nz > 1 && d->nk <= 65536 && adjoint_uses_fold(nx, M);
    a.chunk = adjoint_chunk(nx, M, (size_t)lds_max);
    if (!reg && a.chunk < 1) return MIG_E_ARG;
    hipStream_t s = as_stream(stream);
    char* base = static_cast<char*>(ws);
    const size_t rows = nz > 1 ? (size_t)(nz - 1) : 1;
    a.image = image;
    a.slow = reinterpret_cast<const double*>(base);
    base += demig_slow_bytes(nx, nz);
    int* dense = reinterpret_cast<int*>(base);
    base += kAlign;
    a.chg = reinterpret_cast<AdjRow*>(base);
    base += align_up(rows * sizeof(AdjRow), kAlign);
    a.jpair = reinterpret_cast<int*>(base);
    a.dense = fold ? dense : nullptr;
    a.kmax = fold ? adjoint_fold_kmax(nx, M) : 0;
    a.omega = omega;
    a.tab = reinterpret_cast<const float2*>(tab32);
    a.out = reinterpret_cast<float2*>(data);
    a.nx = nx;
    a.nz = nz;
    a.nw = nw;
    a.ldp = row_stride(nx);
    a.nk = d->nk;
    a.M = M;
    a.dk = (d->kmax - d->kmin) / (double)(d->nk - 1);
    a.b = d->kmin / a.dk;
    if (nz > 1) {
        BatchArgs sa = {};
        sa.nsec = 1;
        sa.one.vel = vel;
        sa.one.slow = a.slow;
        sa.one.nx = nx;
        sa.one.nsteps = nz - 1;
        sa.one.ldp = a.ldp;
        // the slowness launch zeroes the dense flag
        sa.status = dense;
        sa.reset_status = 1;
        // change flags against the row one step deeper: walking depth upward,
        // the register-tap kernels refill a point's taps where its row differs
        // from the row below (the product kernel, whose two alternating tap
        // sets are two rows apart, where either of two rows in a row differs)
        int rc = launch_slowness(sa, nz - 1, a.ldp, -1, s);
        if (rc != MIG_OK) return rc;
    }
    if (!reg) return launch_demigrate(a, s);
    if (fold) {
        // the folded kernel runs unless some row has more change points than
        // it handles; the product kernel, launched after it, runs only then
        int rc = launch_adj_changes(a, s);
        if (rc == MIG_OK) rc = launch_demigrate_fold(a, s);
        if (rc != MIG_OK) return rc;
    }
    return launch_demigrate_reg(a, s);
}

MIG_API size_t mig_transform_workspace_size(int32_t nt, int32_t nw)
{
    if (nt < 1 || nt > MIG_MAX_NT || nw < 1 || nw > MIG_MAX_NW) return 0;
    return align_up((size_t)nt * 2 * nw * sizeof(float), kAlign);
}

MIG_API int mig_transform_t(const float* section, int32_t nx, int32_t nt, double dt,
                            const double* omega, int32_t nw, mig_c64* out, void* ws,
                            size_t ws_bytes, void* stream)
{
    if (!section || !omega || !out || !sizes_ok(nx, nw) || nt < 1 || nt > MIG_MAX_NT ||
        !(dt > 0.0))
        return MIG_E_ARG;
    const size_t need = mig_transform_workspace_size(nt, nw);
    if (!ws || ws_bytes < need) return MIG_E_WORKSPACE;
    if (overlap(section, (size_t)nx * nt * sizeof(float), out, (size_t)nx * nw * sizeof(mig_c64)) ||
        overlap(ws, ws_bytes, out, (size_t)nx * nw * sizeof(mig_c64)))
        return MIG_E_ARG;
    return launch_transform(section, nx, nt, dt, omega, nw, reinterpret_cast<float2*>(out),
                            static_cast<float*>(ws), as_stream(stream));
}

// Internal query used by tests and the benchmark: which extrapolation kernel
// a call with these sizes takes (1 = register-tap kernel, 0 = general).
MIG_API int mig_kernel_kind(int32_t nx, int32_t ntaps)
{
    if (ntaps < 1 || ntaps > MIG_MAX_NTAPS || (ntaps % 2) == 0 || nx < 1) return -1;
    return extrap_kernel_kind(nx, (ntaps - 1) / 2);
}

}  // extern "C"

// ---- 3-D extension ------------------------------------------------------ //

namespace {

bool design2d_desc_valid(const mig_table_desc* d)
{
    return design_desc_valid(d) && d->ntaps <= MIG_MAX_NTAPS_2D &&
           d->ngrid <= MIG_MAX_NGRID_2D && d->ncheck <= MIG_MAX_NCHECK_2D;
}

bool sizes3d_ok(int32_t nx, int32_t ny, int32_t nw, int32_t nz)
{
    // the depth-step kernel addresses one frequency plane with 32-bit offsets
    return nx >= 1 && nx <= MIG_MAX_NXY && ny >= 1 && ny <= MIG_MAX_NXY && nw >= 1 &&
           nw <= MIG_MAX_NW && nz >= 1 &&
           (unsigned long long)nx * (unsigned long long)ny <= MIG_MAX_PLANE_3D;
}

// Frequencies per workgroup group: `want` if given, else enough groups that
// the grid holds two workgroups per CU.
int omegas_per_group3d(int32_t nx, int32_t ny, int32_t nw, int32_t want)
{
    if (want > 0) return want < nw ? want : nw;
    const int tiles = step3d_tiles_x(nx) * step3d_tiles_y(ny);
    int groups = (2 * device_cus() + tiles - 1) / tiles;
    if (groups < 1) groups = 1;
    int wpg = (nw + groups - 1) / groups;
    return wpg < 1 ? 1 : wpg;
}

size_t plane3d_bytes(int32_t nx, int32_t ny, int32_t nw)
{
    return align_up((size_t)nx * ny * nw * sizeof(float2), kAlign);
}

size_t partial3d_bytes(int32_t nx, int32_t ny, int ngroups)
{
    return align_up((size_t)ngroups * nx * ny * sizeof(double), kAlign);
}

}  // namespace

MIG_API size_t mig_design2d_workspace_size(const mig_table_desc* d)
{
    if (!design2d_desc_valid(d)) return 0;
    const size_t M = (size_t)(d->ntaps - 1) / 2, NU = (M + 1) * (M + 2) / 2;
    return align_up((size_t)d->ngrid * d->ngrid * NU * sizeof(double), kAlign) +
           align_up((size_t)d->ncheck * (M + 1) * sizeof(double), kAlign) +
           align_up((size_t)d->nk * sizeof(int), kAlign);
}

MIG_API int mig_design_table_2d(const mig_table_desc* d, mig_c128* tab64, mig_c64* tab32,
                                double* maxgain, double* passerr, void* ws, size_t ws_bytes,
                                void* stream)
{
    if (!design2d_desc_valid(d) || !tab64) return MIG_E_ARG;
    const size_t need = mig_design2d_workspace_size(d);
    if (!ws || ws_bytes < need) return MIG_E_WORKSPACE;
    const size_t M = (size_t)(d->ntaps - 1) / 2, NU = (M + 1) * (M + 2) / 2;
    if (tab32 && overlap(tab64, d->nk * NU * sizeof(mig_c128), tab32, d->nk * NU * sizeof(mig_c64)))
        return MIG_E_ARG;
    hipStream_t s = as_stream(stream);
    char* p = static_cast<char*>(ws);
    double* A = reinterpret_cast<double*>(p);
    p += align_up((size_t)d->ngrid * d->ngrid * NU * sizeof(double), kAlign);
    double* CS = reinterpret_cast<double*>(p);
    p += align_up((size_t)d->ncheck * (M + 1) * sizeof(double), kAlign);
    int* status = reinterpret_cast<int*>(p);

    int rc = launch_design2d_basis(d, A, CS, s);
    if (rc == MIG_OK) rc = launch_design2d(d, A, CS, tab64, tab32, maxgain, passerr, status, s);
    if (rc != MIG_OK) return rc;
    if (hipStreamSynchronize(s) != hipSuccess) return MIG_E_DEVICE;
    std::vector<int> st((size_t)d->nk);
    if (hipMemcpy(st.data(), status, st.size() * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return MIG_E_DEVICE;
    int worst = 0;
    for (int v : st) worst = v > worst ? v : worst;
    if (worst == 2) return MIG_E_ARG;
    if (worst == 1) return MIG_E_UNSTABLE;
    return MIG_OK;
}

MIG_API int mig_omegas_per_group_3d(int32_t nx, int32_t ny, int32_t nw, int32_t want)
{
    if (!sizes3d_ok(nx, ny, nw, 1) || want < 0) return -1;
    return omegas_per_group3d(nx, ny, nw, want);
}

MIG_API size_t mig_migrate3d_workspace_size(int32_t nx, int32_t ny, int32_t nw, int32_t nz,
                                            int32_t omegas_per_group)
{
    if (!sizes3d_ok(nx, ny, nw, nz) || omegas_per_group < 0) return 0;
    const int wpg = omegas_per_group3d(nx, ny, nw, omegas_per_group);
    const int ngroups = (nw + wpg - 1) / wpg;
    return 2 * plane3d_bytes(nx, ny, nw) + 2 * partial3d_bytes(nx, ny, ngroups);
}

MIG_API int mig_migrate3d(const mig_c64* data, const float* vel, const double* omega,
                          const mig_c64* tab32, const mig_table_desc* d, int32_t nx, int32_t ny,
                          int32_t nw, int32_t nz, int32_t omegas_per_group, double* image,
                          mig_c64* plane_out, void* ws, size_t ws_bytes, void* stream)
{
    if (!desc_valid(d) || d->ntaps > MIG_MAX_NTAPS_2D || !data || !vel || !omega || !tab32 ||
        !image || !sizes3d_ok(nx, ny, nw, nz) || omegas_per_group < 0)
        return MIG_E_ARG;
    const size_t need = mig_migrate3d_workspace_size(nx, ny, nw, nz, omegas_per_group);
    if (!ws || ws_bytes < need) return MIG_E_WORKSPACE;
    const size_t plane = (size_t)nx * ny;
    const size_t pb = plane * nw * sizeof(mig_c64);
    if (overlap(ws, ws_bytes, data, pb) || overlap(ws, ws_bytes, image, plane * nz * sizeof(double)) ||
        (plane_out && (overlap(ws, ws_bytes, plane_out, pb) || overlap(data, pb, plane_out, pb))))
        return MIG_E_ARG;
    hipStream_t s = as_stream(stream);
    const int wpg = omegas_per_group3d(nx, ny, nw, omegas_per_group);
    const int ngroups = (nw + wpg - 1) / wpg;
    char* base = static_cast<char*>(ws);
    float2* buf[2] = {reinterpret_cast<float2*>(base),
                      reinterpret_cast<float2*>(base + plane3d_bytes(nx, ny, nw))};
    double* part[2] = {
        reinterpret_cast<double*>(base + 2 * plane3d_bytes(nx, ny, nw)),
        reinterpret_cast<double*>(base + 2 * plane3d_bytes(nx, ny, nw) +
                                  partial3d_bytes(nx, ny, ngroups))};

    const float2* src = reinterpret_cast<const float2*>(data);
    int rc = launch_image3d(src, image, plane, nw, s);
    if (rc != MIG_OK) return rc;
    Step3dArgs a;
    a.tab = reinterpret_cast<const float2*>(tab32);
    a.omega = omega;
    a.nx = nx;
    a.ny = ny;
    a.nw = nw;
    a.nk = d->nk;
    a.wpg = wpg;
    a.ngroups = ngroups;
    a.tiles_x = step3d_tiles_x(nx);
    a.tiles_y = step3d_tiles_y(ny);
    a.dk = (d->kmax - d->kmin) / (double)(d->nk - 1);
    a.b = d->kmin / a.dk;
    const int M = (d->ntaps - 1) / 2;
    for (int k = 1; k < nz; ++k) {
        a.in = src;
        a.out = buf[k & 1];
        a.vel = vel + (size_t)(k - 1) * plane;
        a.part = part[k & 1];
        a.prev = k >= 2 ? part[(k - 1) & 1] : nullptr;
        a.prev_row = k >= 2 ? image + (size_t)(k - 1) * plane : nullptr;
        rc = launch_step3d(a, M, s);
        if (rc != MIG_OK) return rc;
        src = a.out;
    }
    if (nz >= 2) {
        rc = launch_reduce3d(part[(nz - 1) & 1], image + (size_t)(nz - 1) * plane, plane, ngroups, s);
        if (rc != MIG_OK) return rc;
    }
    if (plane_out && hipMemcpyAsync(plane_out, src, pb, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return MIG_E_DEVICE;
    return MIG_OK;
}
