// Batched (2+1)D lattices: many independent lattices of different sizes,
// masses and potentials (per-site theta) advanced together.
//
// Work is a flat list of items (lattice, x strip, y chunk); each item is one
// workgroup's fused (2+1)D pass over its strip and chunk: one step (march2.h)
// or two (march2x2.h), per the tuning candidate.
//  mode 1: one launch per pass over all items of all lattices;
//  mode 0: one persistent launch for all steps, in passes of one step or (the
//          two-step candidates) two steps, an odd remainder then taking one
//          one-step pass after it.  Each workgroup takes items round-robin;
//          before starting pass s of an item of lattice b it waits until all
//          items of b have finished pass s-1 (a per-lattice counter,
//          release/acquire at device scope).  The
//          wait is bounded: a workgroup that waits too long raises a
//          device-wide abort flag and every workgroup leaves, so the launch
//          always ends; the host then reports the failure.  The waits need
//          every workgroup of the grid resident at once, so the launch opens
//          with a census (each workgroup counts in and waits, bounded, for the
//          rest; if they do not all arrive the census closes and every
//          workgroup leaves before touching any state), and the grid is the
//          largest one a census-only launch found resident, measured once per
//          process and kernel, starting from the occupancy calculator's bound
//          (which the device did not always reach with 3- and 5-wave blocks).
// Both modes can be captured once into a HIP graph and replayed.  The tile
// shape (strip width x chunk height) is chosen by timing candidates
// (dirac_batch_autotune), with an optional JSON cache keyed by device and
// batch shape.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dirac.h"
#include "ctx.h"
#include "internal.h"
#include "march2.h"
#include "march2x2.h"

using namespace dirac;

namespace {

struct BatchLat {
    void *st[2][4];    // [0]: bound state buffers, [1]: partner buffers
    void *th[4];
    double r;          // r_x = r_y = dt of this lattice (unit spacing)
    int nx, ny;
    int item0, nitems;
};

struct BatchItem {
    int lat, tx, yc, pad;
};

// strip width x chunk height, and steps per pass (1: march2, 2: march2x2)
struct Cand {
    int txb, ly, spp;
};
const Cand kCands[] = {{64, 16, 1},  {64, 32, 1},  {128, 16, 1}, {128, 32, 1}, {128, 64, 1}, {256, 16, 1},
                       {256, 32, 1}, {256, 64, 1}, {64, 64, 2},  {128, 32, 2}, {128, 64, 2}, {128, 128, 2},
                       {256, 32, 2}, {256, 64, 2}, {256, 128, 2}};
constexpr int kNumCands = (int)(sizeof(kCands) / sizeof(kCands[0]));
constexpr int kDefaultCand = 10;
constexpr long kSpinLimit = 1L << 22;
// counter words of a persistent launch after the per-lattice ones: the abort
// flag, the census word and the census's closing count
constexpr int kDoneExtra = 3;
constexpr unsigned kClosed = 1u << 30;     // census word: closed
constexpr long kCensusSpin = 1L << 18;

int bfail(dirac_ctx *c, int code, const char *fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define BCHK(ctx, expr)                                                                            \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return bfail((ctx), DIRAC_E_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                         __LINE__);                                                                \
    } while (0)

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

int64_t items_for(const dirac_ctx *c, const Cand &k) {
    int64_t n = 0;
    for (int64_t b = 0; b < c->count; ++b)
        n += ((c->bnx[b] + k.txb - 1) / k.txb) * ((c->bny[b] + k.ly - 1) / k.ly);
    return n;
}

// scratch layout of a batch context
struct BLayout {
    size_t lats, items, done, partial, result, total;
};
BLayout blayout(const dirac_ctx *c) {
    int64_t maxi = 0;
    for (int q = 0; q < kNumCands; ++q) maxi = std::max(maxi, items_for(c, kCands[q]));
    BLayout L;
    L.lats = 0;
    L.items = al256((size_t)c->count * sizeof(BatchLat));
    L.done = L.items + al256((size_t)maxi * sizeof(BatchItem));
    L.partial = L.done + al256((size_t)(c->count + kDoneExtra) * sizeof(unsigned));
    L.result = L.partial + al256((size_t)kReduceBlocks * kNormVals * sizeof(double));
    L.total = L.result + al256((size_t)c->count * kNormVals * sizeof(double));
    return L;
}

template <typename R>
__device__ __forceinline__ FusedArgs<R> item_args(const BatchLat &L, int parity, int ly) {
    FusedArgs<R> a;
    for (int q = 0; q < 4; ++q) {
        a.in[q] = L.st[parity][q];
        a.out[q] = L.st[parity ^ 1][q];
        a.th[q] = (const R *)L.th[q];
    }
    for (int q = 4; q < 8; ++q) {
        a.in[q] = nullptr;
        a.out[q] = nullptr;
        a.th[q] = nullptr;
    }
    a.tab = nullptr;
    a.rx = (R)L.r;
    a.ry = (R)L.r;
    a.rz = (R)0;
    a.nx = L.nx;
    a.ny = L.ny;
    a.nz = 1;
    a.zchunk = ly;
    a.nzc = 0;
    a.ntx = 0;
    a.nty = 1;
    a.npart = nullptr;
    a.npart_cap = 0;
    a.zh = 0;
    return a;
}

// Item of block b in a launch of one block per item (n blocks).  Blocks are dealt
// to the eight XCDs in turn (block b to XCD b mod 8); each XCD gets a contiguous
// run of the item list instead, so strips side by side in x run at the same time
// on one XCD and find each other's halo columns in its L2.  XCD x holds
// n/8 + (x < n mod 8) blocks; a bijection for any n.
__device__ __forceinline__ int item_of_block(int b, int n) {
    const int x = b & 7, k = b >> 3, q = n >> 3, r = n & 7;
    return x * q + min(x, r) + k;
}

template <typename R, int TXB>
__global__ __launch_bounds__(TXB) void kb_step(const BatchLat *lats, const BatchItem *items, int ly, int parity) {
    __shared__ cx<R> uu[2][2][TXB + 2];
    const BatchItem w = items[item_of_block(blockIdx.x, gridDim.x)];
    const BatchLat &L = lats[w.lat];
    FusedArgs<R> a = item_args<R>(L, parity, ly);
    march2<R, true, TXB>(a, w.tx, w.yc, uu);
}

// Two steps per launch: every item's strip and chunk by march2x2.
template <typename R, int TW>
__global__ __launch_bounds__(TW + 64) void kb_step2(const BatchLat *lats, const BatchItem *items, int ly, int parity) {
    constexpr int W = TW + 4;
    __shared__ __align__(16) cx<R> sOld[2 + 4 * W + 2];
    __shared__ __align__(16) cx<R> sStage[2 * W];
    __shared__ __align__(16) cx<R> sLev[2 + 6 * W + 2];
    const BatchItem w = items[item_of_block(blockIdx.x, gridDim.x)];
    const BatchLat &L = lats[w.lat];
    FusedArgs<R> a = item_args<R>(L, parity, ly);
    march2x2<R, true, TW>(a, nullptr, w.tx, w.yc, sOld, sStage, sLev);
}

// Per-lattice step barrier of the persistent launches: before pass s of an
// item of lattice lat, wait until all nl items of lat have finished pass s-1
// (done[lat] >= s * nl).  Thread 0 polls with device-scope relaxed loads and,
// once the count is reached, makes one device-scope acquire fence before the
// workgroup barrier (an acquire on every poll would invalidate the caches on
// every spin); the wait is bounded: past kSpinLimit polls it raises the abort
// flag, and a raised flag makes every waiting workgroup leave.  Returns true
// to leave.
__device__ __forceinline__ bool wait_lattice(unsigned *done, int lat, unsigned need, unsigned *abort_flag,
                                             int *s_abort) {
    if (threadIdx.x == 0) {
        int ab = 0;
        long spins = 0;
        for (;;) {
            unsigned v = __hip_atomic_load(&done[lat], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v >= need) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                break;
            }
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                ab = 1;
                break;
            }
            if (++spins > kSpinLimit) {
                __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ab = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        *s_abort = ab;
    }
    __syncthreads();
    return *s_abort != 0;
}
// Census at the start of a persistent launch: every workgroup adds one to the
// census word and waits (bounded) until the whole grid has arrived, so no item
// starts unless the grid is co-resident.  A workgroup whose wait runs out
// closes the census by a compare-and-swap that sets kClosed on the count it
// last saw (which fails if anyone arrived meanwhile: it then waits again) and
// stores that count; a workgroup that sees the bit, on arrival or while
// waiting, leaves.  Every wait ends: arrivals are at most the grid.  Returns
// true to leave.
__device__ __forceinline__ bool census(unsigned *word, unsigned *closed_at, int *s_abort) {
    if (threadIdx.x == 0) {
        int ab = 0;
        const unsigned old = __hip_atomic_fetch_add(word, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (old & kClosed) ab = 1;
        long spins = 0;
        while (!ab) {
            const unsigned v = __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v & kClosed) {
                ab = 1;
                break;
            }
            if (v >= gridDim.x) break;
            if (++spins > kCensusSpin) {
                unsigned expect = v;
                if (__hip_atomic_compare_exchange_strong(word, &expect, v | kClosed, __ATOMIC_RELAXED,
                                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    __hip_atomic_store(closed_at, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ab = 1;
                    break;
                }
                spins = 0;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        *s_abort = ab;
    }
    __syncthreads();
    return *s_abort != 0;
}
// After an item's pass: every thread's stores are done (barrier), then thread 0
// counts the item with a device-scope release, which publishes them.
__device__ __forceinline__ void notify_lattice(unsigned *done, int lat) {
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(&done[lat], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// One persistent launch of nsteps one-step passes (march2 per item).
template <typename R, int TXB>
__global__ __launch_bounds__(TXB) void kb_persist(const BatchLat *lats, const BatchItem *items, int nitems, int ly,
                                                  int parity0, int nsteps, unsigned *done, unsigned *abort_flag) {
    __shared__ cx<R> uu[2][2][TXB + 2];
    __shared__ int s_abort;
    if (census(abort_flag + 1, abort_flag + 2, &s_abort)) return;
    for (int s = 0; s < nsteps; ++s) {
        const int par = (parity0 + s) & 1;
        for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
            const BatchItem w = items[it];
            const BatchLat &L = lats[w.lat];
            if (s > 0 && wait_lattice(done, w.lat, (unsigned)s * (unsigned)L.nitems, abort_flag, &s_abort)) return;
            FusedArgs<R> a = item_args<R>(L, par, ly);
            march2<R, true, TXB>(a, w.tx, w.yc, uu);
            notify_lattice(done, w.lat);
        }
    }
}

// One persistent launch of npass two-step passes (march2x2 per item): the same
// barrier per pass, each pass advancing two steps (its ring is two cells, all
// within the lattice the barrier covers).
template <typename R, int TW>
__global__ __launch_bounds__(TW + 64) void kb_persist2(const BatchLat *lats, const BatchItem *items, int nitems,
                                                       int ly, int parity0, int npass, unsigned *done,
                                                       unsigned *abort_flag) {
    constexpr int W = TW + 4;
    __shared__ __align__(16) cx<R> sOld[2 + 4 * W + 2];
    __shared__ __align__(16) cx<R> sStage[2 * W];
    __shared__ __align__(16) cx<R> sLev[2 + 6 * W + 2];
    __shared__ int s_abort;
    if (census(abort_flag + 1, abort_flag + 2, &s_abort)) return;
    for (int s = 0; s < npass; ++s) {
        const int par = (parity0 + s) & 1;
        for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
            const BatchItem w = items[it];
            const BatchLat &L = lats[w.lat];
            if (s > 0 && wait_lattice(done, w.lat, (unsigned)s * (unsigned)L.nitems, abort_flag, &s_abort)) return;
            FusedArgs<R> a = item_args<R>(L, par, ly);
            march2x2<R, true, TW>(a, nullptr, w.tx, w.yc, sOld, sStage, sLev);
            notify_lattice(done, w.lat);
        }
    }
}

__global__ void kb_zero_u32(unsigned *p, int n) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) p[t] = 0u;
}

// Upper bound on the workgroups of a persistent launch resident at once, from
// the occupancy calculator.  (Measured: with blocks of 3 or 5 waves the device
// did not always hold that many, so the grid actually used comes from a census,
// below.)
template <typename R> int persistent_grid(int txb, bool two, int *grid) {
    int nb = 0, dev = 0, ncu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) {
        if (two) {
            if (txb == 64) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kb_persist2<R, 64>, 128, 0);
            else if (txb == 128) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kb_persist2<R, 128>, 192, 0);
            else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kb_persist2<R, 256>, 320, 0);
        } else {
            if (txb == 64) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kb_persist<R, 64>, 64, 0);
            else if (txb == 128) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kb_persist<R, 128>, 128, 0);
            else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kb_persist<R, 256>, 256, 0);
        }
    }
    if (e != hipSuccess) return -1;
    *grid = nb * ncu;
    return 0;
}

// One persistent launch of the kernel for (R, txb, two) on grid g; npass 0
// runs the census only and touches no state.
template <typename R>
void launch_persist(int txb, bool two, int g, hipStream_t s, const BatchLat *lats, const BatchItem *items,
                    int nitems, int ly, int par, int npass, unsigned *done, unsigned *abort_flag) {
    if (two) {
        if (txb == 64)
            hipLaunchKernelGGL((kb_persist2<R, 64>), dim3(g), dim3(128), 0, s, lats, items, nitems, ly, par, npass,
                               done, abort_flag);
        else if (txb == 128)
            hipLaunchKernelGGL((kb_persist2<R, 128>), dim3(g), dim3(192), 0, s, lats, items, nitems, ly, par, npass,
                               done, abort_flag);
        else
            hipLaunchKernelGGL((kb_persist2<R, 256>), dim3(g), dim3(320), 0, s, lats, items, nitems, ly, par, npass,
                               done, abort_flag);
    } else {
        if (txb == 64)
            hipLaunchKernelGGL((kb_persist<R, 64>), dim3(g), dim3(64), 0, s, lats, items, nitems, ly, par, npass,
                               done, abort_flag);
        else if (txb == 128)
            hipLaunchKernelGGL((kb_persist<R, 128>), dim3(g), dim3(128), 0, s, lats, items, nitems, ly, par, npass,
                               done, abort_flag);
        else
            hipLaunchKernelGGL((kb_persist<R, 256>), dim3(g), dim3(256), 0, s, lats, items, nitems, ly, par, npass,
                               done, abort_flag);
    }
}

// Co-resident grid of each persistent kernel, measured once per process and
// device: census-only launches (no state touched), starting from the
// occupancy bound and retrying with the census's closing count until one
// passes.
std::mutex g_resident_mu;
std::map<int, int> g_resident;
int resident_key(bool fp32, int txb, bool two) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    return (fp32 ? 1 : 0) | (two ? 2 : 0) | (txb << 2) | (dev << 12);
}
template <typename R> int resident_cached(int txb, bool two, int *grid) {
    std::lock_guard<std::mutex> lk(g_resident_mu);
    auto it = g_resident.find(resident_key(sizeof(R) == 4, txb, two));
    if (it == g_resident.end()) return -1;
    *grid = it->second;
    return 0;
}
void resident_forget(bool fp32, int txb, bool two) {
    std::lock_guard<std::mutex> lk(g_resident_mu);
    g_resident.erase(resident_key(fp32, txb, two));
}
// Upload lattice descriptors and the item list of candidate q.
int upload_batch(dirac_ctx *c, int q, hipStream_t s, int64_t *nitems_out) {
    const BLayout Ly = blayout(c);
    const Cand k = kCands[q];
    std::vector<BatchLat> lats((size_t)c->count);
    std::vector<BatchItem> items;
    for (int64_t b = 0; b < c->count; ++b) {
        BatchLat &L = lats[(size_t)b];
        for (int a = 0; a < 4; ++a) {
            L.st[0][a] = c->bstate[(size_t)b * 4 + a];
            L.st[1][a] = c->bpartner[(size_t)b * 4 + a];
            L.th[a] = c->btheta[(size_t)b * 4 + a];
        }
        L.r = c->bdt[(size_t)b];
        L.nx = (int)c->bnx[(size_t)b];
        L.ny = (int)c->bny[(size_t)b];
        L.item0 = (int)items.size();
        const int ntx = (L.nx + k.txb - 1) / k.txb, nyc = (L.ny + k.ly - 1) / k.ly;
        for (int yc = 0; yc < nyc; ++yc)
            for (int tx = 0; tx < ntx; ++tx) items.push_back(BatchItem{(int)b, tx, yc, 0});
        L.nitems = (int)items.size() - L.item0;
    }
    char *base = (char *)c->scratch;
    BCHK(c, hipMemcpyAsync(base + Ly.lats, lats.data(), lats.size() * sizeof(BatchLat), hipMemcpyHostToDevice, s));
    BCHK(c, hipMemcpyAsync(base + Ly.items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice,
                           s));
    BCHK(c, hipStreamSynchronize(s));
    *nitems_out = (int64_t)items.size();
    return DIRAC_OK;
}

// Two-step passes move whole rows in 16-byte units with a per-unit x wrap,
// which needs an even row length for complex64: otherwise one-step passes.
template <typename R> int calibrate_resident(dirac_ctx *c, int txb, bool two, hipStream_t s, int *grid) {
    if (resident_cached<R>(txb, two, grid) == 0) return DIRAC_OK;
    int g = 0;
    if (persistent_grid<R>(txb, two, &g) || g < 1) return bfail(c, DIRAC_E_HIP, "could not size the persistent grid");
    const BLayout Ly = blayout(c);
    unsigned *done = (unsigned *)((char *)c->scratch + Ly.done);
    unsigned *abort_flag = done + c->count;
    for (int attempt = 0; attempt < 16 && g >= 1; ++attempt) {
        hipLaunchKernelGGL(kb_zero_u32, dim3(1), dim3(256), 0, s, done, (int)c->count + kDoneExtra);
        BCHK(c, hipGetLastError());
        launch_persist<R>(txb, two, g, s, nullptr, nullptr, 0, 1, 0, 0, done, abort_flag);
        BCHK(c, hipGetLastError());
        unsigned w[2] = {0u, 0u};
        BCHK(c, hipMemcpyAsync(w, abort_flag + 1, sizeof w, hipMemcpyDeviceToHost, s));
        BCHK(c, hipStreamSynchronize(s));
        if (!(w[0] & kClosed)) {
            std::lock_guard<std::mutex> lk(g_resident_mu);
            g_resident[resident_key(sizeof(R) == 4, txb, two)] = g;
            *grid = g;
            return DIRAC_OK;
        }
        g = (int)w[1] >= 1 && (int)w[1] < g ? (int)w[1] : g - 1;
    }
    return bfail(c, DIRAC_E_HIP, "persistent kernel: no co-resident grid found");
}

bool two_step_ok(const dirac_ctx *c) {
    if (c->dtype != DIRAC_C64) return true;
    for (int64_t b = 0; b < c->count; ++b)
        if (c->bnx[(size_t)b] % 2 != 0) return false;
    return true;
}

// Launch n steps starting from buffer set parity0; *flips receives the number
// of ping-pong launches made (the state ends in set parity0 ^ (flips & 1)).
template <typename R> int enqueue_run(dirac_ctx *c, int q, int64_t nitems, int64_t n, int mode, int parity0,
                                      hipStream_t s, int64_t *flips) {
    const BLayout Ly = blayout(c);
    char *base = (char *)c->scratch;
    const BatchLat *lats = (const BatchLat *)(base + Ly.lats);
    const BatchItem *items = (const BatchItem *)(base + Ly.items);
    unsigned *done = (unsigned *)(base + Ly.done);
    Cand k = kCands[q];
    if (k.spp == 2 && !two_step_ok(c)) k.spp = 1;
    *flips = 0;
    if (n == 0) return DIRAC_OK;
    const dim3 g((unsigned)nitems);
    int par = parity0;
    auto one_step = [&]() -> int {
        if (k.txb == 64) hipLaunchKernelGGL((kb_step<R, 64>), g, dim3(64), 0, s, lats, items, k.ly, par);
        else if (k.txb == 128) hipLaunchKernelGGL((kb_step<R, 128>), g, dim3(128), 0, s, lats, items, k.ly, par);
        else hipLaunchKernelGGL((kb_step<R, 256>), g, dim3(256), 0, s, lats, items, k.ly, par);
        BCHK(c, hipGetLastError());
        par ^= 1;
        ++*flips;
        return DIRAC_OK;
    };
    auto two_steps = [&]() -> int {
        if (k.txb == 64) hipLaunchKernelGGL((kb_step2<R, 64>), g, dim3(128), 0, s, lats, items, k.ly, par);
        else if (k.txb == 128) hipLaunchKernelGGL((kb_step2<R, 128>), g, dim3(192), 0, s, lats, items, k.ly, par);
        else hipLaunchKernelGGL((kb_step2<R, 256>), g, dim3(320), 0, s, lats, items, k.ly, par);
        BCHK(c, hipGetLastError());
        par ^= 1;
        ++*flips;
        return DIRAC_OK;
    };
    int64_t rest = n;
    if (mode == 1) {
        if (k.spp == 2)
            for (; rest >= 2; rest -= 2) {
                int rc = two_steps();
                if (rc) return rc;
            }
        for (; rest > 0; --rest) {
            int rc = one_step();
            if (rc) return rc;
        }
        return DIRAC_OK;
    }
    // mode 0: one persistent launch; two-step passes for the two-step candidates
    // (an odd remainder then takes one one-step pass after it), else one-step passes
    {
        const bool two = k.spp == 2 && n >= 2;
        const int64_t npass = two ? n / 2 : n;
        // the co-resident grid (measured here unless the caller did so before a capture)
        int grid = 0;
        int rc = calibrate_resident<R>(c, k.txb, two, s, &grid);
        if (rc) return rc;
        if ((int64_t)grid > nitems) grid = (int)nitems;
        hipLaunchKernelGGL(kb_zero_u32, dim3(1), dim3(256), 0, s, done, (int)c->count + kDoneExtra);
        BCHK(c, hipGetLastError());
        unsigned *abort_flag = done + c->count;
        launch_persist<R>(k.txb, two, grid, s, lats, items, (int)nitems, k.ly, par, (int)npass, done, abort_flag);
        BCHK(c, hipGetLastError());
        par ^= (int)(npass & 1);
        *flips += npass;
        rest = two ? (n & 1) : 0;
    }
    for (; rest > 0; --rest) {
        int rc = one_step();
        if (rc) return rc;
    }
    return DIRAC_OK;
}

int enqueue(dirac_ctx *c, int q, int64_t nitems, int64_t n, int mode, int parity0, hipStream_t s, int64_t *flips) {
    return c->dtype == DIRAC_C64 ? enqueue_run<float>(c, q, nitems, n, mode, parity0, s, flips)
                                 : enqueue_run<double>(c, q, nitems, n, mode, parity0, s, flips);
}

// The persistent kernel's strip width and steps per pass for candidate q and n steps.
void mode0_config(const dirac_ctx *c, int q, int64_t n, int *txb, bool *two) {
    Cand k = kCands[q];
    if (k.spp == 2 && !two_step_ok(c)) k.spp = 1;
    *txb = k.txb;
    *two = k.spp == 2 && n >= 2;
}

// Measure the co-resident grid of mode 0's kernel before a stream capture
// (the measurement synchronises, which a capture does not allow).
int prepare_mode0(dirac_ctx *c, int q, int64_t n, hipStream_t s) {
    int txb = 0, grid = 0;
    bool two = false;
    mode0_config(c, q, n, &txb, &two);
    return c->dtype == DIRAC_C64 ? calibrate_resident<float>(c, txb, two, s, &grid)
                                 : calibrate_resident<double>(c, txb, two, s, &grid);
}

int check_abort(dirac_ctx *c, int q, int64_t n, hipStream_t s) {
    const BLayout Ly = blayout(c);
    unsigned w[3] = {0u, 0u, 0u};       // abort flag, census word, census closing count
    BCHK(c, hipMemcpyAsync(w, (char *)c->scratch + Ly.done + (size_t)c->count * sizeof(unsigned), sizeof w,
                           hipMemcpyDeviceToHost, s));
    BCHK(c, hipStreamSynchronize(s));
    if (w[1] & kClosed) {
        // the device held fewer workgroups than measured: measure again next time
        int txb = 0;
        bool two = false;
        mode0_config(c, q, n, &txb, &two);
        resident_forget(c->dtype == DIRAC_C64, txb, two);
        return bfail(c, DIRAC_E_HIP, "persistent kernel: only %u workgroups were resident (census closed); the state "
                     "is invalid", w[2]);
    }
    if (w[0]) return bfail(c, DIRAC_E_HIP, "persistent kernel: a per-lattice barrier timed out; the state is invalid");
    return DIRAC_OK;
}

void drop_graph(dirac_ctx *c) {
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    c->graph_n = -1;
}

std::string tune_key(const dirac_ctx *c) {
    hipDeviceProp_t p;
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) {
        arch = p.gcnArchName;
        size_t cpos = arch.find(':');
        if (cpos != std::string::npos) arch = arch.substr(0, cpos);
    }
    int64_t cells = 0, mx = 0, my = 0;
    for (int64_t b = 0; b < c->count; ++b) {
        cells += c->bnx[(size_t)b] * c->bny[(size_t)b];
        mx = std::max(mx, c->bnx[(size_t)b]);
        my = std::max(my, c->bny[(size_t)b]);
    }
    char buf[256];
    snprintf(buf, sizeof buf, "%s/%s/n%lld/cells%lld/max%lldx%lld", arch.c_str(), c->dtype == DIRAC_C64 ? "c64" : "c128",
             (long long)c->count, (long long)cells, (long long)mx, (long long)my);
    return buf;
}

// Minimal reader/writer for the cache: a flat JSON object {"key": [choice_mode1, choice_mode0], ...}.
bool cache_lookup(const char *path, const std::string &key, int out[2]) {
    FILE *f = fopen(path, "r");
    if (!f) return false;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    fclose(f);
    std::string pat = "\"" + key + "\"";
    size_t p = text.find(pat);
    if (p == std::string::npos) return false;
    p = text.find('[', p);
    if (p == std::string::npos) return false;
    int a = -1, b = -1;
    if (sscanf(text.c_str() + p, "[%d , %d]", &a, &b) != 2 && sscanf(text.c_str() + p, "[%d,%d]", &a, &b) != 2)
        return false;
    if (a < 0 || a >= kNumCands || b < 0 || b >= kNumCands) return false;
    out[0] = a;
    out[1] = b;
    return true;
}

void cache_store(const char *path, const std::string &key, const int v[2]) {
    std::string text;
    FILE *f = fopen(path, "r");
    if (f) {
        char buf[4096];
        size_t n;
        while ((n = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
        fclose(f);
    }
    // keep the other entries: collect lines "  "key": [a, b]" that are not ours
    std::vector<std::string> lines;
    size_t pos = 0;
    while ((pos = text.find('"', pos)) != std::string::npos) {
        size_t e = text.find('"', pos + 1);
        if (e == std::string::npos) break;
        std::string k = text.substr(pos + 1, e - pos - 1);
        size_t lb = text.find('[', e), rb = text.find(']', e);
        if (lb == std::string::npos || rb == std::string::npos) break;
        if (k != key) lines.push_back("  \"" + k + "\": " + text.substr(lb, rb - lb + 1));
        pos = rb + 1;
    }
    char mine[512];
    snprintf(mine, sizeof mine, "  \"%s\": [%d, %d]", key.c_str(), v[0], v[1]);
    lines.push_back(mine);
    std::string tmp = std::string(path) + ".tmp";
    f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fputs("{\n", f);
    for (size_t q = 0; q < lines.size(); ++q) fprintf(f, "%s%s\n", lines[q].c_str(), q + 1 < lines.size() ? "," : "");
    fputs("}\n", f);
    fclose(f);
    rename(tmp.c_str(), path);
}

}  // namespace

extern "C" {

int dirac_batch_create_dt(dirac_ctx **out, int64_t count, const int64_t *nx, const int64_t *ny, int dtype,
                          const double *dt, unsigned flags) {
    if (!out) return DIRAC_E_ARG;
    *out = nullptr;
    if (count < 1 || count > (1 << 20) || !nx || !ny || !dt) return DIRAC_E_ARG;
    if (dtype != DIRAC_C64 && dtype != DIRAC_C128) return DIRAC_E_ARG;
    if ((flags & ~DIRAC_ALLOW_UNSTABLE) != 0) return DIRAC_E_ARG;
    for (int64_t b = 0; b < count; ++b)
        if (!isfinite(dt[b]) || dt[b] <= 0.0) return DIRAC_E_ARG;
    for (int64_t b = 0; b < count; ++b)
        if (nx[b] < 1 || ny[b] < 1 || nx[b] > (1 << 24) || ny[b] > (1 << 24) || nx[b] * ny[b] > (1LL << 31))
            return DIRAC_E_SHAPE;
    for (int64_t b = 0; b < count; ++b)
        if (2.0 * dt[b] * dt[b] > 1.0 + 1e-12 && !(flags & DIRAC_ALLOW_UNSTABLE)) return DIRAC_E_UNSTABLE;
    dirac_ctx *c = new (std::nothrow) dirac_ctx();
    if (!c) return DIRAC_E_ARG;
    c->is_batch = true;
    c->ndim = 2;
    c->count = count;
    c->bnx.assign(nx, nx + count);
    c->bny.assign(ny, ny + count);
    c->bdt.assign(dt, dt + count);
    c->dtype = dtype;
    c->dt = dt[0];
    c->rx = c->ry = dt[0];
    c->flags = flags;
    c->batch_scratch_need = blayout(c).total;
    c->tune_choice = -1;
    *out = c;
    return DIRAC_OK;
}

int dirac_batch_create(dirac_ctx **out, int64_t count, const int64_t *nx, const int64_t *ny, int dtype, double dt,
                       unsigned flags) {
    if (!out) return DIRAC_E_ARG;
    *out = nullptr;
    if (count < 1 || count > (1 << 20)) return DIRAC_E_ARG;
    const std::vector<double> dts((size_t)count, dt);
    return dirac_batch_create_dt(out, count, nx, ny, dtype, dts.data(), flags);
}

int dirac_batch_bind(dirac_ctx *c, void *const state[], void *const partner[], void *const theta[], void *scratch,
                     size_t scratch_bytes) {
    if (!c || !state || !partner || !theta || !scratch) return DIRAC_E_ARG;
    if (!c->is_batch) return bfail(c, DIRAC_E_STATE, "not a batch context");
    if (((uintptr_t)scratch & 255) != 0) return bfail(c, DIRAC_E_ARG, "scratch must be 256-byte aligned");
    if (scratch_bytes < c->batch_scratch_need)
        return bfail(c, DIRAC_E_SHAPE, "scratch too small: %zu < %zu", scratch_bytes, c->batch_scratch_need);
    const size_t n = (size_t)c->count * 4;
    for (size_t q = 0; q < n; ++q)
        if (!state[q] || !partner[q] || !theta[q]) return bfail(c, DIRAC_E_ARG, "null pointer at %zu", q);
    c->bstate.assign(state, state + n);
    c->bpartner.assign(partner, partner + n);
    c->btheta.assign(theta, theta + n);
    c->scratch = scratch;
    c->scratch_bytes = scratch_bytes;
    c->bound = true;
    c->cur = 0;
    drop_graph(c);
    return DIRAC_OK;
}

int dirac_batch_run(dirac_ctx *c, int64_t n, int mode, int use_graph, void *stream) {
    if (!c) return DIRAC_E_ARG;
    if (!c->is_batch) return bfail(c, DIRAC_E_STATE, "not a batch context");
    if (!c->bound) return bfail(c, DIRAC_E_STATE, "nothing bound (dirac_batch_bind)");
    if (n < 0 || n > (1LL << 30) || (mode != 0 && mode != 1)) return bfail(c, DIRAC_E_ARG, "bad n or mode");
    hipStream_t s = (hipStream_t)stream;
    const int q = c->tune_choice >= 0 ? (mode == 1 ? (c->tune_choice & 0xff) : (c->tune_choice >> 8)) : kDefaultCand;
    if (!use_graph) {
        drop_graph(c);
        int64_t nitems = 0;
        int rc = upload_batch(c, q, s, &nitems);
        if (rc) return rc;
        int64_t flips = 0;
        rc = enqueue(c, q, nitems, n, mode, c->cur, s, &flips);
        if (rc) return rc;
        if (mode == 0) {
            rc = check_abort(c, q, n, s);
            if (rc) return rc;
        }
        if (flips & 1) c->cur = 1 - c->cur;
    } else {
        if (!(c->graph_exec && c->graph_n == n && c->graph_mode == (mode | (q << 4)) && c->graph_cur == c->cur)) {
            drop_graph(c);
            if (!c->graph_stream) BCHK(c, hipStreamCreateWithFlags(&c->graph_stream, hipStreamNonBlocking));
            int64_t nitems = 0;
            int rc = upload_batch(c, q, c->graph_stream, &nitems);
            if (rc) return rc;
            if (mode == 0) {
                rc = prepare_mode0(c, q, n, c->graph_stream);
                if (rc) return rc;
            }
            BCHK(c, hipStreamBeginCapture(c->graph_stream, hipStreamCaptureModeRelaxed));
            int64_t flips = 0;
            rc = enqueue(c, q, nitems, n, mode, c->cur, c->graph_stream, &flips);
            c->graph_flips = flips;
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(c->graph_stream, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return bfail(c, DIRAC_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
            c->graph = g;
            BCHK(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
            c->graph_n = n;
            c->graph_mode = mode | (q << 4);
            c->graph_cur = c->cur;
        }
        BCHK(c, hipGraphLaunch(c->graph_exec, s));
        if (mode == 0) {
            int rc = check_abort(c, q, n, s);
            if (rc) return rc;
        }
        if (c->graph_flips & 1) c->cur = 1 - c->cur;
    }
    return DIRAC_OK;
}

int dirac_batch_norms(dirac_ctx *c, double *out, void *stream) {
    if (!c || !out) return DIRAC_E_ARG;
    if (!c->is_batch) return bfail(c, DIRAC_E_STATE, "not a batch context");
    if (!c->bound) return bfail(c, DIRAC_E_STATE, "nothing bound");
    hipStream_t s = (hipStream_t)stream;
    const BLayout Ly = blayout(c);
    double *part = (double *)((char *)c->scratch + Ly.partial);
    double *res = (double *)((char *)c->scratch + Ly.result);
    for (int64_t b = 0; b < c->count; ++b) {
        const std::vector<void *> &buf = c->cur == 0 ? c->bstate : c->bpartner;
        if (c->dtype == DIRAC_C64) {
            ReduceArgs<float> a;
            memset(&a, 0, sizeof a);
            for (int q = 0; q < 4; ++q) a.f[q] = buf[(size_t)b * 4 + q];
            a.rx = a.ry = (float)c->bdt[(size_t)b];
            a.nx = (int)c->bnx[(size_t)b];
            a.ny = (int)c->bny[(size_t)b];
            a.nz = 1;
            a.partial = part;
            BCHK(c, launch_norm2<float>(a, s));
        } else {
            ReduceArgs<double> a;
            memset(&a, 0, sizeof a);
            for (int q = 0; q < 4; ++q) a.f[q] = buf[(size_t)b * 4 + q];
            a.rx = a.ry = c->bdt[(size_t)b];
            a.nx = (int)c->bnx[(size_t)b];
            a.ny = (int)c->bny[(size_t)b];
            a.nz = 1;
            a.partial = part;
            BCHK(c, launch_norm2<double>(a, s));
        }
        BCHK(c, launch_final_sum(part, kReduceBlocks, kNormVals, res + (size_t)b * kNormVals, s));
    }
    BCHK(c, hipMemcpyAsync(out, res, (size_t)c->count * kNormVals * sizeof(double), hipMemcpyDeviceToHost, s));
    BCHK(c, hipStreamSynchronize(s));
    for (int64_t q = 0; q < c->count * kNormVals; ++q)
        if (!isfinite(out[q])) return bfail(c, DIRAC_E_NONFINITE, "lattice %lld: non-finite norm", (long long)(q / 3));
    return DIRAC_OK;
}

int dirac_batch_autotune(dirac_ctx *c, const char *cache_path, int *chosen_out, void *stream) {
    if (!c) return DIRAC_E_ARG;
    if (!c->is_batch) return bfail(c, DIRAC_E_STATE, "not a batch context");
    if (!c->bound) return bfail(c, DIRAC_E_STATE, "nothing bound");
    hipStream_t s = (hipStream_t)stream;
    const std::string key = tune_key(c);
    int pick[2] = {-1, -1};
    if (!(cache_path && cache_lookup(cache_path, key, pick))) {
        drop_graph(c);
        hipEvent_t e0, e1;
        BCHK(c, hipEventCreate(&e0));
        BCHK(c, hipEventCreate(&e1));
        const int warm = 2, timed = 8;
        bool aborted = false;
        for (int mode = 1; mode >= 0; --mode) {
            float best = 1e30f;
            for (int q = 0; q < kNumCands; ++q) {
                int64_t nitems = 0;
                int rc = upload_batch(c, q, s, &nitems);
                if (rc) return rc;
                int64_t flips = 0;
                rc = enqueue(c, q, nitems, warm, mode, c->cur, s, &flips);
                if (rc) return rc;
                if (flips & 1) c->cur = 1 - c->cur;
                BCHK(c, hipEventRecord(e0, s));
                rc = enqueue(c, q, nitems, timed, mode, c->cur, s, &flips);
                if (rc) return rc;
                if (flips & 1) c->cur = 1 - c->cur;
                BCHK(c, hipEventRecord(e1, s));
                BCHK(c, hipEventSynchronize(e1));
                if (mode == 0 && check_abort(c, q, timed, s)) {   // candidate unusable here
                    aborted = true;
                    continue;
                }
                float ms = 0.f;
                BCHK(c, hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) {
                    best = ms;
                    pick[mode == 1 ? 0 : 1] = q;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (pick[0] < 0) pick[0] = kDefaultCand;
        if (pick[1] < 0) pick[1] = kDefaultCand;
        if (cache_path) cache_store(cache_path, key, pick);
        if (aborted) {
            // an aborted persistent launch leaves lattices stepped unevenly across
            // both buffer sets: keep the choice, report that the state is gone
            c->tune_choice = pick[0] | (pick[1] << 8);
            if (chosen_out) *chosen_out = c->tune_choice;
            return bfail(c, DIRAC_E_STATE, "autotune: a persistent candidate's per-lattice barrier timed out; "
                                           "the tile choice is kept, the bound state is no longer valid (reload it)");
        }
    }
    c->tune_choice = pick[0] | (pick[1] << 8);
    if (chosen_out) *chosen_out = c->tune_choice;
    return DIRAC_OK;
}

int dirac_autotune(dirac_ctx *c, const char *cache_path) { return dirac_batch_autotune(c, cache_path, nullptr, nullptr); }

}  // extern "C"
