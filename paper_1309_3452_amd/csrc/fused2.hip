// Two time steps per launch ((3+1)D, V(z) coefficient tables or per-site
// records): temporal blocking of the z-march, so each amplitude is read once and written once
// per two steps of Sect. 2 (Eqs. ss1-ss4).
//
// A workgroup owns an x-y tile of TW x TY cells and a chunk [z0, z1) of
// planes.  Four levels run as a pipeline along z, each one plane behind the
// previous:
//   level 1  A,B after step 1 at plane p        (Eqs. ss1, ss2 on the old C,D)
//   level 2  C,D after step 1 at plane p-1      (Eqs. ss3, ss4)
//   level 3  A,B after step 2 at plane p-2      (stored for p-2 in [z0, z1))
//   level 4  C,D after step 2 at plane p-3      (stored for p-3 in [z0, z1))
// Each half-step reaches half a cell in x and y, so the two steps need the
// old C,D on the tile plus a two-cell ring, level 1 on a ring of up to two
// cells, levels 2 and 3 on a one-cell ring and level 4 on the tile.  Every
// level is evaluated on a rectangle that covers what the next one reads; the
// ring is recomputed by each workgroup rather than exchanged, so the state
// ping-pongs between two buffers exactly as in the one-step kernel.
//
// LDS holds, as (TW + 4) x (TY + 4) regions (cell (x, y) of the tile at
// (y + 2)(TW + 4) + x + 2): the old C of plane p and D of planes p and p+1
// (the z-neighbour of B), the next planes in flight, and one plane of each
// level's output.  The old C,D region rows (ring columns included) are copied
// global -> LDS asynchronously, either through a staging area or into three
// sets that rotate (the kernel's ROT layout, described at its LDS arrays).
// Each thread owns one region cell of every level: its z-neighbours and
// previous values X- stay in registers or are re-read from the level planes
// in LDS.
//
// The same stencil and update helpers as the other kernels evaluate every
// value, with the same operation order, so the result is bitwise that of two
// one-step launches.
#include <algorithm>
#include <type_traits>

#include "device.h"
#include "internal.h"
#include "stencil3.h"
#include "march2.h"
#include "march2x2.h"

namespace dirac {

namespace {

__device__ __forceinline__ int logical_block2() {
    const int nb = gridDim.x, b = blockIdx.x;
    if ((nb & 7) == 0) return (b & 7) * (nb >> 3) + (b >> 3);
    return b;
}

// coefficients of class cls (A, B, C, D) at wrapped plane pk; tstride is the
// byte size of one class's table (nz entries of 4 reals)
// Tile and z-chunk of logical block L.  Logical blocks that run at the same
// time on one XCD (consecutive L; about 32 of them, one per CU) cover either
// whole tile rows (px = 0) or a patch of px x 32/px tiles.  Halo rows and
// columns that belong to tiles outside the concurrent set are fetched again
// from HBM (a halo column costs a whole 128-byte line), so the best shape
// depends on the tile's width in bytes.
__device__ __forceinline__ void tile_of(int L, int ntx, int nty, int px, int &tx, int &ty, int &zc) {
    const int PX = px > 0 ? px : 1, PY = px > 0 ? 32 / px : 1;
    if (px > 0 && ntx % PX == 0 && nty % PY == 0) {
        const int within = L % (PX * PY), patch = L / (PX * PY);
        const int npx = ntx / PX, npy = nty / PY;
        tx = (patch % npx) * PX + within % PX;
        const int rest = patch / npx;
        ty = (rest % npy) * PY + within / PX;
        zc = rest / npy;
    } else {
        tx = L % ntx;
        L /= ntx;
        ty = L % nty;
        zc = L / nty;
    }
}

template <typename R> __device__ __forceinline__ Coef<R> tcoef(const R *tab, uint32_t tstride, int cls, int pk) {
    const R *e = (const R *)((const char *)tab + (uint32_t)cls * tstride + (uint32_t)pk * (uint32_t)(4 * sizeof(R)));
    Coef<R> k;
    k.c1 = mk2(e[0], e[1]);
    k.c2 = mk2(e[2], e[3]);
    return k;
}

template <typename C> __device__ __forceinline__ C ld_at(const C *base, uint32_t boff) {
    return *(const C *)((const char *)base + boff);
}
// base + pb + boff: a plane's byte offset pb (wave-uniform) and a lane offset
template <typename C> __device__ __forceinline__ C ld_pl(const C *base, size_t pb, uint32_t boff) {
    return *(const C *)((const char *)base + pb + boff);
}

typedef float nt2f __attribute__((ext_vector_type(2)));
typedef double nt2d __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_nt(float2 *p, float2 v) { __builtin_nontemporal_store(nt2f{v.x, v.y}, (nt2f *)p); }
__device__ __forceinline__ void st_nt(double2 *p, double2 v) { __builtin_nontemporal_store(nt2d{v.x, v.y}, (nt2d *)p); }
template <typename C> __device__ __forceinline__ void st_pl(C *base, size_t pb, uint32_t boff, C v) {
    st_nt((C *)((char *)base + pb + boff), v);
}
// next plane index on the torus of nz planes (k in [0, nz))
__device__ __forceinline__ int wrap_inc(int k, int nz) { return k + 1 == nz ? 0 : k + 1; }

// Asynchronous global -> LDS copy: lane l's 16 bytes land at lds_wave_base + 16 l.
__device__ __forceinline__ void g2lds16(const void *gsrc, void *lds_wave_base) {
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)gsrc,
                                     (__attribute__((address_space(3))) void *)lds_wave_base, 16, 0, 0);
}

// Thread -> region cell.  The tile comes first (wave k holds tile row k, so
// stores are whole aligned rows), then the one-cell ring (levels 1-3), then the
// two-cell ring (level 1 only); with 16 waves the ring cells skip waves 12-14
// so that the four SIMDs (wave w on SIMD w mod 4) get similar work.  Returns
// the slot (-1: no cell) and the cell's coordinates relative to the tile.
template <int TW, int TY, int NT> __device__ __forceinline__ int region_slot(int t, int &xr, int &yr) {
    constexpr int N0 = TW * TY, N1 = 2 * (TW + 2) + 2 * TY, N2 = 2 * (TW + 4) + 2 * (TY + 2);
    constexpr int SKIP0 = NT == 1024 ? 768 : NT, SKIP1 = NT == 1024 ? 960 : NT;
    int r = t < SKIP0 ? t : (t >= SKIP1 ? t - (SKIP1 - SKIP0) : -1);
    if (r >= N0 + N1 + N2) r = -1;
    xr = -3;
    yr = -3;
    if (r < 0) return -1;
    int u = r;
    if (u < N0) {
        xr = u % TW;
        yr = u / TW;
    } else if ((u -= N0) < N1) {
        if (u < TW + 2) { xr = u - 1; yr = -1; }
        else if (u < 2 * (TW + 2)) { xr = u - (TW + 2) - 1; yr = TY; }
        else if (u < 2 * (TW + 2) + TY) { xr = -1; yr = u - 2 * (TW + 2); }
        else { xr = TW; yr = u - 2 * (TW + 2) - TY; }
    } else {
        u -= N1;
        if (u < TW + 4) { xr = u - 2; yr = -2; }
        else if (u < 2 * (TW + 4)) { xr = u - (TW + 4) - 2; yr = TY + 1; }
        else if (u < 2 * (TW + 4) + TY + 2) { xr = -2; yr = u - 2 * (TW + 4) - 1; }
        else { xr = TW + 1; yr = u - 2 * (TW + 4) - (TY + 2) - 1; }
    }
    return r;
}

// Per-site coefficient record: gamma (float2) for complex64 lattices, theta
// (double) for complex128 ones, turned into Cayley coefficients exactly as the
// one-step kernels do.
template <typename R> struct SiteRec;
template <> struct SiteRec<float> {
    typedef float2 T;
    static __device__ __forceinline__ T load(const float *th, size_t pb, uint32_t boff) {
        return *(const float2 *)((const char *)th + pb + boff);
    }
    template <int SITE> static __device__ __forceinline__ Coef<float> coef(T g) {
        return coef_site(g, SITE == 2 ? -1.0f : 1.0f);
    }
};
template <> struct SiteRec<double> {
    typedef double T;
    static __device__ __forceinline__ T load(const double *th, size_t pb, uint32_t boff) {
        return *(const double *)((const char *)th + pb + boff);
    }
    template <int SITE> static __device__ __forceinline__ Coef<double> coef(T th) {
        return coef_theta(SITE == 2 ? -th : th);
    }
};

// SITE: 0 = V(z) tables, 1 = per-site records, 2 = per-site records with
// theta -> -theta (the reversed step's sequence).  ROT: the old C,D planes in
// three rotating LDS sets (below) instead of a staging area copied forward.
template <typename R, int TW, int TY, int NT, bool NORM, int SITE, bool ROT>
__global__ __launch_bounds__(NT) void k3_fused2(FusedArgs<R> a, const R *__restrict__ tab) {
    using C = cx<R>;
    constexpr int W = TW + 4, H = TY + 4, RN = W * H;
    constexpr int PAD = W + 2;                        // keeps +-1, +-W reads of edge cells inside an array set
    constexpr int CPL = 16 / (int)sizeof(C);          // cells per 16-byte unit
    static_assert(RN <= NT - (NT == 1024 ? 192 : 0), "one region cell per thread");
    static_assert((W / CPL) <= 64, "one wave instruction per region row");
    static_assert(PAD % 2 == 0 && W % 2 == 0 && RN % 2 == 0, "16-byte alignment of the LDS rows");
    // LDS (RN cells per array), in one of two layouts.
    // ROT == false: the asynchronous copies land only in a staging area that
    // the stencils never read, so the compiler need not wait for them before
    // the stencils' LDS reads; the staged planes move up at the end of the
    // iteration, and the next plane's copies are issued after that.
    //   sA: 0-1 C(p), 2-3 D(p), 4-5 D(p+1);  sB: 0-1 C(p+1), 2-3 D(p+2) in flight
    // ROT == true: three sets sA, sB, sC, set q holding the C of plane q and
    // the D of plane q+1 (0-1 C0 C1, 2-3 D0 D1), in rotation: plane p's set is
    // number (p - ps) mod 3.  Iteration p reads C(p), D(p+1) from its set and
    // D(p) from the previous one; after its first barrier the previous set is
    // free and receives C(p+2), D(p+3), which then land during the whole next
    // iteration (no copies between LDS arrays, no idle memory pipe while the
    // level planes are written).  The loop is unrolled by three so that every
    // access names its set statically: the compiler then sees that the copies
    // in flight never alias what the stencils read.
    //   sLev: 0-3 level-1 A0 A1 B0 B1, 4-7 level-2 C0 C1 D0 D1, 8-11 level-3 A0 A1 B0 B1
    __shared__ __align__(16) C sA[ROT ? PAD + 4 * RN + PAD : PAD + 6 * RN + PAD];
    __shared__ __align__(16) C sB[ROT ? PAD + 4 * RN + PAD : 4 * RN];
    __shared__ __align__(16) C sC[ROT ? PAD + 4 * RN + PAD : 2];
    __shared__ __align__(16) C sLev[PAD + 12 * RN + PAD];
    auto old_ = [&](int k) -> C * { return sA + PAD + k * RN; };
    auto lev = [&](int k) -> C * { return sLev + PAD + k * RN; };

    int tx, ty, zc;
    tile_of(logical_block2(), a.ntx, a.nty, a.px, tx, ty, zc);
    const int x0 = tx * TW, y0 = ty * TY;
    const int w = min(TW, a.nx - x0), h = min(TY, a.ny - y0);
    const int z0 = zc * a.zchunk, z1 = min(a.nz, z0 + a.zchunk);
    const int t = threadIdx.x;
    // the wave index is uniform: read it into a scalar register so that the
    // per-wave copy bookkeeping below runs on the scalar unit
    const int lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    // z-slab mode: zh halo planes stored on each side of the nz interior ones
    // and no wrap in z; nzt planes (and table entries) are stored
    const int zh = a.zh, nzt = nz + 2 * zh;
    constexpr uint32_t CS = sizeof(C);
    // bytes of one plane (below 4 GiB, checked by the launcher) and of one
    // class of the coefficient table
    const uint32_t pbytes = (uint32_t)nx * (uint32_t)ny * CS;
    const uint32_t tstride = (uint32_t)nzt * (uint32_t)(4 * sizeof(R));
    auto pofs = [&](int k) -> size_t { return (size_t)(uint32_t)k * (size_t)pbytes; };
    // stored index of the next plane, and whether a stored index exists (a
    // slab's march passes two planes beyond its halo on each side; what is
    // computed from those planes reaches no stored value)
    auto next_k = [&](int k) { return zh == 0 ? wrap_inc(k, nz) : k + 1; };
    auto valid = [&](int k) { return (unsigned)k < (unsigned)nzt; };
    auto tk = [&](int k) { return valid(k) ? k : 0; };

    // the region cell of this thread: (xr, yr) relative to the tile origin
    int xr, yr;
    const int r = region_slot<TW, TY, NT>(t, xr, yr);
    int i = (yr + 2) * W + xr + 2;                    // LDS index of the cell
    const bool in1 = r >= 0 && xr < w + 2 && yr < h + 2;                       // levels 1 (ring 2)
    const bool in2 = in1 && xr >= -1 && xr <= w && yr >= -1 && yr <= h;        // levels 2, 3 (ring 1)
    const bool in4 = in1 && xr >= 0 && xr < w && yr >= 0 && yr < h;            // level 4 (tile)
    uint32_t go = in1 ? ((uint32_t)wrapn(y0 + yr, ny) * (uint32_t)nx + (uint32_t)wrapn(x0 + xr, nx)) * CS : 0u;
    // per-site mode: the records of arrays arr0 .. arr0 + 3 at stored plane k
    // and this thread's cell, loaded where a level uses them, addressed as a
    // wave-uniform plane base plus this lane's 32-bit byte offset (a plane not
    // stored reads plane 0; nothing computed from it is stored)
    using Rec = typename SiteRec<R>::T;
    constexpr uint32_t RS = sizeof(Rec);
    const uint32_t rbytes = (uint32_t)nx * (uint32_t)ny * RS;
    auto ld_rec = [&](int arr0, int k, Rec *dst) {
        const size_t pb = (size_t)(uint32_t)tk(k) * (size_t)rbytes;
        const uint32_t ro = go / (CS / RS);
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = SiteRec<R>::load(a.th[arr0 + q], pb, ro);
    };

    const C *in[8];
    C *out[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        in[q] = (const C *)a.in[q];
        out[q] = (C *)a.out[q];
    }
    const R rx = a.rx, ry = a.ry, rz = a.rz;
    const C zero = mk2((R)0, (R)0);

    // whole region rows (ring columns included) of the old C (arrays 4, 5) of
    // one plane and of D (arrays 6, 7) of another; lane j moves cells 2j, 2j+1
    // (complex64) or cell j (complex128) of the row, wrapped in x per 16-byte
    // unit (nx is even for complex64, so no unit straddles the wrap).  Wave wv
    // copies rows cy0, cy0 + WPA, ... of array ck for the whole march, so the
    // wrapped row offsets are computed once.
    constexpr int NW = NT / 64, WPA = NW / 4, NJ = (H + WPA - 1) / WPA;
    static_assert(NW % 4 == 0, "four equal groups of copying waves");
    const int rl = (w + 4) / CPL;                     // active lanes per row
    const uint32_t lxo = (uint32_t)wrapn(x0 - 2 + lane * CPL, nx) * CS;
    const int ck = wv / WPA, cy0 = wv % WPA;
    const C *csrc = ck == 0 ? in[4] : ck == 1 ? in[5] : ck == 2 ? in[6] : in[7];
    uint32_t croff[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) croff[j] = (uint32_t)wrapn(y0 + cy0 + WPA * j - 2, ny) * (uint32_t)nx * CS;
    // kc, kd: stored indices of the C and the D plane (C skipped if !with_c,
    // either skipped if not stored); dst: this wave's LDS array (array ck of
    // the destination)
    auto copy_rows = [&](int kc, int kd, bool with_c, C *dst) {
        if (ck < 2 ? (!with_c || !valid(kc)) : !valid(kd)) return;
        const char *base = (const char *)csrc + pofs(ck < 2 ? kc : kd);
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int yy = cy0 + WPA * j;
            if (yy < h + 4 && lane < rl) g2lds16(base + croff[j] + lxo, dst + yy * W);
        }
    };

    // registers carried along the march (own cell)
    C cprev[2] = {zero, zero}, dprev[2] = {zero, zero};   // old C, D of plane p-1
    C pab[4] = {zero, zero, zero, zero};                  // old A, B of plane p
    C ab1h2[4] = {zero, zero, zero, zero};                // level 1 of plane p-2
    C cd1h2[4] = {zero, zero, zero, zero};                // level 2 of plane p-3
    C b2h2[2] = {zero, zero};                             // level 3 B of plane p-4
    // per-iteration values; declared once so that lanes outside a level's box
    // keep stale (unused) values instead of being cleared every plane
    C pabn[4] = {zero, zero, zero, zero};
    C ab1[4] = {zero, zero, zero, zero}, cown[2] = {zero, zero}, down[2] = {zero, zero};
    C cd1[4] = {zero, zero, zero, zero}, ab1h1[4] = {zero, zero, zero, zero};
    C ab2[4] = {zero, zero, zero, zero}, cd1h1[4] = {zero, zero, zero, zero};
    C ab2h1[4] = {zero, zero, zero, zero};
    double nrm[2] = {0.0, 0.0};

    const int ps = z0 - 3, pe = z1 + 2;
    // stored indices of planes p-3 .. p+2 along the march, advanced by one per plane
    int km3 = zh == 0 ? wrapn(ps - 3, nz) : ps - 3 + zh;
    int km2 = next_k(km3), km1 = next_k(km2), k0 = next_k(km1);
    int kp1 = next_k(k0), kp2 = next_k(kp1), kp3 = next_k(kp2);
    // own-cell prefetch: the old A,B of plane p+1
    auto load_ab_next = [&]() __attribute__((always_inline)) {
        if (in1 && valid(kp1)) {
            const size_t Pn = pofs(kp1);
#pragma unroll
            for (int q = 0; q < 4; ++q) pabn[q] = ld_pl(in[q], Pn, go);
        }
    };
    // the four levels of plane p; oc0, oc1: the LDS arrays of the old C of
    // plane p, od0, od1 of its D, on0, on1 of the D of plane p+1
    auto levels = [&](int p, const C *oc0, const C *oc1, const C *od0, const C *od1, const C *on0,
                      const C *on1) __attribute__((always_inline)) {
        // level 1: A,B of plane p after step 1
        if (in1) {
            Coef<R> kq[4];
            if constexpr (SITE != 0) {
                Rec rr[4];
                ld_rec(0, k0, rr);
#pragma unroll
                for (int q = 0; q < 4; ++q) kq[q] = SiteRec<R>::template coef<SITE>(rr[q]);
            } else {
                kq[0] = kq[1] = tcoef(tab, tstride, 0, tk(k0));
                kq[2] = kq[3] = tcoef(tab, tstride, 1, tk(k0));
            }
            const C *C0 = oc0, *C1 = oc1, *D0 = od0, *D1 = od1, *D0n = on0, *D1n = on1;
            cown[0] = C0[i];
            cown[1] = C1[i];
            down[0] = D0[i];
            down[1] = D1[i];
            const St3<C> S = stencil_ab<C, R>(rx, ry, rz,
                                              cown[0], cprev[0], C0[i + 1], C0[i + W],
                                              cown[1], cprev[1], C1[i - W], C1[i - 1],
                                              down[0], D0[i - 1], D0[i + W], D0n[i],
                                              down[1], D1[i - W], D1[i + 1], D1n[i]);
            ab1[0] = update(pab[0], S.s0, kq[0]);
            ab1[1] = update(pab[1], S.s1, kq[1]);
            ab1[2] = update(pab[2], S.s2, kq[2]);
            ab1[3] = update(pab[3], S.s3, kq[3]);
        }
        // level 2: C,D of plane p-1 after step 1 (LDS: level 1 of plane p-1)
        const int q2 = p - 1;
        // the own values of a level's LDS plane are read whenever that plane
        // was produced (the next plane's window needs them even where this
        // level is not evaluated); the level itself runs on the planes the
        // next level consumes
        const C *A0 = lev(0), *A1 = lev(1), *B0 = lev(2), *B1 = lev(3);
        if (in2 && q2 >= z0 - 3) {
            ab1h1[0] = A0[i];
            ab1h1[1] = A1[i];
            ab1h1[2] = B0[i];
            ab1h1[3] = B1[i];
        }
        if (in2 && q2 >= z0 - 2 && q2 <= z1 + 1) {
            Coef<R> kq[4];
            if constexpr (SITE != 0) {
                Rec rr[4];
                ld_rec(4, km1, rr);
#pragma unroll
                for (int q = 0; q < 4; ++q) kq[q] = SiteRec<R>::template coef<SITE>(rr[q]);
            } else {
                kq[0] = kq[1] = tcoef(tab, tstride, 2, tk(km1));
                kq[2] = kq[3] = tcoef(tab, tstride, 3, tk(km1));
            }
            const St3<C> S = stencil_cd<C, R>(rx, ry, rz,
                                              ab1h1[0], ab1[0], A0[i + 1], A0[i + W],
                                              ab1h1[1], ab1[1], A1[i - 1], A1[i - W],
                                              ab1h1[2], ab1h2[2], B0[i - 1], B0[i + W],
                                              ab1h1[3], ab1h2[3], B1[i + 1], B1[i - W]);
            cd1[0] = update(cprev[0], S.s0, kq[0]);
            cd1[1] = update(cprev[1], S.s1, kq[1]);
            cd1[2] = update(dprev[0], S.s2, kq[2]);
            cd1[3] = update(dprev[1], S.s3, kq[3]);
        }
        // level 3: A,B of plane p-2 after step 2 (LDS: level 2 of plane p-2)
        const int q3 = p - 2;
        const C *C0 = lev(4), *C1 = lev(5), *D0 = lev(6), *D1 = lev(7);
        if (in2 && q3 >= z0 - 2) {
            cd1h1[0] = C0[i];
            cd1h1[1] = C1[i];
            cd1h1[2] = D0[i];
            cd1h1[3] = D1[i];
        }
        if (in2 && q3 >= z0 - 1 && q3 <= z1) {
            Coef<R> kq[4];
            if constexpr (SITE != 0) {
                Rec rr[4];
                ld_rec(0, km2, rr);
#pragma unroll
                for (int q = 0; q < 4; ++q) kq[q] = SiteRec<R>::template coef<SITE>(rr[q]);
            } else {
                kq[0] = kq[1] = tcoef(tab, tstride, 0, tk(km2));
                kq[2] = kq[3] = tcoef(tab, tstride, 1, tk(km2));
            }
            const St3<C> S = stencil_ab<C, R>(rx, ry, rz,
                                              cd1h1[0], cd1h2[0], C0[i + 1], C0[i + W],
                                              cd1h1[1], cd1h2[1], C1[i - W], C1[i - 1],
                                              cd1h1[2], D0[i - 1], D0[i + W], cd1[2],
                                              cd1h1[3], D1[i - W], D1[i + 1], cd1[3]);
            ab2[0] = update(ab1h2[0], S.s0, kq[0]);
            ab2[1] = update(ab1h2[1], S.s1, kq[1]);
            ab2[2] = update(ab1h2[2], S.s2, kq[2]);
            ab2[3] = update(ab1h2[3], S.s3, kq[3]);
            if (in4 && q3 >= z0 && q3 < z1) {
                const size_t Pq = pofs(km2);
#pragma unroll
                for (int q = 0; q < 4; ++q) st_pl(out[q], Pq, go, ab2[q]);
                if constexpr (NORM) {
                    double pp = 0.0;
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        pp += (double)ab2[q].x * (double)ab2[q].x + (double)ab2[q].y * (double)ab2[q].y;
                    nrm[0] += pp;
                    nrm[1] += pp;
                }
            }
        }
        // level 4: C,D of plane p-3 after step 2 on the tile (LDS: level 3 of plane p-3)
        const int q4 = p - 3;
        const C *A20 = lev(8), *A21 = lev(9), *B20 = lev(10), *B21 = lev(11);
        if (in4 && q4 >= z0 - 1) {
            ab2h1[0] = A20[i];
            ab2h1[1] = A21[i];
            ab2h1[2] = B20[i];
            ab2h1[3] = B21[i];
        }
        if (in4 && q4 >= z0 && q4 < z1) {
            Coef<R> kq[4];
            if constexpr (SITE != 0) {
                Rec rr[4];
                ld_rec(4, km3, rr);
#pragma unroll
                for (int q = 0; q < 4; ++q) kq[q] = SiteRec<R>::template coef<SITE>(rr[q]);
            } else {
                kq[0] = kq[1] = tcoef(tab, tstride, 2, tk(km3));
                kq[2] = kq[3] = tcoef(tab, tstride, 3, tk(km3));
            }
            const C *A0 = A20, *A1 = A21, *B0 = B20, *B1 = B21;
            const St3<C> S = stencil_cd<C, R>(rx, ry, rz,
                                              ab2h1[0], ab2[0], A0[i + 1], A0[i + W],
                                              ab2h1[1], ab2[1], A1[i - 1], A1[i - W],
                                              ab2h1[2], b2h2[0], B0[i - 1], B0[i + W],
                                              ab2h1[3], b2h2[1], B1[i + 1], B1[i - W]);
            C o[4];
            o[0] = update(cd1h2[0], S.s0, kq[0]);
            o[1] = update(cd1h2[1], S.s1, kq[1]);
            o[2] = update(cd1h2[2], S.s2, kq[2]);
            o[3] = update(cd1h2[3], S.s3, kq[3]);
            const size_t Pq = pofs(km3);
#pragma unroll
            for (int q = 0; q < 4; ++q) st_pl(out[4 + q], Pq, go, o[q]);
            if constexpr (NORM) {
                // E_r in its C,D-summed form: |Y|^2 + Re conj(Y) S_Y(A,B)
                const C sv[4] = {S.s0, S.s1, S.s2, S.s3};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double yre = (double)o[q].x, yim = (double)o[q].y;
                    const double pp = yre * yre + yim * yim;
                    nrm[0] += pp + (yre * (double)sv[q].x + yim * (double)sv[q].y);
                    nrm[1] += pp;
                }
            }
        }
    };
    // after the first barrier: this iteration's level outputs become the LDS
    // planes of the next one
    auto store_levels = [&]() __attribute__((always_inline)) {
        if (in1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                lev(q)[i] = ab1[q];
                lev(4 + q)[i] = cd1[q];
                lev(8 + q)[i] = ab2[q];
            }
        }
    };
    // advance the z windows
    auto advance = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ab1h2[q] = ab1h1[q];
            cd1h2[q] = cd1h1[q];
            pab[q] = pabn[q];
        }
        b2h2[0] = ab2h1[2];
        b2h2[1] = ab2h1[3];
        cprev[0] = cown[0];
        cprev[1] = cown[1];
        dprev[0] = down[0];
        dprev[1] = down[1];
    };

    if constexpr (!ROT) {
        {
            // old C(ps), D(ps), D(ps+1) regions; C(ps-1) and A,B(ps) at the own cell
            copy_rows(k0, k0, true, old_(ck));
            copy_rows(k0, kp1, false, old_(2 + ck));
            const size_t Pm = pofs(km1), P0 = pofs(k0);
            if (in1 && valid(km1)) {
                cprev[0] = ld_pl(in[4], Pm, go);
                cprev[1] = ld_pl(in[5], Pm, go);
            }
            if (in1 && valid(k0)) {
#pragma unroll
                for (int q = 0; q < 4; ++q) pab[q] = ld_pl(in[q], P0, go);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }

        for (int p = ps; p <= pe; ++p) {
            // keep the per-lane offset opaque, so that addresses stay a wave-uniform
            // plane base plus a 32-bit lane offset instead of hoisted 64-bit pairs
            asm volatile("" : "+v"(go));
            const bool more = p < pe;
            if (more) {
                // prefetch: C(p+1), D(p+2) regions; A,B(p+1) at the own cell
                copy_rows(kp1, kp2, true, sB + ck * RN);
                load_ab_next();
            }
            levels(p, old_(0), old_(1), old_(2), old_(3), old_(4), old_(5));
            // all LDS reads of this iteration done, all copies landed
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            store_levels();
            // the staged old planes move up
            if (more && r >= 0) {
                old_(0)[i] = sB[i];
                old_(1)[i] = sB[RN + i];
                old_(2)[i] = old_(4)[i];
                old_(3)[i] = old_(5)[i];
                old_(4)[i] = sB[2 * RN + i];
                old_(5)[i] = sB[3 * RN + i];
            }
            advance();
            km3 = km2;
            km2 = km1;
            km1 = k0;
            k0 = kp1;
            kp1 = kp2;
            kp2 = next_k(kp2);
            __syncthreads();
        }
    } else {
        {
            // sets of planes ps-1 (its D only: D(ps)), ps and ps+1; C(ps-1) and
            // A,B(ps) at the own cell
            copy_rows(km1, k0, false, sC + PAD + ck * RN);
            copy_rows(k0, kp1, true, sA + PAD + ck * RN);
            copy_rows(kp1, kp2, true, sB + PAD + ck * RN);
            const size_t Pm = pofs(km1), P0 = pofs(k0);
            if (in1 && valid(km1)) {
                cprev[0] = ld_pl(in[4], Pm, go);
                cprev[1] = ld_pl(in[5], Pm, go);
            }
            if (in1 && valid(k0)) {
#pragma unroll
                for (int q = 0; q < 4; ++q) pab[q] = ld_pl(in[q], P0, go);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
        // plane p in set phase PH = (p - ps) mod 3
        auto plane = [&](auto PH, int p) __attribute__((always_inline)) {
            constexpr int ph = decltype(PH)::value;
            C *const Sr = ph == 0 ? sA : ph == 1 ? sB : sC;      // C(p), D(p+1)
            C *const Sp = ph == 0 ? sC : ph == 1 ? sA : sB;      // D(p); then receives C(p+2), D(p+3)
            // the per-lane offsets opaque: addresses stay a wave-uniform base plus
            // a lane offset, and LDS addresses are formed where they are used
            // rather than hoisted out of the loop (one per set, phase and 64 KiB
            // window would not fit the register file)
            asm volatile("" : "+v"(go), "+v"(i));
            if (p < pe) load_ab_next();
            levels(p, Sr + PAD, Sr + PAD + RN, Sp + PAD + 2 * RN, Sp + PAD + 3 * RN, Sr + PAD + 2 * RN,
                   Sr + PAD + 3 * RN);
            // all LDS reads of this iteration done, the next set landed
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (p + 2 <= pe) copy_rows(kp2, kp3, true, Sp + PAD + ck * RN);
            store_levels();
            advance();
            km3 = km2;
            km2 = km1;
            km1 = k0;
            k0 = kp1;
            kp1 = kp2;
            kp2 = kp3;
            kp3 = next_k(kp3);
            // the level planes written: a barrier that waits only for this wave's
            // LDS operations, so that the copies just issued stay in flight (the
            // language's workgroup barrier waits for every memory access)
            asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        };
        for (int p = ps; p <= pe; p += 3) {
            plane(std::integral_constant<int, 0>(), p);
            if (p + 1 > pe) break;
            plane(std::integral_constant<int, 1>(), p + 1);
            if (p + 2 > pe) break;
            plane(std::integral_constant<int, 2>(), p + 2);
        }
    }

    if constexpr (NORM) {
        double *red = (double *)sLev;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) nrm[q] += __shfl_xor(nrm[q], off, 64);
        }
        if (lane == 0) {
            red[2 * wv] = nrm[0];
            red[2 * wv + 1] = nrm[1];
        }
        __syncthreads();
        if (t == 0) {
            double s0 = 0.0, s1 = 0.0;
            for (int q = 0; q < NT / 64; ++q) {
                s0 += red[2 * q];
                s1 += red[2 * q + 1];
            }
            a.npart[2 * blockIdx.x] = s0;
            a.npart[2 * blockIdx.x + 1] = s1;
        }
    }
}

template <typename R, bool SITE, int TW>
__global__ __launch_bounds__(TW + 64) void k2_fused2(FusedArgs<R> a, const R *__restrict__ tab) {
    constexpr int W = TW + 4;
    __shared__ __align__(16) cx<R> sOld[2 + 4 * W + 2];
    __shared__ __align__(16) cx<R> sStage[2 * W];
    __shared__ __align__(16) cx<R> sLev[2 + 6 * W + 2];
    const int L = logical_block2();
    march2x2<R, SITE, TW>(a, tab, L % a.ntx, L / a.ntx, sOld, sStage, sLev);
}

int chunks_for(int64_t tiles, int nz, int target) {
    int64_t c = (target + tiles - 1) / tiles;
    if (c < 1) c = 1;
    if (c > nz) c = nz;
    return (int)c;
}

}  // namespace

// Workgroups of the 3D fused kernels that run at once: one per CU (the
// two-step kernel's LDS allows one; the one-step kernel measured best at the
// same count), queried once.
int resident_per_round() {
    static int n = 0;
    if (n == 0) {
        int dev = 0, cus = 0;
        n = (hipGetDevice(&dev) == hipSuccess &&
             hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
                ? cus : 256;
    }
    return n;
}

// Chunks per tile column of a 3D z-march.  A chunk costs its planes plus
// `fill` of pipeline fill (two-step kernel 6, one-step 3), and the workgroups
// run in rounds of one per CU, so the count minimising rounds x (planes per
// chunk + fill) is taken, the largest within 1% of that minimum (more
// workgroups balance the tail).  It reproduces the best of sweeps at 128^3,
// 256^3, 512^3 (both precisions, both kernels) and a 512 x 512 x 64 slab (e.g.
// 128^3 complex64, two-step: 8 chunks of 16 planes, 0.044 ms per step against
// 0.074 with 32 chunks of 4).  Memoised for repeated calls.
int pick_chunks(int64_t tiles, int nz, int fill) {
    static thread_local int64_t m_tiles = -1;
    static thread_local int m_nz = -1, m_fill = -1, m_res = 1;
    if (tiles == m_tiles && nz == m_nz && fill == m_fill) return m_res;
    const int64_t per = resident_per_round();
    const int64_t cap = std::min<int64_t>(nz, 8 * ((per + tiles - 1) / tiles));
    auto cost = [&](int64_t c) { return (double)((tiles * c + per - 1) / per) * (double)((nz + c - 1) / c + fill); };
    double best = 1e300;
    for (int64_t c = 1; c <= cap; ++c) best = std::min(best, cost(c));
    int res = 1;
    for (int64_t c = 1; c <= cap; ++c)
        if (cost(c) <= 1.01 * best) res = (int)c;
    m_tiles = tiles;
    m_nz = nz;
    m_fill = fill;
    m_res = res;
    return res;
}

bool fused3x2_supported(int nx, bool fp32, bool site) { (void)site; return !fp32 || nx % 2 == 0; }

namespace {
// One launch of the two-step kernel with tile TW x TY and NT threads; px: the
// XCD patch width of its tile order.
template <typename R, int TW, int TY, int NT, bool ROT, bool SITE>
hipError_t launch_x2(FusedArgs<R> a, int px, hipStream_t s, int *nblocks_out) {
    a.ntx = (a.nx + TW - 1) / TW;
    a.nty = (a.ny + TY - 1) / TY;
    const int64_t tiles = (int64_t)a.ntx * a.nty;
    if (a.zchunk <= 0) {
        const int nzc = pick_chunks(tiles, a.nz, 6);
        a.zchunk = (a.nz + nzc - 1) / nzc;
    }
    a.nzc = (a.nz + a.zchunk - 1) / a.zchunk;
    a.px = px;
    const int64_t nblk = tiles * a.nzc;
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    if (nblocks_out) *nblocks_out = (int)nblk;
    const bool norm = a.npart != nullptr;
    if (norm && nblk > a.npart_cap) return hipErrorInvalidValue;
    if (norm && SITE && a.rev) return hipErrorInvalidValue;     // no functional on reversed steps
    const dim3 g((unsigned)nblk), b(NT);
    if constexpr (SITE) {
        if (norm) hipLaunchKernelGGL((k3_fused2<R, TW, TY, NT, true, 1, ROT>), g, b, 0, s, a, a.tab);
        else if (a.rev) hipLaunchKernelGGL((k3_fused2<R, TW, TY, NT, false, 2, ROT>), g, b, 0, s, a, a.tab);
        else hipLaunchKernelGGL((k3_fused2<R, TW, TY, NT, false, 1, ROT>), g, b, 0, s, a, a.tab);
    } else {
        if (norm) hipLaunchKernelGGL((k3_fused2<R, TW, TY, NT, true, 0, ROT>), g, b, 0, s, a, a.tab);
        else hipLaunchKernelGGL((k3_fused2<R, TW, TY, NT, false, 0, ROT>), g, b, 0, s, a, a.tab);
    }
    return hipGetLastError();
}
}  // namespace

// Tiles: complex64 64 x 8 cells (1024 threads); complex128 32 x 8 with
// per-site records, 16 x 16 with tables (512 threads).  The XCD patch: with complex64 tiles whole tile rows keep every x-neighbour
// resident and measured fastest; with complex128 tiles whole tile rows form a
// band only 16 cells tall at 512^3, and patches of 4 x 8 tiles measured ~2%
// faster.  The old C,D planes rotate through three LDS sets (ROT) in the
// complex64 kernels (at 512^3: 3.45 against 4.29 ms per launch with V(z)
// tables, 6.23 against 6.84 with per-site records) and the complex128 ones
// with tables, whose three sets fit only with tiles of 16 x 16 (7.65 against
// 7.82 ms).  The complex128 per-site kernel, bound by the divisions that turn
// its theta records into coefficients, keeps the staging layout and its 32 x 8
// tiles (rotated with 16 x 16 tiles: 8.67 against 8.44 ms per step).
template <typename R>
hipError_t launch_fused3x2(const FusedArgs<R> &a, bool site, hipStream_t s, int *nblocks_out) {
    if ((!site && a.tab == nullptr) || (sizeof(R) == 4 && a.nx % 2 != 0)) return hipErrorInvalidValue;
    if (site)
        for (int q = 0; q < 8; ++q)
            if (a.th[q] == nullptr) return hipErrorInvalidValue;
    // plane byte offsets are 32-bit inside the kernel
    if ((uint64_t)a.nx * (uint64_t)a.ny * sizeof(cx<R>) >= (1ull << 32)) return hipErrorInvalidValue;
    if constexpr (sizeof(R) == 4) {
        if (site) return launch_x2<R, 64, 8, 1024, true, true>(a, 0, s, nblocks_out);
        return launch_x2<R, 64, 8, 1024, true, false>(a, 0, s, nblocks_out);
    } else {
        if (site) return launch_x2<R, 32, 8, 512, false, true>(a, 4, s, nblocks_out);
        return launch_x2<R, 16, 16, 512, true, false>(a, 4, s, nblocks_out);
    }
}

bool fused2x2_supported(int nx, bool fp32) { return !fp32 || nx % 2 == 0; }

template <typename R> hipError_t launch_fused2x2(const FusedArgs<R> &a0, bool site, hipStream_t s) {
    FusedArgs<R> a = a0;
    if ((sizeof(R) == 4 && a.nx % 2 != 0) || (!site && a.tab == nullptr)) return hipErrorInvalidValue;
    constexpr int TW = 128;
    a.ntx = (a.nx + TW - 1) / TW;
    a.nty = 1;
    if (a.zchunk <= 0) {
        // about 1024 workgroups of TW + 64 threads: 2^19-cell lattices march 4-row
        // chunks, 2^21-cell ones 16 (the best of a sweep from 2 to 128 rows)
        const int nc = chunks_for(a.ntx, a.ny, 1024);
        a.zchunk = (a.ny + nc - 1) / nc;
        if (a.zchunk < 4) a.zchunk = a.ny < 4 ? a.ny : 4;
    }
    a.nzc = (a.ny + a.zchunk - 1) / a.zchunk;
    const int64_t nblk = (int64_t)a.ntx * a.nzc;
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    if (site) hipLaunchKernelGGL((k2_fused2<R, true, TW>), dim3((unsigned)nblk), dim3(TW + 64), 0, s, a, a.tab);
    else hipLaunchKernelGGL((k2_fused2<R, false, TW>), dim3((unsigned)nblk), dim3(TW + 64), 0, s, a, a.tab);
    return hipGetLastError();
}

template hipError_t launch_fused2x2<float>(const FusedArgs<float> &, bool, hipStream_t);
template hipError_t launch_fused2x2<double>(const FusedArgs<double> &, bool, hipStream_t);
template hipError_t launch_fused3x2<float>(const FusedArgs<float> &, bool, hipStream_t, int *);
template hipError_t launch_fused3x2<double>(const FusedArgs<double> &, bool, hipStream_t, int *);

}  // namespace dirac
