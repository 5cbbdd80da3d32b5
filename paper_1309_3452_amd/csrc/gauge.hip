// Vector potential by gauge links (Sect. 4, Peierls substitution): one unit
// factor per half-link.  Link arrays U[6 a + t] (3D) / U[4 a + t] (2D) hold,
// for the A,B (u) array a at cell c, the factor of its neighbour in direction
// t = +z, -z, +x, -x, +y, -y (2D: +x, -x, +y, -y): the neighbour value in S_X
// is multiplied by it.  A C,D (v) row uses the conjugate of the factor of the
// same half-link, stored at its A,B (u) end; the mapping, from the stencils of
// Eqs. ss1-ss4 (with d the displacement from the C,D site to its neighbour,
// the A,B end's term is the one pointing back, -d):
//   S_C0: +z A0(zp) t-z, -z A0 t+z, +x B0 t-x, -x B0(xm) t+x, +y B1 t-y, -y B1(ym) t+y
//   S_C1: +z A1(zp) t-z, -z A1 t+z, +x B1(xp) t-x, -x B1 t+x, +y B0(yp) t-y, -y B0 t+y
//   S_D0: +z B0 t-z, -z B0(zm) t+z, +x A0(xp) t-x, -x A0 t+x, +y A1 t-y, -y A1(ym) t+y
//   S_D1: +z B1 t-z, -z B1(zm) t+z, +x A1 t-x, -x A1(xm) t+x, +y A0(yp) t-y, -y A0 t+y
// The coupling stays anti-Hermitian, so E_r with the links in S_X is conserved
// for a static potential.  Kernels: cell-parallel split half-steps (in place;
// the reversed step, (2+1)D) and the E_r reductions, and a (3+1)D z-march that
// does the whole step in one launch, reading every link factor once.  Both
// build each C,D coupling through the same helpers: the same bits.
#include "device.h"
#include "internal.h"
#include "stencil3.h"
#include "march2.h"
#include "gauge.h"
#include "norm3.h"
#include "ntstore.h"

namespace dirac {

namespace {

enum { TZP = 0, TZM = 1, TXP = 2, TXM = 3, TYP = 4, TYM = 5 };

// Loads in the compute type D: the stored type for the half-steps, FP64 for
// the reductions.
template <typename D> struct Ld;
template <> struct Ld<float2> {
    static __device__ __forceinline__ float2 get(float2 v) { return v; }
};
template <> struct Ld<double2> {
    static __device__ __forceinline__ double2 get(double2 v) { return v; }
    static __device__ __forceinline__ double2 get(float2 v) { return make_double2((double)v.x, (double)v.y); }
};

// Field value of array p at cell idx; link factor of A,B (u) array a, term t, at cell idx.
#define FV(p, idx) Ld<D>::get(f[p][idx])
#define LK(a, t, idx) Ld<D>::get(((const CS *)L.u[NT * (a) + (t)])[idx])
#define LKC(a, t, idx) cconj(LK(a, t, idx))

template <typename R, bool SITE>
__device__ __forceinline__ Coef<R> gcoef(const HalfArgs<R> &a, int arr, int q, int k, size_t c) {
    if constexpr (SITE) {
        return coef_site_at<R>(a.th[arr], c, a.tsgn);
    } else {
        const R *e = a.tab + ((size_t)q * a.nz + k) * 4;
        Coef<R> cf;
        cf.c1 = mk2(e[0], e[1]);
        cf.c2 = mk2(e[2], e[3]);
        return cf;
    }
}

// Neighbour cell indices of cell (i, j, k), periodic.
struct Nb3 {
    size_t c, xm, xp, ym, yp, zm, zp;
};
__device__ __forceinline__ Nb3 nb3(int i, int j, int k, int nx, int ny, int nz) {
    const size_t plane = (size_t)nx * ny, row = (size_t)j * nx, kk = (size_t)k * plane;
    Nb3 n;
    n.c = kk + row + i;
    n.xm = kk + row + wrap_dec(i, nx);
    n.xp = kk + row + wrap_inc(i, nx);
    n.ym = kk + (size_t)wrap_dec(j, ny) * nx + i;
    n.yp = kk + (size_t)wrap_inc(j, ny) * nx + i;
    n.zm = (size_t)wrap_dec(k, nz) * plane + row + i;
    n.zp = (size_t)wrap_inc(k, nz) * plane + row + i;
    return n;
}

// ---- (3+1)D ----
// A,B rows with links, one row per array (u: that array's six link factors at
// the cell, term order +z, -z, +x, -x, +y, -y; the C,D values as in stencil_ab).
template <typename C, typename R>
__device__ __forceinline__ C ab_row0(const C *u, C c0, C c0zm, C d0, C d0xm, C d1, C d1ym, R rx, R ry, R rz) {
    return sterm3(rz, csub(cmul(u[TZP], c0), cmul(u[TZM], c0zm)), rx, csub(cmul(u[TXP], d0), cmul(u[TXM], d0xm)),
                  -ry, csub(cmul(u[TYP], d1), cmul(u[TYM], d1ym)));
}
template <typename C, typename R>
__device__ __forceinline__ C ab_row1(const C *u, C c1, C c1zm, C d1xp, C d1, C d0yp, C d0, R rx, R ry, R rz) {
    return sterm3(rz, csub(cmul(u[TZP], c1), cmul(u[TZM], c1zm)), rx, csub(cmul(u[TXP], d1xp), cmul(u[TXM], d1)),
                  -ry, csub(cmul(u[TYP], d0yp), cmul(u[TYM], d0)));
}
template <typename C, typename R>
__device__ __forceinline__ C ab_row2(const C *u, C d0zp, C d0, C c0xp, C c0, C c1, C c1ym, R rx, R ry, R rz) {
    return sterm3(-rz, csub(cmul(u[TZP], d0zp), cmul(u[TZM], d0)), rx, csub(cmul(u[TXP], c0xp), cmul(u[TXM], c0)),
                  ry, csub(cmul(u[TYP], c1), cmul(u[TYM], c1ym)));
}
template <typename C, typename R>
__device__ __forceinline__ C ab_row3(const C *u, C d1zp, C d1, C c1, C c1xm, C c0yp, C c0, R rx, R ry, R rz) {
    return sterm3(-rz, csub(cmul(u[TZP], d1zp), cmul(u[TZM], d1)), rx, csub(cmul(u[TXP], c1), cmul(u[TXM], c1xm)),
                  ry, csub(cmul(u[TYP], c0yp), cmul(u[TYM], c0)));
}

// One C,D coupling: the new A,B value x times the conjugate of its link factor u.
template <typename C> __device__ __forceinline__ C pr(C u, C x) { return cmul(cconj(u), x); }

// C,D rows from their 24 couplings T[6 q + term] (q = C0, C1, D0, D1; term
// order +z, -z, +x, -x, +y, -y), each conj(U) times the new A,B value at the
// neighbour (the table in the header comment):
//   C0: A0(zp).-z  A0.+z  B0.-x  B0(xm).+x  B1.-y  B1(ym).+y
//   C1: A1(zp).-z  A1.+z  B1(xp).-x  B1.+x  B0(yp).-y  B0.+y
//   D0: B0.-z  B0(zm).+z  A0(xp).-x  A0.+x  A1.-y  A1(ym).+y
//   D1: B1.-z  B1(zm).+z  A1.-x  A1(xm).+x  A0(yp).-y  A0.+y
template <typename C, typename R> __device__ __forceinline__ St3<C> cd_rows(const C (&T)[24], R rx, R ry, R rz) {
    St3<C> s;
    s.s0 = sterm3(rz, csub(T[0], T[1]), rx, csub(T[2], T[3]), -ry, csub(T[4], T[5]));
    s.s1 = sterm3(rz, csub(T[6], T[7]), rx, csub(T[8], T[9]), -ry, csub(T[10], T[11]));
    s.s2 = sterm3(-rz, csub(T[12], T[13]), rx, csub(T[14], T[15]), ry, csub(T[16], T[17]));
    s.s3 = sterm3(-rz, csub(T[18], T[19]), rx, csub(T[20], T[21]), ry, csub(T[22], T[23]));
    return s;
}

// Cell-parallel forms (split half-steps, reductions): values loaded in the
// compute type D (FV, LK above).
template <typename D, typename RD, typename CS>
__device__ __forceinline__ St3<D> links_ab(const CS *const f[8], const LinkPtrs &L, const Nb3 &n, RD rx, RD ry, RD rz) {
    constexpr int NT = 6;
    D u[24];
#pragma unroll
    for (int q = 0; q < 24; ++q) u[q] = LK(q / 6, q % 6, n.c);
    St3<D> s;
    s.s0 = ab_row0(u, FV(4, n.c), FV(4, n.zm), FV(6, n.c), FV(6, n.xm), FV(7, n.c), FV(7, n.ym), rx, ry, rz);
    s.s1 = ab_row1(u + 6, FV(5, n.c), FV(5, n.zm), FV(7, n.xp), FV(7, n.c), FV(6, n.yp), FV(6, n.c), rx, ry, rz);
    s.s2 = ab_row2(u + 12, FV(6, n.zp), FV(6, n.c), FV(4, n.xp), FV(4, n.c), FV(5, n.c), FV(5, n.ym), rx, ry, rz);
    s.s3 = ab_row3(u + 18, FV(7, n.zp), FV(7, n.c), FV(5, n.c), FV(5, n.xm), FV(4, n.yp), FV(4, n.c), rx, ry, rz);
    return s;
}

template <typename D, typename RD, typename CS>
__device__ __forceinline__ St3<D> links_cd(const CS *const f[8], const LinkPtrs &L, const Nb3 &n, RD rx, RD ry, RD rz) {
    constexpr int NT = 6;
    const D T[24] = {
        pr(LK(0, TZM, n.zp), FV(0, n.zp)), pr(LK(0, TZP, n.c), FV(0, n.c)),
        pr(LK(2, TXM, n.c), FV(2, n.c)), pr(LK(2, TXP, n.xm), FV(2, n.xm)),
        pr(LK(3, TYM, n.c), FV(3, n.c)), pr(LK(3, TYP, n.ym), FV(3, n.ym)),
        pr(LK(1, TZM, n.zp), FV(1, n.zp)), pr(LK(1, TZP, n.c), FV(1, n.c)),
        pr(LK(3, TXM, n.xp), FV(3, n.xp)), pr(LK(3, TXP, n.c), FV(3, n.c)),
        pr(LK(2, TYM, n.yp), FV(2, n.yp)), pr(LK(2, TYP, n.c), FV(2, n.c)),
        pr(LK(2, TZM, n.c), FV(2, n.c)), pr(LK(2, TZP, n.zm), FV(2, n.zm)),
        pr(LK(0, TXM, n.xp), FV(0, n.xp)), pr(LK(0, TXP, n.c), FV(0, n.c)),
        pr(LK(1, TYM, n.c), FV(1, n.c)), pr(LK(1, TYP, n.ym), FV(1, n.ym)),
        pr(LK(3, TZM, n.c), FV(3, n.c)), pr(LK(3, TZP, n.zm), FV(3, n.zm)),
        pr(LK(1, TXM, n.c), FV(1, n.c)), pr(LK(1, TXP, n.xm), FV(1, n.xm)),
        pr(LK(0, TYM, n.yp), FV(0, n.yp)), pr(LK(0, TYP, n.c), FV(0, n.c))};
    return cd_rows(T, rx, ry, rz);
}

// which == 0: A,B from C,D (Eqs. ss1, ss2); 1: C,D from A,B (ss3, ss4); in place.
template <typename R, bool SITE, int WHICH>
__global__ __launch_bounds__(256) void k3_half_links(HalfArgs<R> a, LinkPtrs L) {
    using C = cx<R>;
    const int64_t ncell = (int64_t)a.nx * a.ny * a.nz;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncell) return;
    const int i = (int)(t % a.nx);
    const int64_t q = t / a.nx;
    const int j = (int)(q % a.ny), k = (int)(q / a.ny);
    const Nb3 n = nb3(i, j, k, a.nx, a.ny, a.nz);
    C *f[8];
    const C *fc[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        f[p] = (C *)a.f[p];
        fc[p] = f[p];
    }
    if constexpr (WHICH == 0) {
        const St3<C> s = links_ab<C, R, C>(fc, L, n, a.rx, a.ry, a.rz);
        // old values and coefficients before the first store: a load issued after a
        // store would wait for it too
        const C o0 = f[0][n.c], o1 = f[1][n.c], o2 = f[2][n.c], o3 = f[3][n.c];
        const Coef<R> k0 = gcoef<R, SITE>(a, 0, 0, k, n.c), k1 = gcoef<R, SITE>(a, 1, 0, k, n.c), k2 = gcoef<R, SITE>(a, 2, 1, k, n.c), k3 = gcoef<R, SITE>(a, 3, 1, k, n.c);
        st_nt(&f[0][n.c], update(o0, s.s0, k0));
        st_nt(&f[1][n.c], update(o1, s.s1, k1));
        st_nt(&f[2][n.c], update(o2, s.s2, k2));
        st_nt(&f[3][n.c], update(o3, s.s3, k3));
    } else {
        const St3<C> s = links_cd<C, R, C>(fc, L, n, a.rx, a.ry, a.rz);
        // old values and coefficients before the first store: a load issued after a
        // store would wait for it too
        const C o4 = f[4][n.c], o5 = f[5][n.c], o6 = f[6][n.c], o7 = f[7][n.c];
        const Coef<R> k4 = gcoef<R, SITE>(a, 4, 2, k, n.c), k5 = gcoef<R, SITE>(a, 5, 2, k, n.c), k6 = gcoef<R, SITE>(a, 6, 3, k, n.c), k7 = gcoef<R, SITE>(a, 7, 3, k, n.c);
        st_nt(&f[4][n.c], update(o4, s.s0, k4));
        st_nt(&f[5][n.c], update(o5, s.s1, k5));
        st_nt(&f[6][n.c], update(o6, s.s2, k6));
        st_nt(&f[7][n.c], update(o7, s.s3, k7));
    }
}

// One step per launch with links, marching along z (ping-pong in -> out).
// A workgroup owns a 64 x TY tile and a chunk [z0, z1) of planes; at plane p it
// computes the new A,B(p) on the tile and on the one-cell ring around it (not
// the corners), then the new C,D(p-1) on the tile.  Each of a cell's 24 C,D
// couplings pr(U, new A,B) is formed once, by the thread that updated the A,B
// end, right after that update, with the link factors it has just loaded for
// it: 12 serve the cell's own C,D rows (kept in registers one plane), 2 the
// C,D rows one plane below (this plane's C,D(p-1)), 2 the rows one plane above
// (kept two planes), and 8 the x-y neighbours' rows, through LDS.  So every
// link factor and every amplitude is read once per step (the ring's recompute
// and cache-served neighbour reads aside), where the split form reads the
// links twice.  Same helpers and operation order as the split kernels: the
// same bits.  Thread layout: 64 TY tile threads (wave y = tile row y), then
// the ring (left and right columns, bottom and top rows), the rest idle.
template <int TW, int TY> constexpr int fl_threads() { return TW * TY + 64 * ((2 * TW + 2 * TY + 63) / 64); }

template <typename R, bool SITE, int TW, int TY, int WPE>
__global__ __launch_bounds__((fl_threads<TW, TY>()), WPE) void k3_fused_links(FusedArgs<R> a, LinkPtrs L,
                                                                             const R *__restrict__ tab) {
    using C = cx<R>;
    constexpr int LW = TW + 2, LN = LW * (TY + 2);
    __shared__ C sE[2][8][LN];      // exports of A,B(p), slot p & 1

    int lb = blockIdx.x;
    if ((gridDim.x & 7) == 0) lb = (lb & 7) * (gridDim.x >> 3) + (lb >> 3);   // one run of tiles per XCD
    // the ~32 tiles an XCD runs at once: whole tile rows (px = 0) or a patch of
    // px x 32/px tiles, whose halo rows and columns stay in that XCD's L2
    int tx, ty, zc;
    const int PX = a.px > 0 ? a.px : 1, PY = a.px > 0 ? 32 / a.px : 1;
    if (a.px > 0 && a.ntx % PX == 0 && a.nty % PY == 0) {
        const int within = lb % (PX * PY), patch = lb / (PX * PY);
        const int npx = a.ntx / PX, npy = a.nty / PY;
        tx = (patch % npx) * PX + within % PX;
        const int rest = patch / npx;
        ty = (rest % npy) * PY + within / PX;
        zc = rest / npy;
    } else {
        tx = lb % a.ntx;
        lb /= a.ntx;
        ty = lb % a.nty;
        zc = lb / a.nty;
    }
    const int x0 = tx * TW, y0 = ty * TY;
    const int w = min(TW, a.nx - x0), h = min(TY, a.ny - y0);
    const int z0 = zc * a.zchunk, z1 = min(a.nz, z0 + a.zchunk);
    const int t = threadIdx.x;
    // rows this cell updates: all four on the tile; on the ring only the two
    // whose couplings point into the tile (left: A1, B0; right: A0, B1; bottom:
    // A1, B1; top: A0, B0)
    int x = 0, y = 0;
    bool tile = false, act = false, nA0 = false, nA1 = false, nB0 = false, nB1 = false;
    if (t < TW * TY) {
        x = t % TW;
        y = t / TW;
        tile = act = nA0 = nA1 = nB0 = nB1 = x < w && y < h;
    } else {
        const int r = t - TW * TY;
        act = true;
        if (r < h) { x = -1; y = r; nA1 = nB0 = true; }
        else if (r < 2 * h) { x = w; y = r - h; nA0 = nB1 = true; }
        else if (r < 2 * h + w) { x = r - 2 * h; y = -1; nA1 = nB1 = true; }
        else if (r < 2 * h + 2 * w) { x = r - 2 * h - w; y = h; nA0 = nB0 = true; }
        else { act = false; }
    }
    const int gx = wrapn(x0 + x, a.nx), gy = wrapn(y0 + y, a.ny);
    const size_t row = (size_t)gy * a.nx;
    const size_t c2 = row + gx;
    const size_t xm2 = row + wrap_dec(gx, a.nx), xp2 = row + wrap_inc(gx, a.nx);
    const size_t ym2 = (size_t)wrap_dec(gy, a.ny) * a.nx + gx, yp2 = (size_t)wrap_inc(gy, a.ny) * a.nx + gx;
    const int li = act ? (y + 1) * LW + (x + 1) : 0;
    const size_t plane = (size_t)a.nx * a.ny;
    const C *in[8];
    C *out[8];
    const C *lk[24];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        in[q] = (const C *)a.in[q];
        out[q] = (C *)a.out[q];
    }
#pragma unroll
    for (int q = 0; q < 24; ++q) lk[q] = (const C *)L.u[q];
    const R rx = a.rx, ry = a.ry, rz = a.rz;
    const C zero = mk2((R)0, (R)0);
    // V(z) table entry of class cls at plane pk: the address is the same for the
    // whole workgroup, and the table is read-only here, so these are scalar loads
    // that never hold up the vector memory counter
    auto tcoef = [&](int cls, int pk) -> Coef<R> {
        const R *e = tab + ((size_t)cls * a.nz + pk) * 4;
        Coef<R> k;
        k.c1 = mk2(e[0], e[1]);
        k.c2 = mk2(e[2], e[3]);
        return k;
    };

    // carried along the march: old C(p-1), D(p), D(p-1) at the cell; the own
    // couplings of A,B(p-1); the upward couplings of A,B(p-1) and A,B(p-2)
    C cm0 = zero, cm1 = zero, dc0 = zero, dc1 = zero, dm0 = zero, dm1 = zero;
    C Q[12], zm1[2] = {zero, zero}, zm2[2] = {zero, zero};
#pragma unroll
    for (int q = 0; q < 12; ++q) Q[q] = zero;
    if (act) {
        const size_t Pc = (size_t)wrapn(z0 - 2, a.nz) * plane, Pd = (size_t)wrapn(z0 - 1, a.nz) * plane;
        cm0 = in[4][Pc + c2];
        cm1 = in[5][Pc + c2];
        dc0 = in[6][Pd + c2];
        dc1 = in[7][Pd + c2];
    }

    for (int p = z0 - 1; p <= z1; ++p) {
        const int pk = wrapn(p, a.nz), pm = wrapn(p - 1, a.nz);
        const size_t P = (size_t)pk * plane, Pn = (size_t)wrapn(p + 1, a.nz) * plane;
        C E[8], Qn[12], zpn[2], zmn[2], cc0 = zero, cc1 = zero, dn0 = zero, dn1 = zero;
        Coef<R> kt[4];      // classes A, B at plane p and C, D at plane p - 1 (tables only)
        if constexpr (!SITE) {
            kt[0] = tcoef(0, pk);
            kt[1] = tcoef(1, pk);
            kt[2] = tcoef(2, pm);
            kt[3] = tcoef(3, pm);
        }
        auto coef = [&](int arr, int cls, size_t idx) -> Coef<R> {
            if constexpr (SITE) return coef_site_at<R>(a.th[arr], idx, (R)1);
            else return kt[cls];
        };
#pragma unroll
        for (int q = 0; q < 8; ++q) E[q] = zero;
#pragma unroll
        for (int q = 0; q < 12; ++q) Qn[q] = zero;
        zpn[0] = zpn[1] = zmn[0] = zmn[1] = zero;
        if (act) {
            const size_t ci = P + c2;
            const bool store = tile && p >= z0 && p < z1;
            C u[24], xo[4], nb[8];
#pragma unroll
            for (int q = 0; q < 24; ++q) u[q] = zero;
#pragma unroll
            for (int q = 0; q < 8; ++q) nb[q] = zero;
            xo[0] = xo[1] = xo[2] = xo[3] = zero;
            cc0 = in[4][ci];
            cc1 = in[5][ci];
            dn0 = in[6][Pn + c2];
            dn1 = in[7][Pn + c2];
            auto ld0 = [&]() {
#pragma unroll
                for (int q = 0; q < 6; ++q) u[q] = lk[q][ci];
                xo[0] = in[0][ci];
                nb[0] = in[6][P + xm2];
                nb[1] = in[7][P + ym2];
            };
            auto ld1 = [&]() {
#pragma unroll
                for (int q = 0; q < 6; ++q) u[6 + q] = lk[6 + q][ci];
                xo[1] = in[1][ci];
                nb[2] = in[7][P + xp2];
                nb[3] = in[6][P + yp2];
            };
            auto ld2 = [&]() {
#pragma unroll
                for (int q = 0; q < 6; ++q) u[12 + q] = lk[12 + q][ci];
                xo[2] = in[2][ci];
                nb[4] = in[4][P + xp2];
                nb[5] = in[5][P + ym2];
            };
            auto ld3 = [&]() {
#pragma unroll
                for (int q = 0; q < 6; ++q) u[18 + q] = lk[18 + q][ci];
                xo[3] = in[3][ci];
                nb[6] = in[5][P + xm2];
                nb[7] = in[4][P + yp2];
            };
            if (nA0) {
                ld0();
                const C na0 = update(xo[0], ab_row0(u, cc0, cm0, dc0, nb[0], dc1, nb[1], rx, ry, rz), coef(0, 0, ci));
                if (store) st_nt(&out[0][ci], na0);
                E[3] = pr(u[TXM], na0);
                E[7] = pr(u[TYM], na0);
                Qn[0] = pr(u[TZP], na0);
                Qn[7] = pr(u[TXP], na0);
                Qn[11] = pr(u[TYP], na0);
                zpn[0] = pr(u[TZM], na0);
            }
            if (nA1) {
                ld1();
                const C *v = u + 6;
                const C na1 = update(xo[1], ab_row1(v, cc1, cm1, nb[2], dc1, nb[3], dc0, rx, ry, rz), coef(1, 0, ci));
                if (store) st_nt(&out[1][ci], na1);
                E[1] = pr(v[TXP], na1);
                E[5] = pr(v[TYP], na1);
                Qn[3] = pr(v[TZP], na1);
                Qn[8] = pr(v[TYM], na1);
                Qn[10] = pr(v[TXM], na1);
                zpn[1] = pr(v[TZM], na1);
            }
            if (nB0) {
                ld2();
                const C *v = u + 12;
                const C nb0 = update(xo[2], ab_row2(v, dn0, dc0, nb[4], cc0, cc1, nb[5], rx, ry, rz), coef(2, 1, ci));
                if (store) st_nt(&out[2][ci], nb0);
                E[0] = pr(v[TXP], nb0);
                E[6] = pr(v[TYM], nb0);
                Qn[1] = pr(v[TXM], nb0);
                Qn[5] = pr(v[TYP], nb0);
                Qn[6] = pr(v[TZM], nb0);
                zmn[0] = pr(v[TZP], nb0);
            }
            if (nB1) {
                ld3();
                const C *v = u + 18;
                const C nb1 = update(xo[3], ab_row3(v, dn1, dc1, cc1, nb[6], nb[7], cc0, rx, ry, rz), coef(3, 1, ci));
                if (store) st_nt(&out[3][ci], nb1);
                E[2] = pr(v[TXM], nb1);
                E[4] = pr(v[TYP], nb1);
                Qn[2] = pr(v[TYM], nb1);
                Qn[4] = pr(v[TXP], nb1);
                Qn[9] = pr(v[TZM], nb1);
                zmn[1] = pr(v[TZP], nb1);
            }
        }
        // C,D of plane p-1 on the tile, from the couplings of A,B(p-1) (LDS and
        // registers), A,B(p) (this plane) and A,B(p-2)
        if (act) {
#pragma unroll
            for (int q = 0; q < 8; ++q) sE[p & 1][q][li] = E[q];
        }
        if (tile && p - 1 >= z0 && p - 1 < z1) {
            const size_t cm = (size_t)pm * plane + c2;
            const C(*e)[LN] = sE[(p - 1) & 1];
            const C T[24] = {zpn[0], Q[0], Q[1], e[0][li - 1], Q[2], e[4][li - LW],
                             zpn[1], Q[3], e[2][li + 1], Q[4], e[6][li + LW], Q[5],
                             Q[6], zm2[0], e[3][li + 1], Q[7], Q[8], e[5][li - LW],
                             Q[9], zm2[1], Q[10], e[1][li - 1], e[7][li + LW], Q[11]};
            const St3<C> s = cd_rows(T, rx, ry, rz);
            // all four coefficients before the first store (per-site records:
            // the loads then need not wait for the stores)
            const Coef<R> k4 = coef(4, 2, cm), k5 = coef(5, 2, cm), k6 = coef(6, 3, cm), k7 = coef(7, 3, cm);
            st_nt(&out[4][cm], update(cm0, s.s0, k4));
            st_nt(&out[5][cm], update(cm1, s.s1, k5));
            st_nt(&out[6][cm], update(dm0, s.s2, k6));
            st_nt(&out[7][cm], update(dm1, s.s3, k7));
        }
        // one barrier per plane: the exports of A,B(p) (slot p & 1) are visible to
        // the next plane's C,D, and this plane's reads of slot (p - 1) & 1 are done
        // before the next plane overwrites it
        __syncthreads();
        cm0 = cc0;
        cm1 = cc1;
        dm0 = dc0;
        dm1 = dc1;
        dc0 = dn0;
        dc1 = dn1;
#pragma unroll
        for (int q = 0; q < 12; ++q) Q[q] = Qn[q];
        zm2[0] = zm1[0];
        zm2[1] = zm1[1];
        zm1[0] = zmn[0];
        zm1[1] = zmn[1];
    }
}

__device__ __forceinline__ double2 dd(double2 v) { return v; }
__device__ __forceinline__ double2 dd(float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ __forceinline__ double re_cs(double2 x, double2 s) { return x.x * s.x + x.y * s.y; }   // Re conj(x) s

// Per-workgroup partials of (E_r, E_r summed on the C,D sites, plain norm) with
// links; kReduceBlocks workgroups take cells with a fixed stride (fixed order).
template <typename R>
__global__ __launch_bounds__(kReduceThreads) void k3_norm_links(ReduceArgs<R> a, LinkPtrs L) {
    using C = cx<R>;
    __shared__ double lds[kNormVals * 16];
    const C *f[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) f[p] = (const C *)a.f[p];
    const int64_t ncell = (int64_t)a.nx * a.ny * a.nz;
    const double rx = a.rx, ry = a.ry, rz = a.rz;
    double v[kNormVals] = {0.0, 0.0, 0.0};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ncell; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % a.nx);
        const int64_t q = t / a.nx;
        const int j = (int)(q % a.ny), k = (int)(q / a.ny);
        const Nb3 n = nb3(i, j, k, a.nx, a.ny, a.nz);
        const St3<double2> sa = links_ab<double2, double, C>(f, L, n, rx, ry, rz);
        const St3<double2> sc = links_cd<double2, double, C>(f, L, n, rx, ry, rz);
        double p2 = 0.0;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const double2 x = dd(f[p][n.c]);
            p2 += x.x * x.x + x.y * x.y;
        }
        const double eab = re_cs(dd(f[0][n.c]), sa.s0) + re_cs(dd(f[1][n.c]), sa.s1) +
                           re_cs(dd(f[2][n.c]), sa.s2) + re_cs(dd(f[3][n.c]), sa.s3);
        const double ecd = re_cs(dd(f[4][n.c]), sc.s0) + re_cs(dd(f[5][n.c]), sc.s1) +
                           re_cs(dd(f[6][n.c]), sc.s2) + re_cs(dd(f[7][n.c]), sc.s3);
        v[0] += p2 - eab;
        v[1] += p2 + ecd;
        v[2] += p2;
    }
    block_sum<kNormVals>(v, lds);
    if (threadIdx.x == 0) {
        double *o = a.partial + (size_t)blockIdx.x * kNormVals;
        for (int p = 0; p < kNormVals; ++p) o[p] = v[p];
    }
}

// ---- (2+1)D ----
struct Nb2 {
    size_t c, xm, xp, ym, yp;
};
__device__ __forceinline__ Nb2 nb2(int i, int j, int nx, int ny) {
    const size_t row = (size_t)j * nx;
    Nb2 n;
    n.c = row + i;
    n.xm = row + wrap_dec(i, nx);
    n.xp = row + wrap_inc(i, nx);
    n.ym = (size_t)wrap_dec(j, ny) * nx + i;
    n.yp = (size_t)wrap_inc(j, ny) * nx + i;
    return n;
}
enum { T2XP = 0, T2XM = 1, T2YP = 2, T2YM = 3 };

// u rows with links, one row per array (u: the array's four link factors at
// the cell, term order +x, -x, +y, -y):
//   u0: +x v0, -x v0[i-1], +y v1, -y v1[j-1];  u1: +x v1[i+1], -x v1, +y v0[j+1], -y v0
template <typename C, typename R>
__device__ __forceinline__ C u_row0(const C *u, C v0, C v0xm, C v1, C v1ym, R rx, R ry) {
    return sterm2(rx, csub(cmul(u[T2XP], v0), cmul(u[T2XM], v0xm)), -ry, csub(cmul(u[T2YP], v1), cmul(u[T2YM], v1ym)));
}
template <typename C, typename R>
__device__ __forceinline__ C u_row1(const C *u, C v1xp, C v1, C v0yp, C v0, R rx, R ry) {
    return sterm2(rx, csub(cmul(u[T2XP], v1xp), cmul(u[T2XM], v1)), -ry, csub(cmul(u[T2YP], v0yp), cmul(u[T2YM], v0)));
}
// v rows from their 8 couplings T[4 q + term] (q = v0, v1; term order +x, -x, +y, -y):
//   v0: u0(xp).-x  u0.+x  u1.-y  u1(ym).+y;   v1: u1.-x  u1(xm).+x  u0(yp).-y  u0.+y
template <typename C, typename R> __device__ __forceinline__ St2<C> v_rows(const C (&T)[8], R rx, R ry) {
    St2<C> s;
    s.s0 = sterm2(rx, csub(T[0], T[1]), ry, csub(T[2], T[3]));
    s.s1 = sterm2(rx, csub(T[4], T[5]), ry, csub(T[6], T[7]));
    return s;
}

template <typename D, typename RD, typename CS>
__device__ __forceinline__ St2<D> links_u(const CS *const f[4], const LinkPtrs &L, const Nb2 &n, RD rx, RD ry) {
    constexpr int NT = 4;
    D u[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) u[q] = LK(q / 4, q % 4, n.c);
    St2<D> s;
    s.s0 = u_row0(u, FV(2, n.c), FV(2, n.xm), FV(3, n.c), FV(3, n.ym), rx, ry);
    s.s1 = u_row1(u + 4, FV(3, n.xp), FV(3, n.c), FV(2, n.yp), FV(2, n.c), rx, ry);
    return s;
}
template <typename D, typename RD, typename CS>
__device__ __forceinline__ St2<D> links_v(const CS *const f[4], const LinkPtrs &L, const Nb2 &n, RD rx, RD ry) {
    constexpr int NT = 4;
    const D T[8] = {pr(LK(0, T2XM, n.xp), FV(0, n.xp)), pr(LK(0, T2XP, n.c), FV(0, n.c)),
                    pr(LK(1, T2YM, n.c), FV(1, n.c)), pr(LK(1, T2YP, n.ym), FV(1, n.ym)),
                    pr(LK(1, T2XM, n.c), FV(1, n.c)), pr(LK(1, T2XP, n.xm), FV(1, n.xm)),
                    pr(LK(0, T2YM, n.yp), FV(0, n.yp)), pr(LK(0, T2YP, n.c), FV(0, n.c))};
    return v_rows(T, rx, ry);
}

template <typename R, bool SITE, int WHICH>
__global__ __launch_bounds__(256) void k2_half_links(HalfArgs<R> a, LinkPtrs L) {
    using C = cx<R>;
    const int64_t ncell = (int64_t)a.nx * a.ny;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncell) return;
    const int i = (int)(t % a.nx), j = (int)(t / a.nx);
    const Nb2 n = nb2(i, j, a.nx, a.ny);
    C *f[4];
    const C *fc[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        f[p] = (C *)a.f[p];
        fc[p] = f[p];
    }
    // 2D tables: u class 0, v class 3 (one plane)
    if constexpr (WHICH == 0) {
        const St2<C> s = links_u<C, R, C>(fc, L, n, a.rx, a.ry);
        // old values and coefficients before the first store: a load issued after a
        // store would wait for it too
        const C o0 = f[0][n.c], o1 = f[1][n.c];
        const Coef<R> k0 = gcoef<R, SITE>(a, 0, 0, 0, n.c), k1 = gcoef<R, SITE>(a, 1, 0, 0, n.c);
        st_nt(&f[0][n.c], update(o0, s.s0, k0));
        st_nt(&f[1][n.c], update(o1, s.s1, k1));
    } else {
        const St2<C> s = links_v<C, R, C>(fc, L, n, a.rx, a.ry);
        // old values and coefficients before the first store: a load issued after a
        // store would wait for it too
        const C o2 = f[2][n.c], o3 = f[3][n.c];
        const Coef<R> k2 = gcoef<R, SITE>(a, 2, 3, 0, n.c), k3 = gcoef<R, SITE>(a, 3, 3, 0, n.c);
        st_nt(&f[2][n.c], update(o2, s.s0, k2));
        st_nt(&f[3][n.c], update(o3, s.s1, k3));
    }
}

// (2+1)D step with links in one launch: a workgroup owns an x strip of TW cells
// and marches a chunk of rows; at row p it updates u(p) on the strip and on a
// one-cell ring (left: u1, right: u0), then v(p-1) on the strip.  Each v
// coupling pr(U, new u) is formed by the thread that updated the u end: four
// serve the cell's own v rows (kept one row), u0's -y one the v1 row below
// (used at once), u1's +y one the v0 row above (kept two rows), and u0's -x and
// u1's +x ones the x neighbours (LDS).  Same helpers as the split kernels.
template <typename R, bool SITE, int TW>
__global__ __launch_bounds__(TW + 64) void k2_fused_links(FusedArgs<R> a, LinkPtrs L, const R *__restrict__ tab) {
    using C = cx<R>;
    constexpr int LW = TW + 2;
    __shared__ C sE[2][2][LW];     // slot p & 1: [0] u0's -x coupling, [1] u1's +x coupling
    const int tx = blockIdx.x % a.ntx, yc = blockIdx.x / a.ntx;
    const int x0 = tx * TW, w = min(TW, a.nx - x0);
    const int y0 = yc * a.zchunk, y1 = min(a.ny, y0 + a.zchunk);
    const int t = threadIdx.x;
    int x = 0;
    bool tile = false, n0 = false, n1 = false;
    if (t < TW) {
        x = t;
        tile = n0 = n1 = x < w;
    } else if (t == TW) {
        x = -1;
        n1 = true;                 // its u1 coupling reaches the strip's first v1
    } else if (t == TW + 1) {
        x = w;
        n0 = true;                 // its u0 coupling reaches the strip's last v0
    }
    const bool act = n0 || n1;
    const int gx = wrapn(x0 + x, a.nx);
    const int gxm = wrap_dec(gx, a.nx), gxp = wrap_inc(gx, a.nx);
    const int li = x + 1;
    const size_t nx = (size_t)a.nx;
    const C *in[4];
    C *out[4];
    const C *lk[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        in[q] = (const C *)a.in[q];
        out[q] = (C *)a.out[q];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) lk[q] = (const C *)L.u[q];
    const R rx = a.rx, ry = a.ry;
    const C zero = mk2((R)0, (R)0);
    // table entries (plane 0 of the u and v classes) read once, as scalar loads
    Coef<R> kt[4];
    if constexpr (!SITE) {
#pragma unroll
        for (int cls = 0; cls < 4; cls += 3) {
            const R *e = tab + (size_t)cls * a.nz * 4;
            kt[cls].c1 = mk2(e[0], e[1]);
            kt[cls].c2 = mk2(e[2], e[3]);
        }
    }
    auto coef = [&](int arr, int cls, size_t idx) -> Coef<R> {
        if constexpr (SITE) return coef_site_at<R>(a.th[arr], idx, (R)1);
        else return kt[cls];
    };
    // carried: old v0 of rows p and p-1, old v1 of row p-1; own couplings of u(p-1);
    // the u1 +y couplings of u(p-1) and u(p-2)
    C v0c = zero, v0m = zero, v1m = zero, Q[4] = {zero, zero, zero, zero}, up1 = zero, up2 = zero;
    if (act) {
        v0c = in[2][(size_t)wrapn(y0 - 1, a.ny) * nx + gx];
        v1m = in[3][(size_t)wrapn(y0 - 2, a.ny) * nx + gx];
    }
    for (int p = y0 - 1; p <= y1; ++p) {
        const size_t row = (size_t)wrapn(p, a.ny) * nx, rown = (size_t)wrapn(p + 1, a.ny) * nx;
        const size_t ci = row + gx;
        C v1c = zero, v0n = zero, Qn[4] = {zero, zero, zero, zero}, dn = zero, upn = zero, eL = zero, eR = zero;
        if (act) {
            v1c = in[3][ci];
            v0n = in[2][rown + gx];
            const bool store = tile && p >= y0 && p < y1;
            C u[4];
            if (n0) {
                const C v0xm = in[2][row + gxm];
#pragma unroll
                for (int q = 0; q < 4; ++q) u[q] = lk[q][ci];
                const C nu0 = update(in[0][ci], u_row0(u, v0c, v0xm, v1c, v1m, rx, ry), coef(0, 0, ci));
                if (store) st_nt(&out[0][ci], nu0);
                eL = pr(u[T2XM], nu0);
                Qn[0] = pr(u[T2XP], nu0);
                Qn[3] = pr(u[T2YP], nu0);
                dn = pr(u[T2YM], nu0);
            }
            if (n1) {
                const C v1xp = in[3][row + gxp];
#pragma unroll
                for (int q = 0; q < 4; ++q) u[q] = lk[4 + q][ci];
                const C nu1 = update(in[1][ci], u_row1(u, v1xp, v1c, v0n, v0c, rx, ry), coef(1, 0, ci));
                if (store) st_nt(&out[1][ci], nu1);
                eR = pr(u[T2XP], nu1);
                Qn[1] = pr(u[T2YM], nu1);
                Qn[2] = pr(u[T2XM], nu1);
                upn = pr(u[T2YP], nu1);
            }
            sE[p & 1][0][li] = eL;
            sE[p & 1][1][li] = eR;
        }
        if (tile && p - 1 >= y0 && p - 1 < y1) {
            const size_t cm = (size_t)wrapn(p - 1, a.ny) * nx + gx;
            const C(*e)[LW] = sE[(p - 1) & 1];
            const C T[8] = {e[0][li + 1], Q[0], Q[1], up2, Q[2], e[1][li - 1], dn, Q[3]};
            const St2<C> s = v_rows(T, rx, ry);
            const Coef<R> k2 = coef(2, 3, cm), k3 = coef(3, 3, cm);   // both loads before the stores
            st_nt(&out[2][cm], update(v0m, s.s0, k2));
            st_nt(&out[3][cm], update(v1m, s.s1, k3));
        }
        __syncthreads();
        v0m = v0c;
        v0c = v0n;
        v1m = v1c;
#pragma unroll
        for (int q = 0; q < 4; ++q) Q[q] = Qn[q];
        up2 = up1;
        up1 = upn;
    }
}

// (2+1)D: (E_r summed on the u sites, E_r summed on the v sites, plain norm);
// both equal the d_+ form of the functional.
template <typename R>
__global__ __launch_bounds__(kReduceThreads) void k2_norm_links(ReduceArgs<R> a, LinkPtrs L) {
    using C = cx<R>;
    __shared__ double lds[kNormVals * 16];
    const C *f[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) f[p] = (const C *)a.f[p];
    const int64_t ncell = (int64_t)a.nx * a.ny;
    const double rx = a.rx, ry = a.ry;
    double v[kNormVals] = {0.0, 0.0, 0.0};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ncell; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % a.nx), j = (int)(t / a.nx);
        const Nb2 n = nb2(i, j, a.nx, a.ny);
        const St2<double2> su = links_u<double2, double, C>(f, L, n, rx, ry);
        const St2<double2> sv = links_v<double2, double, C>(f, L, n, rx, ry);
        double p2 = 0.0;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const double2 x = dd(f[p][n.c]);
            p2 += x.x * x.x + x.y * x.y;
        }
        const double ev = re_cs(dd(f[2][n.c]), sv.s0) + re_cs(dd(f[3][n.c]), sv.s1);
        const double eu = re_cs(dd(f[0][n.c]), su.s0) + re_cs(dd(f[1][n.c]), su.s1);
        v[0] += p2 - eu;
        v[1] += p2 + ev;
        v[2] += p2;
    }
    block_sum<kNormVals>(v, lds);
    if (threadIdx.x == 0) {
        double *o = a.partial + (size_t)blockIdx.x * kNormVals;
        for (int p = 0; p < kNormVals; ++p) o[p] = v[p];
    }
}

}  // namespace

template <typename R>
hipError_t launch_half_links(const HalfArgs<R> &a, const LinkPtrs &L, int ndim, int which, bool site, hipStream_t s) {
    const int64_t ncell = (int64_t)a.nx * a.ny * (ndim == 3 ? a.nz : 1);
    const int64_t nb = (ncell + 255) / 256;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 g((unsigned)nb), b(256);
#define LH(K)                                                                                   \
    do {                                                                                        \
        if (which == 0) {                                                                       \
            if (site) hipLaunchKernelGGL((K<R, true, 0>), g, b, 0, s, a, L);                    \
            else hipLaunchKernelGGL((K<R, false, 0>), g, b, 0, s, a, L);                        \
        } else {                                                                                \
            if (site) hipLaunchKernelGGL((K<R, true, 1>), g, b, 0, s, a, L);                    \
            else hipLaunchKernelGGL((K<R, false, 1>), g, b, 0, s, a, L);                        \
        }                                                                                       \
    } while (0)
    if (ndim == 3) LH(k3_half_links);
    else LH(k2_half_links);
#undef LH
    return hipGetLastError();
}

// tiles across the patch one XCD runs at once (0: whole tile rows); measured at
// 512^3: complex64 fastest in whole rows (4 x 8 and 2 x 16 patches slower),
// complex128 in 4 x 8 patches (about 4% faster than whole rows; 2 x 16, 8 x 4, 16 x 2 between)
constexpr int kLinkPX32 = 0, kLinkPX64 = 4;

template <typename R>
hipError_t launch_fused_links(const FusedArgs<R> &a0, const LinkPtrs &L, bool site, hipStream_t s) {
    FusedArgs<R> a = a0;
    // tiles 64 x 8 (complex64, 704 threads) or 32 x 8 (complex128, 384 threads:
    // registers without spilling); measured best of 64x8, 32x16 (complex64) and
    // 64x4, 32x8 (complex128) at 512^3
    constexpr int TW = sizeof(R) == 4 ? 64 : 32, TY = 8;
    a.ntx = (a.nx + TW - 1) / TW;
    a.nty = (a.ny + TY - 1) / TY;
    const int64_t tiles = (int64_t)a.ntx * a.nty;
    if (a.zchunk <= 0) {
        int64_t nzc = (1024 + tiles - 1) / tiles;
        if (nzc < 1) nzc = 1;
        if (nzc > a.nz) nzc = a.nz;
        a.zchunk = (int)((a.nz + nzc - 1) / nzc);
    }
    a.nzc = (a.nz + a.zchunk - 1) / a.zchunk;
    a.px = sizeof(R) == 4 ? kLinkPX32 : kLinkPX64;
    const int64_t nblk = tiles * a.nzc;
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 g((unsigned)nblk), b(fl_threads<TW, TY>());
    constexpr int WPE = sizeof(R) == 4 ? 3 : 2;
    if (site) hipLaunchKernelGGL((k3_fused_links<R, true, TW, TY, WPE>), g, b, 0, s, a, L, a.tab);
    else hipLaunchKernelGGL((k3_fused_links<R, false, TW, TY, WPE>), g, b, 0, s, a, L, a.tab);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_fused2_links(const FusedArgs<R> &a0, const LinkPtrs &L, bool site, hipStream_t s) {
    FusedArgs<R> a = a0;
    constexpr int TW = 128;
    a.ntx = (a.nx + TW - 1) / TW;
    a.nty = 1;
    if (a.zchunk <= 0) {
        // about 2048 workgroups, chunks of at least 8 rows (each chunk recomputes
        // two); at 2048^2 complex64: 16-row chunks 132 us per step, 32-row 141-144
        int64_t nc = (2048 + a.ntx - 1) / a.ntx;
        if (nc > a.ny) nc = a.ny;
        a.zchunk = (int)((a.ny + nc - 1) / nc);
        if (a.zchunk < 8) a.zchunk = a.ny < 8 ? a.ny : 8;
    }
    a.nzc = (a.ny + a.zchunk - 1) / a.zchunk;
    const int64_t nblk = (int64_t)a.ntx * a.nzc;
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    if (site) hipLaunchKernelGGL((k2_fused_links<R, true, TW>), dim3((unsigned)nblk), dim3(TW + 64), 0, s, a, L, a.tab);
    else hipLaunchKernelGGL((k2_fused_links<R, false, TW>), dim3((unsigned)nblk), dim3(TW + 64), 0, s, a, L, a.tab);
    return hipGetLastError();
}

template <typename R> hipError_t launch_norm_links(const ReduceArgs<R> &a, const LinkPtrs &L, int ndim, hipStream_t s) {
    if (ndim == 3 && norm3_staged_supported(a.nx, sizeof(R) == 4)) return launch_norm3_links_staged<R>(a, L, s);
    if (ndim == 3) hipLaunchKernelGGL((k3_norm_links<R>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, a, L);
    else hipLaunchKernelGGL((k2_norm_links<R>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, a, L);
    return hipGetLastError();
}

template hipError_t launch_half_links<float>(const HalfArgs<float> &, const LinkPtrs &, int, int, bool, hipStream_t);
template hipError_t launch_half_links<double>(const HalfArgs<double> &, const LinkPtrs &, int, int, bool, hipStream_t);
template hipError_t launch_fused_links<float>(const FusedArgs<float> &, const LinkPtrs &, bool, hipStream_t);
template hipError_t launch_fused_links<double>(const FusedArgs<double> &, const LinkPtrs &, bool, hipStream_t);
template hipError_t launch_fused2_links<float>(const FusedArgs<float> &, const LinkPtrs &, bool, hipStream_t);
template hipError_t launch_fused2_links<double>(const FusedArgs<double> &, const LinkPtrs &, bool, hipStream_t);
template hipError_t launch_norm_links<float>(const ReduceArgs<float> &, const LinkPtrs &, int, hipStream_t);
template hipError_t launch_norm_links<double>(const ReduceArgs<double> &, const LinkPtrs &, int, hipStream_t);

}  // namespace dirac
