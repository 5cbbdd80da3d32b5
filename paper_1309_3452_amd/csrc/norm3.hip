// Conserved functional of the (3+1)D scheme (Lemma of Sect. 2) as an
// LDS-staged z-march, without and with gauge links (Sect. 4; the second kernel
// below): per-workgroup partial sums of
//   E_r   = sum |X|^2 - Re sum_{A,B} conj(X) S_X(C,D)
//   E_r'  = sum |X|^2 + Re sum_{C,D} conj(Y) S_Y(A,B)   (the same functional summed on the C,D sites)
//   N     = sum |X|^2
// with S_X from Eqs. ss1-ss4, in FP64.
//
// A workgroup owns an x-y tile of TW x TY cells (one cell per thread) and a
// chunk [z0, z1) of planes.  Each plane of all eight arrays is copied
// global -> LDS asynchronously into one of two sets: plane p+1 lands in one
// set while plane p is read from the other, and each amplitude is fetched
// once per plane instead of once per neighbour read.  Every array is read at
// one x and one y neighbour only, always on the same side (S_X of Eqs.
// ss1-ss4), so its region is the tile plus one ring row and the ring columns
// on that side (two columns for complex64, so that every 16-byte unit is
// aligned).  A thread's own values of plane p-1 stay in registers.
//
// Of the eight difference terms, S_B0, S_B1 reach D at k+1 and S_C0, S_C1
// reach A at k+1.  Their x-y part is formed at plane k and kept in registers;
// the z difference is added at plane k+1, where the upper value is in LDS
// anyway.  Each S is evaluated with the same operations as in the other
// kernels (the z term is the outermost fused multiply-add), so every per-cell
// term has the same bits as there; only the order of the sum over cells
// differs.
#include <type_traits>

#include "device.h"
#include "internal.h"
#include "norm3.h"
#include "stencil3.h"

namespace dirac {

namespace {

// TW x TY tile, XL ring columns copied on one side of it.
template <typename R> struct NormTile;
template <> struct NormTile<float> {
    static constexpr int TW = 64, TY = 16, XL = 2;
};
template <> struct NormTile<double> {
    static constexpr int TW = 32, TY = 16, XL = 1;
};

struct NormMap {
    int ntx, nty, nzc, zchunk, items;
};

// the side of each array's x and y neighbour (arrays A0 A1 B0 B1 C0 C1 D0 D1):
// A1, B0, C1, D0 are read at i-1, the others at i+1; the odd ones at j-1, the
// even ones at j+1
__host__ __device__ constexpr bool x_minus(int q) { return q == 1 || q == 2 || q == 5 || q == 6; }
__host__ __device__ constexpr bool y_minus(int q) { return (q & 1) != 0; }

__device__ __forceinline__ int wrapm(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

__device__ __forceinline__ double2 dbl(double2 v) { return v; }
__device__ __forceinline__ double2 dbl(float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ __forceinline__ double re_cm(double2 x, double2 s) { return x.x * s.x + x.y * s.y; }
__device__ __forceinline__ double sq(double2 x) { return x.x * x.x + x.y * x.y; }

// The x-y part of a difference term b v + i c w (the inner two operations of
// sterm3), and the term completed with its z part a u.
__device__ __forceinline__ double2 xy_part(double b, double2 v, double c, double2 w) {
    return mk2(fmx(b, v.x, -(c * w.y)), fmx(b, v.y, c * w.x));
}
__device__ __forceinline__ double2 add_z(double a, double2 u, double2 g) { return mk2(fmx(a, u.x, g.x), fmx(a, u.y, g.y)); }

__device__ __forceinline__ void g2lds16(const void *gsrc, void *lds_wave_base) {
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)gsrc,
                                     (__attribute__((address_space(3))) void *)lds_wave_base, 16, 0, 0);
}

template <typename R, bool ZB>
__global__ __launch_bounds__(NormTile<R>::TW *NormTile<R>::TY) void k3_norm_lds(ReduceArgs<R> a, NormMap m) {
    using C = cx<R>;
    constexpr int TW = NormTile<R>::TW, TY = NormTile<R>::TY, XL = NormTile<R>::XL, NT = TW * TY;
    constexpr int CPL = 16 / (int)sizeof(C);          // cells per 16-byte copy unit
    constexpr int W = TW + XL, H = TY + 1, RN = W * H;
    constexpr int NW = NT / 64, WPA = NW / 8, NJ = (H + WPA - 1) / WPA;
    static_assert(NW % 8 == 0, "whole waves per array");
    static_assert(W / CPL <= 64, "one wave instruction per region row");
    static_assert((W * sizeof(C)) % 16 == 0 && (RN * sizeof(C)) % 16 == 0, "16-byte aligned LDS rows");
    // two sets of the eight arrays' regions (A0 A1 B0 B1 C0 C1 D0 D1), cell
    // (x, y) of the tile at (y + y_minus) W + x + XL x_minus; separate arrays,
    // so that the compiler sees that copies into one never alias reads of the
    // other
    __shared__ __align__(16) C sP[8 * RN];
    __shared__ __align__(16) C sQ[8 * RN];
    __shared__ double red[kNormVals * 16];

    const int t = threadIdx.x, lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int xr = t % TW, yr = t / TW;
    const int i = yr * W + xr;                         // plus the array's offset ofs(q)
    auto ofs = [](int q) { return (y_minus(q) ? W : 0) + (x_minus(q) ? XL : 0); };
    const int nx = a.nx, ny = a.ny, nz = a.nz, zh = a.zh;
    constexpr uint32_t CS = sizeof(C);
    const size_t rowbytes = (size_t)nx * CS, pbytes = rowbytes * ny;
    const double rx = a.rx, ry = a.ry, rz = a.rz;
    // stored plane of lattice plane pl: periodic wrap, or the interior of a z-slab
    auto zpl = [&](int pl) { return zh ? pl + zh : (pl < 0 ? pl + nz : pl >= nz ? pl - nz : pl); };
    // the wave's array and rows in the copies
    const int ck = wv / WPA, cy0 = wv % WPA;
    const char *csrc = (const char *)a.f[ck];

    const int blk = (gridDim.x & 7) == 0 ? (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3) : blockIdx.x;
    double v[kNormVals] = {0.0, 0.0, 0.0};
    for (int item = blk; item < m.items; item += gridDim.x) {
        int r = item;
        const int tx = r % m.ntx;
        r /= m.ntx;
        const int ty = r % m.nty;
        const int zc = r / m.nty;
        const int x0 = tx * TW, y0 = ty * TY;
        const int w = min(TW, nx - x0), h = min(TY, ny - y0);
        const int z0 = zc * m.zchunk, z1 = min(nz, z0 + m.zchunk);
        const bool act = xr < w && yr < h;
        const int gi = x0 + xr, gj = y0 + yr;
        // zero values outside the lattice (ZB): neighbours across a face read as zero
        const bool oxm = !ZB || gi > 0, oxp = !ZB || gi < nx - 1, oym = !ZB || gj > 0, oyp = !ZB || gj < ny - 1;

        // this wave's rows of one plane: row yy of the region is lattice row
        // y0 - ym + yy, lane l moves cells x0 - xm + CPL l ... (wrapped per
        // 16-byte unit; complex64 rows have an even length)
        const int ym = y_minus(ck) ? 1 : 0, xm = x_minus(ck) ? XL : 0;
        const int rl = (w + XL) / CPL;
        const uint32_t lxo = (uint32_t)wrapm(x0 - xm + lane * CPL, nx) * CS;
        auto copy_plane = [&](int pl, C *set) __attribute__((always_inline)) {
            const char *base = csrc + (size_t)zpl(pl) * pbytes;
            C *dst = set + ck * RN;
#pragma unroll 1
            for (int j = 0; j < NJ; ++j) {
                const int yy = cy0 + WPA * j;
                // rows copied lie in [y0 - 1, y0 + h] and h <= ny: one wrap at most
                int y = y0 - ym + yy;
                y = y < 0 ? y + ny : y >= ny ? y - ny : y;
                if (yy < h + 1 && lane < rl) g2lds16(base + (size_t)y * rowbytes + lxo, dst + yy * W);
            }
        };

        // own values of plane p-1 (A0 A1 B0 B1 C0 C1 D0 D1) and the x-y parts
        // of S_B0, S_B1 (E_r) and S_C0, S_C1 (E_r') at plane p-1
        C pv[8];
        double2 g[4];
#pragma unroll
        for (int q = 0; q < 8; ++q) pv[q] = mk2((R)0, (R)0);
#pragma unroll
        for (int q = 0; q < 4; ++q) g[q] = make_double2(0.0, 0.0);
        if (act && (!ZB || z0 > 0)) {
            const size_t o = (size_t)zpl(z0 - 1) * nx * ny + (size_t)gj * nx + gi;
#pragma unroll
            for (int q = 2; q < 6; ++q) pv[q] = ((const C *)a.f[q])[o];   // B, C of plane z0-1
        }

        // the set of the previous item may still be read: wait for every wave
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        copy_plane(z0, sP);
        auto plane = [&](const C *S, C *Snext, int p) __attribute__((always_inline)) {
            __builtin_amdgcn_s_waitcnt(0);   // this wave's copies of plane p and its reads of plane p-1
            __syncthreads();                 // everyone's: S complete, Snext free
            const bool up = p < z1 && (!ZB || p + 1 < nz);
            if (up) copy_plane(p + 1, Snext);
            if (!act) return;
            // plane p's own values (zero beyond the last plane with ZB)
            C cur[8];
            const bool here = !ZB || p < nz;
#pragma unroll
            for (int q = 0; q < 8; ++q) cur[q] = here ? S[q * RN + ofs(q) + i] : mk2((R)0, (R)0);
            if (p > z0) {
                // finish plane p-1: z differences up to plane p
                const double2 s2 = add_z(-rz, csub(dbl(cur[6]), dbl(pv[6])), g[0]);
                const double2 s3 = add_z(-rz, csub(dbl(cur[7]), dbl(pv[7])), g[1]);
                const double2 t0 = add_z(rz, csub(dbl(cur[0]), dbl(pv[0])), g[2]);
                const double2 t1 = add_z(rz, csub(dbl(cur[1]), dbl(pv[1])), g[3]);
                v[0] -= re_cm(dbl(pv[2]), s2) + re_cm(dbl(pv[3]), s3);
                v[1] += re_cm(dbl(pv[4]), t0) + re_cm(dbl(pv[5]), t1);
            }
            if (p < z1) {
                const double2 a0 = dbl(cur[0]), a1 = dbl(cur[1]), b0 = dbl(cur[2]), b1 = dbl(cur[3]);
                const double2 c0 = dbl(cur[4]), c1 = dbl(cur[5]), d0 = dbl(cur[6]), d1 = dbl(cur[7]);
                auto nb = [&](int q, int off, bool ok) {
                    const C x = S[q * RN + ofs(q) + i + off];
                    return dbl(ok ? x : mk2((R)0, (R)0));
                };
                // E_r: S_A0, S_A1 whole, x-y parts of S_B0, S_B1
                const double2 sa0 = sterm3(rz, csub(c0, dbl(pv[4])), rx, csub(d0, nb(6, -1, oxm)), -ry,
                                           csub(d1, nb(7, -W, oym)));
                const double2 sa1 = sterm3(rz, csub(c1, dbl(pv[5])), rx, csub(nb(7, 1, oxp), d1), -ry,
                                           csub(nb(6, W, oyp), d0));
                g[0] = xy_part(rx, csub(nb(4, 1, oxp), c0), ry, csub(c1, nb(5, -W, oym)));
                g[1] = xy_part(rx, csub(c1, nb(5, -1, oxm)), ry, csub(nb(4, W, oyp), c0));
                // E_r': S_D0, S_D1 whole, x-y parts of S_C0, S_C1
                const double2 sd0 = sterm3(-rz, csub(b0, dbl(pv[2])), rx, csub(nb(0, 1, oxp), a0), ry,
                                           csub(a1, nb(1, -W, oym)));
                const double2 sd1 = sterm3(-rz, csub(b1, dbl(pv[3])), rx, csub(a1, nb(1, -1, oxm)), ry,
                                           csub(nb(0, W, oyp), a0));
                g[2] = xy_part(rx, csub(b0, nb(2, -1, oxm)), -ry, csub(b1, nb(3, -W, oym)));
                g[3] = xy_part(rx, csub(nb(3, 1, oxp), b1), -ry, csub(nb(2, W, oyp), b0));
                const double pp = sq(a0) + sq(a1) + sq(b0) + sq(b1) + sq(c0) + sq(c1) + sq(d0) + sq(d1);
                v[0] += pp - (re_cm(a0, sa0) + re_cm(a1, sa1));
                v[1] += pp + (re_cm(d0, sd0) + re_cm(d1, sd1));
                v[2] += pp;
#pragma unroll
                for (int q = 0; q < 8; ++q) pv[q] = cur[q];
            }
        };
        // planes z0 .. z1: the last one only finishes plane z1 - 1
        for (int p = z0;;) {
            plane(sP, sQ, p);
            if (++p > z1) break;
            plane(sQ, sP, p);
            if (++p > z1) break;
        }
    }

#pragma unroll
    for (int q = 0; q < kNormVals; ++q) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
    }
    __syncthreads();
    if (lane == 0)
        for (int q = 0; q < kNormVals; ++q) red[q * 16 + wv] = v[q];
    __syncthreads();
    if (t == 0) {
        double *o = a.partial + (size_t)blockIdx.x * kNormVals;
        for (int q = 0; q < kNormVals; ++q) {
            double s = 0.0;
            for (int u = 0; u < NW; ++u) s += red[q * 16 + u];
            o[q] = s;
        }
    }
}

// ---- with gauge links (Sect. 4) ----
// The same three sums with every neighbour value in S_X multiplied by its link
// factor: an A,B row by the factor stored with its own array at the cell, a C,D
// row by the conjugate of the factor stored at the A,B end of the half-link.
// The amplitudes are staged as above (the link rows read the same neighbours on
// the same sides).  Each cell loads its own 24 factors, and the 8 factors of
// its x and y neighbours that its C,D rows need, straight from global memory:
// a factor is read by at most two cells, its own and one x or y neighbour,
// mostly in the same workgroup and plane, so the second read finds it in the
// caches and staging would save little.
// Across the plane boundary: S_B0 and S_B1 keep their x-y part, their +z factor
// and their -z coupling, and take D at k+1 at the next plane; S_C0 and S_C1
// keep their x-y part and their -z coupling and take the next plane's A times
// that cell's own -z factor; the -z couplings of S_D0 and S_D1 (B at k-1 times
// its +z factor) come up from the plane below.  Each per-cell term takes the
// operations of the unstaged link reduction in the same order.
template <typename R> struct LinkNormTile;
template <> struct LinkNormTile<float> {
    static constexpr int TW = 64, TY = 8, XL = 2;
};
template <> struct LinkNormTile<double> {
    static constexpr int TW = 32, TY = 16, XL = 1;
};

// link factor index 6 a + t for A,B array a and neighbour term t
enum { LZP = 0, LZM = 1, LXP = 2, LXM = 3, LYP = 4, LYM = 5 };

// Two waves per SIMD is the occupancy the registers allow anyway; told so, the
// compiler issues a plane's link loads together instead of moving each next to
// its use (and waiting for it there) to save registers for an occupancy it
// cannot reach: complex64 at 512^3 7.0 against 8.7 ms; the complex128 code is
// the same either way.

template <typename R>
__global__ __launch_bounds__(LinkNormTile<R>::TW *LinkNormTile<R>::TY) __attribute__((amdgpu_waves_per_eu(2, 2))) void k3_norm_links_lds(ReduceArgs<R> a,
                                                                                              LinkPtrs L, NormMap m) {
    using C = cx<R>;
    constexpr int TW = LinkNormTile<R>::TW, TY = LinkNormTile<R>::TY, XL = LinkNormTile<R>::XL, NT = TW * TY;
    constexpr int CPL = 16 / (int)sizeof(C);
    constexpr int W = TW + XL, H = TY + 1, RN = W * H;
    constexpr int NW = NT / 64, WPA = NW / 8, NJ = (H + WPA - 1) / WPA;
    static_assert(NW % 8 == 0, "whole waves per array");
    static_assert(W / CPL <= 64, "one wave instruction per region row");
    static_assert((W * sizeof(C)) % 16 == 0 && (RN * sizeof(C)) % 16 == 0, "16-byte aligned LDS rows");
    __shared__ __align__(16) C sP[8 * RN];
    __shared__ __align__(16) C sQ[8 * RN];
    __shared__ double red[kNormVals * 16];

    const int t = threadIdx.x, lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int xr = t % TW, yr = t / TW;
    const int i = yr * W + xr;
    auto ofs = [](int q) { return (y_minus(q) ? W : 0) + (x_minus(q) ? XL : 0); };
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    constexpr uint32_t CS = sizeof(C);
    const size_t rowbytes = (size_t)nx * CS, pbytes = rowbytes * ny, plane = (size_t)nx * ny;
    const double rx = a.rx, ry = a.ry, rz = a.rz;
    auto zpl = [&](int pl) { return pl < 0 ? pl + nz : pl >= nz ? pl - nz : pl; };
    const int ck = wv / WPA, cy0 = wv % WPA;
    const char *csrc = (const char *)a.f[ck];
    const C *lk[24];
#pragma unroll
    for (int q = 0; q < 24; ++q) lk[q] = (const C *)L.u[q];
    // link times value, and conjugate link times value, in FP64
    auto lm = [](C u, double2 x) { return cmul(dbl(u), x); };
    auto lc = [](C u, double2 x) { return cmul(cconj(dbl(u)), x); };

    const int blk = (gridDim.x & 7) == 0 ? (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3) : blockIdx.x;
    double v[kNormVals] = {0.0, 0.0, 0.0};
    for (int item = blk; item < m.items; item += gridDim.x) {
        int r = item;
        const int tx = r % m.ntx;
        r /= m.ntx;
        const int ty = r % m.nty;
        const int zc = r / m.nty;
        const int x0 = tx * TW, y0 = ty * TY;
        const int w = min(TW, nx - x0), h = min(TY, ny - y0);
        const int z0 = zc * m.zchunk, z1 = min(nz, z0 + m.zchunk);
        const bool act = xr < w && yr < h;
        const int gi = x0 + xr, gj = y0 + yr;
        const size_t oc = (size_t)gj * nx + gi;
        const size_t oxm = (size_t)gj * nx + (gi == 0 ? nx - 1 : gi - 1);
        const size_t oxp = (size_t)gj * nx + (gi == nx - 1 ? 0 : gi + 1);
        const size_t oym = (size_t)(gj == 0 ? ny - 1 : gj - 1) * nx + gi;
        const size_t oyp = (size_t)(gj == ny - 1 ? 0 : gj + 1) * nx + gi;

        const int ym = y_minus(ck) ? 1 : 0, xm = x_minus(ck) ? XL : 0;
        const int rl = (w + XL) / CPL;
        const uint32_t lxo = (uint32_t)wrapm(x0 - xm + lane * CPL, nx) * CS;
        auto copy_plane = [&](int pl, C *set) __attribute__((always_inline)) {
            const char *base = csrc + (size_t)zpl(pl) * pbytes;
            C *dst = set + ck * RN;
#pragma unroll 1
            for (int j = 0; j < NJ; ++j) {
                const int yy = cy0 + WPA * j;
                int y = y0 - ym + yy;
                y = y < 0 ? y + ny : y >= ny ? y - ny : y;
                if (yy < h + 1 && lane < rl) g2lds16(base + (size_t)y * rowbytes + lxo, dst + yy * W);
            }
        };

        // own values of plane p-1; the x-y parts of S_B0, S_B1, S_C0, S_C1 at
        // plane p-1 (g), the +z factors of B0, B1 (zl) and the -z couplings of
        // S_B0, S_B1 (zr) and of S_C0, S_C1 (tz) there; the -z couplings of
        // S_D0, S_D1 at plane p (zd)
        C pv[8], zl[2];
        double2 g[4], zr[2], tz[2], zd[2];
#pragma unroll
        for (int q = 0; q < 8; ++q) pv[q] = mk2((R)0, (R)0);
        zl[0] = zl[1] = mk2((R)0, (R)0);
#pragma unroll
        for (int q = 0; q < 2; ++q) zr[q] = tz[q] = zd[q] = make_double2(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < 4; ++q) g[q] = make_double2(0.0, 0.0);
        if (act) {
            const size_t o = (size_t)zpl(z0 - 1) * plane + oc;
#pragma unroll
            for (int q = 2; q < 6; ++q) pv[q] = ((const C *)a.f[q])[o];   // B, C of plane z0-1
            zd[0] = lc(lk[12 + LZP][o], dbl(pv[2]));
            zd[1] = lc(lk[18 + LZP][o], dbl(pv[3]));
        }

        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        copy_plane(z0, sP);
        auto plane_step = [&](const C *S, C *Snext, int p) __attribute__((always_inline)) {
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (p < z1) copy_plane(p + 1, Snext);
            if (!act) return;
            const size_t P = (size_t)zpl(p) * plane, c = P + oc;
            C cur[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) cur[q] = S[q * RN + ofs(q) + i];
            if (p > z0) {
                // finish plane p-1: its +z neighbours are this plane's D (S_B) and
                // this plane's A times its own -z factors (S_C)
                const double2 s2 = add_z(-rz, csub(lm(zl[0], dbl(cur[6])), zr[0]), g[0]);
                const double2 s3 = add_z(-rz, csub(lm(zl[1], dbl(cur[7])), zr[1]), g[1]);
                const double2 t0 = add_z(rz, csub(lc(lk[0 + LZM][c], dbl(cur[0])), tz[0]), g[2]);
                const double2 t1 = add_z(rz, csub(lc(lk[6 + LZM][c], dbl(cur[1])), tz[1]), g[3]);
                v[0] -= re_cm(dbl(pv[2]), s2) + re_cm(dbl(pv[3]), s3);
                v[1] += re_cm(dbl(pv[4]), t0) + re_cm(dbl(pv[5]), t1);
            }
            if (p < z1) {
                C u[24];
#pragma unroll
                for (int q = 0; q < 24; ++q) u[q] = lk[q][c];
                // factors of the x and y neighbours that the C,D couplings use
                const C nB0xm = lk[12 + LXP][P + oxm], nB1ym = lk[18 + LYP][P + oym];
                const C nB1xp = lk[18 + LXM][P + oxp], nB0yp = lk[12 + LYM][P + oyp];
                const C nA0xp = lk[0 + LXM][P + oxp], nA1ym = lk[6 + LYP][P + oym];
                const C nA1xm = lk[6 + LXP][P + oxm], nA0yp = lk[0 + LYM][P + oyp];
                const double2 a0 = dbl(cur[0]), a1 = dbl(cur[1]), b0 = dbl(cur[2]), b1 = dbl(cur[3]);
                const double2 c0 = dbl(cur[4]), c1 = dbl(cur[5]), d0 = dbl(cur[6]), d1 = dbl(cur[7]);
                auto nb = [&](int q, int off) { return dbl(S[q * RN + ofs(q) + i + off]); };
                // E_r: S_A0, S_A1 whole
                const double2 sa0 = sterm3(rz, csub(lm(u[LZP], c0), lm(u[LZM], dbl(pv[4]))), rx,
                                           csub(lm(u[LXP], d0), lm(u[LXM], nb(6, -1))), -ry,
                                           csub(lm(u[LYP], d1), lm(u[LYM], nb(7, -W))));
                const double2 sa1 = sterm3(rz, csub(lm(u[6 + LZP], c1), lm(u[6 + LZM], dbl(pv[5]))), rx,
                                           csub(lm(u[6 + LXP], nb(7, 1)), lm(u[6 + LXM], d1)), -ry,
                                           csub(lm(u[6 + LYP], nb(6, W)), lm(u[6 + LYM], d0)));
                // S_B0, S_B1: x-y parts, the z part at the next plane
                g[0] = xy_part(rx, csub(lm(u[12 + LXP], nb(4, 1)), lm(u[12 + LXM], c0)), ry,
                               csub(lm(u[12 + LYP], c1), lm(u[12 + LYM], nb(5, -W))));
                g[1] = xy_part(rx, csub(lm(u[18 + LXP], c1), lm(u[18 + LXM], nb(5, -1))), ry,
                               csub(lm(u[18 + LYP], nb(4, W)), lm(u[18 + LYM], c0)));
                zl[0] = u[12 + LZP];
                zl[1] = u[18 + LZP];
                zr[0] = lm(u[12 + LZM], d0);
                zr[1] = lm(u[18 + LZM], d1);
                // E_r': S_C0, S_C1 x-y parts and -z couplings
                g[2] = xy_part(rx, csub(lc(u[12 + LXM], b0), lc(nB0xm, nb(2, -1))), -ry,
                               csub(lc(u[18 + LYM], b1), lc(nB1ym, nb(3, -W))));
                g[3] = xy_part(rx, csub(lc(nB1xp, nb(3, 1)), lc(u[18 + LXP], b1)), -ry,
                               csub(lc(nB0yp, nb(2, W)), lc(u[12 + LYP], b0)));
                tz[0] = lc(u[LZP], a0);
                tz[1] = lc(u[6 + LZP], a1);
                // S_D0, S_D1 whole (their -z couplings from the plane below)
                const double2 sd0 = sterm3(-rz, csub(lc(u[12 + LZM], b0), zd[0]), rx,
                                           csub(lc(nA0xp, nb(0, 1)), lc(u[LXP], a0)), ry,
                                           csub(lc(u[6 + LYM], a1), lc(nA1ym, nb(1, -W))));
                const double2 sd1 = sterm3(-rz, csub(lc(u[18 + LZM], b1), zd[1]), rx,
                                           csub(lc(u[6 + LXM], a1), lc(nA1xm, nb(1, -1))), ry,
                                           csub(lc(nA0yp, nb(0, W)), lc(u[LYP], a0)));
                zd[0] = lc(u[12 + LZP], b0);
                zd[1] = lc(u[18 + LZP], b1);
                const double pp = sq(a0) + sq(a1) + sq(b0) + sq(b1) + sq(c0) + sq(c1) + sq(d0) + sq(d1);
                v[0] += pp - (re_cm(a0, sa0) + re_cm(a1, sa1));
                v[1] += pp + (re_cm(d0, sd0) + re_cm(d1, sd1));
                v[2] += pp;
#pragma unroll
                for (int q = 0; q < 8; ++q) pv[q] = cur[q];
            }
        };
        for (int p = z0;;) {
            plane_step(sP, sQ, p);
            if (++p > z1) break;
            plane_step(sQ, sP, p);
            if (++p > z1) break;
        }
    }

#pragma unroll
    for (int q = 0; q < kNormVals; ++q) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
    }
    __syncthreads();
    if (lane == 0)
        for (int q = 0; q < kNormVals; ++q) red[q * 16 + wv] = v[q];
    __syncthreads();
    if (t == 0) {
        double *o = a.partial + (size_t)blockIdx.x * kNormVals;
        for (int q = 0; q < kNormVals; ++q) {
            double s = 0.0;
            for (int u = 0; u < NW; ++u) s += red[q * 16 + u];
            o[q] = s;
        }
    }
}

template <int TW, int TY> NormMap tile_map(int nx, int ny, int nz) {
    NormMap m;
    m.ntx = (nx + TW - 1) / TW;
    m.nty = (ny + TY - 1) / TY;
    const int64_t tiles = (int64_t)m.ntx * m.nty;
    int64_t nzc = (kReduceBlocks + tiles - 1) / tiles;
    if (nzc > nz) nzc = nz;
    if (nzc < 1) nzc = 1;
    m.zchunk = (int)((nz + nzc - 1) / nzc);
    m.nzc = (nz + m.zchunk - 1) / m.zchunk;
    m.items = (int)(tiles * m.nzc);
    return m;
}

template <typename R> NormMap norm_map(int nx, int ny, int nz) {
    return tile_map<NormTile<R>::TW, NormTile<R>::TY>(nx, ny, nz);
}

}  // namespace

bool norm3_staged_supported(int nx, bool fp32) { return !fp32 || nx % 2 == 0; }

template <typename R> hipError_t launch_norm3_staged(const ReduceArgs<R> &a, hipStream_t s) {
    if (!norm3_staged_supported(a.nx, sizeof(R) == 4)) return hipErrorInvalidValue;
    if ((int64_t)((a.nx + NormTile<R>::TW - 1) / NormTile<R>::TW) * ((a.ny + NormTile<R>::TY - 1) / NormTile<R>::TY) *
            a.nz > 0x7fffffff)
        return hipErrorInvalidValue;
    const NormMap m = norm_map<R>(a.nx, a.ny, a.nz);
    constexpr int NT = NormTile<R>::TW * NormTile<R>::TY;
    if (a.zbc) hipLaunchKernelGGL((k3_norm_lds<R, true>), dim3(kReduceBlocks), dim3(NT), 0, s, a, m);
    else hipLaunchKernelGGL((k3_norm_lds<R, false>), dim3(kReduceBlocks), dim3(NT), 0, s, a, m);
    return hipGetLastError();
}

template hipError_t launch_norm3_staged<float>(const ReduceArgs<float> &, hipStream_t);
template hipError_t launch_norm3_staged<double>(const ReduceArgs<double> &, hipStream_t);

template <typename R> hipError_t launch_norm3_links_staged(const ReduceArgs<R> &a, const LinkPtrs &L, hipStream_t s) {
    constexpr int TW = LinkNormTile<R>::TW, TY = LinkNormTile<R>::TY;
    if (!norm3_staged_supported(a.nx, sizeof(R) == 4) || a.zh || a.zbc) return hipErrorInvalidValue;
    if ((int64_t)((a.nx + TW - 1) / TW) * ((a.ny + TY - 1) / TY) * a.nz > 0x7fffffff) return hipErrorInvalidValue;
    const NormMap m = tile_map<TW, TY>(a.nx, a.ny, a.nz);
    hipLaunchKernelGGL((k3_norm_links_lds<R>), dim3(kReduceBlocks), dim3(TW * TY), 0, s, a, L, m);
    return hipGetLastError();
}

template hipError_t launch_norm3_links_staged<float>(const ReduceArgs<float> &, const LinkPtrs &, hipStream_t);
template hipError_t launch_norm3_links_staged<double>(const ReduceArgs<double> &, const LinkPtrs &, hipStream_t);

}  // namespace dirac
