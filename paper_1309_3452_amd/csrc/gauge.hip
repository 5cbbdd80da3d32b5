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
// for a static potential.  These are cell-parallel kernels (split half-steps,
// in place, and the E_r reduction); the fused kernels carry no links.
#include "device.h"
#include "internal.h"
#include "stencil3.h"

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

// S_X with links at cell n.c for the A,B arrays (from C,D) or C,D arrays (from A,B).
template <typename D, typename RD, typename CS>
__device__ __forceinline__ St3<D> links_ab(const CS *const f[8], const LinkPtrs &L, const Nb3 &n, RD rx, RD ry, RD rz) {
    constexpr int NT = 6;
    St3<D> s;
    // A0: +z C0, -z C0[k-1], +x D0, -x D0[i-1], +y D1, -y D1[j-1]
    s.s0 = sterm3(rz, csub(cmul(LK(0, TZP, n.c), FV(4, n.c)), cmul(LK(0, TZM, n.c), FV(4, n.zm))),
                  rx, csub(cmul(LK(0, TXP, n.c), FV(6, n.c)), cmul(LK(0, TXM, n.c), FV(6, n.xm))),
                  -ry, csub(cmul(LK(0, TYP, n.c), FV(7, n.c)), cmul(LK(0, TYM, n.c), FV(7, n.ym))));
    // A1: +z C1, -z C1[k-1], +x D1[i+1], -x D1, +y D0[j+1], -y D0
    s.s1 = sterm3(rz, csub(cmul(LK(1, TZP, n.c), FV(5, n.c)), cmul(LK(1, TZM, n.c), FV(5, n.zm))),
                  rx, csub(cmul(LK(1, TXP, n.c), FV(7, n.xp)), cmul(LK(1, TXM, n.c), FV(7, n.c))),
                  -ry, csub(cmul(LK(1, TYP, n.c), FV(6, n.yp)), cmul(LK(1, TYM, n.c), FV(6, n.c))));
    // B0: +z D0[k+1], -z D0, +x C0[i+1], -x C0, +y C1, -y C1[j-1]
    s.s2 = sterm3(-rz, csub(cmul(LK(2, TZP, n.c), FV(6, n.zp)), cmul(LK(2, TZM, n.c), FV(6, n.c))),
                  rx, csub(cmul(LK(2, TXP, n.c), FV(4, n.xp)), cmul(LK(2, TXM, n.c), FV(4, n.c))),
                  ry, csub(cmul(LK(2, TYP, n.c), FV(5, n.c)), cmul(LK(2, TYM, n.c), FV(5, n.ym))));
    // B1: +z D1[k+1], -z D1, +x C1, -x C1[i-1], +y C0[j+1], -y C0
    s.s3 = sterm3(-rz, csub(cmul(LK(3, TZP, n.c), FV(7, n.zp)), cmul(LK(3, TZM, n.c), FV(7, n.c))),
                  rx, csub(cmul(LK(3, TXP, n.c), FV(5, n.c)), cmul(LK(3, TXM, n.c), FV(5, n.xm))),
                  ry, csub(cmul(LK(3, TYP, n.c), FV(4, n.yp)), cmul(LK(3, TYM, n.c), FV(4, n.c))));
    return s;
}

template <typename D, typename RD, typename CS>
__device__ __forceinline__ St3<D> links_cd(const CS *const f[8], const LinkPtrs &L, const Nb3 &n, RD rx, RD ry, RD rz) {
    constexpr int NT = 6;
    St3<D> s;
    // C0: +z A0[k+1], -z A0, +x B0, -x B0[i-1], +y B1, -y B1[j-1]
    s.s0 = sterm3(rz, csub(cmul(LKC(0, TZM, n.zp), FV(0, n.zp)), cmul(LKC(0, TZP, n.c), FV(0, n.c))),
                  rx, csub(cmul(LKC(2, TXM, n.c), FV(2, n.c)), cmul(LKC(2, TXP, n.xm), FV(2, n.xm))),
                  -ry, csub(cmul(LKC(3, TYM, n.c), FV(3, n.c)), cmul(LKC(3, TYP, n.ym), FV(3, n.ym))));
    // C1: +z A1[k+1], -z A1, +x B1[i+1], -x B1, +y B0[j+1], -y B0
    s.s1 = sterm3(rz, csub(cmul(LKC(1, TZM, n.zp), FV(1, n.zp)), cmul(LKC(1, TZP, n.c), FV(1, n.c))),
                  rx, csub(cmul(LKC(3, TXM, n.xp), FV(3, n.xp)), cmul(LKC(3, TXP, n.c), FV(3, n.c))),
                  -ry, csub(cmul(LKC(2, TYM, n.yp), FV(2, n.yp)), cmul(LKC(2, TYP, n.c), FV(2, n.c))));
    // D0: +z B0, -z B0[k-1], +x A0[i+1], -x A0, +y A1, -y A1[j-1]
    s.s2 = sterm3(-rz, csub(cmul(LKC(2, TZM, n.c), FV(2, n.c)), cmul(LKC(2, TZP, n.zm), FV(2, n.zm))),
                  rx, csub(cmul(LKC(0, TXM, n.xp), FV(0, n.xp)), cmul(LKC(0, TXP, n.c), FV(0, n.c))),
                  ry, csub(cmul(LKC(1, TYM, n.c), FV(1, n.c)), cmul(LKC(1, TYP, n.ym), FV(1, n.ym))));
    // D1: +z B1, -z B1[k-1], +x A1, -x A1[i-1], +y A0[j+1], -y A0
    s.s3 = sterm3(-rz, csub(cmul(LKC(3, TZM, n.c), FV(3, n.c)), cmul(LKC(3, TZP, n.zm), FV(3, n.zm))),
                  rx, csub(cmul(LKC(1, TXM, n.c), FV(1, n.c)), cmul(LKC(1, TXP, n.xm), FV(1, n.xm))),
                  ry, csub(cmul(LKC(0, TYM, n.yp), FV(0, n.yp)), cmul(LKC(0, TYP, n.c), FV(0, n.c))));
    return s;
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
        f[0][n.c] = update(f[0][n.c], s.s0, gcoef<R, SITE>(a, 0, 0, k, n.c));
        f[1][n.c] = update(f[1][n.c], s.s1, gcoef<R, SITE>(a, 1, 0, k, n.c));
        f[2][n.c] = update(f[2][n.c], s.s2, gcoef<R, SITE>(a, 2, 1, k, n.c));
        f[3][n.c] = update(f[3][n.c], s.s3, gcoef<R, SITE>(a, 3, 1, k, n.c));
    } else {
        const St3<C> s = links_cd<C, R, C>(fc, L, n, a.rx, a.ry, a.rz);
        f[4][n.c] = update(f[4][n.c], s.s0, gcoef<R, SITE>(a, 4, 2, k, n.c));
        f[5][n.c] = update(f[5][n.c], s.s1, gcoef<R, SITE>(a, 5, 2, k, n.c));
        f[6][n.c] = update(f[6][n.c], s.s2, gcoef<R, SITE>(a, 6, 3, k, n.c));
        f[7][n.c] = update(f[7][n.c], s.s3, gcoef<R, SITE>(a, 7, 3, k, n.c));
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

template <typename D, typename RD, typename CS>
__device__ __forceinline__ St2<D> links_u(const CS *const f[4], const LinkPtrs &L, const Nb2 &n, RD rx, RD ry) {
    constexpr int NT = 4;
    St2<D> s;
    // u0: +x v0, -x v0[i-1], +y v1, -y v1[j-1]
    s.s0 = sterm2(rx, csub(cmul(LK(0, T2XP, n.c), FV(2, n.c)), cmul(LK(0, T2XM, n.c), FV(2, n.xm))),
                  -ry, csub(cmul(LK(0, T2YP, n.c), FV(3, n.c)), cmul(LK(0, T2YM, n.c), FV(3, n.ym))));
    // u1: +x v1[i+1], -x v1, +y v0[j+1], -y v0
    s.s1 = sterm2(rx, csub(cmul(LK(1, T2XP, n.c), FV(3, n.xp)), cmul(LK(1, T2XM, n.c), FV(3, n.c))),
                  -ry, csub(cmul(LK(1, T2YP, n.c), FV(2, n.yp)), cmul(LK(1, T2YM, n.c), FV(2, n.c))));
    return s;
}
template <typename D, typename RD, typename CS>
__device__ __forceinline__ St2<D> links_v(const CS *const f[4], const LinkPtrs &L, const Nb2 &n, RD rx, RD ry) {
    constexpr int NT = 4;
    St2<D> s;
    // v0: +x u0[i+1] (its -x term), -x u0 (+x), +y u1 (-y), -y u1[j-1] (+y)
    s.s0 = sterm2(rx, csub(cmul(LKC(0, T2XM, n.xp), FV(0, n.xp)), cmul(LKC(0, T2XP, n.c), FV(0, n.c))),
                  ry, csub(cmul(LKC(1, T2YM, n.c), FV(1, n.c)), cmul(LKC(1, T2YP, n.ym), FV(1, n.ym))));
    // v1: +x u1 (-x), -x u1[i-1] (+x), +y u0[j+1] (-y), -y u0 (+y)
    s.s1 = sterm2(rx, csub(cmul(LKC(1, T2XM, n.c), FV(1, n.c)), cmul(LKC(1, T2XP, n.xm), FV(1, n.xm))),
                  ry, csub(cmul(LKC(0, T2YM, n.yp), FV(0, n.yp)), cmul(LKC(0, T2YP, n.c), FV(0, n.c))));
    return s;
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
        f[0][n.c] = update(f[0][n.c], s.s0, gcoef<R, SITE>(a, 0, 0, 0, n.c));
        f[1][n.c] = update(f[1][n.c], s.s1, gcoef<R, SITE>(a, 1, 0, 0, n.c));
    } else {
        const St2<C> s = links_v<C, R, C>(fc, L, n, a.rx, a.ry);
        f[2][n.c] = update(f[2][n.c], s.s0, gcoef<R, SITE>(a, 2, 3, 0, n.c));
        f[3][n.c] = update(f[3][n.c], s.s1, gcoef<R, SITE>(a, 3, 3, 0, n.c));
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

template <typename R> hipError_t launch_norm_links(const ReduceArgs<R> &a, const LinkPtrs &L, int ndim, hipStream_t s) {
    if (ndim == 3) hipLaunchKernelGGL((k3_norm_links<R>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, a, L);
    else hipLaunchKernelGGL((k2_norm_links<R>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, a, L);
    return hipGetLastError();
}

template hipError_t launch_half_links<float>(const HalfArgs<float> &, const LinkPtrs &, int, int, bool, hipStream_t);
template hipError_t launch_half_links<double>(const HalfArgs<double> &, const LinkPtrs &, int, int, bool, hipStream_t);
template hipError_t launch_norm_links<float>(const ReduceArgs<float> &, const LinkPtrs &, int, hipStream_t);
template hipError_t launch_norm_links<double>(const ReduceArgs<double> &, const LinkPtrs &, int, hipStream_t);

}  // namespace dirac
