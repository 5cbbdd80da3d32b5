// (3+1)D kernels: split half-steps (in place), conserved-functional and
// observable reductions, adjoint seed and per-site theta fields.
//
// Stencils (cell (i,j,k), periodic; the position of each array's amplitude is
// A0 (i,j,k), A1 (i+1/2,j+1/2,k), B0 (i+1/2,j,k+1/2), B1 (i,j+1/2,k+1/2),
// C0 (i,j,k+1/2), C1 (i+1/2,j+1/2,k+1/2), D0 (i+1/2,j,k), D1 (i,j+1/2,k)).
// Written out from Eqs. ss1-ss4 (centred differences over one cell):
//   S_A0 =  rz(C0 - C0[k-1]) + rx(D0 - D0[i-1]) - i ry(D1 - D1[j-1])
//   S_A1 =  rz(C1 - C1[k-1]) + rx(D1[i+1] - D1) - i ry(D0[j+1] - D0)
//   S_B0 = -rz(D0[k+1] - D0) + rx(C0[i+1] - C0) + i ry(C1 - C1[j-1])
//   S_B1 = -rz(D1[k+1] - D1) + rx(C1 - C1[i-1]) + i ry(C0[j+1] - C0)
//   S_C0 =  rz(A0[k+1] - A0) + rx(B0 - B0[i-1]) - i ry(B1 - B1[j-1])
//   S_C1 =  rz(A1[k+1] - A1) + rx(B1[i+1] - B1) - i ry(B0[j+1] - B0)
//   S_D0 = -rz(B0 - B0[k-1]) + rx(A0[i+1] - A0) + i ry(A1 - A1[j-1])
//   S_D1 = -rz(B1 - B1[k-1]) + rx(A1 - A1[i-1]) + i ry(A0[j+1] - A0)
#include "device.h"
#include "internal.h"
#include "norm3.h"
#include "stencil3.h"
#include "ntstore.h"

namespace dirac {

namespace {

constexpr int kTX = 64, kTY = 4;

template <typename R> __device__ __forceinline__ Coef<R> tab_coef(const R *tab, int q, int nz, int k) {
    const R *e = tab + ((size_t)q * nz + k) * 4;
    Coef<R> c;
    c.c1 = mk2(e[0], e[1]);
    c.c2 = mk2(e[2], e[3]);
    return c;
}

template <typename R, bool SITE>
__device__ __forceinline__ Coef<R> coef_at(const HalfArgs<R> &a, int arr, int q, int k, size_t c) {
    if constexpr (SITE) {
        return coef_site_at<R>(a.th[arr], c, a.tsgn);
    } else {
        return tab_coef(a.tab, q, a.nz, k);
    }
}

// which == 0: A,B from C,D (Eqs. ss1, ss2); which == 1: C,D from A,B (ss3, ss4).
// ZB: zero values outside the lattice (a compile-time choice, so the periodic
// instantiation keeps plain loads).
template <typename R, bool SITE, int WHICH, bool ZB>
__global__ __launch_bounds__(256) void k3_half(HalfArgs<R> a) {
    using C = cx<R>;
    const int nbx = (a.nx + kTX - 1) / kTX, nby = (a.ny + kTY - 1) / kTY;
    int b = blockIdx.x;
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nby;
    const int k = b / nby;
    const int i = bx * kTX + (threadIdx.x & (kTX - 1));
    const int j = by * kTY + (threadIdx.x / kTX);
    if (i >= a.nx || j >= a.ny) return;
    const size_t plane = (size_t)a.nx * a.ny;
    const size_t row = (size_t)j * a.nx;
    const size_t kk = (size_t)k * plane;
    const int im = wrap_dec(i, a.nx), ip = wrap_inc(i, a.nx);
    const int jm = wrap_dec(j, a.ny), jp = wrap_inc(j, a.ny);
    const int km = wrap_dec(k, a.nz), kp = wrap_inc(k, a.nz);
    const size_t c = kk + row + i;
    const size_t xm = kk + row + im, xp = kk + row + ip;
    const size_t ym = kk + (size_t)jm * a.nx + i, yp = kk + (size_t)jp * a.nx + i;
    const size_t zm = (size_t)km * plane + row + i, zp = (size_t)kp * plane + row + i;
    C *f[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) f[q] = (C *)a.f[q];
    // zero values outside the lattice: a neighbour across a face reads as zero
    const bool oxm = !ZB || i > 0, oxp = !ZB || i < a.nx - 1, oym = !ZB || j > 0, oyp = !ZB || j < a.ny - 1;
    const bool ozm = !ZB || k > 0, ozp = !ZB || k < a.nz - 1;
    if constexpr (WHICH == 0) {
        St3<C> s = stencil_ab<C, R>(a.rx, a.ry, a.rz,
                                     f[4][c], ld_or0(f[4], zm, ozm), ld_or0(f[4], xp, oxp), ld_or0(f[4], yp, oyp),
                                     f[5][c], ld_or0(f[5], zm, ozm), ld_or0(f[5], ym, oym), ld_or0(f[5], xm, oxm),
                                     f[6][c], ld_or0(f[6], xm, oxm), ld_or0(f[6], yp, oyp), ld_or0(f[6], zp, ozp),
                                     f[7][c], ld_or0(f[7], ym, oym), ld_or0(f[7], xp, oxp), ld_or0(f[7], zp, ozp));
        // old values and coefficients before the first store: a load issued after a
        // store would wait for it too
        const C o0 = f[0][c], o1 = f[1][c], o2 = f[2][c], o3 = f[3][c];
        const Coef<R> k0 = coef_at<R, SITE>(a, 0, 0, k, c), k1 = coef_at<R, SITE>(a, 1, 0, k, c), k2 = coef_at<R, SITE>(a, 2, 1, k, c), k3 = coef_at<R, SITE>(a, 3, 1, k, c);
        st_nt(&f[0][c], update(o0, s.s0, k0));
        st_nt(&f[1][c], update(o1, s.s1, k1));
        st_nt(&f[2][c], update(o2, s.s2, k2));
        st_nt(&f[3][c], update(o3, s.s3, k3));
    } else {
        St3<C> s = stencil_cd<C, R>(a.rx, a.ry, a.rz,
                                     f[0][c], ld_or0(f[0], zp, ozp), ld_or0(f[0], xp, oxp), ld_or0(f[0], yp, oyp),
                                     f[1][c], ld_or0(f[1], zp, ozp), ld_or0(f[1], xm, oxm), ld_or0(f[1], ym, oym),
                                     f[2][c], ld_or0(f[2], zm, ozm), ld_or0(f[2], xm, oxm), ld_or0(f[2], yp, oyp),
                                     f[3][c], ld_or0(f[3], zm, ozm), ld_or0(f[3], xp, oxp), ld_or0(f[3], ym, oym));
        // old values and coefficients before the first store: a load issued after a
        // store would wait for it too
        const C o4 = f[4][c], o5 = f[5][c], o6 = f[6][c], o7 = f[7][c];
        const Coef<R> k4 = coef_at<R, SITE>(a, 4, 2, k, c), k5 = coef_at<R, SITE>(a, 5, 2, k, c), k6 = coef_at<R, SITE>(a, 6, 3, k, c), k7 = coef_at<R, SITE>(a, 7, 3, k, c);
        st_nt(&f[4][c], update(o4, s.s0, k4));
        st_nt(&f[5][c], update(o5, s.s1, k5));
        st_nt(&f[6][c], update(o6, s.s2, k6));
        st_nt(&f[7][c], update(o7, s.s3, k7));
    }
}

__device__ __forceinline__ double2 to_d(double2 v) { return v; }
__device__ __forceinline__ double2 to_d(float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ __forceinline__ double re_conj_mul(double2 x, double2 s) { return x.x * s.x + x.y * s.y; }
__device__ __forceinline__ double abs2(double2 x) { return x.x * x.x + x.y * x.y; }

// Cell (i,j,k) of a flattened index.
__device__ __forceinline__ void cell_of(int64_t t, int nx, int ny, int &i, int &j, int &k) {
    int64_t q = t / nx;
    i = (int)(t - q * nx);
    k = (int)(q / ny);
    j = (int)(q - (int64_t)k * ny);
}

// Reductions march along z like the step: work items are (64 x 4 column tile,
// z chunk), taken round-robin by the kReduceBlocks workgroups, so the partial
// sums have a fixed count and a fixed order.  Own-column z neighbours ride in
// registers; x-y neighbours come through the caches.
struct MarchMap {
    int ntx, nty, nzc, zchunk, items;
};
__host__ __device__ inline MarchMap march_map(int nx, int ny, int nz) {
    MarchMap m;
    m.ntx = (nx + kTX - 1) / kTX;
    m.nty = (ny + kTY - 1) / kTY;
    const int tiles = m.ntx * m.nty;
    int nzc = (kReduceBlocks + tiles - 1) / tiles;
    if (nzc > nz) nzc = nz;
    if (nzc < 1) nzc = 1;
    m.zchunk = (nz + nzc - 1) / nzc;
    m.nzc = (nz + m.zchunk - 1) / m.zchunk;
    m.items = tiles * m.nzc;
    return m;
}

// Per-workgroup partial sums of (E_r, E_r summed on the C,D sites, plain norm), FP64:
//   E_r   = sum |X|^2 - Re sum_{A,B} conj(X) S_X(C,D)
//   E_r'  = sum |X|^2 + Re sum_{C,D} conj(X) S_X(A,B)
template <typename R, bool ZB>
__global__ __launch_bounds__(kReduceThreads) void k3_norm(ReduceArgs<R> a) {
    using C = cx<R>;
    __shared__ double lds[kNormVals * 16];
    const C *f[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) f[q] = (const C *)a.f[q];
    const double rx = a.rx, ry = a.ry, rz = a.rz;
    double v[kNormVals] = {0.0, 0.0, 0.0};
    const MarchMap mm = march_map(a.nx, a.ny, a.nz);
    const size_t plane = (size_t)a.nx * a.ny;
    const int x = threadIdx.x & (kTX - 1), y = threadIdx.x / kTX;
    // consecutive blocks go to the 8 XCDs in turn: remap so that each XCD takes
    // a contiguous range of tiles, whose y-neighbour rows then sit in its L2
    const int blk = (gridDim.x & 7) == 0 ? (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3) : blockIdx.x;
    for (int item = blk; item < mm.items; item += gridDim.x) {
        int r = item;
        const int tx = r % mm.ntx;
        r /= mm.ntx;
        const int ty = r % mm.nty;
        const int zc = r / mm.nty;
        const int i = tx * kTX + x, j = ty * kTY + y;
        if (i >= a.nx || j >= a.ny) continue;
        const int z0 = zc * mm.zchunk, z1 = min(a.nz, z0 + mm.zchunk);
        const uint32_t c = (uint32_t)j * a.nx + i;
        const uint32_t xm = (uint32_t)j * a.nx + wrap_dec(i, a.nx), xp = (uint32_t)j * a.nx + wrap_inc(i, a.nx);
        const uint32_t ym = (uint32_t)wrap_dec(j, a.ny) * a.nx + i, yp = (uint32_t)wrap_inc(j, a.ny) * a.nx + i;
        // storage planes: periodic wrap, or in z-slab mode the interior offset by the halo
        auto zpl = [&](int pl) { return a.zh ? pl + a.zh : (pl < 0 ? pl + a.nz : pl >= a.nz ? pl - a.nz : pl); };
        // zero values outside the lattice (ZB): neighbours across a face read as zero
        const bool oxm = !ZB || i > 0, oxp = !ZB || i < a.nx - 1, oym = !ZB || j > 0, oyp = !ZB || j < a.ny - 1;
        const size_t Pb = (size_t)zpl(z0 - 1) * plane, P0 = (size_t)zpl(z0) * plane;
        const bool ob = !ZB || z0 > 0;
        double2 cm0 = to_d(ld_or0(f[4], Pb + c, ob)), cm1 = to_d(ld_or0(f[5], Pb + c, ob));      // C(k-1)
        double2 bm0 = to_d(ld_or0(f[2], Pb + c, ob)), bm1 = to_d(ld_or0(f[3], Pb + c, ob));      // B(k-1)
        double2 a0 = to_d(f[0][P0 + c]), a1 = to_d(f[1][P0 + c]), d0 = to_d(f[6][P0 + c]), d1 = to_d(f[7][P0 + c]);
        for (int k = z0; k < z1; ++k) {
            const size_t Pk = (size_t)zpl(k) * plane;
            const size_t Pn = (size_t)zpl(k + 1) * plane;
            const bool on = !ZB || k + 1 < a.nz;
            const double2 an0 = to_d(ld_or0(f[0], Pn + c, on)), an1 = to_d(ld_or0(f[1], Pn + c, on));
            const double2 dn0 = to_d(ld_or0(f[6], Pn + c, on)), dn1 = to_d(ld_or0(f[7], Pn + c, on));
            const double2 b0 = to_d(f[2][Pk + c]), b1 = to_d(f[3][Pk + c]);
            const double2 c0 = to_d(f[4][Pk + c]), c1 = to_d(f[5][Pk + c]);
            St3<double2> sab = stencil_ab<double2, double>(rx, ry, rz,
                c0, cm0, to_d(ld_or0(f[4], Pk + xp, oxp)), to_d(ld_or0(f[4], Pk + yp, oyp)),
                c1, cm1, to_d(ld_or0(f[5], Pk + ym, oym)), to_d(ld_or0(f[5], Pk + xm, oxm)),
                d0, to_d(ld_or0(f[6], Pk + xm, oxm)), to_d(ld_or0(f[6], Pk + yp, oyp)), dn0,
                d1, to_d(ld_or0(f[7], Pk + ym, oym)), to_d(ld_or0(f[7], Pk + xp, oxp)), dn1);
            St3<double2> scd = stencil_cd<double2, double>(rx, ry, rz,
                a0, an0, to_d(ld_or0(f[0], Pk + xp, oxp)), to_d(ld_or0(f[0], Pk + yp, oyp)),
                a1, an1, to_d(ld_or0(f[1], Pk + xm, oxm)), to_d(ld_or0(f[1], Pk + ym, oym)),
                b0, bm0, to_d(ld_or0(f[2], Pk + xm, oxm)), to_d(ld_or0(f[2], Pk + yp, oyp)),
                b1, bm1, to_d(ld_or0(f[3], Pk + xp, oxp)), to_d(ld_or0(f[3], Pk + ym, oym)));
            const double p = abs2(a0) + abs2(a1) + abs2(b0) + abs2(b1) + abs2(c0) + abs2(c1) + abs2(d0) + abs2(d1);
            v[0] += p - (re_conj_mul(a0, sab.s0) + re_conj_mul(a1, sab.s1) + re_conj_mul(b0, sab.s2) +
                         re_conj_mul(b1, sab.s3));
            v[1] += p + (re_conj_mul(c0, scd.s0) + re_conj_mul(c1, scd.s1) + re_conj_mul(d0, scd.s2) +
                         re_conj_mul(d1, scd.s3));
            v[2] += p;
            cm0 = c0;
            cm1 = c1;
            bm0 = b0;
            bm1 = b1;
            a0 = an0;
            a1 = an1;
            d0 = dn0;
            d1 = dn1;
        }
    }
    block_sum<kNormVals>(v, lds);
    if (threadIdx.x == 0) {
        double *o = a.partial + (size_t)blockIdx.x * kNormVals;
        o[0] = v[0];
        o[1] = v[1];
        o[2] = v[2];
    }
}

__constant__ float kOff3[8][3] = {{0.f, 0.f, 0.f}, {.5f, .5f, 0.f}, {.5f, 0.f, .5f}, {0.f, .5f, .5f},
                                  {0.f, 0.f, .5f}, {.5f, .5f, .5f}, {.5f, 0.f, 0.f}, {0.f, .5f, 0.f}};

template <typename R>
__global__ __launch_bounds__(kReduceThreads) void k3_obs(ReduceArgs<R> a) {
    using C = cx<R>;
    __shared__ double lds[kObsVals * 16];
    double v[kObsVals];
#pragma unroll
    for (int q = 0; q < kObsVals; ++q) v[q] = 0.0;
    const MarchMap mm = march_map(a.nx, a.ny, a.nz);
    const size_t plane = (size_t)a.nx * a.ny;
    const int x = threadIdx.x & (kTX - 1), y = threadIdx.x / kTX;
    // consecutive blocks go to the 8 XCDs in turn: remap so that each XCD takes
    // a contiguous range of tiles, whose y-neighbour rows then sit in its L2
    const int blk = (gridDim.x & 7) == 0 ? (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3) : blockIdx.x;
    for (int item = blk; item < mm.items; item += gridDim.x) {
        int r = item;
        const int tx = r % mm.ntx;
        r /= mm.ntx;
        const int ty = r % mm.nty;
        const int zc = r / mm.nty;
        const int i = tx * kTX + x, j = ty * kTY + y;
        if (i >= a.nx || j >= a.ny) continue;
        const int z0 = zc * mm.zchunk, z1 = min(a.nz, z0 + mm.zchunk);
        const uint32_t c = (uint32_t)j * a.nx + i;
        for (int k = z0; k < z1; ++k) {
            const size_t e = (size_t)k * plane + c;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double p = abs2(to_d(((const C *)a.f[q])[e]));
                const double px = (double)i + (double)kOff3[q][0];
                const double py = (double)j + (double)kOff3[q][1];
                const double pz = (double)k + (double)kOff3[q][2];
                if (pz >= a.z0) v[0] += p;
                v[1] += px * p;
                v[2] += py * p;
                v[3] += pz * p;
                v[4] += p;
                v[5 + q / 2] += p;
            }
        }
    }
    block_sum<kObsVals>(v, lds);
    if (threadIdx.x == 0)
        for (int q = 0; q < kObsVals; ++q) a.partial[(size_t)blockIdx.x * kObsVals + q] = v[q];
}

// complex64 lattices with an even row length: each thread sums two adjacent
// cells, read as one 16-byte unit per array (twice the bytes per load
// instruction); tiles of 128 x 4 cells, otherwise as k3_obs.
__global__ __launch_bounds__(kReduceThreads) void k3_obs_pairs(ReduceArgs<float> a) {
    __shared__ double lds[kObsVals * 16];
    double v[kObsVals];
#pragma unroll
    for (int q = 0; q < kObsVals; ++q) v[q] = 0.0;
    constexpr int PW = 2 * kTX;                      // cells per tile row
    const int ntx = (a.nx + PW - 1) / PW, nty = (a.ny + kTY - 1) / kTY;
    const int tiles = ntx * nty;
    int nzc = (kReduceBlocks + tiles - 1) / tiles;
    if (nzc > a.nz) nzc = a.nz;
    if (nzc < 1) nzc = 1;
    const int zchunk = (a.nz + nzc - 1) / nzc;
    nzc = (a.nz + zchunk - 1) / zchunk;
    const int items = tiles * nzc;
    const size_t plane = (size_t)a.nx * a.ny;
    const int x = threadIdx.x & (kTX - 1), y = threadIdx.x / kTX;
    const int blk = (gridDim.x & 7) == 0 ? (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3) : blockIdx.x;
    for (int item = blk; item < items; item += gridDim.x) {
        int r = item;
        const int tx = r % ntx;
        r /= ntx;
        const int ty = r % nty;
        const int zc = r / nty;
        const int i = tx * PW + 2 * x, j = ty * kTY + y;
        if (i >= a.nx || j >= a.ny) continue;             // nx even: i + 1 < nx as well
        const int z0 = zc * zchunk, z1 = min(a.nz, z0 + zchunk);
        const size_t c = (size_t)j * a.nx + i;
        for (int k = z0; k < z1; ++k) {
            const size_t e = (size_t)k * plane + c;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float4 u = *(const float4 *)((const float2 *)a.f[q] + e);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const double p = h == 0 ? abs2(to_d(make_float2(u.x, u.y))) : abs2(to_d(make_float2(u.z, u.w)));
                    const double px = (double)(i + h) + (double)kOff3[q][0];
                    const double py = (double)j + (double)kOff3[q][1];
                    const double pz = (double)k + (double)kOff3[q][2];
                    if (pz >= a.z0) v[0] += p;
                    v[1] += px * p;
                    v[2] += py * p;
                    v[3] += pz * p;
                    v[4] += p;
                    v[5 + q / 2] += p;
                }
            }
        }
    }
    block_sum<kObsVals>(v, lds);
    if (threadIdx.x == 0)
        for (int q = 0; q < kObsVals; ++q) a.partial[(size_t)blockIdx.x * kObsVals + q] = v[q];
}

template <typename R>
__global__ __launch_bounds__(256) void k3_seed(ReduceArgs<R> a, CPtr8 lam) {
    using C = cx<R>;
    const int64_t ncell = (int64_t)a.nx * a.ny * a.nz;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ncell;
         t += (int64_t)gridDim.x * blockDim.x) {
        int i, j, k;
        cell_of(t, a.nx, a.ny, i, j, k);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            double z = (double)k + (double)kOff3[q][2];
            C x = ((const C *)a.f[q])[t];
            R w = (z >= a.z0) ? (R)2 : (R)0;
            ((C *)lam.p[q])[t] = mk2(w * x.x, w * x.y);
        }
    }
}

// Per-site coefficient arrays from V: theta = (dt/2)(+-m + V) in FP64, stored
// as theta (complex128 lattices) or as the rounded gamma pair (complex64).
__device__ __forceinline__ void put_site_coef(double *th, int64_t t, double theta) { th[t] = theta; }
__device__ __forceinline__ void put_site_coef(float *th, int64_t t, double theta) {
    ((float2 *)th)[t] = gamma32_record(theta);
}

template <typename R>
__global__ __launch_bounds__(256) void k_theta_fields(CPtr8 th, CPtr8 v, int narr, int64_t ncell, double half_dt,
                                                       double m) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ncell;
         t += (int64_t)gridDim.x * blockDim.x) {
        for (int q = 0; q < narr; ++q) {
            // + for the first sheet's arrays (A,B / u), - for the second (C,D / v)
            double sgn = (q < narr / 2) ? 1.0 : -1.0;
            double vv = v.p[q] ? (double)((const R *)v.p[q])[t] : 0.0;
            put_site_coef((R *)th.p[q], t, half_dt * (sgn * m + vv));
        }
    }
}

// gamma = 1 - alpha for a complex theta = th + i thi (absorbing potential):
// rounded once from FP64; real theta keeps the unit-modulus search.
__device__ inline float2 gamma32_complex(double th, double thi) {
#pragma clang fp contract(off)
    if (thi == 0.0) return gamma32_record(th);
    const double den = (1.0 - thi) * (1.0 - thi) + th * th;
    const double ar = (1.0 - thi * thi - th * th) / den, ai = -((2.0 * th) / den);
    return make_float2((float)(1.0 - ar), (float)(-ai));
}

__global__ __launch_bounds__(256) void k_coef_from_theta(float2 *coef, const double *theta, const double *theta_im,
                                                         int64_t n) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        coef[t] = gamma32_complex(theta[t], theta_im ? theta_im[t] : 0.0);
}

// Per-site record from the fields of one state array: theta = half_dt (sgn_m +
// V) + i half_dt W in FP64, then gamma (complex64 lattices) or theta itself.
template <bool C64>
__global__ __launch_bounds__(256) void k_coef_from_fields(void *coef, double half_dt, double sgn_m, const double *v,
                                                          const double *w, int64_t n) {
#pragma clang fp contract(off)
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const double th = half_dt * (sgn_m + (v ? v[t] : 0.0));
        if constexpr (C64) {
            ((float2 *)coef)[t] = gamma32_complex(th, w ? half_dt * w[t] : 0.0);
        } else {
            ((double *)coef)[t] = th;
        }
    }
}

__global__ __launch_bounds__(256) void k_final_sum(const double *partial, int nblocks, int nv, double *out) {
    __shared__ double lds[16 * 16];
    // one value at a time, fixed order: thread t sums blocks t, t+256, ...
    for (int q = 0; q < nv; ++q) {
        double v[1] = {0.0};
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v[0] += partial[(size_t)b * nv + q];
        block_sum<1>(v, lds);
        if (threadIdx.x == 0) out[q] = v[0];
        __syncthreads();
    }
}

inline int grid_for(int64_t n, int threads, int cap) {
    int64_t g = (n + threads - 1) / threads;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

template <typename R>
hipError_t launch_half3(const HalfArgs<R> &a, int which, bool site, hipStream_t s) {
    const int64_t nblk = (int64_t)((a.nx + kTX - 1) / kTX) * ((a.ny + kTY - 1) / kTY) * a.nz;
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    dim3 g((unsigned)nblk), b(kTX * kTY);
#define H3(ZB)                                                                          \
    if (which == 0) {                                                                   \
        if (site) hipLaunchKernelGGL((k3_half<R, true, 0, ZB>), g, b, 0, s, a);         \
        else hipLaunchKernelGGL((k3_half<R, false, 0, ZB>), g, b, 0, s, a);             \
    } else {                                                                            \
        if (site) hipLaunchKernelGGL((k3_half<R, true, 1, ZB>), g, b, 0, s, a);         \
        else hipLaunchKernelGGL((k3_half<R, false, 1, ZB>), g, b, 0, s, a);             \
    }
    if (a.zbc) {
        H3(true)
    } else {
        H3(false)
    }
#undef H3
    return hipGetLastError();
}

template <typename R> hipError_t launch_norm3(const ReduceArgs<R> &a, hipStream_t s) {
    if (norm3_staged_supported(a.nx, sizeof(R) == 4)) return launch_norm3_staged<R>(a, s);
    if (a.zbc) hipLaunchKernelGGL((k3_norm<R, true>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, a);
    else hipLaunchKernelGGL((k3_norm<R, false>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, a);
    return hipGetLastError();
}

template <typename R> hipError_t launch_obs3(const ReduceArgs<R> &a, hipStream_t s) {
    if constexpr (sizeof(R) == 4) {
        if (a.nx % 2 == 0) {
            hipLaunchKernelGGL(k3_obs_pairs, dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k3_obs<R>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, a);
    return hipGetLastError();
}

template <typename R> hipError_t launch_seed3(const ReduceArgs<R> &a, void *const lam[8], hipStream_t s) {
    CPtr8 l;
    for (int q = 0; q < 8; ++q) l.p[q] = lam[q];
    const int64_t n = (int64_t)a.nx * a.ny * a.nz;
    hipLaunchKernelGGL((k3_seed<R>), dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, a, l);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_theta_fields(void *const th[8], void *const v[8], int narr, int64_t ncell, double half_dt,
                               double m, hipStream_t s) {
    CPtr8 t, vv;
    for (int q = 0; q < 8; ++q) {
        t.p[q] = q < narr ? th[q] : nullptr;
        vv.p[q] = (q < narr && v) ? v[q] : nullptr;
    }
    hipLaunchKernelGGL((k_theta_fields<R>), dim3(grid_for(ncell, 256, 8192)), dim3(256), 0, s, t, vv, narr, ncell,
                       half_dt, m);
    return hipGetLastError();
}

hipError_t launch_coef_from_theta(void *coef, const double *theta, const double *theta_im, int64_t n,
                                  hipStream_t s) {
    hipLaunchKernelGGL(k_coef_from_theta, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, (float2 *)coef, theta,
                       theta_im, n);
    return hipGetLastError();
}

hipError_t launch_coef_from_fields(void *coef, bool c64, double half_dt, double sgn_m, const double *v,
                                   const double *w, int64_t n, hipStream_t s) {
    if (c64)
        hipLaunchKernelGGL(k_coef_from_fields<true>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, coef, half_dt,
                           sgn_m, v, w, n);
    else
        hipLaunchKernelGGL(k_coef_from_fields<false>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, coef,
                           half_dt, sgn_m, v, w, n);
    return hipGetLastError();
}

hipError_t launch_final_sum(const double *partial, int nblocks, int nv, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(256), 0, s, partial, nblocks, nv, out);
    return hipGetLastError();
}

#define INST(R)                                                                                             \
    template hipError_t launch_half3<R>(const HalfArgs<R> &, int, bool, hipStream_t);                       \
    template hipError_t launch_norm3<R>(const ReduceArgs<R> &, hipStream_t);                                \
    template hipError_t launch_obs3<R>(const ReduceArgs<R> &, hipStream_t);                                 \
    template hipError_t launch_seed3<R>(const ReduceArgs<R> &, void *const[8], hipStream_t);               \
    template hipError_t launch_theta_fields<R>(void *const[8], void *const[8], int, int64_t, double, double, \
                                               hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace dirac
