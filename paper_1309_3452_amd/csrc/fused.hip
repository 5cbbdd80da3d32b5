// Fused one-launch time step: both half-steps of Sect. 2 (Eqs. ss1-ss4) in a
// single pass over the lattice, so every amplitude is read once and written
// once per step (plus cache-resident halo re-reads).
//
// (3+1)D: a workgroup owns an x-y tile of 64 x TY cells and marches along z
// over a chunk of planes.  At plane p it computes the new A,B of plane p
// (Eqs. ss1, ss2) for its tile plus the one-cell halo ring that the C,D
// stencils of the tile need (left column: A1, B0; right: A0, B1; bottom row:
// A1, B1; top row: A0, B0), keeps them in LDS, and then computes the new C,D
// of plane p-1 (Eqs. ss3, ss4) from LDS and registers.  The halo ring is
// recomputed from the old state rather than exchanged, so workgroups never
// read each other's results: the state ping-pongs between two buffers.
// Per cell the old C(p-1), D(p), D(p-1) and new B(p-1), B(p-2) ride along the
// march in registers.  A chunk [z0, z1) runs planes z0-1 .. z1 so that its
// first and last C,D planes have their A,B neighbours; periodic wrap in z is
// a modulo on the plane index.
//
// (2+1)D: the same with rows for planes: a workgroup owns an x strip and
// marches along y; the halo is one column on each side (u1 on the left, u0 on
// the right).
#include "device.h"
#include "internal.h"
#include "stencil3.h"
#include "march2.h"

namespace dirac {

namespace {

constexpr int kTX = 64;

// XCD-aware ordering: blocks are dealt round-robin to the 8 XCDs; give each
// XCD a contiguous run of tiles so neighbouring tiles (which re-read each
// other's edges) share that XCD's L2.
__device__ __forceinline__ int logical_block() {
    const int nb = gridDim.x, b = blockIdx.x;
    if ((nb & 7) == 0) return (b & 7) * (nb >> 3) + (b >> 3);
    return b;
}

template <typename R, bool SITE>
__device__ __forceinline__ Coef<R> fcoef(const FusedArgs<R> &a, int arr, int cls, int pk, size_t idx) {
    if constexpr (SITE) {
        return coef_theta(a.th[arr][idx]);
    } else {
        const R *e = a.tab + ((size_t)cls * a.nz + pk) * 4;
        Coef<R> k;
        k.c1 = mk2(e[0], e[1]);
        k.c2 = mk2(e[2], e[3]);
        return k;
    }
}

// New value of A,B array Q (0: A0, 1: A1, 2: B0, 3: B1) at cell (gi, gj) of
// plane pk, everything loaded from the old state (halo cells).
template <typename R, bool SITE, int Q>
__device__ __forceinline__ cx<R> h1_at(const FusedArgs<R> &a, int gi, int gj, int pk) {
    using C = cx<R>;
    const size_t plane = (size_t)a.nx * a.ny;
    const size_t P = (size_t)pk * plane;
    const size_t row = (size_t)gj * a.nx;
    const size_t c = P + row + gi;
    const C *in[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) in[q] = (const C *)a.in[q];
    const R rx = a.rx, ry = a.ry, rz = a.rz;
    C s;
    if constexpr (Q == 0) {      // S_A0 = rz(C0 - C0[k-1]) + rx(D0 - D0[i-1]) - i ry(D1 - D1[j-1])
        const size_t zm = (size_t)wrap_dec(pk, a.nz) * plane + row + gi;
        const size_t xm = P + row + wrap_dec(gi, a.nx), ym = P + (size_t)wrap_dec(gj, a.ny) * a.nx + gi;
        s = cadd(cadd(cscale(rz, csub(in[4][c], in[4][zm])), cscale(rx, csub(in[6][c], in[6][xm]))),
                 ciscale(-ry, csub(in[7][c], in[7][ym])));
    } else if constexpr (Q == 1) {   // S_A1 = rz(C1 - C1[k-1]) + rx(D1[i+1] - D1) - i ry(D0[j+1] - D0)
        const size_t zm = (size_t)wrap_dec(pk, a.nz) * plane + row + gi;
        const size_t xp = P + row + wrap_inc(gi, a.nx), yp = P + (size_t)wrap_inc(gj, a.ny) * a.nx + gi;
        s = cadd(cadd(cscale(rz, csub(in[5][c], in[5][zm])), cscale(rx, csub(in[7][xp], in[7][c]))),
                 ciscale(-ry, csub(in[6][yp], in[6][c])));
    } else if constexpr (Q == 2) {   // S_B0 = -rz(D0[k+1] - D0) + rx(C0[i+1] - C0) + i ry(C1 - C1[j-1])
        const size_t zp = (size_t)wrap_inc(pk, a.nz) * plane + row + gi;
        const size_t xp = P + row + wrap_inc(gi, a.nx), ym = P + (size_t)wrap_dec(gj, a.ny) * a.nx + gi;
        s = cadd(cadd(cscale(-rz, csub(in[6][zp], in[6][c])), cscale(rx, csub(in[4][xp], in[4][c]))),
                 ciscale(ry, csub(in[5][c], in[5][ym])));
    } else {                         // S_B1 = -rz(D1[k+1] - D1) + rx(C1 - C1[i-1]) + i ry(C0[j+1] - C0)
        const size_t zp = (size_t)wrap_inc(pk, a.nz) * plane + row + gi;
        const size_t xm = P + row + wrap_dec(gi, a.nx), yp = P + (size_t)wrap_inc(gj, a.ny) * a.nx + gi;
        s = cadd(cadd(cscale(-rz, csub(in[7][zp], in[7][c])), cscale(rx, csub(in[5][c], in[5][xm]))),
                 ciscale(ry, csub(in[4][yp], in[4][c])));
    }
    return update(in[Q][c], s, fcoef<R, SITE>(a, Q, Q / 2, pk, c));
}

template <typename R, bool SITE, int TY>
__global__ __launch_bounds__(kTX *TY) void k3_fused(FusedArgs<R> a) {
    using C = cx<R>;
    constexpr int LW = kTX + 2, LN = LW * (TY + 2);
    __shared__ C ab[2][4][LN];

    int L = logical_block();
    const int tx = L % a.ntx;
    L /= a.ntx;
    const int ty = L % a.nty;
    const int zc = L / a.nty;
    const int x0 = tx * kTX, y0 = ty * TY;
    const int w = min(kTX, a.nx - x0), h = min(TY, a.ny - y0);
    const int z0 = zc * a.zchunk, z1 = min(a.nz, z0 + a.zchunk);
    const int x = threadIdx.x & (kTX - 1), y = threadIdx.x / kTX;
    const bool own = x < w && y < h;
    const int i = x0 + (own ? x : 0), j = y0 + (own ? y : 0);
    const size_t plane = (size_t)a.nx * a.ny;
    const size_t rc = (size_t)j * a.nx + i;
    const size_t rxm = (size_t)j * a.nx + wrap_dec(i, a.nx), rxp = (size_t)j * a.nx + wrap_inc(i, a.nx);
    const size_t rym = (size_t)wrap_dec(j, a.ny) * a.nx + i, ryp = (size_t)wrap_inc(j, a.ny) * a.nx + i;
    const int li = (y + 1) * LW + (x + 1);

    // halo item of this thread (t < 2(w + h)); kind 0: left, 1: right, 2: bottom, 3: top
    const int t = threadIdx.x;
    int hk = -1, hx = 0, hy = 0;
    if (t < h) { hk = 0; hx = -1; hy = t; }
    else if (t < 2 * h) { hk = 1; hx = w; hy = t - h; }
    else if (t < 2 * h + w) { hk = 2; hx = t - 2 * h; hy = -1; }
    else if (t < 2 * h + 2 * w) { hk = 3; hx = t - 2 * h - w; hy = h; }
    const int hgi = wrapn(x0 + hx, a.nx), hgj = wrapn(y0 + hy, a.ny);
    const int hli = (hy + 1) * LW + (hx + 1);

    const C *in[8];
    C *out[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        in[q] = (const C *)a.in[q];
        out[q] = (C *)a.out[q];
    }
    const R rx = a.rx, ry = a.ry, rz = a.rz;

    // register windows of the march (own cell)
    C cm0 = mk2((R)0, (R)0), cm1 = cm0;   // old C(p-1)
    C dc0 = cm0, dc1 = cm0;               // old D(p)
    C dm0 = cm0, dm1 = cm0;               // old D(p-1)
    C bm0 = cm0, bm1 = cm0;               // new B(p-1)
    C bmm0 = cm0, bmm1 = cm0;             // new B(p-2)
    if (own) {
        const size_t Pc = (size_t)wrapn(z0 - 2, a.nz) * plane, Pd = (size_t)wrapn(z0 - 1, a.nz) * plane;
        cm0 = in[4][Pc + rc];
        cm1 = in[5][Pc + rc];
        dc0 = in[6][Pd + rc];
        dc1 = in[7][Pd + rc];
    }

    for (int p = z0 - 1; p <= z1; ++p) {
        const int pk = wrapn(p, a.nz);
        const size_t P = (size_t)pk * plane, Pp = (size_t)wrap_inc(pk, a.nz) * plane;
        const int buf = p & 1;
        C nA0 = cm0, nA1 = cm0, nB0 = cm0, nB1 = cm0, c0 = cm0, c1 = cm0, dn0 = cm0, dn1 = cm0;
        if (own) {
            c0 = in[4][P + rc];
            c1 = in[5][P + rc];
            dn0 = in[6][Pp + rc];
            dn1 = in[7][Pp + rc];
            const C a0 = in[0][P + rc], a1 = in[1][P + rc], b0 = in[2][P + rc], b1 = in[3][P + rc];
            St3<C> s = stencil_ab<C, R>(rx, ry, rz,
                                        c0, cm0, in[4][P + rxp], in[4][P + ryp],
                                        c1, cm1, in[5][P + rym], in[5][P + rxm],
                                        dc0, in[6][P + rxm], in[6][P + ryp], dn0,
                                        dc1, in[7][P + rym], in[7][P + rxp], dn1);
            nA0 = update(a0, s.s0, fcoef<R, SITE>(a, 0, 0, pk, P + rc));
            nA1 = update(a1, s.s1, fcoef<R, SITE>(a, 1, 0, pk, P + rc));
            nB0 = update(b0, s.s2, fcoef<R, SITE>(a, 2, 1, pk, P + rc));
            nB1 = update(b1, s.s3, fcoef<R, SITE>(a, 3, 1, pk, P + rc));
            ab[buf][0][li] = nA0;
            ab[buf][1][li] = nA1;
            ab[buf][2][li] = nB0;
            ab[buf][3][li] = nB1;
            if (p >= z0 && p < z1) {
                out[0][P + rc] = nA0;
                out[1][P + rc] = nA1;
                out[2][P + rc] = nB0;
                out[3][P + rc] = nB1;
            }
        }
        if (hk == 0) {
            ab[buf][1][hli] = h1_at<R, SITE, 1>(a, hgi, hgj, pk);
            ab[buf][2][hli] = h1_at<R, SITE, 2>(a, hgi, hgj, pk);
        } else if (hk == 1) {
            ab[buf][0][hli] = h1_at<R, SITE, 0>(a, hgi, hgj, pk);
            ab[buf][3][hli] = h1_at<R, SITE, 3>(a, hgi, hgj, pk);
        } else if (hk == 2) {
            ab[buf][1][hli] = h1_at<R, SITE, 1>(a, hgi, hgj, pk);
            ab[buf][3][hli] = h1_at<R, SITE, 3>(a, hgi, hgj, pk);
        } else if (hk == 3) {
            ab[buf][0][hli] = h1_at<R, SITE, 0>(a, hgi, hgj, pk);
            ab[buf][2][hli] = h1_at<R, SITE, 2>(a, hgi, hgj, pk);
        }
        __syncthreads();
        if (own && p >= z0 + 1) {
            // C,D of plane k = p-1 from the new A,B of planes p-1 (LDS) and p, p-2 (registers)
            const int kq = wrapn(p - 1, a.nz);
            const size_t Pm = (size_t)kq * plane;
            const C *A0 = ab[buf ^ 1][0], *A1 = ab[buf ^ 1][1], *B0 = ab[buf ^ 1][2], *B1 = ab[buf ^ 1][3];
            St3<C> s = stencil_cd<C, R>(rx, ry, rz,
                                        A0[li], nA0, A0[li + 1], A0[li + LW],
                                        A1[li], nA1, A1[li - 1], A1[li - LW],
                                        B0[li], bmm0, B0[li - 1], B0[li + LW],
                                        B1[li], bmm1, B1[li + 1], B1[li - LW]);
            out[4][Pm + rc] = update(cm0, s.s0, fcoef<R, SITE>(a, 4, 2, kq, Pm + rc));
            out[5][Pm + rc] = update(cm1, s.s1, fcoef<R, SITE>(a, 5, 2, kq, Pm + rc));
            out[6][Pm + rc] = update(dm0, s.s2, fcoef<R, SITE>(a, 6, 3, kq, Pm + rc));
            out[7][Pm + rc] = update(dm1, s.s3, fcoef<R, SITE>(a, 7, 3, kq, Pm + rc));
        }
        __syncthreads();
        cm0 = c0;
        cm1 = c1;
        dm0 = dc0;
        dm1 = dc1;
        dc0 = dn0;
        dc1 = dn1;
        bmm0 = bm0;
        bmm1 = bm1;
        bm0 = nB0;
        bm1 = nB1;
    }
}

template <typename R, bool SITE, int TXB>
__global__ __launch_bounds__(TXB) void k2_fused(FusedArgs<R> a) {
    __shared__ cx<R> uu[2][2][TXB + 2];
    const int L = logical_block();
    march2<R, SITE, TXB>(a, L % a.ntx, L / a.ntx, uu);
}

int default_chunks(int64_t tiles, int n_along, int target_blocks) {
    int64_t c = (target_blocks + tiles - 1) / tiles;
    if (c < 1) c = 1;
    if (c > n_along) c = n_along;
    return (int)c;
}

}  // namespace

template <typename R> hipError_t launch_fused3(const FusedArgs<R> &a0, bool site, int tile_y, hipStream_t s) {
    FusedArgs<R> a = a0;
    const int TY = tile_y > 0 ? tile_y : (sizeof(R) == 8 ? 4 : 8);
    if (TY != 4 && TY != 8) return hipErrorInvalidValue;
    a.ntx = (a.nx + kTX - 1) / kTX;
    a.nty = (a.ny + TY - 1) / TY;
    const int64_t tiles = (int64_t)a.ntx * a.nty;
    if (a.zchunk <= 0) {
        const int nzc = default_chunks(tiles, a.nz, 2048);
        a.zchunk = (a.nz + nzc - 1) / nzc;
    }
    a.nzc = (a.nz + a.zchunk - 1) / a.zchunk;
    const int64_t nblk = tiles * a.nzc;
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    dim3 g((unsigned)nblk), b(kTX * TY);
#define L3(T)                                                                 \
    if (TY == T) {                                                            \
        if (site) hipLaunchKernelGGL((k3_fused<R, true, T>), g, b, 0, s, a);  \
        else hipLaunchKernelGGL((k3_fused<R, false, T>), g, b, 0, s, a);      \
    }
    L3(4) L3(8)
#undef L3
    return hipGetLastError();
}

template <typename R> hipError_t launch_fused2(const FusedArgs<R> &a0, bool site, hipStream_t s) {
    FusedArgs<R> a = a0;
    constexpr int TXB = 128;
    a.ntx = (a.nx + TXB - 1) / TXB;
    a.nty = 1;
    if (a.zchunk <= 0) {
        const int nc = default_chunks(a.ntx, a.ny, 4096);
        a.zchunk = (a.ny + nc - 1) / nc;
        if (a.zchunk < 8 && a.ny >= 8) a.zchunk = 8;
    }
    a.nzc = (a.ny + a.zchunk - 1) / a.zchunk;
    const int64_t nblk = (int64_t)a.ntx * a.nzc;
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    if (site) hipLaunchKernelGGL((k2_fused<R, true, TXB>), dim3((unsigned)nblk), dim3(TXB), 0, s, a);
    else hipLaunchKernelGGL((k2_fused<R, false, TXB>), dim3((unsigned)nblk), dim3(TXB), 0, s, a);
    return hipGetLastError();
}

template hipError_t launch_fused3<float>(const FusedArgs<float> &, bool, int, hipStream_t);
template hipError_t launch_fused3<double>(const FusedArgs<double> &, bool, int, hipStream_t);
template hipError_t launch_fused2<float>(const FusedArgs<float> &, bool, hipStream_t);
template hipError_t launch_fused2<double>(const FusedArgs<double> &, bool, hipStream_t);

}  // namespace dirac
