// (2+1)D fused step for one x strip and one y chunk of a lattice, shared by
// the single-lattice kernel and the batched kernels.
#pragma once

#include "device.h"
#include "internal.h"
#include "stencil3.h"

namespace dirac {

__device__ __forceinline__ int wrapn(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// ---------------------------------------------------------------------------
// (2+1)D row march.  u0 (i,j), u1 (i+1/2,j+1/2), v0 (i+1/2,j), v1 (i,j+1/2):
//   S_u0 = rx(v0 - v0[i-1]) - i ry(v1 - v1[j-1])   S_u1 = rx(v1[i+1] - v1) - i ry(v0[j+1] - v0)
//   S_v0 = rx(u0[i+1] - u0) + i ry(u1 - u1[j-1])   S_v1 = rx(u1 - u1[i-1]) + i ry(u0[j+1] - u0)
// ---------------------------------------------------------------------------
template <typename R, bool SITE>
__device__ __forceinline__ Coef<R> fcoef2(const FusedArgs<R> &a, int arr, size_t idx) {
    if constexpr (SITE) {
        return coef_site_at<R>(a.th[arr], idx, (R)1);
    } else {
        const R *e = a.tab + (size_t)(arr < 2 ? 0 : 3) * a.nz * 4;
        Coef<R> k;
        k.c1 = mk2(e[0], e[1]);
        k.c2 = mk2(e[2], e[3]);
        return k;
    }
}

template <typename R, bool SITE, int TXB>
__device__ __forceinline__ void march2(const FusedArgs<R> &a, int tx, int zc, cx<R> (*uu)[2][TXB + 2]) {
    using C = cx<R>;
    const int x0 = tx * TXB;
    const int w = min(TXB, a.nx - x0);
    const int y0 = zc * a.zchunk, y1 = min(a.ny, y0 + a.zchunk);
    const int x = threadIdx.x;
    const bool own = x < w;
    const int i = x0 + (own ? x : 0);
    const int im = wrap_dec(i, a.nx), ip = wrap_inc(i, a.nx);
    const int li = x + 1;
    // halo: thread 0 does the left column (u1 at i = x0-1), thread 1 the right (u0 at x0+w)
    const int hgl = wrapn(x0 - 1, a.nx), hgr = wrapn(x0 + w, a.nx);
    const C *in[4];
    C *out[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        in[q] = (const C *)a.in[q];
        out[q] = (C *)a.out[q];
    }
    const R rx = a.rx, ry = a.ry;
    const size_t nx = a.nx;
    C z = mk2((R)0, (R)0);
    C v1m = z;                // old v1(p-1)
    C v0c = z;                // old v0(p)
    C v0m = z;                // old v0(p-1)
    C u1m = z, u1mm = z;      // new u1(p-1), u1(p-2)
    if (own) {
        v1m = in[3][(size_t)wrapn(y0 - 2, a.ny) * nx + i];
        v0c = in[2][(size_t)wrapn(y0 - 1, a.ny) * nx + i];
    }
    for (int p = y0 - 1; p <= y1; ++p) {
        const int pr = wrapn(p, a.ny);
        const size_t Rw = (size_t)pr * nx, Rp = (size_t)wrap_inc(pr, a.ny) * nx, Rm = (size_t)wrap_dec(pr, a.ny) * nx;
        const int buf = p & 1;
        C nu0 = z, nu1 = z, v1c = z, v0n = z;
        if (own) {
            v1c = in[3][Rw + i];
            v0n = in[2][Rp + i];
            St2<C> s = stencil_u<C, R>(rx, ry, v0c, in[2][Rw + im], v0n, v1c, v1m, in[3][Rw + ip]);
            nu0 = update(in[0][Rw + i], s.s0, fcoef2<R, SITE>(a, 0, Rw + i));
            nu1 = update(in[1][Rw + i], s.s1, fcoef2<R, SITE>(a, 1, Rw + i));
            uu[buf][0][li] = nu0;
            uu[buf][1][li] = nu1;
            if (p >= y0 && p < y1) {
                out[0][Rw + i] = nu0;
                out[1][Rw + i] = nu1;
            }
        }
        if (threadIdx.x == 0) {
            // u1 at the left halo column: S_u1 = rx(v1[i+1] - v1) - i ry(v0[j+1] - v0)
            const int g = hgl;
            C s = sterm2(rx, csub(in[3][Rw + wrap_inc(g, a.nx)], in[3][Rw + g]), -ry,
                         csub(in[2][Rp + g], in[2][Rw + g]));
            uu[buf][1][0] = update(in[1][Rw + g], s, fcoef2<R, SITE>(a, 1, Rw + g));
        } else if (threadIdx.x == 1) {
            // u0 at the right halo column: S_u0 = rx(v0 - v0[i-1]) - i ry(v1 - v1[j-1])
            const int g = hgr;
            C s = sterm2(rx, csub(in[2][Rw + g], in[2][Rw + wrap_dec(g, a.nx)]), -ry,
                         csub(in[3][Rw + g], in[3][Rm + g]));
            uu[buf][0][w + 1] = update(in[0][Rw + g], s, fcoef2<R, SITE>(a, 0, Rw + g));
        }
        __syncthreads();
        if (own && p >= y0 + 1) {
            const size_t Rk = (size_t)wrapn(p - 1, a.ny) * nx;
            const C *U0 = uu[buf ^ 1][0], *U1 = uu[buf ^ 1][1];
            St2<C> s = stencil_v<C, R>(rx, ry, U0[li], U0[li + 1], nu0, U1[li], u1mm, U1[li - 1]);
            out[2][Rk + i] = update(v0m, s.s0, fcoef2<R, SITE>(a, 2, Rk + i));
            out[3][Rk + i] = update(v1m, s.s1, fcoef2<R, SITE>(a, 3, Rk + i));
        }
        __syncthreads();
        v1m = v1c;
        v0m = v0c;
        v0c = v0n;
        u1mm = u1m;
        u1m = nu1;
    }
}


}  // namespace dirac
