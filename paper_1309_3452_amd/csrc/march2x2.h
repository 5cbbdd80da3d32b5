// (2+1)D: two time steps per pass for one x strip and one y chunk of a
// lattice (Sect. 3, Eqs. scheme2Deq-scheme4thline), shared by the
// single-lattice kernel and the batched kernels.
//
// The structure is the (3+1)D two-step march with y in the role of z: four
// levels pipelined along y, each one row behind the previous --
//   level 1  u after step 1 at row p        (from the old v)
//   level 2  v after step 1 at row p-1
//   level 3  u after step 2 at row p-2      (stored for rows in [y0, y1))
//   level 4  v after step 2 at row p-3      (stored for rows in [y0, y1))
// on x ranges shrinking from a two-cell ring (level 1) to the strip (level 4);
// the ring is recomputed, the state ping-pongs between two buffers.
//   S_u0 = rx(v0 - v0[i-1]) - i ry(v1 - v1[j-1])   S_u1 = rx(v1[i+1] - v1) - i ry(v0[j+1] - v0)
//   S_v0 = rx(u0[i+1] - u0) + i ry(u1 - u1[j-1])   S_v1 = rx(u1 - u1[i-1]) + i ry(u0[j+1] - u0)
// Thread t < TW owns strip column t, threads TW..TW+3 the ring columns
// -2, -1, TW, TW+1; LDS rows are (TW + 4) cells with x stored at x + 2.  The
// old v rows of p and p+1 sit in `old`, row p+2 is copied global -> LDS
// asynchronously into `stage` (never read by the stencils, so no wait is
// needed before them), and one row of each level's output sits in `lev`.
// z-like neighbours (rows j-1, j+1) and the previous values X- of the own
// column stay in registers, as do the per-site coefficient records of the
// rows in flight.  The helpers and operation order are those of the one-step
// march, so the result is bitwise that of two one-step passes.
#pragma once

#include "device.h"
#include "internal.h"
#include "stencil3.h"
#include "march2.h"

namespace dirac {

// Per-site coefficient record: gamma pair (complex64 lattices) or theta.
template <typename R> struct SiteRec;
template <> struct SiteRec<float> { using T = float2; };
template <> struct SiteRec<double> { using T = double; };
__device__ __forceinline__ Coef<float> coef_rec(float2 g) { return coef_site(g, 1.0f); }
__device__ __forceinline__ Coef<double> coef_rec(double th) { return coef_theta(th); }

// Asynchronous global -> LDS copy: lane l's 16 bytes land at lds_wave_base + 16 l.
__device__ __forceinline__ void m2_g2lds16(const void *gsrc, void *lds_wave_base) {
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)gsrc,
                                     (__attribute__((address_space(3))) void *)lds_wave_base, 16, 0, 0);
}

template <typename R> __device__ __forceinline__ Coef<R> m2_tcoef(const R *tab, int cls) {
    // 2D tables have one plane: [class][0][4]
    const R *e = tab + (size_t)cls * 4;
    Coef<R> k;
    k.c1 = mk2(e[0], e[1]);
    k.c2 = mk2(e[2], e[3]);
    return k;
}

template <typename C> __device__ __forceinline__ void m2_st(C *base, size_t cell, C v);
template <> __device__ __forceinline__ void m2_st<float2>(float2 *base, size_t cell, float2 v) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(f2v{v.x, v.y}, (f2v *)(base + cell));
}
template <> __device__ __forceinline__ void m2_st<double2>(double2 *base, size_t cell, double2 v) {
    typedef double d2v __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(d2v{v.x, v.y}, (d2v *)(base + cell));
}

// Block of TW + 64 threads.  sOld: PAD + 4 W + PAD cells, sStage: 2 W,
// sLev: PAD + 6 W + PAD, W = TW + 4, PAD = 2 (three distinct LDS arrays).
template <typename R, bool SITE, int TW>
__device__ __forceinline__ void march2x2(const FusedArgs<R> &a, const R *__restrict__ tab, int tx, int yc,
                                         cx<R> *sOld, cx<R> *sStage, cx<R> *sLev) {
    using C = cx<R>;
    using Rec = typename SiteRec<R>::T;
    constexpr int W = TW + 4, PAD = 2;
    constexpr int CPL = 16 / (int)sizeof(C);
    constexpr int NW = (TW + 64) / 64;
    const int nx = a.nx, ny = a.ny;
    const int x0 = tx * TW, w = min(TW, nx - x0);
    const int y0 = yc * a.zchunk, y1 = min(ny, y0 + a.zchunk);
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;

    int x = -3;
    if (t < TW) x = t;
    else if (t < TW + 4) x = (t - TW) < 2 ? (t - TW) - 2 : TW + (t - TW - 2);
    const bool in1 = x >= -2 && x < w + 2;
    const bool in2 = in1 && x >= -1 && x <= w;
    const bool in4 = in1 && x >= 0 && x < w;
    const int i = x + 2;
    const int gx = in1 ? wrapn(x0 + x, nx) : 0;

    auto old_ = [&](int k) -> C * { return sOld + PAD + k * W; };
    auto lev = [&](int k) -> C * { return sLev + PAD + k * W; };
    const C *in[4];
    C *out[4];
    const Rec *rec[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        in[q] = (const C *)a.in[q];
        out[q] = (C *)a.out[q];
        rec[q] = (const Rec *)a.th[q];
    }
    const R rx = a.rx, ry = a.ry;
    const C zero = mk2((R)0, (R)0);
    auto row = [&](int r) -> size_t { return (size_t)wrapn(r, ny) * (size_t)nx; };

    // whole region rows of the old v0, v1 of row r into dst(k), k = 0, 1
    const int rl = (w + 4) / CPL;                   // 16-byte units per region row
    const int nch = (rl + 63) / 64;
    auto copy_row = [&](int r, auto dst_of) {
        const size_t R0 = row(r);
        for (int item = wv; item < 2 * nch; item += NW) {
            const int k = item / nch, c = item % nch;
            const int j = c * 64 + lane;
            if (j < rl) {
                const size_t cell = R0 + (size_t)wrapn(x0 - 2 + j * CPL, nx);
                m2_g2lds16(in[2 + k] + cell, dst_of(k) + c * 64 * CPL);
            }
        }
    };

    Coef<R> kU0{}, kU1{}, kV0{}, kV1{};
    if constexpr (!SITE) {
        kU0 = kU1 = m2_tcoef(tab, 0);
        kV0 = kV1 = m2_tcoef(tab, 3);
    }

    // registers along the march (own column)
    C vprev[2] = {zero, zero};        // old v of row p-1
    C pu[2] = {zero, zero};           // old u of row p
    C u1h2[2] = {zero, zero};         // level 1 of row p-2
    C v2h2[2] = {zero, zero};         // level 2 of row p-3
    C u3h2 = zero;                    // level 3 u1 of row p-4
    C pun[2] = {zero, zero};
    C u1L[2] = {zero, zero}, vown[2] = {zero, zero}, vL2[2] = {zero, zero}, uL3[2] = {zero, zero};
    C uh1[2] = {zero, zero}, vh1[2] = {zero, zero}, uh13[2] = {zero, zero};
    Rec gu0[2] = {}, gu1[2] = {}, gu2[2] = {}, gun[2] = {};     // u records of rows p, p-1, p-2; p+1
    Rec gv1[2] = {}, gv2[2] = {}, gv3[2] = {}, gvn[2] = {};     // v records of rows p-1, p-2, p-3; p

    const int ps = y0 - 3, pe = y1 + 2;
    {
        copy_row(ps, [&](int k) { return old_(k); });
        copy_row(ps + 1, [&](int k) { return old_(2 + k); });
        if (in1) {
            const size_t Rm = row(ps - 1) + gx, R0 = row(ps) + gx;
            vprev[0] = in[2][Rm];
            vprev[1] = in[3][Rm];
            pu[0] = in[0][R0];
            pu[1] = in[1][R0];
            if constexpr (SITE) {
                gu0[0] = rec[0][R0];
                gu0[1] = rec[1][R0];
                gv1[0] = rec[2][Rm];
                gv1[1] = rec[3][Rm];
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }

    for (int p = ps; p <= pe; ++p) {
        const bool more = p < pe;
        if (more) {
            if (in1) {
                const size_t Rn = row(p + 1) + gx;
                pun[0] = in[0][Rn];
                pun[1] = in[1][Rn];
                if constexpr (SITE) {
                    const size_t Rp = row(p) + gx;
                    gun[0] = rec[0][Rn];
                    gun[1] = rec[1][Rn];
                    gvn[0] = rec[2][Rp];
                    gvn[1] = rec[3][Rp];
                }
            }
            copy_row(p + 2, [&](int k) { return sStage + k * W; });
        }
        if constexpr (SITE) {
            kU0 = coef_rec(gu0[0]);
            kU1 = coef_rec(gu0[1]);
        }
        // level 1: u of row p after step 1
        if (in1) {
            const C *V0 = old_(0), *V1 = old_(1), *V0n = old_(2);
            vown[0] = V0[i];
            vown[1] = V1[i];
            const St2<C> s = stencil_u<C, R>(rx, ry, vown[0], V0[i - 1], V0n[i], vown[1], vprev[1], V1[i + 1]);
            u1L[0] = update(pu[0], s.s0, kU0);
            u1L[1] = update(pu[1], s.s1, kU1);
        }
        // level 2: v of row p-1 after step 1 (LDS: level 1 of row p-1)
        const int q2 = p - 1;
        const C *U0 = lev(0), *U1 = lev(1);
        if (in2 && q2 >= y0 - 3) {
            uh1[0] = U0[i];
            uh1[1] = U1[i];
        }
        if (in2 && q2 >= y0 - 2 && q2 <= y1 + 1) {
            if constexpr (SITE) {
                kV0 = coef_rec(gv1[0]);
                kV1 = coef_rec(gv1[1]);
            }
            const St2<C> s = stencil_v<C, R>(rx, ry, uh1[0], U0[i + 1], u1L[0], uh1[1], u1h2[1], U1[i - 1]);
            vL2[0] = update(vprev[0], s.s0, kV0);
            vL2[1] = update(vprev[1], s.s1, kV1);
        }
        // level 3: u of row p-2 after step 2 (LDS: level 2 of row p-2)
        const int q3 = p - 2;
        const C *V20 = lev(2), *V21 = lev(3);
        if (in2 && q3 >= y0 - 2) {
            vh1[0] = V20[i];
            vh1[1] = V21[i];
        }
        if (in2 && q3 >= y0 - 1 && q3 <= y1) {
            if constexpr (SITE) {
                kU0 = coef_rec(gu2[0]);
                kU1 = coef_rec(gu2[1]);
            }
            const St2<C> s = stencil_u<C, R>(rx, ry, vh1[0], V20[i - 1], vL2[0], vh1[1], v2h2[1], V21[i + 1]);
            uL3[0] = update(u1h2[0], s.s0, kU0);
            uL3[1] = update(u1h2[1], s.s1, kU1);
            if (in4 && q3 >= y0 && q3 < y1) {
                const size_t cell = row(q3) + gx;
                m2_st(out[0], cell, uL3[0]);
                m2_st(out[1], cell, uL3[1]);
            }
        }
        // level 4: v of row p-3 after step 2 on the strip (LDS: level 3 of row p-3)
        const int q4 = p - 3;
        const C *U30 = lev(4), *U31 = lev(5);
        if (in4 && q4 >= y0 - 1) {
            uh13[0] = U30[i];
            uh13[1] = U31[i];
        }
        if (in4 && q4 >= y0 && q4 < y1) {
            if constexpr (SITE) {
                kV0 = coef_rec(gv3[0]);
                kV1 = coef_rec(gv3[1]);
            }
            const St2<C> s = stencil_v<C, R>(rx, ry, uh13[0], U30[i + 1], uL3[0], uh13[1], u3h2, U31[i - 1]);
            const size_t cell = row(q4) + gx;
            m2_st(out[2], cell, update(v2h2[0], s.s0, kV0));
            m2_st(out[3], cell, update(v2h2[1], s.s1, kV1));
        }

        // all LDS reads of this row done, all copies landed
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (in1) {
            lev(0)[i] = u1L[0];
            lev(1)[i] = u1L[1];
            lev(2)[i] = vL2[0];
            lev(3)[i] = vL2[1];
            lev(4)[i] = uL3[0];
            lev(5)[i] = uL3[1];
        }
        if (more && x >= -2) {
            old_(0)[i] = old_(2)[i];
            old_(1)[i] = old_(3)[i];
            old_(2)[i] = sStage[i];
            old_(3)[i] = sStage[W + i];
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            u1h2[q] = uh1[q];
            v2h2[q] = vh1[q];
            vprev[q] = vown[q];
            pu[q] = pun[q];
            if constexpr (SITE) {
                gu2[q] = gu1[q];
                gu1[q] = gu0[q];
                gu0[q] = gun[q];
                gv3[q] = gv2[q];
                gv2[q] = gv1[q];
                gv1[q] = gvn[q];
            }
        }
        u3h2 = uh13[1];
        __syncthreads();
    }
}

}  // namespace dirac
