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
// The old C,D planes are staged in LDS by coalesced row loads (one plane ahead,
// software-prefetched into registers), so the ring needs no extra global reads.  A chunk [z0, z1) runs planes z0-1 .. z1 so that its
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

// Storage plane of plane index pl: periodic wrap, or in z-slab mode the plane
// counted from the first halo plane (reads reach at most zh planes beyond the
// interior).
template <typename R> __device__ __forceinline__ int zplane(const FusedArgs<R> &a, int pl) {
    return a.zh ? pl + a.zh : wrapn(pl, a.nz);
}

// SITE: 0 = V(z) tables, 1 = per-site records, 2 = per-site records with
// theta -> -theta (the reversed step's sequence).
template <typename R, int SITE>
__device__ __forceinline__ Coef<R> fcoef(const FusedArgs<R> &a, int arr, int cls, int pk, size_t idx) {
    if constexpr (SITE != 0) {
        return coef_site_at<R>(a.th[arr], idx, SITE == 2 ? (R)-1 : (R)1);
    } else {
        const R *e = a.tab + ((size_t)cls * (a.nz + 2 * a.zh) + pk) * 4;
        Coef<R> k;
        k.c1 = mk2(e[0], e[1]);
        k.c2 = mk2(e[2], e[3]);
        return k;
    }
}

// Load/store through a wave-uniform base pointer and a 32-bit per-lane byte
// offset (scalar-base addressing: one VGPR per offset instead of a 64-bit
// address per load).
template <typename C> __device__ __forceinline__ C ldo(const C *base, uint32_t boff) {
    return *(const C *)((const char *)base + boff);
}
template <typename C> __device__ __forceinline__ void sto(C *base, uint32_t boff, C v) {
    *(C *)((char *)base + boff) = v;
}

// CPT consecutive cells along x moved as one access (two complex64 = 16 bytes).
template <typename C, int CPT> struct Cells {
    C v[CPT];
};
// Streaming (nontemporal) accesses for data touched once per step: the own
// cells' A,B and every output.  Halo-shared C,D rows keep the normal policy.
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void nt_store(float2 *p, float2 v) { __builtin_nontemporal_store(nt_f2{v.x, v.y}, (nt_f2 *)p); }
__device__ __forceinline__ void nt_store(double2 *p, double2 v) { __builtin_nontemporal_store(nt_d2{v.x, v.y}, (nt_d2 *)p); }
__device__ __forceinline__ float2 nt_load(const float2 *p) {
    nt_f2 t = __builtin_nontemporal_load((const nt_f2 *)p);
    return make_float2(t.x, t.y);
}
__device__ __forceinline__ double2 nt_load(const double2 *p) {
    nt_d2 t = __builtin_nontemporal_load((const nt_d2 *)p);
    return make_double2(t.x, t.y);
}

template <typename C, int CPT> __device__ __forceinline__ Cells<C, CPT> ldv(const C *base, uint32_t boff) {
    Cells<C, CPT> r;
    if constexpr (CPT == 1) {
        r.v[0] = ldo(base, boff);
    } else {
        const float4 q = *(const float4 *)((const char *)base + boff);
        r.v[0] = mk2(q.x, q.y);
        r.v[1] = mk2(q.z, q.w);
    }
    return r;
}
// streaming load of the own cells
template <typename C, int CPT> __device__ __forceinline__ Cells<C, CPT> ldv_nt(const C *base, uint32_t boff) {
    Cells<C, CPT> r;
    if constexpr (CPT == 1) {
        r.v[0] = nt_load((const C *)((const char *)base + boff));
    } else {
        const nt_f4 q = __builtin_nontemporal_load((const nt_f4 *)((const char *)base + boff));
        r.v[0] = mk2(q.x, q.y);
        r.v[1] = mk2(q.z, q.w);
    }
    return r;
}
template <typename C, int CPT> __device__ __forceinline__ void stv(C *base, uint32_t boff, const Cells<C, CPT> &c) {
    if constexpr (CPT == 1) {
        nt_store((C *)((char *)base + boff), c.v[0]);
    } else {
        __builtin_nontemporal_store(nt_f4{c.v[0].x, c.v[0].y, c.v[1].x, c.v[1].y}, (nt_f4 *)((char *)base + boff));
    }
}
template <typename C, int CPT> __device__ __forceinline__ Cells<C, CPT> lds_v(const C *p) {
    Cells<C, CPT> r;
    if constexpr (CPT == 1) {
        r.v[0] = p[0];
    } else {
        const float4 q = *(const float4 *)p;
        r.v[0] = mk2(q.x, q.y);
        r.v[1] = mk2(q.z, q.w);
    }
    return r;
}
template <typename C, int CPT> __device__ __forceinline__ void lds_st(C *p, const Cells<C, CPT> &c) {
    if constexpr (CPT == 1) {
        p[0] = c.v[0];
    } else {
        *(float4 *)p = make_float4(c.v[0].x, c.v[0].y, c.v[1].x, c.v[1].y);
    }
}

// Asynchronous global -> LDS copy of LB bytes per lane: lane l's bytes land at
// lds_wave_base + l * LB (lds_wave_base must be the same for the whole wave).
// Completion is tracked by the vector-memory counter (wait vmcnt(0), then a
// barrier, before the LDS is read).
template <int LB> __device__ __forceinline__ void g2lds(const void *gsrc, void *lds_wave_base) {
    static_assert(LB == 16 || LB == 4, "copy width");
    if constexpr (LB == 16)
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)gsrc,
                                         (__attribute__((address_space(3))) void *)lds_wave_base, 16, 0, 0);
    else
        __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)gsrc,
                                         (__attribute__((address_space(3))) void *)lds_wave_base, 4, 0, 0);
}

// Plane-by-plane schedule of one workgroup (tile (64 CPT) x TY cells, chunk
// [z0, z1) of planes; lane l of row y owns the CPT cells x = l CPT + c):
//   iteration p:  (the old C(p) and D(p+1) regions -- tile plus a one-cell
//                 ring, corners included -- are already in LDS)
//                 start the global->LDS copies of C(p+1), D(p+2) and register
//                 loads of the next A,B; new A,B(p) for the tile and for the
//                 ring cells the C,D stencils need (Eqs. ss1, ss2); new
//                 C,D(p-1) for the tile from the new A,B(p-1) in LDS and
//                 registers (Eqs. ss3, ss4); barrier; new A,B(p) into LDS;
//                 wait for the copies; barrier.
// Ring cells (the new A,B the tile's C,D stencils read outside it): left
// column x = -1: A1, B0; right column x = w: A0, B1; bottom row y = -1: A1,
// B1; top row y = h: A0, B0.  LDS holds C of 2 planes (2 arrays each), D of
// 3 planes (2 arrays each) and the new A,B(p-1) (4 arrays), each a
// (64 CPT + 4) x (TY + 2) region with x stored at index x + 2.  The interior
// rows of the regions are copied global -> LDS without passing through
// registers; the two halo columns go through registers.  Registers carry each
// cell's old C(p-1), D(p-1) and new B(p-1), B(p-2) along the march.
// NORM: also accumulate, per workgroup, the conserved functional of the new
// state in its C,D-summed form E_r = sum |X|^2 + Re sum_{C,D} conj(Y) S_Y(A,B)
// (Lemma of Sect. 2 after summation by parts; S_Y(A,B) is exactly the stencil
// the C,D update evaluates) and the plain norm, into a.npart.
template <typename R, int SITE, int TY, int CPT, bool NORM>
__global__ __launch_bounds__(kTX *TY, sizeof(R) * CPT == 4 ? 3 : 2) void k3_fused(FusedArgs<R> a) {
    using C = cx<R>;
    using V = Cells<C, CPT>;
    constexpr int NT = kTX * TY, TXC = kTX * CPT;
    constexpr int LW = TXC + 4, LN = LW * (TY + 2);
    constexpr int LB = sizeof(C) * CPT >= 16 ? 16 : 4;         // bytes per lane per copy
    constexpr int NI = (TXC * (int)sizeof(C)) / (kTX * LB);     // copies per region row
    constexpr int NROW = 4 * (TY + 2);                          // C0, C1, D0, D1 rows
    static_assert(2 * (TY + 2) <= NT, "halo slots");
    __shared__ __align__(16) C sC[2][2][LN];
    __shared__ __align__(16) C sD[3][2][LN];
    __shared__ __align__(16) C sAB[4][LN];

    int L = logical_block();
    const int tx = L % a.ntx;
    L /= a.ntx;
    const int ty = L % a.nty;
    const int zc = L / a.nty;
    const int x0 = tx * TXC, y0 = ty * TY;
    const int w = min(TXC, a.nx - x0), h = min(TY, a.ny - y0);
    const int z0 = zc * a.zchunk, z1 = min(a.nz, z0 + a.zchunk);
    const int t = threadIdx.x;
    const int lane = t & (kTX - 1), y = t / kTX;
    const int xl = lane * CPT;                       // first cell of this lane
    const bool own = xl < w && y < h;                // w is a multiple of CPT
    const size_t plane = (size_t)a.nx * a.ny;
    constexpr uint32_t CS = sizeof(C);
    const uint32_t nxu = (uint32_t)a.nx;
    const uint32_t rc = ((uint32_t)(y0 + (own ? y : 0)) * nxu + (uint32_t)(x0 + (own ? xl : 0))) * CS;
    const int li = (y + 1) * LW + xl + 2;

    // region halo-column slots (x = -1 and x = w of rows -1..h), through registers
    const bool sv = t < 2 * (TY + 2) && (t / 2 - 1) <= h;
    const int sx = (t & 1) ? w : -1, sy = t / 2 - 1;
    const int sl = sv ? (sy + 1) * LW + sx + 2 : 0;
    const uint32_t so = ((uint32_t)wrapn(y0 + sy, a.ny) * nxu + (uint32_t)wrapn(x0 + sx, a.nx)) * CS;

    // ring unit of this thread: columns (one cell) then rows (CPT cells)
    //   kind 0 left (A1, B0), 1 right (A0, B1), 2 bottom (A1, B1), 3 top (A0, B0)
    int rk = -1, rxc = 0, ryc = 0;
    if (t < h) { rk = 0; rxc = -1; ryc = t; }
    else if (t < 2 * h) { rk = 1; rxc = w; ryc = t - h; }
    else if (t < 2 * h + w / CPT) { rk = 2; rxc = (t - 2 * h) * CPT; ryc = -1; }
    else if (t < 2 * h + 2 * (w / CPT)) { rk = 3; rxc = (t - 2 * h - w / CPT) * CPT; ryc = h; }
    const bool ring = rk >= 0;
    const int rnc = rk >= 2 ? CPT : 1;               // cells in this unit
    const bool qa0 = rk == 1 || rk == 3, qb2 = rk == 0 || rk == 3;
    const int hli = (ryc + 1) * LW + rxc + 2;
    const uint32_t ho = ((uint32_t)wrapn(y0 + ryc, a.ny) * nxu + (uint32_t)wrapn(x0 + rxc, a.nx)) * CS;
    C *ringA_lds = qa0 ? sAB[0] : sAB[1];
    C *ringB_lds = qb2 ? sAB[2] : sAB[3];

    const C *in[8];
    C *out[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        in[q] = (const C *)a.in[q];
        out[q] = (C *)a.out[q];
    }
    const R rx = a.rx, ry = a.ry, rz = a.rz;
    const C zero = mk2((R)0, (R)0);
    V vz;
#pragma unroll
    for (int c = 0; c < CPT; ++c) vz.v[c] = zero;
    double nrm[2] = {0.0, 0.0};

    // Global -> LDS copies of the interior rows of C(pl) (slot pl & 1) and
    // D(pl+1) (slot (pl+1) mod 3); wave y takes rows y, y + TY, ...
    auto copy_rows = [&](int pl) {
        const size_t Pc = (size_t)zplane(a, pl) * plane, Pd = (size_t)zplane(a, pl + 1) * plane;
        const int cs = pl & 1, ds = wrapn(pl + 1, 3);
        for (int item = y; item < NROW; item += TY) {
            const int arr = item / (TY + 2), ry0 = item % (TY + 2) - 1;
            if (ry0 > h) continue;
            const C *src = arr == 0 ? in[4] + Pc : arr == 1 ? in[5] + Pc : arr == 2 ? in[6] + Pd : in[7] + Pd;
            C *dst = (arr < 2 ? sC[cs][arr] : sD[ds][arr - 2]) + (ry0 + 1) * LW + 2;
            const char *row = (const char *)(src + (size_t)wrapn(y0 + ry0, a.ny) * a.nx + x0);
#pragma unroll
            for (int j = 0; j < NI; ++j) {
                const int b = (j * kTX + lane) * LB;             // byte within the row
                if (b < w * (int)CS) g2lds<LB>(row + b, (char *)dst + j * kTX * LB);
            }
        }
    };
    C psc[2] = {zero, zero}, psd[2] = {zero, zero};
    V pa[4] = {vz, vz, vz, vz}, pra = vz, prb = vz;
    auto ring_load = [&](const C *base, uint32_t off) -> V {
        if (rnc == CPT) return ldv<C, CPT>(base, off);
        V r = vz;
        r.v[0] = ldo(base, off);
        return r;
    };
    // register loads for plane pl: halo columns of C(pl), D(pl+1); own and ring A,B(pl)
    auto load_regs = [&](int pl) {
        const size_t P = (size_t)zplane(a, pl) * plane, Pp = (size_t)zplane(a, pl + 1) * plane;
        if (sv) {
            psc[0] = ldo(in[4] + P, so);
            psc[1] = ldo(in[5] + P, so);
            psd[0] = ldo(in[6] + Pp, so);
            psd[1] = ldo(in[7] + Pp, so);
        }
        if (own) {
#pragma unroll
            for (int q = 0; q < 4; ++q) pa[q] = ldv_nt<C, CPT>(in[q] + P, rc);
        }
        if (ring) {
            pra = qa0 ? ring_load(in[0] + P, ho) : ring_load(in[1] + P, ho);
            prb = qb2 ? ring_load(in[2] + P, ho) : ring_load(in[3] + P, ho);
        }
    };
    auto store_halo = [&](int pl) {
        if (sv) {
            sC[pl & 1][0][sl] = psc[0];
            sC[pl & 1][1][sl] = psc[1];
            sD[wrapn(pl + 1, 3)][0][sl] = psd[0];
            sD[wrapn(pl + 1, 3)][1][sl] = psd[1];
        }
    };

    // march windows
    V cm0 = vz, cm1 = vz, dm0 = vz, dm1 = vz, bm0 = vz, bm1 = vz, bmm0 = vz, bmm1 = vz;
    V rcm = vz;   // old C(p-1) at the ring cells (C0 for A0 ring cells, C1 for A1)
    {
        // D(z0-1) region (slot (z0-1) mod 3), C(z0-2) at the own and ring cells
        const int dsl = wrapn(z0 - 1, 3);
        const size_t Pd = (size_t)zplane(a, z0 - 1) * plane, Pc = (size_t)zplane(a, z0 - 2) * plane;
        for (int item = y; item < 2 * (TY + 2); item += TY) {
            const int arr = item / (TY + 2), ry0 = item % (TY + 2) - 1;
            if (ry0 > h) continue;
            C *dst = sD[dsl][arr] + (ry0 + 1) * LW + 2;
            const char *row = (const char *)((arr == 0 ? in[6] : in[7]) + Pd + (size_t)wrapn(y0 + ry0, a.ny) * a.nx + x0);
#pragma unroll
            for (int j = 0; j < NI; ++j) {
                const int b = (j * kTX + lane) * LB;
                if (b < w * (int)CS) g2lds<LB>(row + b, (char *)dst + j * kTX * LB);
            }
        }
        if (sv) {
            sD[dsl][0][sl] = ldo(in[6] + Pd, so);
            sD[dsl][1][sl] = ldo(in[7] + Pd, so);
        }
        if (own) {
            cm0 = ldv<C, CPT>(in[4] + Pc, rc);
            cm1 = ldv<C, CPT>(in[5] + Pc, rc);
        }
        if (ring) rcm = qa0 ? ring_load(in[4] + Pc, ho) : ring_load(in[5] + Pc, ho);
        copy_rows(z0 - 1);
        load_regs(z0 - 1);
        store_halo(z0 - 1);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }

    for (int p = z0 - 1; p <= z1; ++p) {
        const int cs = p & 1;
        const int ds = wrapn(p, 3), dsn = wrapn(p + 1, 3);
        const int pk = zplane(a, p);
        const size_t P = (size_t)pk * plane;
        const V a0 = pa[0], a1 = pa[1], b0 = pa[2], b1 = pa[3], ra = pra, rb = prb;
        if (p < z1) {
            copy_rows(p + 1);
            load_regs(p + 1);
        }

        const C *C0 = sC[cs][0], *C1 = sC[cs][1];
        const C *D0 = sD[ds][0], *D1 = sD[ds][1], *D0n = sD[dsn][0], *D1n = sD[dsn][1];
        V nA0 = vz, nA1 = vz, nB0 = vz, nB1 = vz, c0v = vz, c1v = vz, d0v = vz, d1v = vz;
        if (own) {
            c0v = lds_v<C, CPT>(&C0[li]);
            c1v = lds_v<C, CPT>(&C1[li]);
            d0v = lds_v<C, CPT>(&D0[li]);
            d1v = lds_v<C, CPT>(&D1[li]);
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int e = li + c;
                St3<C> s = stencil_ab<C, R>(rx, ry, rz,
                                            c0v.v[c], cm0.v[c], C0[e + 1], C0[e + LW],
                                            c1v.v[c], cm1.v[c], C1[e - LW], C1[e - 1],
                                            d0v.v[c], D0[e - 1], D0[e + LW], D0n[e],
                                            d1v.v[c], D1[e - LW], D1[e + 1], D1n[e]);
                const size_t g = P + rc / CS + c;
                nA0.v[c] = update(a0.v[c], s.s0, fcoef<R, SITE>(a, 0, 0, pk, g));
                nA1.v[c] = update(a1.v[c], s.s1, fcoef<R, SITE>(a, 1, 0, pk, g));
                nB0.v[c] = update(b0.v[c], s.s2, fcoef<R, SITE>(a, 2, 1, pk, g));
                nB1.v[c] = update(b1.v[c], s.s3, fcoef<R, SITE>(a, 3, 1, pk, g));
            }
        }
        V ringA = vz, ringB = vz;
        if (ring) {
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                if (c >= rnc) break;
                const int e = hli + c;
                C sa, sb;
                // the same expressions as the owners' (stencil_ab), hence the same bits
                if (qa0)   // S_A0 = rz(C0 - C0[k-1]) + rx(D0 - D0[i-1]) - i ry(D1 - D1[j-1])
                    sa = sterm3(rz, csub(C0[e], rcm.v[c]), rx, csub(D0[e], D0[e - 1]), -ry, csub(D1[e], D1[e - LW]));
                else       // S_A1 = rz(C1 - C1[k-1]) + rx(D1[i+1] - D1) - i ry(D0[j+1] - D0)
                    sa = sterm3(rz, csub(C1[e], rcm.v[c]), rx, csub(D1[e + 1], D1[e]), -ry, csub(D0[e + LW], D0[e]));
                if (qb2)   // S_B0 = -rz(D0[k+1] - D0) + rx(C0[i+1] - C0) + i ry(C1 - C1[j-1])
                    sb = sterm3(-rz, csub(D0n[e], D0[e]), rx, csub(C0[e + 1], C0[e]), ry, csub(C1[e], C1[e - LW]));
                else       // S_B1 = -rz(D1[k+1] - D1) + rx(C1 - C1[i-1]) + i ry(C0[j+1] - C0)
                    sb = sterm3(-rz, csub(D1n[e], D1[e]), rx, csub(C1[e], C1[e - 1]), ry, csub(C0[e + LW], C0[e]));
                const size_t g = P + ho / CS + c;
                ringA.v[c] = update(ra.v[c], sa, qa0 ? fcoef<R, SITE>(a, 0, 0, pk, g) : fcoef<R, SITE>(a, 1, 0, pk, g));
                ringB.v[c] = update(rb.v[c], sb, qb2 ? fcoef<R, SITE>(a, 2, 1, pk, g) : fcoef<R, SITE>(a, 3, 1, pk, g));
                rcm.v[c] = qa0 ? C0[e] : C1[e];
            }
        }
        if (own && p >= z0 + 1) {
            // C,D of plane k = p-1 from the new A,B of planes p-1 (LDS), p and p-2 (registers)
            const int kq = zplane(a, p - 1);
            const size_t Pm = (size_t)kq * plane;
            const C *A0 = sAB[0], *A1 = sAB[1], *B0 = sAB[2], *B1 = sAB[3];
            V o4, o5, o6, o7;
            St3<C> sv[CPT];
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int e = li + c;
                St3<C> s = stencil_cd<C, R>(rx, ry, rz,
                                            A0[e], nA0.v[c], A0[e + 1], A0[e + LW],
                                            A1[e], nA1.v[c], A1[e - 1], A1[e - LW],
                                            B0[e], bmm0.v[c], B0[e - 1], B0[e + LW],
                                            B1[e], bmm1.v[c], B1[e + 1], B1[e - LW]);
                const size_t g = Pm + rc / CS + c;
                o4.v[c] = update(cm0.v[c], s.s0, fcoef<R, SITE>(a, 4, 2, kq, g));
                o5.v[c] = update(cm1.v[c], s.s1, fcoef<R, SITE>(a, 5, 2, kq, g));
                o6.v[c] = update(dm0.v[c], s.s2, fcoef<R, SITE>(a, 6, 3, kq, g));
                o7.v[c] = update(dm1.v[c], s.s3, fcoef<R, SITE>(a, 7, 3, kq, g));
                if constexpr (NORM) sv[c] = s;
            }
            stv<C, CPT>(out[4] + Pm, rc, o4);
            stv<C, CPT>(out[5] + Pm, rc, o5);
            stv<C, CPT>(out[6] + Pm, rc, o6);
            stv<C, CPT>(out[7] + Pm, rc, o7);
            if constexpr (NORM) {
                // conj(Y) S_Y(A,B) with the S the update used (FP64 in the
                // complex128 form; FP32-evaluated in complex64), summed in FP64
                auto D2 = [](C v) { return make_double2((double)v.x, (double)v.y); };
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const double2 y4 = D2(o4.v[c]), y5 = D2(o5.v[c]), y6 = D2(o6.v[c]), y7 = D2(o7.v[c]);
                    const double2 s4 = D2(sv[c].s0), s5 = D2(sv[c].s1), s6 = D2(sv[c].s2), s7 = D2(sv[c].s3);
                    const double pp = y4.x * y4.x + y4.y * y4.y + y5.x * y5.x + y5.y * y5.y + y6.x * y6.x +
                                      y6.y * y6.y + y7.x * y7.x + y7.y * y7.y;
                    nrm[0] += pp + (y4.x * s4.x + y4.y * s4.y) + (y5.x * s5.x + y5.y * s5.y) +
                              (y6.x * s6.x + y6.y * s6.y) + (y7.x * s7.x + y7.y * s7.y);
                    nrm[1] += pp;
                }
            }
        }
        if (own && p >= z0 && p < z1) {
            stv<C, CPT>(out[0] + P, rc, nA0);
            stv<C, CPT>(out[1] + P, rc, nA1);
            stv<C, CPT>(out[2] + P, rc, nB0);
            stv<C, CPT>(out[3] + P, rc, nB1);
            if constexpr (NORM) {
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    double pp = 0.0;
                    const C q4[4] = {nA0.v[c], nA1.v[c], nB0.v[c], nB1.v[c]};
#pragma unroll
                    for (int u = 0; u < 4; ++u) pp += (double)q4[u].x * (double)q4[u].x + (double)q4[u].y * (double)q4[u].y;
                    nrm[0] += pp;
                    nrm[1] += pp;
                }
            }
        }
        __syncthreads();
        if (own) {
            lds_st<C, CPT>(&sAB[0][li], nA0);
            lds_st<C, CPT>(&sAB[1][li], nA1);
            lds_st<C, CPT>(&sAB[2][li], nB0);
            lds_st<C, CPT>(&sAB[3][li], nB1);
        }
        if (ring) {
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                if (c >= rnc) break;
                ringA_lds[hli + c] = ringA.v[c];
                ringB_lds[hli + c] = ringB.v[c];
            }
        }
        if (p < z1) store_halo(p + 1);
        cm0 = c0v;
        cm1 = c1v;
        dm0 = d0v;
        dm1 = d1v;
        bmm0 = bm0;
        bmm1 = bm1;
        bm0 = nB0;
        bm1 = nB1;
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
    if constexpr (NORM) {
        // reuse the C region of LDS for the block reduction (all reads are done)
        double *red = (double *)&sC[0][0][0];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) nrm[q] += __shfl_xor(nrm[q], off, 64);
        }
        if (lane == 0) {
            red[2 * y] = nrm[0];
            red[2 * y + 1] = nrm[1];
        }
        __syncthreads();
        if (t == 0) {
            double s0 = 0.0, s1 = 0.0;
            for (int q = 0; q < TY; ++q) {
                s0 += red[2 * q];
                s1 += red[2 * q + 1];
            }
            a.npart[2 * blockIdx.x] = s0;
            a.npart[2 * blockIdx.x + 1] = s1;
        }
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

template <typename R>
hipError_t launch_fused3(const FusedArgs<R> &a0, bool site, int tile_y, hipStream_t s, int *nblocks_out) {
    FusedArgs<R> a = a0;
    const int TY = tile_y > 0 ? tile_y : 8;
    if (TY != 4 && TY != 8) return hipErrorInvalidValue;
    // complex64 with an even row length: two cells per lane (16-byte accesses)
    const int CPT = (sizeof(R) == 4 && (a.nx % 2) == 0) ? 2 : 1;
    a.ntx = (a.nx + kTX * CPT - 1) / (kTX * CPT);
    a.nty = (a.ny + TY - 1) / TY;
    const int64_t tiles = (int64_t)a.ntx * a.nty;
    if (a.zchunk <= 0) {
        const int nzc = pick_chunks(tiles, a.nz, 3);
        a.zchunk = (a.nz + nzc - 1) / nzc;
    }
    a.nzc = (a.nz + a.zchunk - 1) / a.zchunk;
    const int64_t nblk = tiles * a.nzc;
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    if (nblocks_out) *nblocks_out = (int)nblk;
    const bool norm = a.npart != nullptr;
    if (norm && nblk > a.npart_cap) return hipErrorInvalidValue;   // caller falls back
    dim3 g((unsigned)nblk), b(kTX * TY);
    if (norm && site && a.rev) return hipErrorInvalidValue;     // no functional on reversed steps
#define L3(T, P)                                                                              \
    if (TY == T && CPT == P) {                                                                \
        if (norm) {                                                                           \
            if (site) hipLaunchKernelGGL((k3_fused<R, 1, T, P, true>), g, b, 0, s, a);         \
            else hipLaunchKernelGGL((k3_fused<R, 0, T, P, true>), g, b, 0, s, a);              \
        } else {                                                                              \
            if (site && a.rev) hipLaunchKernelGGL((k3_fused<R, 2, T, P, false>), g, b, 0, s, a); \
            else if (site) hipLaunchKernelGGL((k3_fused<R, 1, T, P, false>), g, b, 0, s, a);  \
            else hipLaunchKernelGGL((k3_fused<R, 0, T, P, false>), g, b, 0, s, a);             \
        }                                                                                     \
    }
    L3(4, 1) L3(8, 1)
    if constexpr (sizeof(R) == 4) {
        L3(4, 2) L3(8, 2)
    }
#undef L3
    return hipGetLastError();
}

template <typename R> hipError_t launch_fused2(const FusedArgs<R> &a0, bool site, hipStream_t s) {
    FusedArgs<R> a = a0;
    // small lattices (cache-resident, latency-bound): 64-wide strips and the
    // shortest chunks that keep about 2048 workgroups (one row each up to
    // 256^2: 4.9 us per step at 128^2 against 8.3 with four-row chunks; two
    // rows at 510^2)
    const bool small = (int64_t)a.nx * a.ny < ((int64_t)1 << 18);
    const int TXB = small ? 64 : 128;
    a.ntx = (a.nx + TXB - 1) / TXB;
    a.nty = 1;
    if (a.zchunk <= 0) {
        const int nc = default_chunks(a.ntx, a.ny, small ? 2048 : 4096);
        a.zchunk = (a.ny + nc - 1) / nc;
        if (!small && a.zchunk < 8 && a.ny >= 8) a.zchunk = 8;
    }
    a.nzc = (a.ny + a.zchunk - 1) / a.zchunk;
    const int64_t nblk = (int64_t)a.ntx * a.nzc;
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    if (TXB == 64) {
        if (site) hipLaunchKernelGGL((k2_fused<R, true, 64>), dim3((unsigned)nblk), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k2_fused<R, false, 64>), dim3((unsigned)nblk), dim3(64), 0, s, a);
    } else {
        if (site) hipLaunchKernelGGL((k2_fused<R, true, 128>), dim3((unsigned)nblk), dim3(128), 0, s, a);
        else hipLaunchKernelGGL((k2_fused<R, false, 128>), dim3((unsigned)nblk), dim3(128), 0, s, a);
    }
    return hipGetLastError();
}

template hipError_t launch_fused3<float>(const FusedArgs<float> &, bool, int, hipStream_t, int *);
template hipError_t launch_fused3<double>(const FusedArgs<double> &, bool, int, hipStream_t, int *);
template hipError_t launch_fused2<float>(const FusedArgs<float> &, bool, hipStream_t);
template hipError_t launch_fused2<double>(const FusedArgs<double> &, bool, hipStream_t);

}  // namespace dirac
