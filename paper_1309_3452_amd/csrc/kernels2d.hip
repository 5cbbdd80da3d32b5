// (2+1)D kernels: split half-steps (in place), reductions, adjoint seed.
// Arrays u0 (i,j), u1 (i+1/2,j+1/2) on sheet n-1/2 and v0 (i+1/2,j),
// v1 (i,j+1/2) on sheet n (Sect. 3).  Stencils in stencil3.h.
#include "device.h"
#include "internal.h"
#include "stencil3.h"
#include "ntstore.h"

namespace dirac {

namespace {

constexpr int kTX = 64, kTY = 4;

template <typename R, bool SITE>
__device__ __forceinline__ Coef<R> coef2(const HalfArgs<R> &a, int arr, int q, size_t c) {
    if constexpr (SITE) {
        return coef_site_at<R>(a.th[arr], c, a.tsgn);
    } else {
        const R *e = a.tab + (size_t)q * a.nz * 4;    // plane 0 of class q
        Coef<R> k;
        k.c1 = mk2(e[0], e[1]);
        k.c2 = mk2(e[2], e[3]);
        return k;
    }
}

// WHICH == 0: u from v; WHICH == 1: v from the new u.
template <typename R, bool SITE, int WHICH, bool ZB>
__global__ __launch_bounds__(256) void k2_half(HalfArgs<R> a) {
    using C = cx<R>;
    const int nbx = (a.nx + kTX - 1) / kTX;
    const int bx = blockIdx.x % nbx, by = blockIdx.x / nbx;
    const int i = bx * kTX + (threadIdx.x & (kTX - 1));
    const int j = by * kTY + (threadIdx.x / kTX);
    if (i >= a.nx || j >= a.ny) return;
    const size_t row = (size_t)j * a.nx;
    const size_t c = row + i;
    const size_t xm = row + wrap_dec(i, a.nx), xp = row + wrap_inc(i, a.nx);
    const size_t ym = (size_t)wrap_dec(j, a.ny) * a.nx + i, yp = (size_t)wrap_inc(j, a.ny) * a.nx + i;
    C *f[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) f[q] = (C *)a.f[q];
    // zero values outside the lattice (ZB): a neighbour across an edge reads as zero
    const bool oxm = !ZB || i > 0, oxp = !ZB || i < a.nx - 1, oym = !ZB || j > 0, oyp = !ZB || j < a.ny - 1;
    if constexpr (WHICH == 0) {
        St2<C> s = stencil_u<C, R>(a.rx, a.ry, f[2][c], ld_or0(f[2], xm, oxm), ld_or0(f[2], yp, oyp), f[3][c],
                                   ld_or0(f[3], ym, oym), ld_or0(f[3], xp, oxp));
        // old values and coefficients before the first store: a load issued after a
        // store would wait for it too
        const C o0 = f[0][c], o1 = f[1][c];
        const Coef<R> k0 = coef2<R, SITE>(a, 0, 0, c), k1 = coef2<R, SITE>(a, 1, 0, c);
        st_nt(&f[0][c], update(o0, s.s0, k0));
        st_nt(&f[1][c], update(o1, s.s1, k1));
    } else {
        St2<C> s = stencil_v<C, R>(a.rx, a.ry, f[0][c], ld_or0(f[0], xp, oxp), ld_or0(f[0], yp, oyp), f[1][c],
                                   ld_or0(f[1], ym, oym), ld_or0(f[1], xm, oxm));
        // old values and coefficients before the first store: a load issued after a
        // store would wait for it too
        const C o2 = f[2][c], o3 = f[3][c];
        const Coef<R> k2 = coef2<R, SITE>(a, 2, 3, c), k3 = coef2<R, SITE>(a, 3, 3, c);
        st_nt(&f[2][c], update(o2, s.s0, k2));
        st_nt(&f[3][c], update(o3, s.s1, k3));
    }
}

__device__ __forceinline__ double2 to_d(double2 v) { return v; }
__device__ __forceinline__ double2 to_d(float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ __forceinline__ double re_conj_mul(double2 x, double2 s) { return x.x * s.x + x.y * s.y; }
__device__ __forceinline__ double abs2(double2 x) { return x.x * x.x + x.y * x.y; }

// E_r = ||u||^2 + ||v||^2 - Re sum_u conj(u) S_u(v)  (= ... + Re sum_v conj(v) S_v(u))
template <typename R, bool ZB>
__global__ __launch_bounds__(kReduceThreads) void k2_norm(ReduceArgs<R> a) {
    using C = cx<R>;
    __shared__ double lds[kNormVals * 16];
    const C *f[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) f[q] = (const C *)a.f[q];
    const double rx = a.rx, ry = a.ry;
    double v[kNormVals] = {0.0, 0.0, 0.0};
    const int64_t ncell = (int64_t)a.nx * a.ny;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ncell;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(t / a.nx), i = (int)(t - (int64_t)j * a.nx);
        const size_t row = (size_t)j * a.nx, c = row + i;
        const size_t xm = row + wrap_dec(i, a.nx), xp = row + wrap_inc(i, a.nx);
        const size_t ym = (size_t)wrap_dec(j, a.ny) * a.nx + i, yp = (size_t)wrap_inc(j, a.ny) * a.nx + i;
        double2 x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = to_d(f[q][c]);
        const bool oxm = !ZB || i > 0, oxp = !ZB || i < a.nx - 1, oym = !ZB || j > 0, oyp = !ZB || j < a.ny - 1;
        St2<double2> su = stencil_u<double2, double>(rx, ry, x[2], to_d(ld_or0(f[2], xm, oxm)),
                                                      to_d(ld_or0(f[2], yp, oyp)), x[3], to_d(ld_or0(f[3], ym, oym)),
                                                      to_d(ld_or0(f[3], xp, oxp)));
        St2<double2> sv = stencil_v<double2, double>(rx, ry, x[0], to_d(ld_or0(f[0], xp, oxp)),
                                                      to_d(ld_or0(f[0], yp, oyp)), x[1], to_d(ld_or0(f[1], ym, oym)),
                                                      to_d(ld_or0(f[1], xm, oxm)));
        v[0] -= re_conj_mul(x[0], su.s0) + re_conj_mul(x[1], su.s1);
        v[1] += re_conj_mul(x[2], sv.s0) + re_conj_mul(x[3], sv.s1);
        const double p = abs2(x[0]) + abs2(x[1]) + abs2(x[2]) + abs2(x[3]);
        v[0] += p;
        v[1] += p;
        v[2] += p;
    }
    block_sum<kNormVals>(v, lds);
    if (threadIdx.x == 0)
        for (int q = 0; q < kNormVals; ++q) a.partial[(size_t)blockIdx.x * kNormVals + q] = v[q];
}

__constant__ float kOff2[4][2] = {{0.f, 0.f}, {.5f, .5f}, {.5f, 0.f}, {0.f, .5f}};

template <typename R>
__global__ __launch_bounds__(kReduceThreads) void k2_obs(ReduceArgs<R> a) {
    using C = cx<R>;
    __shared__ double lds[kObsVals * 16];
    double v[kObsVals];
#pragma unroll
    for (int q = 0; q < kObsVals; ++q) v[q] = 0.0;
    const int64_t ncell = (int64_t)a.nx * a.ny;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ncell;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(t / a.nx), i = (int)(t - (int64_t)j * a.nx);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double p = abs2(to_d(((const C *)a.f[q])[t]));
            double x = (double)i + (double)kOff2[q][0];
            double y = (double)j + (double)kOff2[q][1];
            if (x >= a.z0) v[0] += p;
            v[1] += x * p;
            v[2] += y * p;
            v[3] += p;
            v[4 + q / 2] += p;
        }
    }
    block_sum<kObsVals>(v, lds);
    if (threadIdx.x == 0)
        for (int q = 0; q < kObsVals; ++q) a.partial[(size_t)blockIdx.x * kObsVals + q] = v[q];
}

template <typename R>
__global__ __launch_bounds__(256) void k2_seed(ReduceArgs<R> a, CPtr8 lam) {
    using C = cx<R>;
    const int64_t ncell = (int64_t)a.nx * a.ny;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < ncell;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(t / a.nx), i = (int)(t - (int64_t)j * a.nx);
        (void)j;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double x = (double)i + (double)kOff2[q][0];
            C v = ((const C *)a.f[q])[t];
            R w = (x >= a.z0) ? (R)2 : (R)0;
            ((C *)lam.p[q])[t] = mk2(w * v.x, w * v.y);
        }
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
hipError_t launch_half2(const HalfArgs<R> &a, int which, bool site, hipStream_t s) {
    const int64_t nblk = (int64_t)((a.nx + kTX - 1) / kTX) * ((a.ny + kTY - 1) / kTY);
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    dim3 g((unsigned)nblk), b(kTX * kTY);
#define H2(ZB)                                                                          \
    if (which == 0) {                                                                   \
        if (site) hipLaunchKernelGGL((k2_half<R, true, 0, ZB>), g, b, 0, s, a);         \
        else hipLaunchKernelGGL((k2_half<R, false, 0, ZB>), g, b, 0, s, a);             \
    } else {                                                                            \
        if (site) hipLaunchKernelGGL((k2_half<R, true, 1, ZB>), g, b, 0, s, a);         \
        else hipLaunchKernelGGL((k2_half<R, false, 1, ZB>), g, b, 0, s, a);             \
    }
    if (a.zbc) {
        H2(true)
    } else {
        H2(false)
    }
#undef H2
    return hipGetLastError();
}

template <typename R> hipError_t launch_norm2(const ReduceArgs<R> &a, hipStream_t s) {
    if (a.zbc) hipLaunchKernelGGL((k2_norm<R, true>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, a);
    else hipLaunchKernelGGL((k2_norm<R, false>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, a);
    return hipGetLastError();
}

template <typename R> hipError_t launch_obs2(const ReduceArgs<R> &a, hipStream_t s) {
    hipLaunchKernelGGL((k2_obs<R>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s, a);
    return hipGetLastError();
}

template <typename R> hipError_t launch_seed2(const ReduceArgs<R> &a, void *const lam[8], hipStream_t s) {
    CPtr8 l;
    for (int q = 0; q < 8; ++q) l.p[q] = q < 4 ? lam[q] : nullptr;
    const int64_t n = (int64_t)a.nx * a.ny;
    hipLaunchKernelGGL((k2_seed<R>), dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, a, l);
    return hipGetLastError();
}

#define INST(R)                                                                          \
    template hipError_t launch_half2<R>(const HalfArgs<R> &, int, bool, hipStream_t);    \
    template hipError_t launch_norm2<R>(const ReduceArgs<R> &, hipStream_t);             \
    template hipError_t launch_obs2<R>(const ReduceArgs<R> &, hipStream_t);              \
    template hipError_t launch_seed2<R>(const ReduceArgs<R> &, void *const[8], hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace dirac
