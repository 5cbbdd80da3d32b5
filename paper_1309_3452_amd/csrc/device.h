// Device-side helpers shared by the HIP kernels of this library: complex
// arithmetic on interleaved (re, im) pairs, the per-site update of the
// time-averaged mass/potential term, and the coefficient records.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cayley32.h"

namespace dirac {

template <typename R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };

template <typename R> using cx = typename V2<R>::T;

__device__ __forceinline__ double2 mk2(double x, double y) { return make_double2(x, y); }
__device__ __forceinline__ float2 mk2(float x, float y) { return make_float2(x, y); }

// Load p[idx], or zero when ok is false (a zero value outside the lattice).
template <typename C> __device__ __forceinline__ C ld_or0(const C *p, size_t idx, bool ok) {
    if (ok) return p[idx];
    C z;
    z.x = 0;
    z.y = 0;
    return z;
}

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return mk2(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return mk2(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    return mk2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return mk2(a.x, -a.y); }
// r * z for real r
template <typename C, typename R> __device__ __forceinline__ C cscale(R r, C z) { return mk2(r * z.x, r * z.y); }
// i * r * z
template <typename C, typename R> __device__ __forceinline__ C ciscale(R r, C z) { return mk2(-r * z.y, r * z.x); }

// Coefficient pair of one site's update.
//   FP64: c1 = alpha = (1 - i th)/(1 + i th), c2 = beta = 1/(1 + i th);  X+ = c1 X- - c2 S
//   FP32: c1 = gamma = 1 - alpha = 2 i th beta, c2 = beta;              X+ = X- - (c1 X- + c2 S)
// (the FP32 increment form keeps the unit-modulus factor's rounding away
// from the leading 1, so |1 - gamma| stays 1 to ~1e-9).
template <typename R> struct Coef {
    cx<R> c1, c2;
};

// Fused multiply-adds are written out explicitly (the library is built
// without automatic contraction), so every code path that evaluates the same
// expression produces the same bits.
__device__ __forceinline__ float fmx(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmx(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ double2 update(double2 xm, double2 s, const Coef<double> &k) {
    return mk2(fmx(k.c1.x, xm.x, fmx(-k.c1.y, xm.y, fmx(-k.c2.x, s.x, k.c2.y * s.y))),
               fmx(k.c1.x, xm.y, fmx(k.c1.y, xm.x, fmx(-k.c2.x, s.y, -(k.c2.y * s.x)))));
}
__device__ __forceinline__ float2 update(float2 xm, float2 s, const Coef<float> &k) {
    const float re = fmx(k.c1.x, xm.x, fmx(-k.c1.y, xm.y, fmx(k.c2.x, s.x, -(k.c2.y * s.y))));
    const float im = fmx(k.c1.x, xm.y, fmx(k.c1.y, xm.x, fmx(k.c2.x, s.y, k.c2.y * s.x)));
    return mk2(xm.x - re, xm.y - im);
}

// Cayley coefficients from a per-site theta.  FP64: with one IEEE division,
//   r = 1/(1 + th^2), alpha = ((1 - th^2) r, -(2 th) r), beta = (r, -th r)
// with every operation rounded separately (contraction off), so the
// coefficients are the same bits on any IEEE host.
__device__ __forceinline__ Coef<double> coef_theta(double th) {
#pragma clang fp contract(off)
    double t2 = th * th;
    double r = 1.0 / (1.0 + t2);
    Coef<double> k;
    k.c1 = mk2((1.0 - t2) * r, -((2.0 * th) * r));
    k.c2 = mk2(r, -(th * r));
    return k;
}
// FP32: evaluated in FP64 and rounded; gamma_re is re-derived from the rounded
// gamma_im so that (1 - gamma_re)^2 + gamma_im^2 = 1 up to one rounding of gamma_re.
__device__ __forceinline__ Coef<float> coef_theta(float thf) {
#pragma clang fp contract(off)
    double th = (double)thf;
    double d = 1.0 + th * th;
    float gi = (float)(2.0 * th / d);
    double gid = (double)gi;
    double gr = gid * gid / (1.0 + sqrt(1.0 - gid * gid));
    Coef<float> k;
    k.c1 = mk2((float)gr, gi);
    k.c2 = mk2((float)(1.0 / d), (float)(-th / d));
    return k;
}

// Per-site coefficients of the FP32 form.  Only gamma = 1 - alpha is stored
// (two floats per site, chosen once by gamma32_search); beta follows from it
// exactly, since 1 + alpha = 2 beta gives beta = 1 - gamma/2 (one rounding).
// The reversed step (theta -> -theta) uses conj(gamma): sgn = -1.
__device__ __forceinline__ Coef<float> coef_site(float2 g, float sgn) {
    Coef<float> k;
    k.c1 = mk2(g.x, sgn * g.y);
    k.c2 = mk2(fmx(-0.5f, g.x, 1.0f), -0.5f * (sgn * g.y));
    return k;
}
// Per-site coefficient record at site idx of a coefficient array: complex64
// lattices store gamma (float2 per site), complex128 lattices store theta.
template <typename R> __device__ __forceinline__ Coef<R> coef_site_at(const R *th, size_t idx, R sgn);
template <> __device__ __forceinline__ Coef<float> coef_site_at<float>(const float *th, size_t idx, float sgn) {
    return coef_site(((const float2 *)th)[idx], sgn);
}
template <> __device__ __forceinline__ Coef<double> coef_site_at<double>(const double *th, size_t idx, double sgn) {
    return coef_theta(sgn * th[idx]);
}

// Unit-modulus rounding of the complex64 record gamma = 1 - alpha (the search
// itself is shared with the host tables).
__device__ inline float2 gamma32_record(double th) {
    float2 g;
    gamma32_search(th, &g.x, &g.y);
    return g;
}

// dX+/dtheta = -i (X+ + X-) beta ; contribution Re[conj(lam) dX+/dtheta] in FP64
template <typename C, typename R>
__device__ __forceinline__ double dtheta_term(C lam, C xp, C xm, const Coef<R> &k) {
    double sr = (double)xp.x + (double)xm.x, si = (double)xp.y + (double)xm.y;
    // w = -i (s) beta
    double br = (double)k.c2.x, bi = (double)k.c2.y;
    double pr = sr * br - si * bi, pi = sr * bi + si * br;   // s * beta
    double wr = pi, wi = -pr;                                 // -i * (s beta)
    return (double)lam.x * wr + (double)lam.y * wi;           // Re(conj(lam) w)
}

// Periodic neighbour offsets.
__device__ __forceinline__ int wrap_dec(int i, int n) { return i == 0 ? n - 1 : i - 1; }
__device__ __forceinline__ int wrap_inc(int i, int n) { return i == n - 1 ? 0 : i + 1; }

// FP64 block reduction of NV values per thread; result valid in thread 0.
// blockDim.x must be a multiple of 64 and <= 1024.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds /* >= NV*16 */) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
    }
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0)
        for (int q = 0; q < NV; ++q) lds[q * 16 + wave] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < NV; ++q) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += lds[q * 16 + w];
            v[q] = s;
        }
    }
    __syncthreads();
}

}  // namespace dirac
