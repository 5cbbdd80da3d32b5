// Reverse-mode gradient of a function of the final (3+1)D state with respect
// to a z-dependent potential, rebuilding earlier states by the exact reversed
// step instead of storing them.
//
// One forward step is H1: X+ = alpha1 X- - beta1 K1 Y (A,B rows, Eqs. ss1, ss2)
// followed by H2: Y+ = alpha2 Y- - beta2 K2 X+ (C,D rows, Eqs. ss3, ss4), with
// K1, K2 the difference operators of the two sheets.  The operators satisfy
// K1^H = -K2 (the antisymmetry behind the conserved functional, Lemma of
// Sect. 2), so the transposed stencils are the other sheet's stencils.  With
// lam = dL/dRe + i dL/dIm, one backward step runs three sweeps:
//   sweep 0 (C,D sites): Y- = reversed H2; dL/dtheta2 += Re[conj(lamY) dY+/dtheta2]
//   sweep 1 (A,B sites): lamX += K1(conj(beta2) lamY); X- = reversed H1;
//                        dL/dtheta1 += Re[conj(lamX) dX+/dtheta1]; lamX <- conj(alpha1) lamX
//   sweep 2 (C,D sites): lamY <- conj(alpha2) lamY + K2(beta1 lamX)
// (in sweep 2, conj(beta1) times the unscaled lamX equals beta1 times the
// stored conj(alpha1) lamX, since conj(beta) alpha = beta for real theta).
// dY+/dtheta = -i (Y+ + Y-) beta.  Sweep 2 of one backward step and sweep 0
// of the next act on the same C,D site and read only A,B values written
// before them (lamX and X- at the neighbours), so they run as one launch
// (sweep 3): lamY is then read and written once for both.  Per-(tile, plane) FP64 sums are
// accumulated in place by the one workgroup owning them: no atomics, so the
// gradient is bitwise reproducible.
#include "device.h"
#include "internal.h"
#include "stencil3.h"
#include "ntstore.h"

namespace dirac {

namespace {

constexpr int kTX = 64, kTY = 4;

template <typename R> __device__ __forceinline__ Coef<R> tcoef(const R *tab, int q, int nz, int k) {
    const R *e = tab + ((size_t)q * nz + k) * 4;
    Coef<R> c;
    c.c1 = mk2(e[0], e[1]);
    c.c2 = mk2(e[2], e[3]);
    return c;
}

__device__ __forceinline__ double2 alpha_of(const Coef<double> &k) { return k.c1; }
__device__ __forceinline__ float2 alpha_of(const Coef<float> &k) { return mk2(1.0f - k.c1.x, -k.c1.y); }

// conj(b) * z
template <typename C> __device__ __forceinline__ C cmulc(C b, C z) { return cmul(cconj(b), z); }

template <typename R, int SWEEP>
__global__ __launch_bounds__(256) void k3_adj(AdjArgs<R> a) {
    using C = cx<R>;
    __shared__ double lds[2 * 16];
    const int nbx = (a.nx + kTX - 1) / kTX, nby = (a.ny + kTY - 1) / kTY;
    // consecutive blocks go to the 8 XCDs in turn; for complex64 remap them so
    // that each XCD takes a contiguous range of planes, whose y and z
    // neighbours then sit in its L2 (128^3 backward: 66.5 -> 53.8 ms for 400
    // steps; complex128 measured 135 -> 141 ms with the remap, so it keeps the
    // plain order)
    int b = blockIdx.x;
    if (sizeof(R) == 4 && (gridDim.x & 7) == 0) b = (b & 7) * (gridDim.x >> 3) + (b >> 3);
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nby;
    const int k = b / nby;
    const int tile = bx + nbx * by;
    const int i = bx * kTX + (threadIdx.x & (kTX - 1));
    const int j = by * kTY + (threadIdx.x / kTX);
    const bool live = i < a.nx && j < a.ny;
    double g[2] = {0.0, 0.0};   // (V at integer z, V at half-integer z)
    if (live) {
        const size_t plane = (size_t)a.nx * a.ny;
        const size_t row = (size_t)j * a.nx;
        const size_t kk = (size_t)k * plane;
        const int km = wrap_dec(k, a.nz), kp = wrap_inc(k, a.nz);
        const size_t c = kk + row + i;
        const size_t xm = kk + row + wrap_dec(i, a.nx), xp = kk + row + wrap_inc(i, a.nx);
        const size_t ym = kk + (size_t)wrap_dec(j, a.ny) * a.nx + i, yp = kk + (size_t)wrap_inc(j, a.ny) * a.nx + i;
        const size_t zm = (size_t)km * plane + row + i, zp = (size_t)kp * plane + row + i;
        C *f[8], *l[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            f[q] = (C *)a.f[q];
            l[q] = (C *)a.lam[q];
        }
        const R rx = a.rx, ry = a.ry, rz = a.rz;
        if constexpr (SWEEP == 0) {
            // C,D: rebuild Y- from Y+ and X+ (current A,B)
            St3<C> s = stencil_cd<C, R>(rx, ry, rz, f[0][c], f[0][zp], f[0][xp], f[0][yp], f[1][c], f[1][zp],
                                        f[1][xm], f[1][ym], f[2][c], f[2][zm], f[2][xm], f[2][yp], f[3][c],
                                        f[3][zm], f[3][xp], f[3][ym]);
            C ss[4] = {s.s0, s.s1, s.s2, s.s3};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int cls = 2 + q / 2;                 // C, C, D, D
                Coef<R> kf = tcoef(a.tab_f, cls, a.nz, k), kr = tcoef(a.tab_r, cls, a.nz, k);
                C yp_ = f[4 + q][c];
                C ym_ = update(yp_, mk2(-ss[q].x, -ss[q].y), kr);
                g[cls == 2 ? 1 : 0] += dtheta_term(l[4 + q][c], yp_, ym_, kf);
                st_nt(&f[4 + q][c], ym_);
            }
        } else if constexpr (SWEEP == 1) {
            // w = conj(beta2) lamY at every C,D value the A,B stencil reads
            auto w = [&](int arr, size_t idx, int kpl) -> C {
                return cmulc(tcoef(a.tab_f, 2 + (arr - 4) / 2, a.nz, kpl).c2, l[arr][idx]);
            };
            St3<C> sl = stencil_ab<C, R>(rx, ry, rz, w(4, c, k), w(4, zm, km), w(4, xp, k), w(4, yp, k),
                                         w(5, c, k), w(5, zm, km), w(5, ym, k), w(5, xm, k),
                                         w(6, c, k), w(6, xm, k), w(6, yp, k), w(6, zp, kp),
                                         w(7, c, k), w(7, ym, k), w(7, xp, k), w(7, zp, kp));
            // rebuild X- from X+ and the rebuilt Y-
            St3<C> s = stencil_ab<C, R>(rx, ry, rz, f[4][c], f[4][zm], f[4][xp], f[4][yp], f[5][c], f[5][zm],
                                        f[5][ym], f[5][xm], f[6][c], f[6][xm], f[6][yp], f[6][zp], f[7][c],
                                        f[7][ym], f[7][xp], f[7][zp]);
            C sls[4] = {sl.s0, sl.s1, sl.s2, sl.s3};
            C ss[4] = {s.s0, s.s1, s.s2, s.s3};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int cls = q / 2;                     // A, A, B, B
                Coef<R> kf = tcoef(a.tab_f, cls, a.nz, k), kr = tcoef(a.tab_r, cls, a.nz, k);
                C lx = cadd(l[q][c], sls[q]);
                C xp_ = f[q][c];
                C xm_ = update(xp_, mk2(-ss[q].x, -ss[q].y), kr);
                g[cls == 0 ? 0 : 1] += dtheta_term(lx, xp_, xm_, kf);
                st_nt(&f[q][c], xm_);
                st_nt(&l[q][c], cmulc(alpha_of(kf), lx));
            }
        } else {
            // (sweep 2, and sweep 3's first half)
            // u = beta1 lamX (stored, already scaled) at every A,B value the C,D stencil reads
            auto u = [&](int arr, size_t idx, int kpl) -> C {
                return cmul(tcoef(a.tab_f, arr / 2, a.nz, kpl).c2, l[arr][idx]);
            };
            St3<C> s = stencil_cd<C, R>(rx, ry, rz, u(0, c, k), u(0, zp, kp), u(0, xp, k), u(0, yp, k),
                                        u(1, c, k), u(1, zp, kp), u(1, xm, k), u(1, ym, k),
                                        u(2, c, k), u(2, zm, km), u(2, xm, k), u(2, yp, k),
                                        u(3, c, k), u(3, zm, km), u(3, xp, k), u(3, ym, k));
            C ss[4] = {s.s0, s.s1, s.s2, s.s3};
            C lyn[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int cls = 2 + q / 2;
                Coef<R> kf = tcoef(a.tab_f, cls, a.nz, k);
                lyn[q] = cadd(cmulc(alpha_of(kf), l[4 + q][c]), ss[q]);
            }
            if constexpr (SWEEP == 3) {
                // sweep 0 of the next backward step at the same site, with the new lamY
                St3<C> s0 = stencil_cd<C, R>(rx, ry, rz, f[0][c], f[0][zp], f[0][xp], f[0][yp], f[1][c], f[1][zp],
                                             f[1][xm], f[1][ym], f[2][c], f[2][zm], f[2][xm], f[2][yp], f[3][c],
                                             f[3][zm], f[3][xp], f[3][ym]);
                C ss0[4] = {s0.s0, s0.s1, s0.s2, s0.s3};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int cls = 2 + q / 2;
                    Coef<R> kf = tcoef(a.tab_f, cls, a.nz, k), kr = tcoef(a.tab_r, cls, a.nz, k);
                    C yp_ = f[4 + q][c];
                    C ym_ = update(yp_, mk2(-ss0[q].x, -ss0[q].y), kr);
                    g[cls == 2 ? 1 : 0] += dtheta_term(lyn[q], yp_, ym_, kf);
                    st_nt(&f[4 + q][c], ym_);
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) st_nt(&l[4 + q][c], lyn[q]);
        }
    }
    if constexpr (SWEEP != 2) {
        block_sum<2>(g, lds);
        if (threadIdx.x == 0) {
            double *o = a.gpart + ((size_t)tile * a.nz + k) * 2;
            o[0] += g[0];
            o[1] += g[1];
        }
    }
}

__global__ __launch_bounds__(256) void k_adj_finish(const double *gpart, int ntiles, int nz, double half_dt,
                                                    double *dv_int, double *dv_half) {
    __shared__ double lds[2 * 16];
    const int k = blockIdx.x;
    double v[2] = {0.0, 0.0};
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
        v[0] += gpart[((size_t)t * nz + k) * 2 + 0];
        v[1] += gpart[((size_t)t * nz + k) * 2 + 1];
    }
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
        dv_int[k] = half_dt * v[0];
        dv_half[k] = half_dt * v[1];
    }
}

__global__ __launch_bounds__(256) void k_zero(double *p, int64_t n) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = 0.0;
}

}  // namespace

int adj_tiles3(int nx, int ny) { return ((nx + kTX - 1) / kTX) * ((ny + kTY - 1) / kTY); }

template <typename R> hipError_t launch_adj3(const AdjArgs<R> &a, int sweep, hipStream_t s) {
    const int64_t nblk = (int64_t)adj_tiles3(a.nx, a.ny) * a.nz;
    if (nblk > 0x7fffffff) return hipErrorInvalidValue;
    dim3 g((unsigned)nblk), b(kTX * kTY);
    if (sweep == 0) hipLaunchKernelGGL((k3_adj<R, 0>), g, b, 0, s, a);
    else if (sweep == 1) hipLaunchKernelGGL((k3_adj<R, 1>), g, b, 0, s, a);
    else if (sweep == 2) hipLaunchKernelGGL((k3_adj<R, 2>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k3_adj<R, 3>), g, b, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adj_finish(const double *gpart, int ntiles, int nz, double half_dt, double *dv_int,
                             double *dv_half, hipStream_t s) {
    hipLaunchKernelGGL(k_adj_finish, dim3(nz), dim3(256), 0, s, gpart, ntiles, nz, half_dt, dv_int, dv_half);
    return hipGetLastError();
}

hipError_t launch_zero(double *p, int64_t n, hipStream_t s) {
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)g), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

template hipError_t launch_adj3<float>(const AdjArgs<float> &, int, hipStream_t);
template hipError_t launch_adj3<double>(const AdjArgs<double> &, int, hipStream_t);

}  // namespace dirac
