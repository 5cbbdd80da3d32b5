// Host-side declarations shared between the ABI layer and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dirac {

// Eight pointers passed by value to a kernel.
struct CPtr8 {
    void *p[8];
};

// Arguments of one half-step launch (split kernels) over a single lattice.
// `f` holds the 8 (3D) or 4 (2D) state arrays, updated in place.
template <typename R> struct HalfArgs {
    void *f[8];
    const R *th[8];       // per-site coefficients (site mode: theta, or gamma pairs for FP32), else null
    const R *tab;         // [class][nz][4] coefficient table (profile mode), else null
    R rx, ry, rz;         // signed: negated for the reversed step
    R tsgn;               // +1 forward, -1 reversed (site mode)
    int nx, ny, nz;
    int zbc;              // 1: zero values outside the lattice; 0: periodic
};

// Fused one-step launch (3D z-march / 2D y-march), ping-pong in -> out.
template <typename R> struct FusedArgs {
    const void *in[8];
    void *out[8];
    const R *th[8];
    const R *tab;
    R rx, ry, rz;
    int nx, ny, nz;
    int zchunk;           // planes per workgroup along the march
    int nzc;              // number of chunks = ceil(nz / zchunk)
    int ntx, nty;         // tiles in x, y
    double *npart;        // if set: per-workgroup (E_r, plain norm) of the new state, FP64
    int npart_cap;        // capacity of npart in workgroups
    int zh;               // z-slab mode: halo planes per side (arrays hold nz + 2 zh planes,
                          // interior planes zh .. zh + nz - 1, no wrap in z); 0 = periodic
    int px;               // two-step 3D kernel: tiles across one XCD's concurrent patch
                          // (0 = whole tile rows); set by its launcher
    int rev;              // 3D: per-site records taken with theta -> -theta (steps of the
                          // reversed sequence; r and the table pointer are set by the caller)
};

// Reduction launch over a single lattice.
template <typename R> struct ReduceArgs {
    const void *f[8];
    R rx, ry, rz;
    int nx, ny, nz;
    double z0;
    double *partial;      // [nblocks][nv]
    int zh;               // z-slab mode (as in FusedArgs); 0 = periodic
    int zbc;              // 1: zero values outside the lattice (x, y, z); 0: periodic
};

// Gauge-link arrays (vector potential, Sect. 4): u[6 a + t] (3D) or u[4 a + t]
// (2D) for A,B (u) array a and neighbour term t, one unit complex per cell in
// the lattice's storage type.
struct LinkPtrs {
    const void *u[24];
};

// Adjoint sweep launch (V(z) profile mode).
template <typename R> struct AdjArgs {
    void *f[8];           // state, rebuilt in place
    void *lam[8];         // adjoint, updated in place
    const R *tab_f;       // forward coefficient table [class][nz][4]
    const R *tab_r;       // reversed-step coefficient table
    R rx, ry, rz;
    int nx, ny, nz;
    double *gpart;        // [tiles][nz][2] per-(tile, plane) dL/dtheta sums (int, half)
};

constexpr int kReduceBlocks = 1024;   // fixed partial count: reproducible sums
constexpr int kReduceThreads = 256;
constexpr int kNormVals = 3;
constexpr int kObsVals = 9;

// 3D split kernels (kernels3d.hip)
template <typename R> hipError_t launch_half3(const HalfArgs<R> &a, int which /*0: A,B  1: C,D*/, bool site,
                                              hipStream_t s);
template <typename R> hipError_t launch_fused3(const FusedArgs<R> &a, bool site, int tile_y, hipStream_t s,
                                               int *nblocks_out = nullptr);
// Two steps per launch (fused2.hip); V(z) tables or per-site records, nx even for complex64.
bool fused3x2_supported(int nx, bool fp32, bool site);
template <typename R>
hipError_t launch_fused3x2(const FusedArgs<R> &a, bool site, hipStream_t s, int *nblocks_out = nullptr);
// (2+1)D two steps per launch (fused2.hip, march2x2.h); nx even for complex64.
bool fused2x2_supported(int nx, bool fp32);
template <typename R> hipError_t launch_fused2x2(const FusedArgs<R> &a, bool site, hipStream_t s);
template <typename R> hipError_t launch_norm3(const ReduceArgs<R> &a, hipStream_t s);
template <typename R> hipError_t launch_obs3(const ReduceArgs<R> &a, hipStream_t s);
template <typename R> hipError_t launch_seed3(const ReduceArgs<R> &a, void *const lam[8], hipStream_t s);
template <typename R> hipError_t launch_theta_fields(void *const th[8], void *const v[8], int narr, int64_t ncell,
                                                     double half_dt, double m, hipStream_t s);
hipError_t launch_coef_from_theta(void *coef, const double *theta, const double *theta_im, int64_t n,
                                  hipStream_t s);
hipError_t launch_coef_from_fields(void *coef, bool c64, double half_dt, double sgn_m, const double *v,
                                   const double *w, int64_t n, hipStream_t s);
hipError_t launch_final_sum(const double *partial, int nblocks, int nv, double *out, hipStream_t s);

// 2D split kernels (kernels2d.hip)
template <typename R> hipError_t launch_half2(const HalfArgs<R> &a, int which /*0: u  1: v*/, bool site,
                                              hipStream_t s);
template <typename R> hipError_t launch_fused2(const FusedArgs<R> &a, bool site, hipStream_t s);
// Chunks per tile column of a 3D z-march of `tiles` tile columns over nz planes,
// each chunk paying `fill` planes of pipeline fill (see fused2.hip).
int pick_chunks(int64_t tiles, int nz, int fill);
template <typename R> hipError_t launch_norm2(const ReduceArgs<R> &a, hipStream_t s);
template <typename R> hipError_t launch_obs2(const ReduceArgs<R> &a, hipStream_t s);
template <typename R> hipError_t launch_seed2(const ReduceArgs<R> &a, void *const lam[8], hipStream_t s);

// Split half-step (which: 0 A,B / u, 1 C,D / v) and E_r reduction with gauge
// links (gauge.hip); ndim 3 or 2.
template <typename R> hipError_t launch_half_links(const HalfArgs<R> &a, const LinkPtrs &L, int ndim, int which,
                                                   bool site, hipStream_t s);
template <typename R> hipError_t launch_norm_links(const ReduceArgs<R> &a, const LinkPtrs &L, int ndim,
                                                   hipStream_t s);
// 3D one step per launch with links, z-march, ping-pong in -> out (gauge.hip).
template <typename R> hipError_t launch_fused_links(const FusedArgs<R> &a, const LinkPtrs &L, bool site,
                                                    hipStream_t s);

// Adjoint (adjoint.hip)
template <typename R> hipError_t launch_adj3(const AdjArgs<R> &a, int sweep, hipStream_t s);
hipError_t launch_adj_finish(const double *gpart, int ntiles, int nz, double half_dt, double *dv_int,
                             double *dv_half, hipStream_t s);
int adj_tiles3(int nx, int ny);
hipError_t launch_zero(double *p, int64_t n, hipStream_t s);

}  // namespace dirac
