// C ABI of the library: context, validation, coefficient tables, dispatch of
// the single-lattice kernels.  The batched entry points live in batch.hip.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/dirac.h"
#include "cayley32.h"
#include "ctx.h"
#include "gauge.h"
#include "internal.h"

using namespace dirac;

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
namespace {

int fail(dirac_ctx *c, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(dirac_ctx *c, int code, const char *fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPCHK(ctx, expr)                                                                         \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail((ctx), DIRAC_E_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                                \
    } while (0)

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// FP64 Cayley coefficients, every operation rounded on its own.
void cayley64(double th, double out[4]) {
#pragma clang fp contract(off)
    double t2 = th * th;
    double d = 1.0 + t2;
    out[0] = (1.0 - t2) / d;
    out[1] = -((2.0 * th) / d);
    out[2] = 1.0 / d;
    out[3] = -(th / d);
}

// FP32 increment-form coefficients: gamma = 2 i th / (1 + i th) by the
// unit-modulus rounding shared with the device records (cayley32.h), beta =
// 1 / (1 + i th) rounded from FP64.
void cayley32(double th, float out[4]) {
#pragma clang fp contract(off)
    const double d = 1.0 + th * th;
    gamma32_search(th, &out[0], &out[1]);
    out[2] = (float)(1.0 / d);
    out[3] = (float)(-th / d);
}

// Complex theta = th + i thi (a complex potential; Im V damps for Im V < 0):
// with 1 + i theta = (1 - thi) + i th and 1 - i theta = (1 + thi) - i th,
//   beta = ((1 - thi) - i th)/den,  alpha = ((1 - thi^2 - th^2) - 2 i th)/den,
//   den = (1 - thi)^2 + th^2.
void cayley64c(double th, double thi, double out[4]) {
#pragma clang fp contract(off)
    if (thi == 0.0) {
        cayley64(th, out);
        return;
    }
    const double den = (1.0 - thi) * (1.0 - thi) + th * th;
    out[0] = (1.0 - thi * thi - th * th) / den;
    out[1] = -((2.0 * th) / den);
    out[2] = (1.0 - thi) / den;
    out[3] = -(th / den);
}
// FP32 increment form for a complex theta: gamma = 1 - alpha and beta rounded
// from FP64 (|alpha| != 1, so the unit-modulus search does not apply).
void cayley32c(double th, double thi, float out[4]) {
    if (thi == 0.0) {
        cayley32(th, out);
        return;
    }
    double c[4];
    cayley64c(th, thi, c);
    out[0] = (float)(1.0 - c[0]);
    out[1] = (float)(-c[1]);
    out[2] = (float)c[2];
    out[3] = (float)c[3];
}

// Planes of the V(z) tables and per-site fields: the interior plus, in z-slab
// mode, the halo planes on both sides.
int64_t planes_of(const dirac_ctx *c) { return c->nz + 2 * c->zh; }

// theta of class q (A, B, C, D) at plane k: (dt/2)(+-m + V at the class's z).
double theta_of(const dirac_ctx *c, int q, int64_t k) {
    double h = 0.5 * c->dt;
    double v = 0.0;
    if (!c->v_int.empty()) v = (q == 0 || q == 3) ? c->v_int[k] : c->v_half[k];
    double sgn = (q < 2) ? 1.0 : -1.0;
    return h * (sgn * c->m + v);
}
// Im theta of class q at plane k: (dt/2) Im V at the class's z (m is real).
double theta_im_of(const dirac_ctx *c, int q, int64_t k) {
    if (c->w_int.empty()) return 0.0;
    return 0.5 * c->dt * ((q == 0 || q == 3) ? c->w_int[k] : c->w_half[k]);
}

template <typename R> size_t tab_bytes(const dirac_ctx *c) { return (size_t)4 * planes_of(c) * 4 * sizeof(R); }

size_t tab_bytes_of(const dirac_ctx *c) {
    return c->dtype == DIRAC_C64 ? tab_bytes<float>(c) : tab_bytes<double>(c);
}

// scratch layout
// Per-workgroup partials of the in-step functional (two doubles each): every
// z-march launch has at most nz chunks per tile column, and its tiles are at
// least 32 x 4 or 16 x 16 cells, so the area is sized for the larger tile
// count of the two and an in-step reduction is never refused for lack of
// slots.  The standalone reductions use kReduceBlocks x kObsVals doubles of the
// same area.
size_t step_partials(const dirac_ctx *c) {
    const size_t t1 = (size_t)((c->nx + 31) / 32) * (size_t)((c->ny + 3) / 4);
    const size_t t2 = (size_t)((c->nx + 15) / 16) * (size_t)((c->ny + 15) / 16);
    return (t1 > t2 ? t1 : t2) * (size_t)c->nz;
}
size_t partial_doubles(const dirac_ctx *c) {
    const size_t red = (size_t)kReduceBlocks * kObsVals, stp = 2 * step_partials(c);
    return red > stp ? red : stp;
}
size_t off_partial(const dirac_ctx *) { return 0; }
size_t off_result(const dirac_ctx *c) { return align256(partial_doubles(c) * sizeof(double)); }
size_t off_tab(const dirac_ctx *c) { return off_result(c) + 256; }
size_t off_gpart(const dirac_ctx *c) { return off_tab(c) + 2 * align256(tab_bytes_of(c)); }
size_t scratch_need(const dirac_ctx *c) {
    size_t g = 0;
    if (c->ndim == 3) g = (size_t)adj_tiles3((int)c->nx, (int)c->ny) * c->nz * 2 * sizeof(double);
    return off_gpart(c) + align256(g);
}

char *scratch_at(const dirac_ctx *c, size_t off) { return (char *)c->scratch + off; }

int upload_tables(dirac_ctx *c, hipStream_t s) {
    if (!c->tab_dirty) return DIRAC_OK;
    if (!c->scratch) return fail(c, DIRAC_E_STATE, "scratch must be bound before stepping");
    const int64_t nz = planes_of(c);
    if (c->dtype == DIRAC_C128) {
        c->tab_host64.assign((size_t)2 * 4 * nz * 4, 0.0);
        for (int dir = 0; dir < 2; ++dir)
            for (int q = 0; q < 4; ++q)
                for (int64_t k = 0; k < nz; ++k) {
                    double th = theta_of(c, q, k), thi = theta_im_of(c, q, k);
                    cayley64c(dir == 0 ? th : -th, dir == 0 ? thi : -thi,
                              &c->tab_host64[(((size_t)dir * 4 + q) * nz + k) * 4]);
                }
        size_t half = tab_bytes<double>(c);
        HIPCHK(c, hipMemcpyAsync(scratch_at(c, off_tab(c)), c->tab_host64.data(), half, hipMemcpyHostToDevice, s));
        HIPCHK(c, hipMemcpyAsync(scratch_at(c, off_tab(c) + align256(half)), c->tab_host64.data() + 4 * nz * 4,
                                 half, hipMemcpyHostToDevice, s));
    } else {
        c->tab_host32.assign((size_t)2 * 4 * nz * 4, 0.0f);
        for (int dir = 0; dir < 2; ++dir)
            for (int q = 0; q < 4; ++q)
                for (int64_t k = 0; k < nz; ++k) {
                    double th = theta_of(c, q, k), thi = theta_im_of(c, q, k);
                    cayley32c(dir == 0 ? th : -th, dir == 0 ? thi : -thi,
                              &c->tab_host32[(((size_t)dir * 4 + q) * nz + k) * 4]);
                }
        size_t half = tab_bytes<float>(c);
        HIPCHK(c, hipMemcpyAsync(scratch_at(c, off_tab(c)), c->tab_host32.data(), half, hipMemcpyHostToDevice, s));
        HIPCHK(c, hipMemcpyAsync(scratch_at(c, off_tab(c) + align256(half)), c->tab_host32.data() + 4 * nz * 4,
                                 half, hipMemcpyHostToDevice, s));
    }
    // the host staging vectors stay alive in the context until the next upload
    HIPCHK(c, hipStreamSynchronize(s));
    c->tab_dirty = false;
    return DIRAC_OK;
}

template <typename R> HalfArgs<R> half_args(dirac_ctx *c, bool reverse) {
    HalfArgs<R> a;
    memset(&a, 0, sizeof a);
    int narr = c->ndim == 3 ? 8 : 4;
    for (int q = 0; q < narr; ++q) {
        a.f[q] = c->buf[c->cur][q];
        a.th[q] = c->site_mode ? (const R *)c->theta[q] : nullptr;
    }
    size_t half = align256(tab_bytes<R>(c));
    a.tab = c->site_mode ? nullptr : (const R *)scratch_at(c, off_tab(c) + (reverse ? half : 0));
    R sg = reverse ? (R)-1 : (R)1;
    a.rx = sg * (R)c->rx;
    a.ry = sg * (R)c->ry;
    a.rz = sg * (R)c->rz;
    a.tsgn = sg;
    a.nx = (int)c->nx;
    a.ny = (int)c->ny;
    a.nz = (int)c->nz;
    a.zbc = c->zbc ? 1 : 0;
    return a;
}

template <typename R> FusedArgs<R> fused_args(dirac_ctx *c) {
    FusedArgs<R> a;
    memset(&a, 0, sizeof a);
    int narr = c->ndim == 3 ? 8 : 4;
    for (int q = 0; q < narr; ++q) {
        a.in[q] = c->buf[c->cur][q];
        a.out[q] = c->buf[1 - c->cur][q];
        a.th[q] = c->site_mode ? (const R *)c->theta[q] : nullptr;
    }
    a.tab = c->site_mode ? nullptr : (const R *)scratch_at(c, off_tab(c));
    a.rx = (R)c->rx;
    a.ry = (R)c->ry;
    a.rz = (R)c->rz;
    a.nx = (int)c->nx;
    a.ny = (int)c->ny;
    a.nz = (int)c->nz;
    a.zchunk = c->zchunk;
    a.zh = c->zh;
    return a;
}

int kernel_choice(const dirac_ctx *c) {
    // the fused kernels address a plane with 32-bit byte offsets
    const uint64_t plane_bytes = (uint64_t)c->nx * (uint64_t)c->ny * (c->dtype == DIRAC_C64 ? 8u : 16u);
    if (c->zh) {
        // z-slab mode: the two-step march where it applies (the two halo planes
        // serve two steps), else the one-step march; never the split kernels
        if (c->kernel != DIRAC_KERNEL_FUSED && plane_bytes < (1ull << 32) &&
            fused3x2_supported((int)c->nx, c->dtype == DIRAC_C64, c->site_mode))
            return DIRAC_KERNEL_FUSED2;
        return DIRAC_KERNEL_FUSED;
    }
    if (c->kernel == DIRAC_KERNEL_SPLIT) return DIRAC_KERNEL_SPLIT;
    // zero values outside the lattice: the split kernels (in place)
    if (c->zbc) return DIRAC_KERNEL_SPLIT;
    // links: the link marches (one step per launch)
    if (c->links_on) return DIRAC_KERNEL_FUSED;
    if (plane_bytes >= (1ull << 32)) return DIRAC_KERNEL_SPLIT;
    if (c->kernel == DIRAC_KERNEL_FUSED) return DIRAC_KERNEL_FUSED;
    if (c->ndim == 3 && fused3x2_supported((int)c->nx, c->dtype == DIRAC_C64, c->site_mode))
        return DIRAC_KERNEL_FUSED2;
    // (2+1)D: a two-step pass recomputes a six-row pipeline per chunk, so small
    // lattices (under 2^18 cells, cache-resident) keep the one-step march, which
    // spreads them over more workgroups; an explicit FUSED2 request is honoured
    if (c->ndim == 2 && fused2x2_supported((int)c->nx, c->dtype == DIRAC_C64) &&
        (c->kernel == DIRAC_KERNEL_FUSED2 || c->nx * c->ny >= (int64_t)1 << 18))
        return DIRAC_KERNEL_FUSED2;
    return DIRAC_KERNEL_FUSED;
}

// z-slab mode: the most steps one call may advance between halo refills
int halo_steps(const dirac_ctx *c) { return kernel_choice(c) == DIRAC_KERNEL_FUSED2 ? 2 : 1; }

int slab_step_check(dirac_ctx *c, int64_t n) {
    if (c->zh && n > halo_steps(c))
        return fail(c, DIRAC_E_ARG, halo_steps(c) == 2 ? "z-slab mode: at most 2 steps per call, halos refilled between calls"
                                                       : "z-slab mode: 1 step per call, halos refilled between calls");
    return DIRAC_OK;
}

LinkPtrs link_ptrs(const dirac_ctx *c) {
    LinkPtrs L;
    for (int q = 0; q < 24; ++q) L.u[q] = c->links[q];
    return L;
}

// The forward march kernels run the reversed sequence: with r -> -r, the
// reversed coefficient tables (theta -> -theta) and per-site records read with
// theta -> -theta they apply H1' then H2', the two half-steps solved backwards
// (H1' undoes ss1, ss2; H2' undoes ss3, ss4).  n reversed steps are
// (H1' H2')^n = H1' (H2' H1')^(n-1) H2': one split H2', n - 1 march steps, one
// split H1'.
template <typename R> FusedArgs<R> fused_args_rev(dirac_ctx *c) {
    FusedArgs<R> a = fused_args<R>(c);
    a.rx = -a.rx;
    a.ry = -a.ry;
    a.rz = -a.rz;
    if (!c->site_mode) a.tab = (const R *)scratch_at(c, off_tab(c) + align256(tab_bytes<R>(c)));
    a.rev = 1;
    return a;
}

// 3D lattices whose forward steps take a march kernel reverse on it too
bool reverse_on_march(const dirac_ctx *c) {
    if (c->ndim != 3 || c->links_on || c->zh) return false;
    const int kc = kernel_choice(c);
    return kc == DIRAC_KERNEL_FUSED || kc == DIRAC_KERNEL_FUSED2;
}

template <typename R> int run_reverse_march(dirac_ctx *c, int64_t n, hipStream_t s) {
    if (n <= 0) return DIRAC_OK;
    const bool site = c->site_mode;
    HIPCHK(c, launch_half3<R>(half_args<R>(c, true), 1, site, s));      // H2'
    int64_t t = 1;
    if (kernel_choice(c) == DIRAC_KERNEL_FUSED2) {
        for (; t + 2 <= n; t += 2) {
            HIPCHK(c, launch_fused3x2<R>(fused_args_rev<R>(c), site, s));
            c->cur = 1 - c->cur;
        }
    }
    for (; t < n; ++t) {
        HIPCHK(c, launch_fused3<R>(fused_args_rev<R>(c), site, c->tile_y, s));
        c->cur = 1 - c->cur;
    }
    HIPCHK(c, launch_half3<R>(half_args<R>(c, true), 0, site, s));      // H1'
    return DIRAC_OK;
}

template <typename R> int run_steps(dirac_ctx *c, int64_t n, bool reverse, hipStream_t s) {
    int rc = upload_tables(c, s);
    if (rc) return rc;
    if (reverse && reverse_on_march(c)) return run_reverse_march<R>(c, n, s);
    const bool site = c->site_mode;
    const int kc = reverse ? DIRAC_KERNEL_SPLIT : kernel_choice(c);
    const bool fused = kc == DIRAC_KERNEL_FUSED || kc == DIRAC_KERNEL_FUSED2;
    int64_t t = 0;
    if (kc == DIRAC_KERNEL_FUSED2) {
        for (; t + 2 <= n; t += 2) {
            FusedArgs<R> a = fused_args<R>(c);
            if (c->ndim == 3) HIPCHK(c, launch_fused3x2<R>(a, site, s));
            else HIPCHK(c, launch_fused2x2<R>(a, site, s));
            c->cur = 1 - c->cur;
        }
    }
    for (; t < n; ++t) {
        if (fused && c->links_on) {
            FusedArgs<R> a = fused_args<R>(c);
            if (c->ndim == 3) HIPCHK(c, launch_fused_links<R>(a, link_ptrs(c), site, s));
            else HIPCHK(c, launch_fused2_links<R>(a, link_ptrs(c), site, s));
            c->cur = 1 - c->cur;
        } else if (fused) {
            FusedArgs<R> a = fused_args<R>(c);
            if (c->ndim == 3) HIPCHK(c, launch_fused3<R>(a, site, c->tile_y, s));
            else HIPCHK(c, launch_fused2<R>(a, site, s));
            c->cur = 1 - c->cur;
        } else {
            HalfArgs<R> a = half_args<R>(c, reverse);
            int first = reverse ? 1 : 0;
            if (c->links_on) {
                const LinkPtrs L = link_ptrs(c);
                HIPCHK(c, launch_half_links<R>(a, L, c->ndim, first, site, s));
                HIPCHK(c, launch_half_links<R>(a, L, c->ndim, 1 - first, site, s));
            } else if (c->ndim == 3) {
                HIPCHK(c, launch_half3<R>(a, first, site, s));
                HIPCHK(c, launch_half3<R>(a, 1 - first, site, s));
            } else {
                HIPCHK(c, launch_half2<R>(a, first, site, s));
                HIPCHK(c, launch_half2<R>(a, 1 - first, site, s));
            }
        }
    }
    return DIRAC_OK;
}

template <typename R> ReduceArgs<R> reduce_args(dirac_ctx *c, double z0) {
    ReduceArgs<R> a;
    memset(&a, 0, sizeof a);
    int narr = c->ndim == 3 ? 8 : 4;
    for (int q = 0; q < narr; ++q) a.f[q] = c->buf[c->cur][q];
    a.rx = (R)c->rx;
    a.ry = (R)c->ry;
    a.rz = (R)c->rz;
    a.nx = (int)c->nx;
    a.ny = (int)c->ny;
    a.nz = (int)c->nz;
    a.z0 = z0;
    a.partial = (double *)scratch_at(c, off_partial(c));
    a.zh = c->zh;
    a.zbc = c->zbc ? 1 : 0;
    return a;
}

int check_ready(dirac_ctx *c, bool need_scratch) {
    if (!c) return DIRAC_E_ARG;
    if (c->is_batch) return fail(c, DIRAC_E_STATE, "batch context: use the dirac_batch_* calls");
    if (!c->bound) return fail(c, DIRAC_E_STATE, "no state bound (dirac_bind_state)");
    if (need_scratch && !c->scratch) return fail(c, DIRAC_E_STATE, "no scratch bound (dirac_bind_scratch)");
    return DIRAC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *dirac_status_string(int status) {
    switch (status) {
    case DIRAC_OK: return "ok";
    case DIRAC_E_ARG: return "invalid argument";
    case DIRAC_E_SHAPE: return "invalid shape";
    case DIRAC_E_UNSTABLE: return "step above the stability bound";
    case DIRAC_E_NONFINITE: return "non-finite value";
    case DIRAC_E_HIP: return "HIP runtime error";
    case DIRAC_E_STATE: return "call out of order";
    default: return "unknown status";
    }
}

int dirac_create(dirac_ctx **out, int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype, double dt, double dx,
                 double dy, double dz, unsigned flags) {
    if (!out) return DIRAC_E_ARG;
    *out = nullptr;
    if (ndim != 2 && ndim != 3) return DIRAC_E_ARG;
    if (dtype != DIRAC_C64 && dtype != DIRAC_C128) return DIRAC_E_ARG;
    if ((flags & ~(DIRAC_ALLOW_UNSTABLE | DIRAC_SLAB_Z | DIRAC_ZERO_BC)) != 0) return DIRAC_E_ARG;
    if ((flags & DIRAC_SLAB_Z) && ndim != 3) return DIRAC_E_ARG;
    if ((flags & DIRAC_SLAB_Z) && (flags & DIRAC_ZERO_BC)) return DIRAC_E_ARG;
    if (nx < 1 || ny < 1 || nz < 1) return DIRAC_E_SHAPE;
    if (ndim == 2 && nz != 1) return DIRAC_E_SHAPE;
    if (nx > (1 << 30) || ny > (1 << 30) || nz > (1 << 30)) return DIRAC_E_SHAPE;
    if ((double)nx * (double)ny * (double)nz >= 1099511627776.0) return DIRAC_E_SHAPE;
    if (!finite_pos(dt) || !finite_pos(dx) || !finite_pos(dy) || (ndim == 3 && !finite_pos(dz))) return DIRAC_E_ARG;
    double rx = dt / dx, ry = dt / dy, rz = ndim == 3 ? dt / dz : 0.0;
    double r2 = rx * rx + ry * ry + rz * rz;
    if (r2 > 1.0 + 1e-12 && !(flags & DIRAC_ALLOW_UNSTABLE)) return DIRAC_E_UNSTABLE;
    dirac_ctx *c = new (std::nothrow) dirac_ctx();
    if (!c) return DIRAC_E_ARG;
    c->ndim = ndim;
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->dtype = dtype;
    c->dt = dt;
    c->rx = rx;
    c->ry = ry;
    c->rz = rz;
    c->flags = flags;
    c->zh = (flags & DIRAC_SLAB_Z) ? 2 : 0;
    c->zbc = (flags & DIRAC_ZERO_BC) != 0;
    *out = c;
    return DIRAC_OK;
}

void dirac_destroy(dirac_ctx *c) {
    if (!c) return;
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    delete c;
}

const char *dirac_last_error(const dirac_ctx *c) { return c ? c->err.c_str() : "null context"; }

int dirac_bind_state(dirac_ctx *c, void *const buf0[], void *const buf1[]) {
    if (!c || !buf0 || !buf1) return DIRAC_E_ARG;
    if (c->is_batch) return fail(c, DIRAC_E_STATE, "batch context: use dirac_batch_bind");
    int narr = c->ndim == 3 ? 8 : 4;
    for (int q = 0; q < narr; ++q)
        if (!buf0[q] || !buf1[q]) return fail(c, DIRAC_E_ARG, "null state array %d", q);
    for (int q = 0; q < 8; ++q) {
        c->buf[0][q] = q < narr ? buf0[q] : nullptr;
        c->buf[1][q] = q < narr ? buf1[q] : nullptr;
    }
    c->bound = true;
    c->cur = 0;
    return DIRAC_OK;
}

int dirac_current(const dirac_ctx *c, int *which) {
    if (!c || !which) return DIRAC_E_ARG;
    *which = c->cur;
    return DIRAC_OK;
}

int dirac_set_current(dirac_ctx *c, int which) {
    if (!c || (which != 0 && which != 1)) return DIRAC_E_ARG;
    c->cur = which;
    return DIRAC_OK;
}

int dirac_halo_steps(const dirac_ctx *c, int *steps) {
    if (!c || !steps) return DIRAC_E_ARG;
    *steps = (!c->is_batch && c->zh) ? halo_steps(c) : 0;
    return DIRAC_OK;
}

int dirac_scratch_bytes(const dirac_ctx *c, size_t *bytes) {
    if (!c || !bytes) return DIRAC_E_ARG;
    *bytes = c->is_batch ? c->batch_scratch_need : scratch_need(c);
    return DIRAC_OK;
}

int dirac_bind_scratch(dirac_ctx *c, void *dev, size_t bytes) {
    if (!c || !dev) return DIRAC_E_ARG;
    if (((uintptr_t)dev & 255) != 0) return fail(c, DIRAC_E_ARG, "scratch must be 256-byte aligned");
    size_t need = c->is_batch ? c->batch_scratch_need : scratch_need(c);
    if (bytes < need) return fail(c, DIRAC_E_SHAPE, "scratch too small: %zu < %zu bytes", bytes, need);
    c->scratch = dev;
    c->scratch_bytes = bytes;
    c->tab_dirty = true;
    return DIRAC_OK;
}

int dirac_set_potential_im_z(dirac_ctx *c, const double *w_int, const double *w_half, int64_t nz) {
    if (!c) return DIRAC_E_ARG;
    if (c->is_batch) return fail(c, DIRAC_E_STATE, "batch context");
    if (nz != planes_of(c))
        return fail(c, DIRAC_E_SHAPE, "nz %lld != lattice planes %lld", (long long)nz, (long long)planes_of(c));
    if ((w_int == nullptr) != (w_half == nullptr)) return fail(c, DIRAC_E_ARG, "w_int and w_half: both or neither");
    std::vector<double> wi, wh;
    if (w_int) {
        wi.assign(w_int, w_int + nz);
        wh.assign(w_half, w_half + nz);
        bool any = false;
        for (int64_t k = 0; k < nz; ++k) {
            if (!isfinite(wi[k]) || !isfinite(wh[k]))
                return fail(c, DIRAC_E_NONFINITE, "non-finite Im V at k=%lld", (long long)k);
            any = any || wi[k] != 0.0 || wh[k] != 0.0;
        }
        if (!any) {
            wi.clear();
            wh.clear();
        }
    }
    c->w_int.swap(wi);
    c->w_half.swap(wh);
    c->tab_dirty = true;
    return DIRAC_OK;
}

int dirac_set_mass_potential_z(dirac_ctx *c, double m, const double *v_int, const double *v_half, int64_t nz) {
    if (!c || !isfinite(m)) return DIRAC_E_ARG;
    if (c->is_batch) return fail(c, DIRAC_E_STATE, "batch context");
    if (nz != planes_of(c))
        return fail(c, DIRAC_E_SHAPE, "nz %lld != lattice planes %lld", (long long)nz, (long long)planes_of(c));
    if ((v_int == nullptr) != (v_half == nullptr)) return fail(c, DIRAC_E_ARG, "v_int and v_half: both or neither");
    if (v_int && c->ndim == 2) return fail(c, DIRAC_E_ARG, "2D: use dirac_theta_from_fields for V(x, y)");
    std::vector<double> vi, vh;
    if (v_int) {
        vi.assign(v_int, v_int + nz);
        vh.assign(v_half, v_half + nz);
        for (int64_t k = 0; k < nz; ++k)
            if (!isfinite(vi[k]) || !isfinite(vh[k])) return fail(c, DIRAC_E_NONFINITE, "non-finite V at k=%lld",
                                                                   (long long)k);
    }
    c->m = m;
    c->v_int.swap(vi);
    c->v_half.swap(vh);
    c->site_mode = false;
    c->tab_dirty = true;
    return DIRAC_OK;
}

int dirac_set_mass(dirac_ctx *c, double m) {
    if (!c) return DIRAC_E_ARG;
    if (c->v_int.empty()) return dirac_set_mass_potential_z(c, m, nullptr, nullptr, planes_of(c));
    const std::vector<double> vi = c->v_int, vh = c->v_half;
    return dirac_set_mass_potential_z(c, m, vi.data(), vh.data(), planes_of(c));
}

int dirac_set_potential_z(dirac_ctx *c, const double *v_int, const double *v_half, int64_t nz) {
    if (!c) return DIRAC_E_ARG;
    return dirac_set_mass_potential_z(c, c->m, v_int, v_half, nz);
}

int dirac_set_theta_field(dirac_ctx *c, void *const theta[]) {
    if (!c || !theta) return DIRAC_E_ARG;
    if (c->is_batch) return fail(c, DIRAC_E_STATE, "batch context");
    int narr = c->ndim == 3 ? 8 : 4;
    for (int q = 0; q < narr; ++q)
        if (!theta[q]) return fail(c, DIRAC_E_ARG, "null theta array %d", q);
    for (int q = 0; q < 8; ++q) c->theta[q] = q < narr ? theta[q] : nullptr;
    c->site_mode = true;
    return DIRAC_OK;
}

int dirac_set_links(dirac_ctx *c, void *const links[]) {
    if (!c) return DIRAC_E_ARG;
    if (c->is_batch) return fail(c, DIRAC_E_STATE, "batch context");
    if (c->zh && links) return fail(c, DIRAC_E_STATE, "links are not available in z-slab mode");
    if (c->zbc && links) return fail(c, DIRAC_E_STATE, "links are not available with DIRAC_ZERO_BC");
    for (int q = 0; q < 24; ++q) c->links[q] = nullptr;
    c->links_on = false;
    if (!links) return DIRAC_OK;
    const int nl = c->ndim == 3 ? 24 : 8;
    for (int q = 0; q < nl; ++q)
        if (!links[q]) return fail(c, DIRAC_E_ARG, "null link array %d", q);
    for (int q = 0; q < nl; ++q) c->links[q] = links[q];
    c->links_on = true;
    return DIRAC_OK;
}

int dirac_coef_from_theta_host(float *coef, const double *theta, int64_t n) {
    if (!coef || !theta || n < 0) return DIRAC_E_ARG;
    for (int64_t t = 0; t < n; ++t) {
        if (!isfinite(theta[t])) return DIRAC_E_NONFINITE;
        gamma32_search(theta[t], &coef[2 * t], &coef[2 * t + 1]);
    }
    return DIRAC_OK;
}

int dirac_coef_from_theta(void *coef, const void *theta, int64_t n, void *stream) {
    return dirac_coef_from_theta_c(coef, theta, nullptr, n, stream);
}

int dirac_coef_from_theta_c(void *coef, const void *theta, const void *theta_im, int64_t n, void *stream) {
    if (!coef || !theta || n < 0) return DIRAC_E_ARG;
    if (n == 0) return DIRAC_OK;
    if (launch_coef_from_theta(coef, (const double *)theta, (const double *)theta_im, n, (hipStream_t)stream) !=
        hipSuccess)
        return DIRAC_E_HIP;
    return DIRAC_OK;
}

int dirac_coef_from_fields(void *coef, int dtype, double dt, double sgn_m, const void *v, const void *w, int64_t n,
                           void *stream) {
    if (!coef || n < 0 || !isfinite(dt) || !isfinite(sgn_m)) return DIRAC_E_ARG;
    if (dtype != DIRAC_C64 && dtype != DIRAC_C128) return DIRAC_E_ARG;
    if (dtype == DIRAC_C128 && w) return DIRAC_E_ARG;     // complex128 records hold a real theta
    if (n == 0) return DIRAC_OK;
    if (launch_coef_from_fields(coef, dtype == DIRAC_C64, 0.5 * dt, sgn_m, (const double *)v, (const double *)w, n,
                                (hipStream_t)stream) != hipSuccess)
        return DIRAC_E_HIP;
    return DIRAC_OK;
}

int dirac_theta_from_fields(dirac_ctx *c, double m, void *const v_site[], void *const theta[], void *stream) {
    if (!c || !theta || !isfinite(m)) return DIRAC_E_ARG;
    if (c->is_batch) return fail(c, DIRAC_E_STATE, "batch context");
    int narr = c->ndim == 3 ? 8 : 4;
    for (int q = 0; q < narr; ++q)
        if (!theta[q]) return fail(c, DIRAC_E_ARG, "null theta array %d", q);
    void *th8[8] = {0}, *v8[8] = {0};
    for (int q = 0; q < narr; ++q) {
        th8[q] = theta[q];
        v8[q] = v_site ? v_site[q] : nullptr;
    }
    hipStream_t s = (hipStream_t)stream;
    int64_t ncell = c->nx * c->ny * planes_of(c);
    if (c->dtype == DIRAC_C64) HIPCHK(c, launch_theta_fields<float>(th8, v8, narr, ncell, 0.5 * c->dt, m, s));
    else HIPCHK(c, launch_theta_fields<double>(th8, v8, narr, ncell, 0.5 * c->dt, m, s));
    c->m = m;
    return dirac_set_theta_field(c, theta);
}

int dirac_set_kernel(dirac_ctx *c, int kernel, int tile_y, int zchunk) {
    if (!c) return DIRAC_E_ARG;
    if (kernel < DIRAC_KERNEL_AUTO || kernel > DIRAC_KERNEL_FUSED2) return fail(c, DIRAC_E_ARG, "bad kernel %d", kernel);
    if (tile_y != 0 && tile_y != 4 && tile_y != 8) return fail(c, DIRAC_E_ARG, "tile_y must be 0, 4 or 8");
    if (zchunk < 0) return fail(c, DIRAC_E_ARG, "zchunk must be >= 0");
    c->kernel = kernel;
    c->tile_y = tile_y;
    c->zchunk = zchunk;
    return DIRAC_OK;
}

int dirac_step(dirac_ctx *c, int64_t n, void *stream) {
    int rc = check_ready(c, !c || !c->site_mode);
    if (rc) return rc;
    if (n < 0) return fail(c, DIRAC_E_ARG, "n must be >= 0");
    rc = slab_step_check(c, n);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    return c->dtype == DIRAC_C64 ? run_steps<float>(c, n, false, s) : run_steps<double>(c, n, false, s);
}

int dirac_reverse(dirac_ctx *c, int64_t n, void *stream) {
    int rc = check_ready(c, !c || !c->site_mode);
    if (rc) return rc;
    if (c->zh) return fail(c, DIRAC_E_STATE, "z-slab contexts step forward only");
    if (n < 0) return fail(c, DIRAC_E_ARG, "n must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    return c->dtype == DIRAC_C64 ? run_steps<float>(c, n, true, s) : run_steps<double>(c, n, true, s);
}

int dirac_step_norm(dirac_ctx *c, int64_t n, void *dev_out, void *stream) {
    int rc = check_ready(c, true);
    if (rc) return rc;
    if (n < 1 || !dev_out) return fail(c, DIRAC_E_ARG, "need n >= 1 and an output");
    rc = slab_step_check(c, n);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    double *part = (double *)scratch_at(c, off_partial(c));
    const size_t cap_sz = partial_doubles(c) / 2;
    const int cap = cap_sz > 0x7fffffff ? 0x7fffffff : (int)cap_sz;
    const int kc = kernel_choice(c);
    if (c->ndim == 3 && kc == DIRAC_KERNEL_FUSED2 && n >= 2 && !c->links_on) {
        rc = dirac_step(c, n - 2, stream);
        if (rc) return rc;
        rc = upload_tables(c, s);
        if (rc) return rc;
        int nb = 0;
        hipError_t e;
        if (c->dtype == DIRAC_C64) {
            FusedArgs<float> a = fused_args<float>(c);
            a.npart = part;
            a.npart_cap = cap;
            e = launch_fused3x2<float>(a, c->site_mode, s, &nb);
        } else {
            FusedArgs<double> a = fused_args<double>(c);
            a.npart = part;
            a.npart_cap = cap;
            e = launch_fused3x2<double>(a, c->site_mode, s, &nb);
        }
        if (e == hipSuccess) {
            c->cur = 1 - c->cur;
            HIPCHK(c, launch_final_sum(part, nb, 2, (double *)dev_out, s));
            return DIRAC_OK;
        }
        if (nb <= cap) HIPCHK(c, e);   // a real launch failure
        // more workgroups than partial slots (the area is sized so that this
        // does not happen).  A z-slab's halos are stale after a launch, so a
        // reduction after the step would be wrong there: refuse.  Otherwise the
        // same two steps without the in-step sum, then the reduction.
        if (c->zh) return fail(c, DIRAC_E_SHAPE, "z-slab mode: %d workgroups exceed the %d partial slots", nb, cap);
        if (c->dtype == DIRAC_C64) HIPCHK(c, launch_fused3x2<float>(fused_args<float>(c), c->site_mode, s));
        else HIPCHK(c, launch_fused3x2<double>(fused_args<double>(c), c->site_mode, s));
        c->cur = 1 - c->cur;
        double *res = (double *)scratch_at(c, off_result(c));
        rc = dirac_norm_device(c, res, stream);
        if (rc) return rc;
        HIPCHK(c, hipMemcpyAsync(dev_out, res + 1, 2 * sizeof(double), hipMemcpyDeviceToDevice, s));
        return DIRAC_OK;
    } else {
        rc = dirac_step(c, n - 1, stream);
        if (rc) return rc;
    }
    if (c->ndim == 3 && (kc == DIRAC_KERNEL_FUSED || kc == DIRAC_KERNEL_FUSED2) && !c->links_on) {
        int nb = 0;
        hipError_t e;
        if (c->dtype == DIRAC_C64) {
            FusedArgs<float> a = fused_args<float>(c);
            a.npart = part;
            a.npart_cap = cap;
            e = launch_fused3<float>(a, c->site_mode, c->tile_y, s, &nb);
        } else {
            FusedArgs<double> a = fused_args<double>(c);
            a.npart = part;
            a.npart_cap = cap;
            e = launch_fused3<double>(a, c->site_mode, c->tile_y, s, &nb);
        }
        if (e == hipSuccess) {
            c->cur = 1 - c->cur;
            HIPCHK(c, launch_final_sum(part, nb, 2, (double *)dev_out, s));
            return DIRAC_OK;
        }
        if (nb <= cap) HIPCHK(c, e);   // a real launch failure
        if (c->zh) return fail(c, DIRAC_E_SHAPE, "z-slab mode: %d workgroups exceed the %d partial slots", nb, cap);
    }
    rc = dirac_step(c, 1, stream);
    if (rc) return rc;
    double *res = (double *)scratch_at(c, off_result(c));
    rc = dirac_norm_device(c, res, stream);
    if (rc) return rc;
    HIPCHK(c, hipMemcpyAsync(dev_out, res + 1, 2 * sizeof(double), hipMemcpyDeviceToDevice, s));
    return DIRAC_OK;
}

int dirac_norm_device(dirac_ctx *c, void *dev_out, void *stream) {
    int rc = check_ready(c, true);
    if (rc) return rc;
    if (!dev_out) return fail(c, DIRAC_E_ARG, "null output");
    hipStream_t s = (hipStream_t)stream;
    double *part = (double *)scratch_at(c, off_partial(c));
    if (c->links_on) {
        const LinkPtrs L = link_ptrs(c);
        if (c->dtype == DIRAC_C64) HIPCHK(c, launch_norm_links<float>(reduce_args<float>(c, 0.0), L, c->ndim, s));
        else HIPCHK(c, launch_norm_links<double>(reduce_args<double>(c, 0.0), L, c->ndim, s));
    } else if (c->dtype == DIRAC_C64) {
        ReduceArgs<float> a = reduce_args<float>(c, 0.0);
        HIPCHK(c, c->ndim == 3 ? launch_norm3<float>(a, s) : launch_norm2<float>(a, s));
    } else {
        ReduceArgs<double> a = reduce_args<double>(c, 0.0);
        HIPCHK(c, c->ndim == 3 ? launch_norm3<double>(a, s) : launch_norm2<double>(a, s));
    }
    HIPCHK(c, launch_final_sum(part, kReduceBlocks, kNormVals, (double *)dev_out, s));
    return DIRAC_OK;
}

int dirac_norm(dirac_ctx *c, double out[3], void *stream) {
    if (!out) return c ? fail(c, DIRAC_E_ARG, "null output") : DIRAC_E_ARG;
    int rc = check_ready(c, true);
    if (rc) return rc;
    double *res = (double *)scratch_at(c, off_result(c));
    rc = dirac_norm_device(c, res, stream);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipMemcpyAsync(out, res, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    for (int q = 0; q < 3; ++q)
        if (!isfinite(out[q])) return fail(c, DIRAC_E_NONFINITE, "norm value %d is not finite", q);
    return DIRAC_OK;
}

int dirac_observables(dirac_ctx *c, double z0, double out[9], void *stream) {
    int rc = check_ready(c, true);
    if (rc) return rc;
    if (c->zh) return fail(c, DIRAC_E_STATE, "not available in z-slab mode (dirac_norm is)");
    if (!out || !isfinite(z0)) return fail(c, DIRAC_E_ARG, "bad output or z0");
    hipStream_t s = (hipStream_t)stream;
    double *part = (double *)scratch_at(c, off_partial(c));
    double *res = (double *)scratch_at(c, off_result(c));
    if (c->dtype == DIRAC_C64) {
        ReduceArgs<float> a = reduce_args<float>(c, z0);
        HIPCHK(c, c->ndim == 3 ? launch_obs3<float>(a, s) : launch_obs2<float>(a, s));
    } else {
        ReduceArgs<double> a = reduce_args<double>(c, z0);
        HIPCHK(c, c->ndim == 3 ? launch_obs3<double>(a, s) : launch_obs2<double>(a, s));
    }
    HIPCHK(c, launch_final_sum(part, kReduceBlocks, kObsVals, res, s));
    HIPCHK(c, hipMemcpyAsync(out, res, kObsVals * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    for (int q = 0; q < kObsVals; ++q)
        if (!isfinite(out[q])) return fail(c, DIRAC_E_NONFINITE, "observable %d is not finite", q);
    return DIRAC_OK;
}

int dirac_seed_region(dirac_ctx *c, double z0, void *const lam[], void *stream) {
    int rc = check_ready(c, false);
    if (rc) return rc;
    if (c->zh) return fail(c, DIRAC_E_STATE, "not available in z-slab mode");
    if (!lam || !isfinite(z0)) return fail(c, DIRAC_E_ARG, "bad lam or z0");
    int narr = c->ndim == 3 ? 8 : 4;
    void *l8[8] = {0};
    for (int q = 0; q < narr; ++q) {
        if (!lam[q]) return fail(c, DIRAC_E_ARG, "null lam array %d", q);
        l8[q] = lam[q];
    }
    hipStream_t s = (hipStream_t)stream;
    if (c->dtype == DIRAC_C64) {
        ReduceArgs<float> a = reduce_args<float>(c, z0);
        HIPCHK(c, c->ndim == 3 ? launch_seed3<float>(a, l8, s) : launch_seed2<float>(a, l8, s));
    } else {
        ReduceArgs<double> a = reduce_args<double>(c, z0);
        HIPCHK(c, c->ndim == 3 ? launch_seed3<double>(a, l8, s) : launch_seed2<double>(a, l8, s));
    }
    return DIRAC_OK;
}

int dirac_adjoint(dirac_ctx *c, int64_t n, void *const lam[], double z0, void *dLdV_int, void *dLdV_half,
                  void *stream) {
    int rc = dirac_seed_region(c, z0, lam, stream);
    if (rc) return rc;
    return dirac_adjoint_vz(c, n, lam, dLdV_int, dLdV_half, stream);
}

int dirac_adjoint_vz(dirac_ctx *c, int64_t n, void *const lam[], void *dLdV_int, void *dLdV_half, void *stream) {
    int rc = check_ready(c, true);
    if (rc) return rc;
    if (c->ndim != 3) return fail(c, DIRAC_E_STATE, "the V(z) gradient is defined for 3D lattices");
    if (c->zh) return fail(c, DIRAC_E_STATE, "not available in z-slab mode");
    if (c->site_mode) return fail(c, DIRAC_E_STATE, "needs a V(z) profile (dirac_set_mass_potential_z)");
    if (!c->w_int.empty())
        return fail(c, DIRAC_E_STATE, "the reversal-based adjoint needs a real potential (no absorbing layers)");
    if (c->links_on) return fail(c, DIRAC_E_STATE, "the V(z) gradient kernels carry no gauge links");
    if (c->zbc) return fail(c, DIRAC_E_STATE, "the V(z) gradient kernels are periodic (no DIRAC_ZERO_BC)");
    if (n < 0 || !lam || !dLdV_int || !dLdV_half) return fail(c, DIRAC_E_ARG, "bad arguments");
    for (int q = 0; q < 8; ++q)
        if (!lam[q]) return fail(c, DIRAC_E_ARG, "null lam array %d", q);
    hipStream_t s = (hipStream_t)stream;
    rc = upload_tables(c, s);
    if (rc) return rc;
    const int ntiles = adj_tiles3((int)c->nx, (int)c->ny);
    double *gpart = (double *)scratch_at(c, off_gpart(c));
    HIPCHK(c, launch_zero(gpart, (int64_t)ntiles * c->nz * 2, s));
    auto run = [&](auto zero) -> int {
        using R = decltype(zero);
        AdjArgs<R> a;
        memset(&a, 0, sizeof a);
        for (int q = 0; q < 8; ++q) {
            a.f[q] = c->buf[c->cur][q];
            a.lam[q] = lam[q];
        }
        size_t half = align256(tab_bytes<R>(c));
        a.tab_f = (const R *)scratch_at(c, off_tab(c));
        a.tab_r = (const R *)scratch_at(c, off_tab(c) + half);
        a.rx = (R)c->rx;
        a.ry = (R)c->ry;
        a.rz = (R)c->rz;
        a.nx = (int)c->nx;
        a.ny = (int)c->ny;
        a.nz = (int)c->nz;
        a.gpart = gpart;
        // sweeps 0, 1, 2 per backward step; sweep 2 of a step and sweep 0 of the
        // next run as one launch (sweep 3)
        if (n > 0) HIPCHK(c, launch_adj3<R>(a, 0, s));
        for (int64_t t = 0; t < n; ++t) {
            HIPCHK(c, launch_adj3<R>(a, 1, s));
            HIPCHK(c, launch_adj3<R>(a, t + 1 < n ? 3 : 2, s));
        }
        return DIRAC_OK;
    };
    rc = c->dtype == DIRAC_C64 ? run(0.0f) : run(0.0);
    if (rc) return rc;
    HIPCHK(c, launch_adj_finish(gpart, ntiles, (int)c->nz, 0.5 * c->dt, (double *)dLdV_int, (double *)dLdV_half, s));
    return DIRAC_OK;
}

}  // extern "C"
