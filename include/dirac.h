/*
 * dirac.h -- C ABI of the MI355X (gfx950) implementation of the single-cone
 * staggered leap-frog scheme for the time-dependent Dirac equation
 * (R. Hammer, W. Poetz, A. Arnold, arXiv:1309.3452).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units: hbar = c = 1.  r_j = dt / d_j (Sect. 2.2, "r_j = Delta_o/Delta_j").
 *
 * State (Sect. 2, Eq. ABCDgrid; Sect. 3 for 2D).  A (3+1)D state is 8 device
 * arrays, in this order:
 *     A0 (i,j,k)        A1 (i+1/2,j+1/2,k)      -- time sheet n-1/2
 *     B0 (i+1/2,j,k+1/2) B1 (i,j+1/2,k+1/2)     -- time sheet n-1/2
 *     C0 (i,j,k+1/2)    C1 (i+1/2,j+1/2,k+1/2)  -- time sheet n
 *     D0 (i+1/2,j,k)    D1 (i,j+1/2,k)          -- time sheet n
 * where the position is that of the amplitude stored for cell (i,j,k).  A
 * (2+1)D state is 4 arrays u0 (i,j), u1 (i+1/2,j+1/2) on sheet n-1/2 and
 * v0 (i+1/2,j), v1 (i,j+1/2) on sheet n.  Each array holds one complex
 * amplitude per cell, interleaved (re, im), [k][j][i] with i fastest, no
 * padding: complex64 (DIRAC_C64) or complex128 (DIRAC_C128).  Boundaries are
 * periodic in every direction (zero outside the lattice with DIRAC_ZERO_BC).
 *
 * Ownership: every device buffer is allocated by the caller and borrowed by
 * raw pointer; it must stay valid while bound.  The library allocates only its
 * host-side context; it never frees caller memory.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 * stream).  Launching calls are asynchronous on it unless said otherwise.
 *
 * Errors: every int-returning call returns DIRAC_OK (0) or a negative
 * DIRAC_E_* code.  Arguments are validated before any HIP call; a failed call
 * leaves the context unchanged.  dirac_last_error() gives a message for the
 * last failure on a context.  Nothing aborts or throws across the ABI.
 * A context is not thread-safe; use one per stream.
 */
#ifndef DIRAC_H
#define DIRAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dirac_ctx dirac_ctx;

enum dirac_dtype { DIRAC_C64 = 1, DIRAC_C128 = 2 };

enum dirac_status {
    DIRAC_OK = 0,
    DIRAC_E_ARG = -1,        /* null pointer, bad enum or value out of range      */
    DIRAC_E_SHAPE = -2,      /* lattice sizes or buffer sizes do not fit          */
    DIRAC_E_UNSTABLE = -3,   /* r_x^2 + r_y^2 (+ r_z^2) > 1 without ALLOW_UNSTABLE */
    DIRAC_E_NONFINITE = -4,  /* a reduction met NaN or Inf                        */
    DIRAC_E_HIP = -5,        /* a HIP runtime call failed (message has details)   */
    DIRAC_E_STATE = -6       /* call out of order (e.g. no state bound yet)       */
};

/* dirac_create flags */
#define DIRAC_ALLOW_UNSTABLE 1u
/*
 * z-slab mode (3D): the context is one z-slab of a larger lattice, the unit a
 * multi-GPU run gives each device (the paper's closing remark on splitting
 * space into sub-domains that trade boundary values).  Every bound array
 * (state, per-site fields) holds nz + 4 planes: two halo planes below, the nz
 * interior planes, two halo planes above; V(z) tables take nz + 4 entries, one
 * per stored plane.  z is not periodic: a call of dirac_step reads the halo
 * planes and writes the interior only, so before each call the caller fills
 * the halos of the current buffer set with the neighbouring slabs' outermost
 * two interior planes (all 8 arrays).  With nx even for complex64 (any nx for
 * complex128) a call may advance two steps in one launch of the two-step
 * kernel, whose reach in z over two steps is the two halo planes; otherwise
 * (odd nx in complex64, or DIRAC_KERNEL_FUSED set) one step by the one-step
 * kernel.
 * dirac_halo_steps tells which; a larger n is refused (DIRAC_E_ARG).  Each
 * launch moves the state to the other buffer set.  dirac_step_norm and
 * dirac_norm sum the interior (slab sums add up to the whole lattice's).  dirac_reverse, dirac_observables,
 * dirac_seed_region, dirac_adjoint_vz and links are refused (DIRAC_E_STATE).
 */
#define DIRAC_SLAB_Z 2u
/*
 * Zero values outside the lattice (2D and 3D): every neighbour that lies
 * across a face of the box of cells reads as zero, in the steps, the reversed
 * steps and the conserved functional, instead of wrapping periodically.  The
 * summation by parts in the proofs of the Lemmas (Sect. 2, Sect. 3) leaves no
 * boundary terms with zero values outside either, so E_r stays exactly
 * conserved.  Steps run on the split kernels (one launch per half-step, in
 * place).  Not combined with DIRAC_SLAB_Z (DIRAC_E_ARG); dirac_set_links and
 * dirac_adjoint_vz are refused (DIRAC_E_STATE).
 */
#define DIRAC_ZERO_BC 4u

/* step kernels (dirac_set_kernel) */
enum dirac_kernel {
    DIRAC_KERNEL_AUTO = 0,   /* FUSED2 where it applies, else FUSED                */
    DIRAC_KERNEL_SPLIT = 1,  /* one launch per half-step, in place                 */
    DIRAC_KERNEL_FUSED = 2,  /* one launch per step, ping-pong between the buffers */
    DIRAC_KERNEL_FUSED2 = 3  /* one launch per two steps (3D: V(z) tables or
                                per-site records, nx even for complex64; 2D), ping-
                                pong; an odd remainder and other cases take FUSED */
};

/* Human-readable name of a status code (static storage). */
const char *dirac_status_string(int status);

/*
 * Create a lattice context.
 *   ndim   2 or 3.  For ndim == 2, nz must be 1 and dz is ignored.
 *   nx, ny, nz  cells per direction, each >= 1; nx*ny*nz < 2^40.
 *   dtype  DIRAC_C64 (complex64 storage and FP32 arithmetic, FP64 reductions)
 *          or DIRAC_C128 (FP64 throughout).
 *   dt     time step (Delta_o = dt); dx, dy, dz > 0 grid spacings.
 *   flags  DIRAC_ALLOW_UNSTABLE to accept sum r_j^2 > 1 (the scheme then
 *          grows, Sect. 2.2 and Sect. 3 "reality condition"); DIRAC_SLAB_Z
 *          (ndim == 3) for z-slab mode, nz then counting interior planes;
 *          DIRAC_ZERO_BC for zero values outside the lattice.
 * Validates the stability bound sum_j r_j^2 <= 1 of Sect. 2.2 (3D) / Sect. 3
 * (2D).  The context starts with m = 0, V = 0.  Makes no HIP call.
 */
int dirac_create(dirac_ctx **out, int ndim, int64_t nx, int64_t ny, int64_t nz, int dtype,
                 double dt, double dx, double dy, double dz, unsigned flags);

/* Release the context (and any graph it owns).  Safe on NULL. */
void dirac_destroy(dirac_ctx *ctx);

/* Message of the last failure on ctx ("" if none); valid until the next call. */
const char *dirac_last_error(const dirac_ctx *ctx);

/*
 * Bind the state: the staggered amplitudes of Sect. 2 (A, B on sheet n-1/2,
 * C, D on sheet n; Fig. 1) or Sect. 3 (u, v).  buf0 and buf1 each give 8 (3D)
 * or 4 (2D) device arrays of nx*ny*nz amplitudes in the layout above.  buf0
 * holds the initial state; buf1 is the partner the fused kernel writes into
 * (it may alias nothing the caller still needs).  The current state flips
 * between them as fused steps run; dirac_current() says where it is.  The
 * arrays stay caller-owned and must outlive their use; DIRAC_E_ARG for null
 * pointers.  No HIP call.
 */
int dirac_bind_state(dirac_ctx *ctx, void *const buf0[], void *const buf1[]);

/* which = 0 if buf0 holds the current state, 1 if buf1 does. */
int dirac_current(const dirac_ctx *ctx, int *which);

/* Declare which bound buffer set holds the current state (after the caller
 * wrote a new state into it). */
int dirac_set_current(dirac_ctx *ctx, int which);

/* z-slab mode: *steps = the most steps one dirac_step / dirac_step_norm call
 * may advance between halo refills (2 when the two-step kernel applies, else
 * 1); 0 for other contexts (no limit).  Makes no HIP call; DIRAC_E_ARG for
 * null arguments. */
int dirac_halo_steps(const dirac_ctx *ctx, int *steps);

/*
 * Scratch for reductions and gradients.  dirac_scratch_bytes reports the size
 * this context needs; the caller allocates at least that much device memory
 * (256-byte aligned) and binds it.  Required before norm/observables/adjoint.
 */
int dirac_scratch_bytes(const dirac_ctx *ctx, size_t *bytes);
int dirac_bind_scratch(dirac_ctx *ctx, void *dev, size_t bytes);

/*
 * Mass and a potential that depends on z only (3D) or is zero (2D), Eqs. ss1-ss4:
 * theta = (dt/2)(m + V) at A,B sites on sheet n and (dt/2)(-m + V) at C,D
 * sites on sheet n+1/2, each at the amplitude's own z.
 *   v_int[k]  = V(z = k)      (used at A and D sites),
 *   v_half[k] = V(z = k+1/2)  (used at B and C sites),
 * host arrays of nz doubles, or both NULL for V = 0.  In 2D pass nz = 1 and
 * NULL arrays (use dirac_theta_from_fields for V(x, y)).  Replaces any
 * per-site field.  Copies the tables to the device on the next launch.
 */
int dirac_set_mass_potential_z(dirac_ctx *ctx, double m, const double *v_int, const double *v_half,
                               int64_t nz);

/* The mass alone (the m of Eqs. ss1-ss4), keeping the V(z) tables last set (V = 0
 * if none): dirac_set_mass_potential_z(ctx, m, <current tables>).  Leaves a
 * per-site mode for the V(z) mode.  No HIP call; errors as that call. */
int dirac_set_mass(dirac_ctx *ctx, double m);

/* The V(z) tables alone (as dirac_set_mass_potential_z), keeping the mass last
 * set.  No HIP call; errors as that call. */
int dirac_set_potential_z(dirac_ctx *ctx, const double *v_int, const double *v_half, int64_t nz);

/*
 * Imaginary part of a z-dependent potential, V(z) = V_re(z) + i W(z): absorbing
 * layers (the growth factors of Sect. 3's stability analysis have modulus
 * below one where the imaginary part has the damping sign; in the Cayley form
 * alpha = (1 - i theta)/(1 + i theta) used here that is W < 0).  w_int[k] =
 * W(z = k) (A, D sites), w_half[k] = W(z = k+1/2) (B, C sites): host arrays of
 * nz doubles, or both NULL (or all zero) for none.  Combines with
 * dirac_set_mass_potential_z; the tables hold the complex Cayley factors from
 * the next launch on.  With W != 0 the functional E_r decreases by
 * sum Im(theta) |X+ + X-|^2 per step; the reversed step amplifies (it is the
 * exact inverse) and dirac_adjoint_vz is refused (DIRAC_E_STATE).
 */
int dirac_set_potential_im_z(dirac_ctx *ctx, const double *w_int, const double *w_half, int64_t nz);

/*
 * Per-site mass and potential (the time-averaged term of Eqs. ss1-ss4 with
 * theta = (dt/2)(+-m + V) at every amplitude's own site: + for A,B / u, - for
 * C,D / v).  v_site[a] is a device array (real, float for DIRAC_C64 and double
 * for DIRAC_C128, one value per cell) holding V at the sites of state array a,
 * or NULL for V = 0 there.  coef[a] are caller-owned device arrays, one record
 * per cell, that receive the per-site coefficient record:
 *   DIRAC_C128: theta itself (double);
 *   DIRAC_C64:  gamma = 1 - alpha = 2 i theta / (1 + i theta) as a complex64
 *               (8 bytes per site), rounded once to the float pair closest to
 *               |1 - gamma| = 1 (beta = 1 - gamma/2 is derived in the kernels),
 *               so no step re-evaluates the Cayley factors.
 * theta is formed in FP64.  The arrays stay bound and are read by every later
 * step until replaced.  Asynchronous on stream.
 */
int dirac_theta_from_fields(dirac_ctx *ctx, double m, void *const v_site[], void *const coef[],
                            void *stream);

/* Bind already computed per-site coefficient arrays (format as above): the
 * time-averaged mass and potential term of Eqs. ss1-ss4 (Sect. 3 in 2D).
 * Caller-owned, read by every later step until replaced.  No HIP call. */
int dirac_set_theta_field(dirac_ctx *ctx, void *const coef[]);

/*
 * The complex64 per-site coefficient record from theta: coef[t] = gamma(theta[t])
 * (format of dirac_theta_from_fields; the Cayley form of the time-averaged term
 * of Eqs. ss1-ss4) for t < n.  theta: device array of n
 * doubles; coef: device array of n complex64.  Context-free.  Asynchronous on
 * stream; DIRAC_E_ARG for null pointers or n < 0, DIRAC_E_HIP on launch failure.
 */
int dirac_coef_from_theta(void *coef, const void *theta, int64_t n, void *stream);

/*
 * dirac_coef_from_theta computed on the host: coef[2t], coef[2t+1] = the
 * complex64 record gamma(theta[t]) (the same rounding, from the same source,
 * as the device records and the V(z) tables) for t < n.  theta: host array of
 * n doubles; coef: host array of 2n floats.  Context-free, synchronous, makes
 * no HIP call; DIRAC_E_ARG for null pointers or n < 0, DIRAC_E_NONFINITE for a
 * non-finite theta (records before it are written).
 */
int dirac_coef_from_theta_host(float *coef, const double *theta, int64_t n);

/*
 * As dirac_coef_from_theta for a complex theta = theta[t] + i theta_im[t]
 * (theta_im: device array of n doubles, (dt/2) Im V per site, or NULL): the
 * complex64 record gamma = 1 - alpha, rounded once from FP64 where Im theta !=
 * 0 (|alpha| != 1 there) and by the unit-modulus search elsewhere (absorbing
 * potentials, after Sect. 3's remark on imaginary potentials).  Per-site
 * complex potentials are supported for complex64 lattices and batches.
 * Context-free, asynchronous; DIRAC_E_ARG for null coef/theta or n < 0.
 */
int dirac_coef_from_theta_c(void *coef, const void *theta, const void *theta_im, int64_t n, void *stream);

/*
 * Vector potential by gauge links (Sect. 4: the Peierls substitution applied
 * to each neighbour coupling of Eqs. ss1-ss4 / scheme2Deq-scheme4thline).
 * links: 24 (3D) or 8 (2D) caller-owned device arrays, one complex per cell in
 * the lattice's storage type (complex64 for DIRAC_C64, complex128 for
 * DIRAC_C128), laid out like the state arrays.  links[6 a + t] (3D) /
 * links[4 a + t] (2D) belongs to state array a of the A,B group (A0, A1, B0,
 * B1) / u group (u0, u1) and neighbour term t in the order +z, -z, +x, -x, +y,
 * -y (2D: +x, -x, +y, -y): in S_X of that array at cell c, the neighbour
 * value reached in direction t is multiplied by links[6 a + t][c].  The C,D /
 * v rows use the complex conjugate of the factor of the same half-link, taken
 * at its A,B / u end.  For U = exp(-i a_j(mid) d_j) (a_j the Peierls phase per
 * unit length at the half-link midpoint, d_j the signed displacement) the
 * coupling is gauge covariant: with U = exp(i (chi(Y) - chi(X))) a step maps
 * exp(-i chi) psi to exp(-i chi) times the free step of psi.  Unit-modulus
 * links keep E_r (dirac_norm, evaluated with the links) exactly conserved.
 * While links are bound, a step takes one launch (a z-march in 3D, a y-march in
 * 2D) that moves the state to the other buffer set, unless DIRAC_KERNEL_SPLIT
 * is set; the reversed step and DIRAC_KERNEL_SPLIT use the in-place split
 * kernels; all give the same bits.  dirac_step_norm steps, then reduces.
 * dirac_adjoint_vz is refused.  links == NULL unbinds them.  The arrays must stay valid while
 * bound.  DIRAC_E_ARG for a null link array (nothing is bound then),
 * DIRAC_E_STATE for a batch context.  Makes no HIP call.
 */
int dirac_set_links(dirac_ctx *ctx, void *const links[]);

/*
 * The per-site coefficient record of one state array from its fields (the
 * time-averaged term of Eqs. ss1-ss4 / scheme2Deq-scheme4thline), for lattices
 * and batches: theta[t] = (dt/2)(sgn_m + v[t]) + i (dt/2) w[t], formed in FP64
 * and written in the record format of dtype (see dirac_theta_from_fields):
 * DIRAC_C128 theta (double; w must be NULL), DIRAC_C64 gamma (complex64).
 * sgn_m: the mass with the array's sign, +m for A,B / u arrays, -m for C,D / v.
 * v, w: device arrays of n doubles (V and Im V at the array's sites), or NULL
 * for zero.  coef: device array of n records.  Context-free, asynchronous on
 * stream; DIRAC_E_ARG for bad arguments, DIRAC_E_HIP on launch failure.
 */
int dirac_coef_from_fields(void *coef, int dtype, double dt, double sgn_m, const void *v, const void *w,
                           int64_t n, void *stream);

/* Choose the step kernel and its tiling; 0 = library default for a knob.
 *   tile_y: cells along y per workgroup of the 3D one-step fused kernel: 4 or 8
 *           (default 8); its tile is 64 cells in x (128 for complex64 with nx even)
 *   zchunk: planes (3D) or rows (2D) per workgroup along the march of the fused
 *           kernels (default: chosen per kernel and lattice from the number of
 *           workgroups the device runs at once and each chunk's pipeline fill)
 * The two-step kernel uses 64 x 8 tiles (complex64) or 32 x 8 (complex128).
 * Every kernel gives the same bits.  The reversed step always uses the split
 * kernels, the adjoint its own in-place sweeps. */
int dirac_set_kernel(dirac_ctx *ctx, int kernel, int tile_y, int zchunk);

/*
 * Advance the bound state by n >= 0 full steps (Sect. 2: A,B from n-1/2 to
 * n+1/2 by Eqs. ss1, ss2, then C,D from n to n+1 by Eqs. ss3, ss4; Sect. 3:
 * u then v by Eqs. scheme2Deq-scheme4thline).  Asynchronous on stream.
 * Each fused launch moves the state to the other bound buffer set (FUSED2:
 * floor(n/2) two-step launches plus one one-step launch if n is odd; FUSED: n
 * launches; SPLIT: in place).  A stream capture of step calls replays
 * correctly any number of times only if the captured calls leave the state in
 * the buffer set they started from: compare dirac_current before and after.
 */
int dirac_step(dirac_ctx *ctx, int64_t n, void *stream);

/*
 * Undo n full steps exactly (up to rounding): the relations of Eqs. ss3, ss4
 * solved for the old C,D, then those of ss1, ss2 for the old A,B -- the step
 * with dt -> -dt in the opposite half-step order.  Asynchronous on stream.
 */
int dirac_reverse(dirac_ctx *ctx, int64_t n, void *stream);

/*
 * Conserved functional of Lemma, Sect. 2, Eq. (EPM) (3D) / Lemma, Sect. 3,
 * Eq. (E) with the delta_+ sign that the update equations conserve (2D):
 *   dev_out[0] = sum |X|^2 - Re sum_{A,B sites} conj(X) S_X(C,D)
 *   dev_out[1] = sum |X|^2 + Re sum_{C,D sites} conj(X) S_X(A,B)   (equal to [0])
 *   dev_out[2] = sum |X|^2 (the plain norm, conserved only on average)
 * accumulated in FP64 in a fixed order (run-to-run bitwise reproducible).
 * dirac_norm_device writes 3 doubles to device memory, asynchronously;
 * dirac_norm copies them to host `out` and synchronises the stream, and
 * returns DIRAC_E_NONFINITE if any is NaN/Inf.
 */
int dirac_norm_device(dirac_ctx *ctx, void *dev_out, void *stream);
int dirac_norm(dirac_ctx *ctx, double out[3], void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * dirac_norm_device without bound scratch.  Same values, same bits: the same
 * reduction kernels, whose partial sums go to a library-owned device array of
 * DIRAC_STATIC_SCRATCH_BYTES bytes per GPU (held until the process ends)
 * instead of the caller-bound scratch.  The reduction needs kReduceBlocks x 3
 * doubles (24 KiB) whatever the lattice size; a layout that did not fit would
 * be refused with DIRAC_E_SHAPE.  Allocates nothing (no hipMalloc, no
 * allocating library call); the array's device address is looked up once per
 * GPU on the first call there.  Every call on one GPU shares that array: calls
 * that overlap in time on one GPU (other streams, other threads, other
 * contexts) race and must be ordered by the caller.  Asynchronous on stream;
 * writes 3 doubles to dev_out.  DIRAC_E_ARG for a null context or output,
 * DIRAC_E_STATE without a bound state or for a batch context, DIRAC_E_HIP on a
 * failed lookup or launch.
 */
#define DIRAC_STATIC_SCRATCH_BYTES 65536
int dirac_norm_device_static(dirac_ctx *ctx, void *dev_out, void *stream);

/*
 * n >= 1 steps (as dirac_step) whose last step also evaluates, on the state it
 * produces, the conserved functional (Lemma of Sect. 2.2, Eq. EPM; Sect. 3 in
 * 2D) in its C,D-summed form (dev_out[0], equal to dirac_norm's values) and
 * the plain norm (dev_out[1]); two FP64 values
 * written to device memory, asynchronously, in a fixed order.  With the fused
 * (3+1)D kernel the functional is accumulated inside the step at no extra
 * pass over memory; otherwise a step is followed by the reduction.
 */
int dirac_step_norm(dirac_ctx *ctx, int64_t n, void *dev_out, void *stream);

/*
 * Observables of the plain density |X|^2 over all sites (its sum is the naive
 * norm of Sects. 2.2 and 3; a region sum is a transmitted or reflected
 * fraction as in the Klein-step simulation of Sect. 5), FP64, positions in
 * cell units (each amplitude at its own site):
 *   3D: out[0] = sum over sites with z >= z0, out[1..3] = sum x|X|^2, y|X|^2,
 *       z|X|^2, out[4] = sum |X|^2, out[5..8] = per component A, B, C, D.
 *   2D: out[0] = sum over sites with x >= z0, out[1..2] = sum x|X|^2, y|X|^2,
 *       out[3] = sum |X|^2, out[4..5] = per component u, v; out[6..8] = 0.
 * Synchronous; out has 9 doubles; DIRAC_E_NONFINITE if a value is not finite.
 */
int dirac_observables(dirac_ctx *ctx, double z0, double out[9], void *stream);

/*
 * Seed of the adjoint of L = sum_{z_s >= z0} |psi_s|^2 (3D; x_s >= z0 in 2D),
 * the region probability of dirac_observables: lam[a] = 2 psi on the region, 0
 * elsewhere, with lam = dL/dRe + i dL/dIm.  lam: caller-owned device arrays
 * shaped like the state.  Asynchronous; DIRAC_E_ARG for null arrays.
 */
int dirac_seed_region(dirac_ctx *ctx, double z0, void *const lam[], void *stream);

/*
 * Reverse-mode gradient of a function of the final state with respect to the
 * z-profile of V (3D, after dirac_set_mass_potential_z).  On entry the bound
 * state is psi after n steps and lam[] holds dL/dRe + i dL/dIm at that state.
 * Runs n backward steps, each rebuilding the previous state by the exact
 * reversed step (no stored trajectory) and carrying lam back by the chain rule
 * through Eqs. ss3, ss4 then ss1, ss2.  On return the state is the rebuilt
 * initial state, lam the adjoint at it, and the device FP64 arrays
 * dLdV_int[nz] (V at z = k: A, D sites) and dLdV_half[nz] (V at z = k+1/2:
 * B, C sites) hold dL/dV summed over all steps (overwritten, deterministic).
 * Works in place (state and lam): three per-cell sweeps per backward step in
 * two launches, the last sweep of a step sharing one with the first of the
 * next.  Asynchronous on stream.
 */
int dirac_adjoint_vz(dirac_ctx *ctx, int64_t n, void *const lam[], void *dLdV_int, void *dLdV_half,
                     void *stream);

/* The gradient of the region probability L = sum_{z_s >= z0} |psi_s|^2 after n
 * steps with respect to V(z): dirac_seed_region(ctx, z0, lam) then
 * dirac_adjoint_vz(ctx, n, lam, dLdV_int, dLdV_half).  lam: caller-owned work
 * arrays shaped like the state (on return the adjoint at the initial state).
 * Errors as those two calls. */
int dirac_adjoint(dirac_ctx *ctx, int64_t n, void *const lam[], double z0, void *dLdV_int, void *dLdV_half,
                  void *stream);

/* ------------------------------------------------------------------------ */
/* Batched (2+1)D lattices: many independent lattices of different size,    */
/* mass and potential advanced together.                                     */
/* ------------------------------------------------------------------------ */

/*
 * Create a batch of `count` 2D lattices advanced by the scheme of Sect. 3
 * (Eqs. scheme2Deq-scheme4thline), lattice b having nx[b] x ny[b] cells (each
 * >= 1), common dtype and dt (unit spacing), per-site theta supplied by
 * dirac_batch_bind.  Stability is checked as for dirac_create (Sect. 3's
 * bound).  No HIP call; DIRAC_E_ARG / DIRAC_E_UNSTABLE as for dirac_create.
 */
int dirac_batch_create(dirac_ctx **out, int64_t count, const int64_t *nx, const int64_t *ny, int dtype,
                       double dt, unsigned flags);

/*
 * As dirac_batch_create with a time step per lattice: dt[b] (host array of
 * count doubles, each finite and > 0) for lattice b, so r_x = r_y = dt[b] in
 * its steps and its functional (Sect. 3); the stability bound of Sect. 3 is
 * checked per lattice.  The per-site coefficient records bound with
 * dirac_batch_bind must be built with each lattice's own dt (theta =
 * (dt[b]/2)(+-m + V)).  dirac_batch_create(..., dt, ...) is this call with every
 * dt[b] = dt.  No HIP call; DIRAC_E_ARG for a null or non-positive dt,
 * DIRAC_E_UNSTABLE for a lattice above the bound without ALLOW_UNSTABLE.
 */
int dirac_batch_create_dt(dirac_ctx **out, int64_t count, const int64_t *nx, const int64_t *ny, int dtype,
                          const double *dt, unsigned flags);

/*
 * Bind the buffers of every lattice: state[4*b + a], partner[4*b + a] and
 * coef[4*b + a] for array a (u0 u1 v0 v1) of lattice b -- device pointers in
 * the single-lattice layout; coef holds the per-site coefficient record of
 * theta = (dt/2)(+-m + V) in the format of dirac_theta_from_fields (double
 * theta for C128, complex64 gamma for C64, e.g. from dirac_coef_from_theta).
 * Also binds the scratch (see dirac_scratch_bytes on the batch context).
 */
int dirac_batch_bind(dirac_ctx *ctx, void *const state[], void *const partner[], void *const theta[],
                     void *scratch, size_t scratch_bytes);

/*
 * Advance every lattice by n steps.  mode 0: one persistent launch for all n
 * steps with a per-lattice barrier between passes; mode 1: one launch per pass
 * over all lattices (both replayed from a captured HIP graph when use_graph !=
 * 0).  A pass advances one step or, with the tuned tile candidate's two-step
 * march (even nx for complex64), two; an odd remainder takes one one-step pass.
 * After an odd n the partner buffers hold the state (dirac_current).  Mode 0
 * needs its whole grid resident at once: the first mode-0 call for a kernel in
 * a process measures that grid by census-only launches (synchronous; no state
 * touched), and every persistent launch opens with a census that leaves
 * before any step if not all workgroups arrived.  Every per-lattice wait of
 * mode 0 is bounded.  If a wait times out, or a launch's census closes, every
 * workgroup leaves, the call returns DIRAC_E_HIP, and the lattices may be left
 * stepped unevenly across both buffer sets -- the bound state is then invalid
 * and must be reloaded.  Mode 0 calls synchronise with the stream.
 */
int dirac_batch_run(dirac_ctx *ctx, int64_t n, int mode, int use_graph, void *stream);

/* The conserved functional of Sect. 3 in both summed-by-parts forms and the
 * plain norm of every lattice: host out[3*count], FP64.  Synchronous. */
int dirac_batch_norms(dirac_ctx *ctx, double *out, void *stream);

/*
 * Pick the batched kernel's tile shape (x strip width, y chunk height) for
 * each mode by timing every candidate for a few steps on the bound lattices.
 * This advances the bound state by an even number of steps (it stays in the
 * same buffer set); callers that need the state unchanged save and restore it.
 * If a persistent (mode 0) candidate times out (see dirac_batch_run) it is
 * skipped, the choice is still made, stored and written to chosen_out, and the
 * call returns DIRAC_E_STATE: the bound state is no longer valid (reload it).
 * cache_path: JSON file consulted first and updated (NULL = no cache), keyed
 * by device architecture, dtype and batch shape.  The choice is kept in the
 * context.  Synchronous.  chosen_out (may be NULL) receives
 * (candidate for mode 1) | (candidate for mode 0) << 8.
 */
int dirac_batch_autotune(dirac_ctx *ctx, const char *cache_path, int *chosen_out, void *stream);

/* dirac_batch_autotune(ctx, cache_path, NULL, default stream): tile shapes are an
 * implementation choice with no counterpart in the paper.  DIRAC_E_STATE for a
 * single-lattice context (its knobs are dirac_set_kernel's). */
int dirac_autotune(dirac_ctx *ctx, const char *cache_path);

/*
 * Measurement utility, not a step of the method: a plain streaming copy of
 * `bytes` bytes from src to dst (device pointers, 8-byte aligned, not
 * overlapping; bytes a multiple of 8), each byte read once and written once.
 * It is the reference dispatch for the device's copy bandwidth and for scaling
 * the memory byte counters next to the library's kernels.  Context-free,
 * asynchronous on stream, allocates nothing.  DIRAC_E_ARG for null pointers, a
 * negative or unaligned size or address, or overlapping ranges; DIRAC_E_HIP on
 * launch failure.
 */
int dirac_stream_copy(void *dst, const void *src, int64_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DIRAC_H */
