/*
 * CPU FP64 oracle for the single-cone staggered leap-frog scheme of
 * R. Hammer, W. Poetz, A. Arnold, "Single-cone real-space finite difference
 * scheme for the time-dependent Dirac equation" (arXiv:1309.3452).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the HIP library.
 *
 * Plain and slow on purpose: every amplitude is addressed through its
 * physical position on the space-time staggered grid (in doubled
 * coordinates, so that half-integer positions are integers), and every
 * update is the paper's implicit relation solved for the new amplitude.
 *
 *   Grid (Sect. 2, Eq. list after Dirac-A; Eq. ABCDgrid), doubled coords:
 *     A : (2i,2j,2k)     and (2i+1,2j+1,2k)      arrays A0, A1
 *     B : (2i+1,2j,2k+1) and (2i,2j+1,2k+1)      arrays B0, B1
 *     C : (2i,2j,2k+1)   and (2i+1,2j+1,2k+1)    arrays C0, C1
 *     D : (2i+1,2j,2k)   and (2i,2j+1,2k)        arrays D0, D1
 *   (2+1)D grid (Sect. 3, text before Eq. scheme2Deq):
 *     u : (2i,2j) and (2i+1,2j+1)                arrays u0, u1
 *     v : (2i+1,2j) and (2i,2j+1)                arrays v0, v1
 *
 * Each array holds one complex amplitude per cell (i,j,k), stored
 * [k][j][i] with i fastest; all indices wrap periodically.
 *
 * Time convention (Sect. 2, Fig. 1 caption): A,B (u) sit on the half-integer
 * sheet n-1/2, C,D (v) on the integer sheet n.  One step first moves A,B to
 * n+1/2 from C,D at n (Eqs. ss1, ss2), then C,D to n+1 from the new A,B
 * (Eqs. ss3, ss4).  Mass and potential enter as the time average of
 * Eq. (3+3Ddis): with theta = (dt/2)(+-m + V) at the updated site,
 *     (X+ - X-) + S_X = -i theta (X+ + X-),
 * which this file solves as X+ = alpha X- - beta S_X,
 *     beta  = 1/(1 + i theta)       = (1 - i theta)/(1 + theta^2),
 *     alpha = (1 - i theta) beta    = (1 - theta^2 - 2 i theta)/(1 + theta^2).
 * The caller supplies theta per site (it folds m, V and dt).
 *
 * Readings taken where the paper is silent or garbled: periodic boundaries; V and m sampled at the updated
 * amplitude's own site and sheet; hbar = c = 1, so Delta_o = dt and
 * r_j = dt/Delta_j; in 2D the conserved functional carries delta_+ (the sign
 * that the printed update equations conserve), the printed delta_- form is
 * evaluated alongside for comparison.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

enum { CA = 0, CB = 1, CC = 2, CD = 3 };       /* 3D components */
enum { CU = 0, CV = 1 };                       /* 2D components */

static int g_bad_lookup = 0;                   /* set when a position is not a site */
/* Boundary: 0 = periodic wrap in every direction; 1 = zero values outside the
 * lattice (a site whose doubled coordinate leaves [0, 2n) holds 0).  The
 * summation by parts of the Lemmas (Sect. 2, Sect. 3) then has no boundary
 * terms either, so E_r stays exactly conserved. */
static int g_zero_bc = 0;

static int64_t wrap(int64_t a, int64_t n) {
    a %= n;
    return a < 0 ? a + n : a;
}

/* ------------------------------------------------------------------------ */
/* (3+1)D lattice                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t nx, ny, nz;
    cplx *f[8];                                /* A0 A1 B0 B1 C0 C1 D0 D1 */
} lat3;

/* parity of the doubled coordinates of each array's sites */
static const int OFF3[8][3] = {
    {0, 0, 0}, {1, 1, 0},                      /* A0, A1 */
    {1, 0, 1}, {0, 1, 1},                      /* B0, B1 */
    {0, 0, 1}, {1, 1, 1},                      /* C0, C1 */
    {1, 0, 0}, {0, 1, 0},                      /* D0, D1 */
};

/* Address of component `comp` at doubled position (X,Y,Z); NULL if no such site. */
static cplx *site3(const lat3 *L, int comp, int64_t X, int64_t Y, int64_t Z) {
    if (g_zero_bc && (X < 0 || X >= 2 * L->nx || Y < 0 || Y >= 2 * L->ny || Z < 0 || Z >= 2 * L->nz))
        return NULL;                           /* outside: a zero ghost, not a lookup error */
    X = wrap(X, 2 * L->nx);
    Y = wrap(Y, 2 * L->ny);
    Z = wrap(Z, 2 * L->nz);
    for (int s = 0; s < 2; ++s) {
        int a = 2 * comp + s;
        if ((X & 1) == OFF3[a][0] && (Y & 1) == OFF3[a][1] && (Z & 1) == OFF3[a][2])
            return &L->f[a][((Z >> 1) * L->ny + (Y >> 1)) * L->nx + (X >> 1)];
    }
    g_bad_lookup = 1;
    return NULL;
}

static cplx get3(const lat3 *L, int comp, int64_t X, int64_t Y, int64_t Z) {
    cplx *p = site3(L, comp, X, Y, Z);
    return p ? *p : 0.0;
}

/* One stencil term: coefficient class, source component, doubled offset. */
typedef struct { int cls; int comp; int dx, dy, dz; } term;
/* coefficient classes: +-r_z, +-r_x, +-i r_y */
enum { PZ, MZ, PX, MX, PIY, MIY };

static cplx coef(int cls, const double r[3]) {
    switch (cls) {
    case PZ:  return r[2];
    case MZ:  return -r[2];
    case PX:  return r[0];
    case MX:  return -r[0];
    case PIY: return I * r[1];
    default:  return -I * r[1];
    }
}

/*
 * The difference terms S_X of Eqs. ss1-ss4 (Lemma proof, Sect. 2), one row per
 * term, offsets of +-1 in doubled coordinates being +-1/2 cell:
 *   ss1  S_A =  r_z dz C + r_x dx D - i r_y dy D
 *   ss2  S_B = -r_z dz D + r_x dx C + i r_y dy C
 *   ss3  S_C =  r_z dz A + r_x dx B - i r_y dy B
 *   ss4  S_D = -r_z dz B + r_x dx A + i r_y dy A
 * with (d_j F)(s) = F(s + e_j/2) - F(s - e_j/2).
 */
static const term ST3[4][6] = {
    /* A */ {{PZ, CC, 0, 0, 1}, {MZ, CC, 0, 0, -1}, {PX, CD, 1, 0, 0}, {MX, CD, -1, 0, 0},
             {MIY, CD, 0, 1, 0}, {PIY, CD, 0, -1, 0}},
    /* B */ {{MZ, CD, 0, 0, 1}, {PZ, CD, 0, 0, -1}, {PX, CC, 1, 0, 0}, {MX, CC, -1, 0, 0},
             {PIY, CC, 0, 1, 0}, {MIY, CC, 0, -1, 0}},
    /* C */ {{PZ, CA, 0, 0, 1}, {MZ, CA, 0, 0, -1}, {PX, CB, 1, 0, 0}, {MX, CB, -1, 0, 0},
             {MIY, CB, 0, 1, 0}, {PIY, CB, 0, -1, 0}},
    /* D */ {{MZ, CB, 0, 0, 1}, {PZ, CB, 0, 0, -1}, {PX, CA, 1, 0, 0}, {MX, CA, -1, 0, 0},
             {PIY, CA, 0, 1, 0}, {MIY, CA, 0, -1, 0}},
};

static cplx stencil3(const lat3 *L, int comp, int64_t X, int64_t Y, int64_t Z, const double r[3]) {
    cplx s = 0.0;
    for (int t = 0; t < 6; ++t) {
        const term *q = &ST3[comp][t];
        s += coef(q->cls, r) * get3(L, q->comp, X + q->dx, Y + q->dy, Z + q->dz);
    }
    return s;
}

/*
 * Gauge links (a vector potential by the Peierls substitution of Sect. 4).  A
 * unit factor per half-link: in term t of S_X at an A,B site X (term order of
 * ST3: +z -z +x -x +y -y) the neighbour value is multiplied by U[6 a + t] at
 * X's cell, a the array of X.  At a C,D site Y the same half-link enters
 * conjugated: Y's neighbour X contributes with conj of X's factor for Y.  With
 * U = exp(-i q/(hbar c) times the line integral of A from X to Y) this is the
 * Peierls substitution, and to first order in A it is the rule of Sect. 4,
 * d_j psi -> d_j psi - i (q/(hbar c)) A_j times the mean of the two values.
 * The coupling stays anti-Hermitian, so E_r (with the same factors in S_X)
 * is conserved for a static potential.
 */
static int locate3(const lat3 *L, int comp, int64_t X, int64_t Y, int64_t Z, int64_t *cell) {
    X = wrap(X, 2 * L->nx);
    Y = wrap(Y, 2 * L->ny);
    Z = wrap(Z, 2 * L->nz);
    for (int s = 0; s < 2; ++s) {
        int a = 2 * comp + s;
        if ((X & 1) == OFF3[a][0] && (Y & 1) == OFF3[a][1] && (Z & 1) == OFF3[a][2]) {
            *cell = ((Z >> 1) * L->ny + (Y >> 1)) * L->nx + (X >> 1);
            return a;
        }
    }
    g_bad_lookup = 1;
    *cell = 0;
    return 0;
}

static cplx stencil3_links(const lat3 *L, int comp, int64_t X, int64_t Y, int64_t Z, const double r[3],
                           const cplx *const U[24]) {
    cplx s = 0.0;
    int64_t cx;
    int ax = locate3(L, comp, X, Y, Z, &cx);
    for (int t = 0; t < 6; ++t) {
        const term *q = &ST3[comp][t];
        int64_t QX = X + q->dx, QY = Y + q->dy, QZ = Z + q->dz;
        cplx u;
        if (comp == CA || comp == CB) {
            u = U[6 * ax + t][cx];
        } else {
            int64_t cq;
            int aq = locate3(L, q->comp, QX, QY, QZ, &cq);
            int tb = -1;                        /* the term of S at Q that points back to X */
            for (int t2 = 0; t2 < 6; ++t2) {
                const term *b = &ST3[q->comp][t2];
                if (b->dx == -q->dx && b->dy == -q->dy && b->dz == -q->dz) tb = t2;
            }
            if (tb < 0) {
                g_bad_lookup = 1;
                tb = 0;
            }
            u = conj(U[6 * aq + tb][cq]);
        }
        s += coef(q->cls, r) * u * get3(L, q->comp, QX, QY, QZ);
    }
    return s;
}

/* Cayley factors of the time average, from (1 + i th) X+ = (1 - i th) X- - S. */
static void cayley(double th, cplx *alpha, cplx *beta) {
    double d = 1.0 + th * th;
    *alpha = (1.0 - th * th) / d - I * ((2.0 * th) / d);
    *beta = 1.0 / d - I * (th / d);
}

/* The same relation for a complex theta = th + i thi (a complex potential V,
 * whose imaginary part damps or amplifies, Sect. 3 stability discussion):
 * alpha = (1 - i theta)/(1 + i theta), beta = 1/(1 + i theta) in complex
 * arithmetic.  thi = 0 is left to cayley() above. */
static void cayley_c(double th, double thi, cplx *alpha, cplx *beta) {
    if (thi == 0.0) {
        cayley(th, alpha, beta);
        return;
    }
    cplx t = th + I * thi;
    cplx d = 1.0 + I * t;
    *beta = 1.0 / d;
    *alpha = (1.0 - I * t) / d;
}

/* doubled position of cell (i,j,k) of array a */
#define POS3(a, i, j, k) (2 * (i) + OFF3[a][0]), (2 * (j) + OFF3[a][1]), (2 * (k) + OFF3[a][2])

/*
 * Half-step for the two components of one time sheet: every site of arrays
 * a_lo..a_lo+3 gets X+ = alpha X- - sgn*beta S_X.  sgn = +1 is the forward
 * half-step; sgn = -1 together with theta -> -theta solves the same relation
 * for X- (the reversed half-step).  S_X only reads the other sheet's two
 * components, so the update is done in place.
 */
static void half3(const lat3 *L, int a_lo, const double r[3], const double *const th[8],
                  const double *const thi[8], double tsgn, double sgn, const cplx *const *U) {
    for (int a = a_lo; a < a_lo + 4; ++a) {
        int comp = a / 2;
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < L->nz; ++k)
            for (int64_t j = 0; j < L->ny; ++j)
                for (int64_t i = 0; i < L->nx; ++i) {
                    int64_t c = (k * L->ny + j) * L->nx + i;
                    cplx al, be;
                    if (thi) cayley_c(tsgn * th[a][c], tsgn * thi[a][c], &al, &be);
                    else cayley(tsgn * th[a][c], &al, &be);
                    cplx s = U ? stencil3_links(L, comp, POS3(a, i, j, k), r, U)
                               : stencil3(L, comp, POS3(a, i, j, k), r);
                    L->f[a][c] = al * L->f[a][c] - sgn * be * s;
                }
    }
}

static int mk3(lat3 *L, const int64_t n[3], void *const f[8]) {
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) return -1;
    L->nx = n[0]; L->ny = n[1]; L->nz = n[2];
    for (int a = 0; a < 8; ++a) {
        if (!f[a]) return -1;
        L->f[a] = (cplx *)f[a];
    }
    return 0;
}

/* One forward step: Eqs. ss1, ss2 (A,B from C,D) then ss3, ss4 (C,D from new A,B).
 * th[0..3]: theta at the A0,A1,B0,B1 sites on sheet n; th[4..7]: at the
 * C0,C1,D0,D1 sites on sheet n+1/2. */
int oracle_step3(const int64_t n[3], const double r[3], void *const f[8], const double *const th[8]) {
    lat3 L;
    if (mk3(&L, n, f)) return -1;
    g_bad_lookup = 0;
    half3(&L, 0, r, th, NULL, 1.0, 1.0, NULL);
    half3(&L, 4, r, th, NULL, 1.0, 1.0, NULL);
    return g_bad_lookup ? -2 : 0;
}

/* oracle_step3 with a complex theta: thi[a] holds Im theta at the sites of
 * array a, i.e. (dt/2) Im V (the mass is real). */
int oracle_step3c(const int64_t n[3], const double r[3], void *const f[8], const double *const th[8],
                  const double *const thi[8]) {
    lat3 L;
    if (mk3(&L, n, f) || !thi) return -1;
    g_bad_lookup = 0;
    half3(&L, 0, r, th, thi, 1.0, 1.0, NULL);
    half3(&L, 4, r, th, thi, 1.0, 1.0, NULL);
    return g_bad_lookup ? -2 : 0;
}

/* One reversed step: the relation of ss3, ss4 solved for the old C,D, then
 * that of ss1, ss2 solved for the old A,B (same theta sheets). */
int oracle_reverse3(const int64_t n[3], const double r[3], void *const f[8], const double *const th[8]) {
    lat3 L;
    if (mk3(&L, n, f)) return -1;
    g_bad_lookup = 0;
    half3(&L, 4, r, th, NULL, -1.0, -1.0, NULL);
    half3(&L, 0, r, th, NULL, -1.0, -1.0, NULL);
    return g_bad_lookup ? -2 : 0;
}

/* One forward step with gauge links U[24] (see stencil3_links). */
int oracle_step3_links(const int64_t n[3], const double r[3], void *const f[8], const double *const th[8],
                       void *const U[24]) {
    if (g_zero_bc) return -1;                  /* links: periodic lattices only */
    lat3 L;
    if (mk3(&L, n, f)) return -1;
    for (int q = 0; q < 24; ++q)
        if (!U[q]) return -1;
    g_bad_lookup = 0;
    half3(&L, 0, r, th, NULL, 1.0, 1.0, (const cplx *const *)U);
    half3(&L, 4, r, th, NULL, 1.0, 1.0, (const cplx *const *)U);
    return g_bad_lookup ? -2 : 0;
}

/* Kahan-compensated accumulation, per plane then over planes in order. */
typedef struct { double s, c; } ksum;
static void kadd(ksum *k, double x) {
    double y = x - k->c;
    double t = k->s + y;
    k->c = (t - k->s) - y;
    k->s = t;
}

/*
 * Conserved functional, Lemma of Sect. 2, Eq. (EPM), term by term:
 *   E_r = (A,A)+(B,B)+(C,C)+(D,D)
 *         - r_z Re[(d_z C, A) - (d_z D, B)] - r_x Re[(d_x D, A) + (d_x C, B)]
 *         + r_y Re[i (d_y D, A) - i (d_y C, B)],
 * with (F,G) = sum_j F_j conj(G_j) over the sites of G.
 * out[0] = E_r as above; out[1] = the same functional written on the C,D
 * sites after summation by parts, |psi|^2 + Re sum_{C,D} conj(X) S_X(A,B);
 * out[2] = the plain sum of |amplitude|^2 over all sites.
 */
int oracle_energy3(const int64_t n[3], const double r[3], void *const f[8], double out[3]) {
    lat3 L;
    if (mk3(&L, n, f)) return -1;
    g_bad_lookup = 0;
    int64_t nz = L.nz;
    double *pl = (double *)calloc((size_t)(3 * nz), sizeof(double));
    if (!pl) return -3;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k) {
        ksum e1 = {0, 0}, e2 = {0, 0}, nv = {0, 0};
        for (int64_t j = 0; j < L.ny; ++j)
            for (int64_t i = 0; i < L.nx; ++i) {
                int64_t c = (k * L.ny + j) * L.nx + i;
                for (int a = 0; a < 8; ++a) {
                    double m2 = creal(L.f[a][c]) * creal(L.f[a][c]) + cimag(L.f[a][c]) * cimag(L.f[a][c]);
                    kadd(&nv, m2);
                }
                for (int s = 0; s < 2; ++s) {
                    /* A site */
                    int a = CA * 2 + s;
                    int64_t X = 2 * i + OFF3[a][0], Y = 2 * j + OFF3[a][1], Z = 2 * k + OFF3[a][2];
                    cplx A = L.f[a][c];
                    cplx dzC = get3(&L, CC, X, Y, Z + 1) - get3(&L, CC, X, Y, Z - 1);
                    cplx dxD = get3(&L, CD, X + 1, Y, Z) - get3(&L, CD, X - 1, Y, Z);
                    cplx dyD = get3(&L, CD, X, Y + 1, Z) - get3(&L, CD, X, Y - 1, Z);
                    double t = -r[2] * creal(dzC * conj(A)) - r[0] * creal(dxD * conj(A))
                               + r[1] * creal(I * dyD * conj(A));
                    kadd(&e1, t);
                    /* B site */
                    a = CB * 2 + s;
                    X = 2 * i + OFF3[a][0]; Y = 2 * j + OFF3[a][1]; Z = 2 * k + OFF3[a][2];
                    cplx B = L.f[a][c];
                    cplx dzD = get3(&L, CD, X, Y, Z + 1) - get3(&L, CD, X, Y, Z - 1);
                    cplx dxC = get3(&L, CC, X + 1, Y, Z) - get3(&L, CC, X - 1, Y, Z);
                    cplx dyC = get3(&L, CC, X, Y + 1, Z) - get3(&L, CC, X, Y - 1, Z);
                    t = r[2] * creal(dzD * conj(B)) - r[0] * creal(dxC * conj(B))
                        - r[1] * creal(I * dyC * conj(B));
                    kadd(&e1, t);
                    /* C and D sites: the summed-by-parts form */
                    for (int comp = CC; comp <= CD; ++comp) {
                        int b = comp * 2 + s;
                        cplx x = L.f[b][c];
                        cplx sx = stencil3(&L, comp, POS3(b, i, j, k), r);
                        kadd(&e2, creal(conj(x) * sx));
                    }
                }
            }
        pl[3 * k + 0] = e1.s;
        pl[3 * k + 1] = e2.s;
        pl[3 * k + 2] = nv.s;
    }
    ksum t1 = {0, 0}, t2 = {0, 0}, t3 = {0, 0};
    for (int64_t k = 0; k < nz; ++k) {
        kadd(&t1, pl[3 * k]);
        kadd(&t2, pl[3 * k + 1]);
        kadd(&t3, pl[3 * k + 2]);
    }
    free(pl);
    out[0] = t3.s + t1.s;
    out[1] = t3.s + t2.s;
    out[2] = t3.s;
    return g_bad_lookup ? -2 : 0;
}

/*
 * E_r with gauge links: out[0] = sum |psi|^2 - Re sum_{A,B} conj(X) S_X(C,D),
 * out[1] = sum |psi|^2 + Re sum_{C,D} conj(Y) S_Y(A,B) (S with the links),
 * out[2] = sum |psi|^2.
 */
int oracle_energy3_links(const int64_t n[3], const double r[3], void *const f[8], void *const U[24],
                         double out[3]) {
    if (g_zero_bc) return -1;                  /* links: periodic lattices only */
    lat3 L;
    if (mk3(&L, n, f)) return -1;
    for (int q = 0; q < 24; ++q)
        if (!U[q]) return -1;
    const cplx *const *u = (const cplx *const *)U;
    g_bad_lookup = 0;
    int64_t nz = L.nz;
    double *pl = (double *)calloc((size_t)(3 * nz), sizeof(double));
    if (!pl) return -3;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nz; ++k) {
        ksum e1 = {0, 0}, e2 = {0, 0}, nv = {0, 0};
        for (int64_t j = 0; j < L.ny; ++j)
            for (int64_t i = 0; i < L.nx; ++i) {
                int64_t c = (k * L.ny + j) * L.nx + i;
                for (int a = 0; a < 8; ++a) {
                    double m2 = creal(L.f[a][c]) * creal(L.f[a][c]) + cimag(L.f[a][c]) * cimag(L.f[a][c]);
                    kadd(&nv, m2);
                    cplx sx = stencil3_links(&L, a / 2, POS3(a, i, j, k), r, u);
                    if (a < 4) kadd(&e1, -creal(conj(L.f[a][c]) * sx));
                    else kadd(&e2, creal(conj(L.f[a][c]) * sx));
                }
            }
        pl[3 * k + 0] = e1.s;
        pl[3 * k + 1] = e2.s;
        pl[3 * k + 2] = nv.s;
    }
    ksum t1 = {0, 0}, t2 = {0, 0}, t3 = {0, 0};
    for (int64_t k = 0; k < nz; ++k) {
        kadd(&t1, pl[3 * k]);
        kadd(&t2, pl[3 * k + 1]);
        kadd(&t3, pl[3 * k + 2]);
    }
    free(pl);
    out[0] = t3.s + t1.s;
    out[1] = t3.s + t2.s;
    out[2] = t3.s;
    return g_bad_lookup ? -2 : 0;
}

/*
 * Observables of the plain density |amplitude|^2 summed over all sites
 * (positions in cell units, i.e. doubled coordinate / 2):
 *   out[0] = sum over sites with z >= z0,  out[1..3] = sum x|.|^2, y|.|^2, z|.|^2,
 *   out[4] = sum |.|^2,  out[5..8] = per component A, B, C, D.
 */
int oracle_observe3(const int64_t n[3], void *const f[8], double z0, double out[9]) {
    lat3 L;
    if (mk3(&L, n, f)) return -1;
    ksum acc[9];
    memset(acc, 0, sizeof(acc));
    for (int64_t k = 0; k < L.nz; ++k)
        for (int64_t j = 0; j < L.ny; ++j)
            for (int64_t i = 0; i < L.nx; ++i) {
                int64_t c = (k * L.ny + j) * L.nx + i;
                for (int a = 0; a < 8; ++a) {
                    cplx x = L.f[a][c];
                    double p = creal(x) * creal(x) + cimag(x) * cimag(x);
                    double px = 0.5 * (double)(2 * i + OFF3[a][0]);
                    double py = 0.5 * (double)(2 * j + OFF3[a][1]);
                    double pz = 0.5 * (double)(2 * k + OFF3[a][2]);
                    if (pz >= z0) kadd(&acc[0], p);
                    kadd(&acc[1], px * p);
                    kadd(&acc[2], py * p);
                    kadd(&acc[3], pz * p);
                    kadd(&acc[4], p);
                    kadd(&acc[5 + a / 2], p);
                }
            }
    for (int q = 0; q < 9; ++q) out[q] = acc[q].s;
    return 0;
}

/*
 * Reverse-mode derivative of one forward step, by the chain rule applied to
 * the step's two half-steps in reverse order.  Inputs: the state before the
 * step (pre) and after it (post), the theta sheets used, and the adjoint
 * lam = dL/dRe(psi) + i dL/dIm(psi) with respect to `post`.  On return lam
 * holds the adjoint with respect to `pre`, and gth[a][c] has been increased by
 * dL/dtheta at every site.
 *
 * For X+ = alpha X- - beta S with S = sum_t c_t Y_t:
 *   dX+/dtheta = -i (X+ + X-)/(1 + i theta)     (differentiating the relation),
 *   lam_X-  = conj(alpha) lam_X+,   lam_Yt += conj(-beta c_t) lam_X+,
 *   dL/dtheta = Re[conj(lam_X+) dX+/dtheta].
 * The scatter to Y_t walks the same stencil table as the forward step, so no
 * symmetry of the operator is assumed.  Single-threaded (scatter).
 */
static void adj_half3(const lat3 *post, const lat3 *pre, lat3 *lam, int a_lo, const double r[3],
                      const double *const th[8], double *const gth[8]) {
    /* pass 1: theta derivative and scatter into the other sheet's adjoint */
    for (int a = a_lo; a < a_lo + 4; ++a) {
        int comp = a / 2;
        for (int64_t k = 0; k < post->nz; ++k)
            for (int64_t j = 0; j < post->ny; ++j)
                for (int64_t i = 0; i < post->nx; ++i) {
                    int64_t c = (k * post->ny + j) * post->nx + i;
                    double t = th[a][c];
                    cplx al, be;
                    cayley(t, &al, &be);
                    cplx lx = lam->f[a][c];
                    cplx dx = -I * (post->f[a][c] + pre->f[a][c]) / (1.0 + I * t);
                    gth[a][c] += creal(conj(lx) * dx);
                    int64_t X = 2 * i + OFF3[a][0], Y = 2 * j + OFF3[a][1], Z = 2 * k + OFF3[a][2];
                    for (int q = 0; q < 6; ++q) {
                        const term *u = &ST3[comp][q];
                        cplx *p = site3(lam, u->comp, X + u->dx, Y + u->dy, Z + u->dz);
                        if (p) *p += conj(-be * coef(u->cls, r)) * lx;
                    }
                }
    }
    /* pass 2: through the alpha X- term */
    for (int a = a_lo; a < a_lo + 4; ++a)
        for (int64_t c = 0; c < post->nx * post->ny * post->nz; ++c) {
            cplx al, be;
            cayley(th[a][c], &al, &be);
            lam->f[a][c] = conj(al) * lam->f[a][c];
        }
}

/* pre/post/lam: 8 arrays each; mid = the state between the half-steps is
 * rebuilt here from pre (new A,B with old C,D). */
int oracle_adjoint3(const int64_t n[3], const double r[3], void *const pre[8], void *const post[8],
                    void *const lam[8], const double *const th[8], double *const gth[8]) {
    lat3 Lpre, Lpost, Llam, Lmid;
    if (mk3(&Lpre, n, pre) || mk3(&Lpost, n, post) || mk3(&Llam, n, lam)) return -1;
    int64_t nc = n[0] * n[1] * n[2];
    cplx *mid[8];
    for (int a = 0; a < 8; ++a) {
        /* A,B of mid = post's A,B; C,D of mid = pre's C,D */
        mid[a] = (cplx *)((a < 4) ? post[a] : pre[a]);
    }
    if (mk3(&Lmid, n, (void *const *)mid)) return -1;
    (void)nc;
    g_bad_lookup = 0;
    /* second half-step (C,D): pre-image is mid, image is post */
    adj_half3(&Lpost, &Lmid, &Llam, 4, r, th, gth);
    /* first half-step (A,B): pre-image is pre, image is mid */
    adj_half3(&Lmid, &Lpre, &Llam, 0, r, th, gth);
    return g_bad_lookup ? -2 : 0;
}

/* ------------------------------------------------------------------------ */
/* (2+1)D lattice                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t nx, ny;
    cplx *f[4];                                /* u0 u1 v0 v1 */
} lat2;

static const int OFF2[4][2] = {{0, 0}, {1, 1}, {1, 0}, {0, 1}};

static cplx *site2(const lat2 *L, int comp, int64_t X, int64_t Y) {
    if (g_zero_bc && (X < 0 || X >= 2 * L->nx || Y < 0 || Y >= 2 * L->ny))
        return NULL;                           /* outside: a zero ghost */
    X = wrap(X, 2 * L->nx);
    Y = wrap(Y, 2 * L->ny);
    for (int s = 0; s < 2; ++s) {
        int a = 2 * comp + s;
        if ((X & 1) == OFF2[a][0] && (Y & 1) == OFF2[a][1])
            return &L->f[a][(Y >> 1) * L->nx + (X >> 1)];
    }
    g_bad_lookup = 1;
    return NULL;
}

static cplx get2(const lat2 *L, int comp, int64_t X, int64_t Y) {
    cplx *p = site2(L, comp, X, Y);
    return p ? *p : 0.0;
}

/*
 * Difference terms of Eqs. scheme2Deq - scheme4thline moved to the left:
 *   u:  S_u = r_x dx v - i r_y dy v      (scheme2Deq, scheme3rdline)
 *   v:  S_v = r_x dx u + i r_y dy u      (scheme2ndline, scheme4thline)
 * theta_u = (dt/2)(m + V) on sheet n, theta_v = (dt/2)(-m + V) on n+1/2.
 */
static const term ST2[2][4] = {
    /* u */ {{PX, CV, 1, 0, 0}, {MX, CV, -1, 0, 0}, {MIY, CV, 0, 1, 0}, {PIY, CV, 0, -1, 0}},
    /* v */ {{PX, CU, 1, 0, 0}, {MX, CU, -1, 0, 0}, {PIY, CU, 0, 1, 0}, {MIY, CU, 0, -1, 0}},
};

static cplx stencil2(const lat2 *L, int comp, int64_t X, int64_t Y, const double r[3]) {
    cplx s = 0.0;
    for (int t = 0; t < 4; ++t) {
        const term *q = &ST2[comp][t];
        s += coef(q->cls, r) * get2(L, q->comp, X + q->dx, Y + q->dy);
    }
    return s;
}

/* Gauge links in 2D: as stencil3_links with U[4 a + t] at the u sites (term
 * order of ST2: +x -x +y -y) and the conjugates at the v sites. */
static int locate2(const lat2 *L, int comp, int64_t X, int64_t Y, int64_t *cell) {
    X = wrap(X, 2 * L->nx);
    Y = wrap(Y, 2 * L->ny);
    for (int s = 0; s < 2; ++s) {
        int a = 2 * comp + s;
        if ((X & 1) == OFF2[a][0] && (Y & 1) == OFF2[a][1]) {
            *cell = (Y >> 1) * L->nx + (X >> 1);
            return a;
        }
    }
    g_bad_lookup = 1;
    *cell = 0;
    return 0;
}

static cplx stencil2_links(const lat2 *L, int comp, int64_t X, int64_t Y, const double r[3],
                           const cplx *const U[8]) {
    cplx s = 0.0;
    int64_t cx;
    int ax = locate2(L, comp, X, Y, &cx);
    for (int t = 0; t < 4; ++t) {
        const term *q = &ST2[comp][t];
        int64_t QX = X + q->dx, QY = Y + q->dy;
        cplx u;
        if (comp == CU) {
            u = U[4 * ax + t][cx];
        } else {
            int64_t cq;
            int aq = locate2(L, q->comp, QX, QY, &cq);
            int tb = -1;
            for (int t2 = 0; t2 < 4; ++t2) {
                const term *b = &ST2[q->comp][t2];
                if (b->dx == -q->dx && b->dy == -q->dy) tb = t2;
            }
            if (tb < 0) {
                g_bad_lookup = 1;
                tb = 0;
            }
            u = conj(U[4 * aq + tb][cq]);
        }
        s += coef(q->cls, r) * u * get2(L, q->comp, QX, QY);
    }
    return s;
}

static void half2(const lat2 *L, int a_lo, const double r[3], const double *const th[4],
                  const double *const thi[4], double tsgn, double sgn, const cplx *const *U) {
    for (int a = a_lo; a < a_lo + 2; ++a) {
        int comp = a / 2;
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < L->ny; ++j)
            for (int64_t i = 0; i < L->nx; ++i) {
                int64_t c = j * L->nx + i;
                cplx al, be;
                if (thi) cayley_c(tsgn * th[a][c], tsgn * thi[a][c], &al, &be);
                else cayley(tsgn * th[a][c], &al, &be);
                cplx s = U ? stencil2_links(L, comp, 2 * i + OFF2[a][0], 2 * j + OFF2[a][1], r, U)
                           : stencil2(L, comp, 2 * i + OFF2[a][0], 2 * j + OFF2[a][1], r);
                L->f[a][c] = al * L->f[a][c] - sgn * be * s;
            }
    }
}

static int mk2(lat2 *L, const int64_t n[2], void *const f[4]) {
    if (n[0] < 1 || n[1] < 1) return -1;
    L->nx = n[0]; L->ny = n[1];
    for (int a = 0; a < 4; ++a) {
        if (!f[a]) return -1;
        L->f[a] = (cplx *)f[a];
    }
    return 0;
}

/* r[0] = r_x, r[1] = r_y (r[2] unused).  th[0..1]: u0,u1 sites on sheet n;
 * th[2..3]: v0,v1 sites on sheet n+1/2. */
int oracle_step2(const int64_t n[2], const double r[3], void *const f[4], const double *const th[4]) {
    lat2 L;
    if (mk2(&L, n, f)) return -1;
    g_bad_lookup = 0;
    half2(&L, 0, r, th, NULL, 1.0, 1.0, NULL);
    half2(&L, 2, r, th, NULL, 1.0, 1.0, NULL);
    return g_bad_lookup ? -2 : 0;
}

/* oracle_step2 with a complex theta (thi = Im theta per site, see oracle_step3c). */
int oracle_step2c(const int64_t n[2], const double r[3], void *const f[4], const double *const th[4],
                  const double *const thi[4]) {
    lat2 L;
    if (mk2(&L, n, f) || !thi) return -1;
    g_bad_lookup = 0;
    half2(&L, 0, r, th, thi, 1.0, 1.0, NULL);
    half2(&L, 2, r, th, thi, 1.0, 1.0, NULL);
    return g_bad_lookup ? -2 : 0;
}

int oracle_reverse2(const int64_t n[2], const double r[3], void *const f[4], const double *const th[4]) {
    lat2 L;
    if (mk2(&L, n, f)) return -1;
    g_bad_lookup = 0;
    half2(&L, 2, r, th, NULL, -1.0, -1.0, NULL);
    half2(&L, 0, r, th, NULL, -1.0, -1.0, NULL);
    return g_bad_lookup ? -2 : 0;
}

/* One forward (2+1)D step with gauge links U[8] (see stencil2_links). */
int oracle_step2_links(const int64_t n[2], const double r[3], void *const f[4], const double *const th[4],
                       void *const U[8]) {
    if (g_zero_bc) return -1;                  /* links: periodic lattices only */
    lat2 L;
    if (mk2(&L, n, f)) return -1;
    for (int q = 0; q < 8; ++q)
        if (!U[q]) return -1;
    g_bad_lookup = 0;
    half2(&L, 0, r, th, NULL, 1.0, 1.0, (const cplx *const *)U);
    half2(&L, 2, r, th, NULL, 1.0, 1.0, (const cplx *const *)U);
    return g_bad_lookup ? -2 : 0;
}

/* (2+1)D functional with links (d_+ form): out[0] = sum |psi|^2 + Re sum_v conj(v) S_v(u),
 * out[1] = sum |psi|^2 - Re sum_u conj(u) S_u(v), out[2] = sum |psi|^2. */
int oracle_energy2_links(const int64_t n[2], const double r[3], void *const f[4], void *const U[8],
                         double out[3]) {
    if (g_zero_bc) return -1;                  /* links: periodic lattices only */
    lat2 L;
    if (mk2(&L, n, f)) return -1;
    for (int q = 0; q < 8; ++q)
        if (!U[q]) return -1;
    const cplx *const *u = (const cplx *const *)U;
    g_bad_lookup = 0;
    ksum ev = {0, 0}, eu = {0, 0}, nv = {0, 0};
    for (int64_t j = 0; j < L.ny; ++j)
        for (int64_t i = 0; i < L.nx; ++i) {
            int64_t c = j * L.nx + i;
            for (int a = 0; a < 4; ++a) {
                kadd(&nv, creal(L.f[a][c]) * creal(L.f[a][c]) + cimag(L.f[a][c]) * cimag(L.f[a][c]));
                cplx sx = stencil2_links(&L, a / 2, 2 * i + OFF2[a][0], 2 * j + OFF2[a][1], r, u);
                if (a < 2) kadd(&eu, -creal(conj(L.f[a][c]) * sx));
                else kadd(&ev, creal(conj(L.f[a][c]) * sx));
            }
        }
    out[0] = nv.s + ev.s;
    out[1] = nv.s + eu.s;
    out[2] = nv.s;
    return g_bad_lookup ? -2 : 0;
}

/*
 * (2+1)D functional, Lemma of Sect. 3, Eq. (E), with (f,g) = sum f conj(g)
 * over the v sites and d_+- = d_x +- i d_y:
 *   out[0] = ||u||^2 + ||v||^2 + r_x Re(d_x u, v) + r_y Re(i d_y u, v)   (d_+ form)
 *   out[1] = ||u||^2 + ||v||^2 + r_x Re(d_x u, v) - r_y Re(i d_y u, v)   (d_- form, as printed)
 *   out[2] = ||u||^2 + ||v||^2
 * The d_+ form is the one the update equations scheme2Deq-scheme4thline
 * conserve; the printed d_- form oscillates whenever the state has k_y != 0.
 */
int oracle_energy2(const int64_t n[2], const double r[3], void *const f[4], double out[3]) {
    lat2 L;
    if (mk2(&L, n, f)) return -1;
    g_bad_lookup = 0;
    ksum ep = {0, 0}, em = {0, 0}, nv = {0, 0};
    for (int64_t j = 0; j < L.ny; ++j)
        for (int64_t i = 0; i < L.nx; ++i) {
            int64_t c = j * L.nx + i;
            for (int a = 0; a < 4; ++a)
                kadd(&nv, creal(L.f[a][c]) * creal(L.f[a][c]) + cimag(L.f[a][c]) * cimag(L.f[a][c]));
            for (int s = 0; s < 2; ++s) {
                int a = 2 + s;                 /* v site */
                int64_t X = 2 * i + OFF2[a][0], Y = 2 * j + OFF2[a][1];
                cplx v = L.f[a][c];
                cplx dxu = get2(&L, CU, X + 1, Y) - get2(&L, CU, X - 1, Y);
                cplx dyu = get2(&L, CU, X, Y + 1) - get2(&L, CU, X, Y - 1);
                double tx = r[0] * creal(dxu * conj(v));
                double ty = r[1] * creal(I * dyu * conj(v));
                kadd(&ep, tx + ty);
                kadd(&em, tx - ty);
            }
        }
    out[0] = nv.s + ep.s;
    out[1] = nv.s + em.s;
    out[2] = nv.s;
    return g_bad_lookup ? -2 : 0;
}

/* out[0] = sum over sites with x >= x0; out[1..2] = sum x|.|^2, y|.|^2;
 * out[3] = sum |.|^2; out[4..5] = per component u, v. */
int oracle_observe2(const int64_t n[2], void *const f[4], double x0, double out[6]) {
    lat2 L;
    if (mk2(&L, n, f)) return -1;
    ksum acc[6];
    memset(acc, 0, sizeof(acc));
    for (int64_t j = 0; j < L.ny; ++j)
        for (int64_t i = 0; i < L.nx; ++i) {
            int64_t c = j * L.nx + i;
            for (int a = 0; a < 4; ++a) {
                cplx x = L.f[a][c];
                double p = creal(x) * creal(x) + cimag(x) * cimag(x);
                double px = 0.5 * (double)(2 * i + OFF2[a][0]);
                double py = 0.5 * (double)(2 * j + OFF2[a][1]);
                if (px >= x0) kadd(&acc[0], p);
                kadd(&acc[1], px * p);
                kadd(&acc[2], py * p);
                kadd(&acc[3], p);
                kadd(&acc[4 + a / 2], p);
            }
        }
    for (int q = 0; q < 6; ++q) out[q] = acc[q].s;
    return 0;
}

static void adj_half2(const lat2 *post, const lat2 *pre, lat2 *lam, int a_lo, const double r[3],
                      const double *const th[4], double *const gth[4]) {
    for (int a = a_lo; a < a_lo + 2; ++a) {
        int comp = a / 2;
        for (int64_t j = 0; j < post->ny; ++j)
            for (int64_t i = 0; i < post->nx; ++i) {
                int64_t c = j * post->nx + i;
                double t = th[a][c];
                cplx al, be;
                cayley(t, &al, &be);
                cplx lx = lam->f[a][c];
                cplx dx = -I * (post->f[a][c] + pre->f[a][c]) / (1.0 + I * t);
                gth[a][c] += creal(conj(lx) * dx);
                int64_t X = 2 * i + OFF2[a][0], Y = 2 * j + OFF2[a][1];
                for (int q = 0; q < 4; ++q) {
                    const term *u = &ST2[comp][q];
                    cplx *p = site2(lam, u->comp, X + u->dx, Y + u->dy);
                    if (p) *p += conj(-be * coef(u->cls, r)) * lx;
                }
            }
    }
    for (int a = a_lo; a < a_lo + 2; ++a)
        for (int64_t c = 0; c < post->nx * post->ny; ++c) {
            cplx al, be;
            cayley(th[a][c], &al, &be);
            lam->f[a][c] = conj(al) * lam->f[a][c];
        }
}

int oracle_adjoint2(const int64_t n[2], const double r[3], void *const pre[4], void *const post[4],
                    void *const lam[4], const double *const th[4], double *const gth[4]) {
    lat2 Lpre, Lpost, Llam, Lmid;
    if (mk2(&Lpre, n, pre) || mk2(&Lpost, n, post) || mk2(&Llam, n, lam)) return -1;
    void *mid[4] = {post[0], post[1], pre[2], pre[3]};
    if (mk2(&Lmid, n, mid)) return -1;
    g_bad_lookup = 0;
    adj_half2(&Lpost, &Lmid, &Llam, 2, r, th, gth);
    adj_half2(&Lmid, &Lpre, &Llam, 0, r, th, gth);
    return g_bad_lookup ? -2 : 0;
}

/* Number of OpenMP threads the oracle runs with (reported by the benchmark). */
int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of OpenMP threads of later calls (n >= 1); returns the
 * number now in effect.  The benchmark times the oracle on one thread and on
 * all host cores. */
int oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Boundary of later calls: zero != 0 for zero values outside the lattice,
 * 0 for periodic wrap (the default).  Gauge-link calls are periodic only and
 * return -1 while zero boundaries are set.  Returns the previous setting. */
int oracle_set_zero_bc(int zero) {
    int old = g_zero_bc;
    g_zero_bc = zero != 0;
    return old;
}
