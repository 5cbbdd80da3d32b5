"""Planted mistakes in the oracle must fail its pins.

Each case copies dirac_oracle.c with one plausible mistake (a sign, an offset,
a missing conjugate, a swapped half-step order, ...), builds it on the CPU,
swaps it in for the real oracle and runs the pins chosen for that part: at
least one must fail.  The unmodified source passes the same pins, so a failure
is the mistake's, not the harness's.  No mutant is ever used outside this file.
"""
import os

import pytest

import oracle
import test_oracle_pins as pins

PINS = {
    "dense3": lambda: pins.test_dense_matches_oracle_3d((3, 2, 2)),
    "dense2": lambda: pins.test_dense_matches_oracle_2d((5, 3)),
    "gram3": lambda: pins.test_gram_invariant_and_energy_form(3),
    "aniso": lambda: pins.test_plane_wave_anisotropic_spacing(),
    "reverse": lambda: pins.test_reverse_is_inverse_dense(),
    "complex3": lambda: pins.test_complex_theta_dense_matches_oracle(3),
    "links3": lambda: pins.test_links_match_dense_from_potential(3),
    "obs3": lambda: (pins.test_observables_single_site_3d(), pins.test_observables_eigen_plane_wave_3d((1, 2))),
    "obs2": lambda: (pins.test_observables_single_site_2d(), pins.test_observables_eigen_plane_wave_2d(1)),
    "zbc3": lambda: (pins.test_zero_bc_dense_matches_oracle_3d((3, 2, 4)), pins.test_zero_bc_conserves_functional(3)),
    "zbc2": lambda: (pins.test_zero_bc_dense_matches_oracle_2d((4, 3)), pins.test_zero_bc_conserves_functional(2)),
}

# (name, text in dirac_oracle.c, replacement, pins expected to catch it)
MUTANTS = [
    ("S_A y-difference sign",
     "{MIY, CD, 0, 1, 0}, {PIY, CD, 0, -1, 0}},\n    /* B */",
     "{PIY, CD, 0, 1, 0}, {MIY, CD, 0, -1, 0}},\n    /* B */", ["dense3"]),
    ("S_C x neighbour offset",
     "{PX, CB, 1, 0, 0}, {MX, CB, -1, 0, 0},", "{PX, CB, 1, 0, 0}, {MX, CB, 1, 0, 0},", ["dense3"]),
    ("S_D z-difference sign",
     "/* D */ {{MZ, CB, 0, 0, 1}, {PZ, CB, 0, 0, -1},", "/* D */ {{PZ, CB, 0, 0, 1}, {MZ, CB, 0, 0, -1},",
     ["dense3"]),
    ("alpha imaginary part sign",
     "*alpha = (1.0 - th * th) / d - I * ((2.0 * th) / d);", "*alpha = (1.0 - th * th) / d + I * ((2.0 * th) / d);",
     ["dense3"]),
    ("beta imaginary part sign",
     "*beta = 1.0 / d - I * (th / d);", "*beta = 1.0 / d + I * (th / d);", ["dense3"]),
    ("half-steps in the wrong order",
     "    g_bad_lookup = 0;\n    half3(&L, 0, r, th, NULL, 1.0, 1.0, NULL);\n    half3(&L, 4, r, th, NULL, 1.0, 1.0, NULL);\n",
     "    g_bad_lookup = 0;\n    half3(&L, 4, r, th, NULL, 1.0, 1.0, NULL);\n    half3(&L, 0, r, th, NULL, 1.0, 1.0, NULL);\n",
     ["dense3"]),
    ("sign of S in the update",
     ": stencil3(L, comp, POS3(a, i, j, k), r);\n                    L->f[a][c] = al * L->f[a][c] - sgn * be * s;",
     ": stencil3(L, comp, POS3(a, i, j, k), r);\n                    L->f[a][c] = al * L->f[a][c] + sgn * be * s;",
     ["dense3"]),
    ("r_x in place of r_z",
     "case PZ:  return r[2];", "case PZ:  return r[0];", ["aniso", "dense3"]),
    ("reversed step with the forward theta",
     "half3(&L, 4, r, th, NULL, -1.0, -1.0, NULL);", "half3(&L, 4, r, th, NULL, 1.0, -1.0, NULL);", ["reverse"]),
    ("complex theta: wrong denominator sign",
     "cplx d = 1.0 + I * t;", "cplx d = 1.0 - I * t;", ["complex3"]),
    ("links: C,D rows without the conjugate",
     "u = conj(U[6 * aq + tb][cq]);", "u = U[6 * aq + tb][cq];", ["links3"]),
    ("links: C,D rows take the wrong term of the A,B end",
     "if (b->dx == -q->dx && b->dy == -q->dy && b->dz == -q->dz) tb = t2;",
     "if (b->dx == q->dx && b->dy == q->dy && b->dz == q->dz) tb = t2;", ["links3"]),
    ("functional: sign of the y term at A sites",
     "+ r[1] * creal(I * dyD * conj(A));", "- r[1] * creal(I * dyD * conj(A));", ["gram3"]),
    ("2D: S_v y-difference sign",
     "/* v */ {{PX, CU, 1, 0, 0}, {MX, CU, -1, 0, 0}, {PIY, CU, 0, 1, 0}, {MIY, CU, 0, -1, 0}},",
     "/* v */ {{PX, CU, 1, 0, 0}, {MX, CU, -1, 0, 0}, {MIY, CU, 0, 1, 0}, {PIY, CU, 0, -1, 0}},", ["dense2"]),
    ("2D: S_u x neighbour offset",
     "/* u */ {{PX, CV, 1, 0, 0}, {MX, CV, -1, 0, 0},", "/* u */ {{PX, CV, 1, 0, 0}, {MX, CV, 1, 0, 0},",
     ["dense2"]),
    ("observables: z offset of the half-integer sites doubled",
     "double pz = 0.5 * (double)(2 * k + OFF3[a][2]);", "double pz = 0.5 * (double)(2 * k + 2 * OFF3[a][2]);",
     ["obs3"]),
    ("observables: x offset halved",
     "double px = 0.5 * (double)(2 * i + OFF3[a][0]);", "double px = 0.5 * (double)(2 * i) + 0.25 * OFF3[a][0];",
     ["obs3"]),
    ("observables: strict > for the region boundary",
     "if (pz >= z0) kadd(&acc[0], p);", "if (pz > z0) kadd(&acc[0], p);", ["obs3"]),
    ("observables: per-component sum indexed by array",
     "kadd(&acc[5 + a / 2], p);", "kadd(&acc[5 + a % 4], p);", ["obs3"]),
    ("2D observables: y offset taken from x",
     "double py = 0.5 * (double)(2 * j + OFF2[a][1]);", "double py = 0.5 * (double)(2 * j + OFF2[a][0]);",
     ["obs2"]),
    ("2D observables: strict > for the region boundary",
     "if (px >= x0) kadd(&acc[0], p);", "if (px > x0) kadd(&acc[0], p);", ["obs2"]),
    ("2D observables: per-component sum indexed by array",
     "kadd(&acc[4 + a / 2], p);", "kadd(&acc[4 + a % 2], p);", ["obs2"]),
    ("zero boundary: upper x face off by one (the outside site wraps)",
     "if (g_zero_bc && (X < 0 || X >= 2 * L->nx || Y < 0 || Y >= 2 * L->ny || Z < 0 || Z >= 2 * L->nz))",
     "if (g_zero_bc && (X < 0 || X > 2 * L->nx || Y < 0 || Y >= 2 * L->ny || Z < 0 || Z >= 2 * L->nz))",
     ["zbc3"]),
    ("zero boundary: z left periodic",
     "if (g_zero_bc && (X < 0 || X >= 2 * L->nx || Y < 0 || Y >= 2 * L->ny || Z < 0 || Z >= 2 * L->nz))",
     "if (g_zero_bc && (X < 0 || X >= 2 * L->nx || Y < 0 || Y >= 2 * L->ny))", ["zbc3"]),
    ("2D zero boundary: lower y face missing",
     "if (g_zero_bc && (X < 0 || X >= 2 * L->nx || Y < 0 || Y >= 2 * L->ny))\n        return NULL;                           /* outside: a zero ghost */",
     "if (g_zero_bc && (X < 0 || X >= 2 * L->nx || Y >= 2 * L->ny))\n        return NULL;                           /* outside: a zero ghost */",
     ["zbc2"]),
]


def _with_library(path, names):
    """Run the pins with the oracle library at path; return the names that failed."""
    saved = oracle._lib
    oracle._lib = oracle.load(path)
    failed = []
    try:
        for n in names:
            try:
                PINS[n]()
            except AssertionError:
                failed.append(n)
    finally:
        oracle._lib = saved
    return failed


def test_unmodified_oracle_passes_the_pins():
    assert _with_library(oracle.build(), list(PINS)) == []


@pytest.mark.parametrize("case", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(case, tmp_path):
    name, old, new, names = case
    src = open(oracle._SRC).read()
    assert src.count(old) == 1, "mutation site not unique or missing: %s" % name
    mutant = os.path.join(str(tmp_path), "mutant.c")
    with open(mutant, "w") as fh:
        fh.write(src.replace(old, new))
    so = oracle.compile_source(mutant, os.path.join(str(tmp_path), "libmutant.so"))
    assert _with_library(so, names), "no pin caught: %s" % name
