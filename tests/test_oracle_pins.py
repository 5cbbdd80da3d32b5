"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them re-types the oracle's own
formula: they use the closed-form dispersion and eigenkets, an independently
assembled dense one-step matrix, proven invariants and inequalities, and
brute-force finite differences.
"""
import numpy as np
import pytest

import oracle
from oracle.dense import Dense2, Dense3
from closed_form import (links_from_potential2, links_from_potential3, links_from_site_phase2,
                         links_from_site_phase3, links_uniform_field2, smooth_potential3)
from closed_form import (eigenket2, eigenket3, growth_factor, lattice_momentum, omega,
                         plane_wave2, plane_wave3, rel_l2)

DT3 = 0.9 / np.sqrt(3.0)
DT2 = 0.9 / np.sqrt(2.0)


def rng(seed):
    return np.random.default_rng(seed)


def rand_state(shape, count, g):
    return [np.ascontiguousarray(g.standard_normal(shape) + 1j * g.standard_normal(shape)) for _ in range(count)]


def rand_theta(shape, count, g, scale=0.4):
    return [np.ascontiguousarray(scale * g.standard_normal(shape)) for _ in range(count)]


# --------------------------------------------------------------------------
# Plane waves: Eq. (planeonlattice) with eigenkets psi^(1..4) and w from
# Eq. (pwdsip) evolve as exp(-i w n dt) exactly (Sect. 2.1; Sect. 3 for 2D).
# k includes k_y != 0 and extended-zone modes (k_x beyond 2*pi: the
# sublattice-staggered copies of the fcr sublattices).
# Tolerance: every step rounds each amplitude a handful of times (about four
# ulps of relative error, coherent for an eigenmode), so the bound is
# 1e-15 per step: 2e-13 after 200 steps.
# --------------------------------------------------------------------------
PW_TOL_PER_STEP = 1e-15
K3 = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (3, 2, 7), (5, -3, 2), (9, 1, 3), (4, 3, 5), (12, 5, 1)]


@pytest.mark.parametrize("branch", [1, 2, 3, 4])
@pytest.mark.parametrize("m", [0.0, 0.5])
def test_plane_wave_3d(branch, m):
    nx, ny, nz = 8, 6, 10
    lat = oracle.Lattice3(nx, ny, nz, DT3)
    th = lat.theta(m)
    for n in K3:
        k = (2 * np.pi * n[0] / nx, 2 * np.pi * n[1] / ny, 2 * np.pi * n[2] / nz)
        w, amps = eigenket3(k, m, DT3, branch)
        f = plane_wave3(lat.shape, k, amps, w, DT3)
        g = [a.copy() for a in f]
        lat.step(g, th, 200)
        expect = plane_wave3(lat.shape, k, amps, w, DT3, t_shift=200 * DT3)
        assert rel_l2(g, expect) < 200 * PW_TOL_PER_STEP, (n, branch, m)


K2 = [(1, 0), (0, 1), (3, 5), (17, -29), (6, 0), (64, 64), (70, 3), (1, 130)]


@pytest.mark.parametrize("branch", [1, 2])
@pytest.mark.parametrize("m", [0.0, 0.7])
def test_plane_wave_2d(branch, m):
    nx = ny = 128
    lat = oracle.Lattice2(nx, ny, DT2)
    th = lat.theta(m)
    for n in K2:
        k = (2 * np.pi * n[0] / nx, 2 * np.pi * n[1] / ny)
        w, amps = eigenket2(k, m, DT2, branch)
        f = plane_wave2(lat.shape, k, amps, w, DT2)
        g = [a.copy() for a in f]
        lat.step(g, th, 200)
        expect = plane_wave2(lat.shape, k, amps, w, DT2, t_shift=200 * DT2)
        assert rel_l2(g, expect) < 200 * PW_TOL_PER_STEP, (n, branch, m)


def test_plane_wave_anisotropic_spacing():
    """Unequal d_j: P_j = (2/d_j) sin(k_j d_j / 2), r_j = dt/d_j (Eq. substp, Sect. 2.2)."""
    nx, ny, nz = 6, 8, 4
    d = (1.0, 0.7, 1.3)
    dt = 0.8 / np.sqrt(sum(1.0 / dj ** 2 for dj in d))
    lat = oracle.Lattice3(nx, ny, nz, dt, *d)
    m = 0.3
    n = (2, 3, 1)
    k = tuple(2 * np.pi * n[q] / ((nx, ny, nz)[q] * d[q]) for q in range(3))
    w, amps = eigenket3(k, m, dt, 1, d)
    # positions are in cell units; the phase per cell is k_j * d_j
    kc = tuple(k[q] * d[q] for q in range(3))
    f = plane_wave3(lat.shape, kc, amps, w, dt)
    lat.step(f, lat.theta(m), 100)
    expect = plane_wave3(lat.shape, kc, amps, w, dt, t_shift=100 * dt)
    assert rel_l2(f, expect) < 100 * PW_TOL_PER_STEP


def test_single_cone_in_first_zone():
    """Sect. 2.1: for m = 0, w(k) vanishes only at k = 0 within (-pi, pi]^3 and is
    largest at the zone corner; the dispersion is monotonic along each axis."""
    ks = np.linspace(-np.pi, np.pi, 41)[1:]
    KX, KY, KZ = np.meshgrid(ks, ks, ks, indexing="ij")
    w = omega((KX, KY, KZ), 0.0, DT3)
    zero = np.argwhere(np.abs(w) < 1e-12)
    assert len(zero) == 1 and np.allclose(ks[zero[0]], 0.0)
    assert np.isclose(w.max(), omega((np.pi,) * 3, 0.0, DT3))
    axis = omega((ks[ks >= 0], 0 * ks[ks >= 0], 0 * ks[ks >= 0]), 0.0, DT3)
    assert np.all(np.diff(axis) > 0)


# --------------------------------------------------------------------------
# Dense matrix assembled independently in numpy (oracle/dense.py).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(2, 2, 4), (3, 2, 2), (4, 4, 4)])
def test_dense_matches_oracle_3d(shape):
    nx, ny, nz = shape
    g = rng(1)
    lat = oracle.Lattice3(nx, ny, nz, DT3)
    D = Dense3(nx, ny, nz, DT3)
    f = rand_state(lat.shape, 8, g)
    x = D.pack(f)
    for _ in range(4):                         # time-dependent theta
        th = rand_theta(lat.shape, 8, g)
        lat.step(f, th)
        x = D.step_matrix(D.pack(th).real) @ x
    assert rel_l2([D.pack(f)], [x]) < 1e-13


@pytest.mark.parametrize("shape", [(4, 4), (5, 3), (2, 6)])
def test_dense_matches_oracle_2d(shape):
    nx, ny = shape
    g = rng(2)
    lat = oracle.Lattice2(nx, ny, DT2)
    D = Dense2(nx, ny, DT2)
    f = rand_state(lat.shape, 4, g)
    x = D.pack(f)
    for _ in range(4):
        th = rand_theta(lat.shape, 4, g)
        lat.step(f, th)
        x = D.step_matrix(D.pack(th).real) @ x
    assert rel_l2([D.pack(f)], [x]) < 1e-13


def test_reverse_is_inverse_dense():
    """The reversed step (relations of Eqs. ss3, ss4 then ss1, ss2 solved for the
    old amplitudes) is the inverse of the dense one-step matrix."""
    g = rng(3)
    lat = oracle.Lattice3(2, 3, 4, DT3)
    D = Dense3(2, 3, 4, DT3)
    th = rand_theta(lat.shape, 8, g)
    f = rand_state(lat.shape, 8, g)
    x = np.linalg.solve(D.step_matrix(D.pack(th).real), D.pack(f))
    lat.reverse(f, th)
    assert rel_l2([D.pack(f)], [x]) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_gram_invariant_and_energy_form(dim):
    """Lemmas of Sects. 2 and 3: E_r is conserved for arbitrary real, site- and
    time-dependent m, V, i.e. M^H G M = G; and the oracle's reduction equals the
    Hermitian form psi^H G psi (both of its E_r evaluations)."""
    g = rng(4)
    if dim == 3:
        lat, D, cnt = oracle.Lattice3(2, 2, 4, DT3), Dense3(2, 2, 4, DT3), 8
    else:
        lat, D, cnt = oracle.Lattice2(4, 3, DT2), Dense2(4, 3, DT2), 4
    th = rand_theta(lat.shape, cnt, g, 1.0)
    M = D.step_matrix(D.pack(th).real)
    G = D.gram()
    assert np.abs(M.conj().T @ G @ M - G).max() < 1e-13
    f = rand_state(lat.shape, cnt, g)
    x = D.pack(f)
    e_form = float(np.real(np.vdot(x, G @ x)))
    e = lat.energy(f)
    assert abs(e[0] - e_form) < 1e-12 * abs(e_form)
    if dim == 3:
        assert abs(e[1] - e_form) < 1e-12 * abs(e_form)
    assert abs(e[-1] - float(np.vdot(x, x).real)) < 1e-12 * e[-1]


def _extended_zone_phases(nx, ny, nz, m, dt):
    """Closed-form eigen-phases w*dt of the one-step map for constant m, V = 0.
    Distinct plane waves on the fcr sublattices: k_x, k_y in 2*pi*Z/N modulo
    4*pi and modulo the reciprocal vector (2*pi, 2*pi); k_z in 2*pi*Z/N_z."""
    out = []
    for ix in range(2 * nx):
        for iy in range(ny):
            for iz in range(nz):
                k = (2 * np.pi * ix / nx, 2 * np.pi * iy / ny, 2 * np.pi * iz / nz)
                out.append(omega(k, m, dt) * dt)
    return np.array(out)


@pytest.mark.parametrize("m", [0.0, 0.6])
def test_spectrum_3d(m):
    """Eigenvalues of the one-step map are exp(-+i w(k) dt), w from Eq. (pwdsip),
    each twice (spin) per distinct plane wave."""
    nx, ny, nz = 2, 2, 4
    D = Dense3(nx, ny, nz, DT3)
    lat = oracle.Lattice3(nx, ny, nz, DT3)
    th = D.pack(lat.theta(m)).real
    ev = np.linalg.eigvals(D.step_matrix(th))
    assert np.allclose(np.abs(ev), 1.0, atol=1e-12)
    got = np.sort(np.angle(ev))
    ph = _extended_zone_phases(nx, ny, nz, m, DT3)
    expect = np.sort(np.concatenate([ph, ph, -ph, -ph]))
    assert got.shape == expect.shape
    assert np.abs(got - expect).max() < 1e-10


@pytest.mark.parametrize("m", [0.0, 0.4])
def test_spectrum_2d(m):
    nx, ny = 4, 6
    D = Dense2(nx, ny, DT2)
    lat = oracle.Lattice2(nx, ny, DT2)
    ev = np.linalg.eigvals(D.step_matrix(D.pack(lat.theta(m)).real))
    got = np.sort(np.angle(ev))
    ph = []
    for ix in range(2 * nx):
        for iy in range(ny):
            k = (2 * np.pi * ix / nx, 2 * np.pi * iy / ny)
            P2 = lattice_momentum(k[0]) ** 2 + lattice_momentum(k[1]) ** 2
            ph.append(2 * np.arcsin(np.sqrt((m * m + P2) / (m * m + (2 / DT2) ** 2))))
    ph = np.array(ph)
    expect = np.sort(np.concatenate([ph, -ph]))
    assert np.abs(got - expect).max() < 1e-10


def test_gram_min_eigenvalue():
    """Derived from Eq. (EPM): G has eigenvalues 1 +- |rho(k)|/2, rho_j = dt P_j, so its
    smallest is 1 - sqrt(sum r_j^2), reached at the zone corner (consistent with
    the reality condition r_x^2 + r_y^2 + r_z^2 <= 1 of Sect. 2.2)."""
    for dt, (nx, ny, nz) in [(DT3, (2, 2, 2)), (0.3, (4, 2, 2))]:
        G = Dense3(nx, ny, nz, dt).gram()
        lo = np.linalg.eigvalsh(G).min()
        assert abs(lo - (1 - np.sqrt(3) * dt)) < 1e-12
    G = Dense2(4, 4, DT2).gram()
    assert abs(np.linalg.eigvalsh(G).min() - (1 - np.sqrt(2) * DT2)) < 1e-12


# --------------------------------------------------------------------------
# Conservation (Lemmas of Sects. 2, 3) on larger random data with random
# site- and time-dependent m, V.
# --------------------------------------------------------------------------
def test_conservation_3d_time_dependent():
    g = rng(5)
    lat = oracle.Lattice3(8, 6, 10, DT3)
    f = rand_state(lat.shape, 8, g)
    e0 = lat.energy(f)
    assert abs(e0[0] - e0[1]) < 1e-13 * abs(e0[0])
    for _ in range(100):
        lat.step(f, rand_theta(lat.shape, 8, g, 0.5))
    e1 = lat.energy(f)
    assert abs(e1[0] - e0[0]) < 1e-13 * abs(e0[0])
    assert abs(e1[1] - e1[0]) < 1e-13 * abs(e0[0])
    assert abs(e1[2] - e0[2]) > 1e-6 * e0[2]     # the plain norm is not conserved


def test_conservation_2d_and_printed_sign():
    """Sect. 3, Eq. (E): the functional the update equations conserve carries
    delta_+; the printed delta_- form is not conserved once k_y != 0."""
    g = rng(6)
    lat = oracle.Lattice2(16, 12, DT2)
    f = rand_state(lat.shape, 4, g)
    e0 = lat.energy(f)
    for _ in range(200):
        lat.step(f, rand_theta(lat.shape, 4, g, 0.5))
    e1 = lat.energy(f)
    assert abs(e1[0] - e0[0]) < 1e-13 * abs(e0[0])
    assert abs(e1[1] - e0[1]) > 1e-4 * abs(e0[1])


def test_energy_plane_wave_closed_form():
    """E_r of a plane wave psi^(1) with A~ = 1 (from Eq. EPM and the substitution
    rules): n_A [1 + |P|^2/(E+m k)^2 - (dt^2/2) E |P|^2/(E+m k)], and the plain
    norm n_A [1 + |P|^2/(E+m k)^2], with n_A the number of A sites."""
    nx, ny, nz = 8, 6, 10
    for m in (0.0, 0.5):
        lat = oracle.Lattice3(nx, ny, nz, DT3)
        for n in [(1, 2, 3), (3, -1, 4), (9, 2, 1)]:
            k = (2 * np.pi * n[0] / nx, 2 * np.pi * n[1] / ny, 2 * np.pi * n[2] / nz)
            w, amps = eigenket3(k, m, DT3, 1)
            f = plane_wave3(lat.shape, k, amps, w, DT3)
            P2 = sum(lattice_momentum(kj) ** 2 for kj in k)
            X = np.sin(w * DT3 / 2)
            E = 2 / DT3 * X
            den = E + m * np.sqrt(1 - X * X)
            nA = 2 * nx * ny * nz
            e = lat.energy(f)
            assert abs(e[2] - nA * (1 + P2 / den ** 2)) < 1e-11 * e[2]
            expect = nA * (1 + P2 / den ** 2 - 0.5 * DT3 ** 2 * E * P2 / den)
            assert abs(e[0] - expect) < 1e-11 * e[2]
            assert abs(e[1] - expect) < 1e-11 * e[2]
    lat2 = oracle.Lattice2(16, 16, DT2)
    for n in [(1, 3), (5, -2)]:
        k = (2 * np.pi * n[0] / 16, 2 * np.pi * n[1] / 16)
        w, amps = eigenket2(k, 0.3, DT2, 1)
        f = plane_wave2(lat2.shape, k, amps, w, DT2)
        P2 = sum(lattice_momentum(kj) ** 2 for kj in k)
        X = np.sin(w * DT2 / 2)
        E = 2 / DT2 * X
        den = E + 0.3 * np.sqrt(1 - X * X)
        nA = 2 * 16 * 16
        expect = nA * (1 + P2 / den ** 2 - 0.5 * DT2 ** 2 * E * P2 / den)
        assert abs(lat2.energy(f)[0] - expect) < 1e-11 * expect


# --------------------------------------------------------------------------
# Stability (Sect. 2.2, Props. 2 and 4; Sect. 3)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_growth_just_beyond_bound(dim):
    """At r = 1.01 x bound (m = 0) the zone-corner mode has X = 1.01 > 1 and the
    plain norm grows by |lambda|^2 = (X + sqrt(X^2 - 1))^4 per step."""
    g = rng(7)
    if dim == 3:
        dt = 1.01 / np.sqrt(3)
        lat, cnt = oracle.Lattice3(4, 4, 4, dt), 8
    else:
        dt = 1.01 / np.sqrt(2)
        lat, cnt = oracle.Lattice2(4, 4, dt), 4
    th = lat.theta(0.0)
    f = rand_state(lat.shape, cnt, g)
    lat.step(f, th, 40)
    n0 = lat.energy(f)[-1]
    lat.step(f, th)
    n1 = lat.energy(f)[-1]
    assert abs(n1 / n0 - growth_factor(1.01) ** 2) < 1e-6
    assert abs(growth_factor(1.01) - 1.32658) < 1e-5


def test_bounds_below_threshold():
    """C2-type bound from the Gram eigenvalues: plain norm <= E_r / (1 - sqrt(sum r^2))
    at r = 0.99 x bound; Prop. 2 (sum r_j < 1) and Prop. 4 (2D) bounds."""
    g = rng(8)
    for dt, bound in [(0.99 / np.sqrt(3), lambda r: 1 - np.sqrt(3) * r), (0.3, lambda r: 1 - 3 * r)]:
        lat = oracle.Lattice3(4, 4, 4, dt)
        f = rand_state(lat.shape, 8, g)
        E0 = lat.energy(f)[0]
        for _ in range(300):
            lat.step(f, rand_theta(lat.shape, 8, g, 0.3))
            assert lat.energy(f)[-1] <= E0 / bound(dt) * (1 + 1e-12)
    dt = 0.45
    lat = oracle.Lattice2(6, 6, dt)
    f = rand_state(lat.shape, 4, g)
    E0 = lat.energy(f)[0]
    for _ in range(300):
        lat.step(f, rand_theta(lat.shape, 4, g, 0.3))
        assert lat.energy(f)[-1] <= E0 / (1 - 2 * dt) * (1 + 1e-12)


def test_prop3_2d_averaged_norm_at_bound():
    """Sect. 3, last Proposition: at r = 1/sqrt(2) the averaged norms satisfy
    ||u~||^2 + ||v~||^2 <= 2 E^0 for arbitrary m, V.  ||v~|| uses the same
    construction on the v sublattices shifted by half a cell in x."""
    g = rng(9)
    dt = 1 / np.sqrt(2)
    lat = oracle.Lattice2(8, 8, dt)
    f = rand_state(lat.shape, 4, g)
    E0 = lat.energy(f)[0]

    def avg_norm(p0, p1):
        # p0 on the integer cells, p1 on the (i+1/2, j+1/2) cells of one fcr sublattice:
        # sum over both sub-grids of |(p(x+1,y) - i p(x+1/2,y+1/2) + p(x,y) - i p(x+1/2,y-1/2)) / (2 sqrt 2)|^2
        t0 = (np.roll(p0, -1, 1) - 1j * p1 + p0 - 1j * np.roll(p1, 1, 0)) / (2 * np.sqrt(2))
        t1 = (np.roll(p1, -1, 1) - 1j * np.roll(p0, (-1, -1), (0, 1)) + p1 - 1j * np.roll(p0, -1, 1)) \
            / (2 * np.sqrt(2))
        return float(np.sum(np.abs(t0) ** 2) + np.sum(np.abs(t1) ** 2))

    for _ in range(200):
        lat.step(f, rand_theta(lat.shape, 4, g, 0.5))
        u = avg_norm(f[0], f[1])
        v = avg_norm(f[2], np.roll(f[3], -1, 1))
        assert u + v <= 2 * E0 * (1 + 1e-12)


# --------------------------------------------------------------------------
# Time reversal and 2D <-> 3D
# --------------------------------------------------------------------------
def test_reversibility_3d():
    g = rng(10)
    lat = oracle.Lattice3(6, 4, 8, DT3)
    th = rand_theta(lat.shape, 8, g, 0.5)
    f0 = rand_state(lat.shape, 8, g)
    f = [a.copy() for a in f0]
    lat.step(f, th, 1000)
    lat.reverse(f, th, 1000)
    assert rel_l2(f, f0) < 1e-13


def test_reversibility_2d():
    g = rng(11)
    lat = oracle.Lattice2(12, 10, DT2)
    th = rand_theta(lat.shape, 4, g, 0.5)
    f0 = rand_state(lat.shape, 4, g)
    f = [a.copy() for a in f0]
    lat.step(f, th, 1000)
    lat.reverse(f, th, 1000)
    assert rel_l2(f, f0) < 1e-13


def test_2d_is_the_AD_block_of_3d():
    """With N_z = 1 the z differences vanish: (A, D) evolve as the (2+1)D scheme with
    (u, v) = (A, D), and (C, B) as the (2+1)D scheme with u = C, v = B, m -> -m."""
    g = rng(12)
    nx, ny, dt, m = 7, 5, DT2 * 0.8, 0.35
    l3 = oracle.Lattice3(nx, ny, 1, dt)
    l2 = oracle.Lattice2(nx, ny, dt)
    Vf = lambda x, y, z=None: 0.3 * np.sin(0.9 * x) * np.cos(0.7 * y)
    th3 = l3.theta(m, lambda x, y, z: Vf(x, y))
    f3 = rand_state(l3.shape, 8, g)
    f3[2][:] = 0
    f3[3][:] = 0
    f3[4][:] = 0
    f3[5][:] = 0
    f2 = [f3[0][0].copy(), f3[1][0].copy(), f3[6][0].copy(), f3[7][0].copy()]
    l3.step(f3, th3, 50)
    l2.step(f2, l2.theta(m, Vf), 50)
    assert rel_l2([f3[0][0], f3[1][0], f3[6][0], f3[7][0]], f2) < 1e-14
    assert np.abs(l3.energy(f3)[0] - l2.energy(f2)[0]) < 1e-13 * l2.energy(f2)[0]
    # the B-C block: B is updated first (from C) with the delta_+ stencil, C second
    # with delta_-, so it is the 2D scheme for u = C, v = B, m -> -m, started from
    # (u, v) = (C^0, B^{1/2}).  After n 2D steps u = C^n and v = B^{n+1/2}.
    f3 = rand_state(l3.shape, 8, g)
    for a in (0, 1, 6, 7):
        f3[a][:] = 0
    c0 = [f3[4][0].copy(), f3[5][0].copy()]
    l3.step(f3, th3, 1)
    f2 = [c0[0], c0[1], f3[2][0].copy(), f3[3][0].copy()]
    th2 = l2.theta(-m, Vf)
    n = 30
    l3.step(f3, th3, n - 1)
    c_n = [f3[4][0].copy(), f3[5][0].copy()]
    l3.step(f3, th3, 1)
    l2.step(f2, th2, n)
    assert rel_l2(f2[:2], c_n) < 1e-14
    assert rel_l2(f2[2:], [f3[2][0], f3[3][0]]) < 1e-14


# --------------------------------------------------------------------------
# Adjoint: dot-product test against the dense matrix, and finite differences.
# --------------------------------------------------------------------------
def test_adjoint_matches_dense_transpose():
    g = rng(13)
    lat = oracle.Lattice3(2, 3, 4, DT3)
    D = Dense3(2, 3, 4, DT3)
    th = rand_theta(lat.shape, 8, g)
    pre = rand_state(lat.shape, 8, g)
    post = [a.copy() for a in pre]
    lat.step(post, th)
    lam = rand_state(lat.shape, 8, g)
    lam_v = D.pack(lam)
    gth = [np.zeros(lat.shape) for _ in range(8)]
    lat.adjoint(pre, post, lam, th, gth)
    M = D.step_matrix(D.pack(th).real)
    assert rel_l2([D.pack(lam)], [M.conj().T @ lam_v]) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_adjoint_theta_gradient_fd(dim):
    """dL/dtheta per site from the chain rule vs central differences (h = 1e-6),
    L = probability in the region z >= z0 (x >= x0 in 2D) after n steps."""
    g = rng(14 + dim)
    nsteps = 6
    if dim == 3:
        lat, cnt = oracle.Lattice3(3, 2, 6, DT3), 8
        z0 = 3.0

        def loss(f):
            return lat.observe(f, z0)[0]

        def seed(f):
            mask = [lat.positions(a)[2] >= z0 for a in range(8)]
            return loss(f), [2 * f[a] * mask[a] for a in range(8)]
        run = oracle.run_with_adjoint3
    else:
        lat, cnt = oracle.Lattice2(6, 4, DT2), 4
        z0 = 3.0

        def loss(f):
            return lat.observe(f, z0)[0]

        def seed(f):
            mask = [lat.positions(a)[0] >= z0 for a in range(4)]
            return loss(f), [2 * f[a] * mask[a] for a in range(4)]
        run = oracle.run_with_adjoint2
    th = rand_theta(lat.shape, cnt, g, 0.4)
    f0 = rand_state(lat.shape, cnt, g)
    _, _, gth, _ = run(lat, f0, th, nsteps, seed)
    h = 1e-6
    for _ in range(12):
        a = int(g.integers(cnt))
        idx = tuple(int(g.integers(s)) for s in lat.shape)
        vals = []
        for s in (+1, -1):
            t2 = [x.copy() for x in th]
            t2[a][idx] += s * h
            f = [x.copy() for x in f0]
            lat.step(f, t2, nsteps)
            vals.append(loss(f))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - gth[a][idx]) < 1e-6 * max(1.0, abs(fd)), (a, idx, fd, gth[a][idx])


# --------------------------------------------------------------------------
# Complex potential (absorbing layers): theta = (dt/2)(+-m + V) with complex V.
# Sect. 3 stability discussion: the growth factors have modulus below one when
# the imaginary part has the damping sign.  In the Cayley form used here that
# sign is Im V < 0 (|1 - i theta| < |1 + i theta| iff Im theta < 0).
# --------------------------------------------------------------------------
def _rand_thi(shape, count, g, lo=-0.4, hi=0.2):
    return [np.ascontiguousarray(g.uniform(lo, hi, shape)) for _ in range(count)]


@pytest.mark.parametrize("dim", [2, 3])
def test_complex_theta_dense_matches_oracle(dim):
    """Brute force: the oracle's complex-theta step equals the dense one-step
    matrix assembled from coordinates with alpha, beta of the complex theta."""
    g = rng(201)
    if dim == 3:
        lat, D, cnt = oracle.Lattice3(3, 2, 4, DT3), Dense3(3, 2, 4, DT3), 8
    else:
        lat, D, cnt = oracle.Lattice2(4, 3, DT2), Dense2(4, 3, DT2), 4
    f = rand_state(lat.shape, cnt, g)
    x = D.pack(f)
    for _ in range(3):
        th = rand_theta(lat.shape, cnt, g)
        thi = _rand_thi(lat.shape, cnt, g)
        lat.step(f, th, thi=thi)
        x = D.step_matrix(D.pack(th).real + 1j * D.pack(thi).real) @ x
    assert rel_l2([D.pack(f)], [x]) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_complex_theta_dissipation_identity(dim):
    """Multiplying (X+ - X-) + S_X = -i theta (X+ + X-) by conj(X+ + X-), taking
    real parts and summing over both half-steps, the cross terms telescope into
    the conserved functional (anti-Hermitian stencils), leaving
      E_r(n+1) - E_r(n) = sum_sites Im(theta) |X+ + X-|^2
    exactly; it vanishes for real theta (the Lemma of Sect. 2) and is <= 0 when
    Im theta <= 0 everywhere."""
    g = rng(202)
    if dim == 3:
        lat, cnt = oracle.Lattice3(6, 5, 7, DT3), 8
    else:
        lat, cnt = oracle.Lattice2(9, 8, DT2), 4
    f0 = rand_state(lat.shape, cnt, g)
    th = rand_theta(lat.shape, cnt, g)
    for lo, hi in ((-0.3, 0.25), (-0.3, 0.0)):
        thi = _rand_thi(lat.shape, cnt, g, lo, hi)
        f = [a.copy() for a in f0]
        e0 = lat.energy(f)[0]
        lat.step(f, th, thi=thi)
        e1 = lat.energy(f)[0]
        rhs = sum(float(np.sum(thi[a] * np.abs(f[a] + f0[a]) ** 2)) for a in range(cnt))
        scale = sum(float(np.sum(np.abs(a) ** 2)) for a in f0)
        assert abs((e1 - e0) - rhs) <= 1e-13 * scale, (e1 - e0, rhs)
        if hi <= 0.0:
            assert e1 < e0


def _amplification_2d(k, m, V, dt):
    """2x2 amplification matrix of the (2+1)D scheme for a plane wave (u at
    n-1/2, v at n) with uniform complex V: Fourier symbols of the stencils of
    Eqs. scheme2Deq-scheme4thline on the staggered positions,
      (1 + i th_u) u+ = (1 - i th_u) u- - s_u v-,
      (1 + i th_v) v+ = (1 - i th_v) v- - s_v u+,
    s_u = r (2i sin(kx/2) + 2 sin(ky/2)), s_v = r (2i sin(kx/2) - 2 sin(ky/2))."""
    r = dt
    th_u, th_v = 0.5 * dt * (m + V), 0.5 * dt * (-m + V)
    su = r * (2j * np.sin(k[0] / 2) + 2 * np.sin(k[1] / 2))
    sv = r * (2j * np.sin(k[0] / 2) - 2 * np.sin(k[1] / 2))
    S = np.array([[1 + 1j * th_u, 0], [sv, 1 + 1j * th_v]])
    T = np.array([[1 - 1j * th_u, -su], [0, 1 - 1j * th_v]])
    return np.linalg.solve(S, T)


@pytest.mark.parametrize("V", [-0.2j, 0.3 - 0.4j, 0.8j, 0.5])
def test_complex_potential_plane_wave_2d(V):
    """A plane-wave eigenvector of the amplification matrix decays (or grows) by
    its eigenvalue per step in the oracle; the matrix's determinant and trace
    are the paper's Q and P (P with the Delta_t^2 factor on the 4 c^2 term
    restored); |lambda| < 1 exactly when Im V < 0."""
    m, dt, n = 0.3, DT2, 32
    k = (2 * np.pi * 3 / n, 2 * np.pi * 5 / n)
    G = _amplification_2d(k, m, V, dt)
    # the paper's closed forms (hbar = c = 1, unit spacing)
    N = 4 + (m * m - V * V) * dt * dt + 4j * V * dt
    Q = (4 + (m * m - V * V) * dt * dt - 4j * V * dt) / N
    P = -2 * ((m * m - V * V) * dt * dt - 4 * (1 - 2 * dt * dt)
              - 4 * dt * dt * (np.cos(k[0]) + np.cos(k[1]))) / N
    assert abs(np.linalg.det(G) - Q) < 1e-13 and abs(np.trace(G) - P) < 1e-13
    lam, vec = np.linalg.eig(G)
    for q in range(2):
        if np.imag(V) < 0:
            assert abs(lam[q]) < 1.0
        elif np.imag(V) > 0:
            assert abs(lam[q]) > 1.0
        else:
            assert abs(abs(lam[q]) - 1.0) < 1e-14
        f = plane_wave2((n, n), k, vec[:, q], 0.0, dt)
        lat = oracle.Lattice2(n, n, dt)
        th = [np.full((n, n), 0.5 * dt * ((1.0 if a < 2 else -1.0) * m + np.real(V))) for a in range(4)]
        thi = [np.full((n, n), 0.5 * dt * np.imag(V)) for a in range(4)]
        f0 = [a.copy() for a in f]
        steps = 20
        lat.step(f, th, steps, thi=thi)
        assert rel_l2(f, [lam[q] ** steps * a for a in f0]) < 1e-12


# --------------------------------------------------------------------------
# Vector potential by gauge links (Sect. 4, Peierls substitution).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_links_pure_gauge_is_a_phase(dim):
    """Links built from a site function chi, U(X -> Y) = exp(i(chi(Y) - chi(X))),
    are a pure gauge: the evolved state is exp(-i chi) times the free evolution
    of exp(i chi) psi0, exactly.  A wrong orientation or a missing conjugate on
    either sheet breaks this."""
    g = rng(301)
    if dim == 3:
        lat, cnt = oracle.Lattice3(5, 4, 6, DT3), 8
        make = links_from_site_phase3
    else:
        lat, cnt = oracle.Lattice2(7, 6, DT2), 4
        make = links_from_site_phase2
    chi = [g.uniform(-np.pi, np.pi, lat.shape) for _ in range(cnt)]
    U = make(lat.shape, chi)
    f0 = rand_state(lat.shape, cnt, g)
    th = rand_theta(lat.shape, cnt, g)
    f = [a.copy() for a in f0]
    lat.step(f, th, 6, links=U)
    h = [np.exp(1j * chi[a]) * f0[a] for a in range(cnt)]
    lat.step(h, th, 6)
    assert rel_l2(f, [np.exp(-1j * chi[a]) * h[a] for a in range(cnt)]) < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_links_unit_and_conservation(dim):
    """Unit links give the plain scheme; a static link field that is not a pure
    gauge (random phases; a uniform magnetic flux in 2D) keeps E_r, with the
    links in S_X, exactly conserved, and its two forms agree."""
    g = rng(302)
    if dim == 3:
        lat, cnt, nl = oracle.Lattice3(6, 5, 7, DT3), 8, 24
    else:
        lat, cnt, nl = oracle.Lattice2(9, 8, DT2), 4, 8
    f0 = rand_state(lat.shape, cnt, g)
    th = rand_theta(lat.shape, cnt, g)
    ones = [np.ones(lat.shape, np.complex128) for _ in range(nl)]
    f1, f2 = [a.copy() for a in f0], [a.copy() for a in f0]
    lat.step(f1, th, 3, links=ones)
    lat.step(f2, th, 3)
    assert rel_l2(f1, f2) < 1e-15
    # smooth fields with curl (a physical vector potential varies slowly on the
    # grid; uniformly random link phases would make E_r indefinite, and the
    # state then grows although E_r is still an exact invariant)
    if dim == 3:
        fields = [links_from_potential3(lat.shape, smooth_potential3(lat.shape, 0.5, 7))]
    else:
        fields = [links_uniform_field2(lat.shape, 0.05),
                  links_from_potential2(lat.shape, lambda x, y: (0.4 * np.sin(2 * np.pi * y / 8.0),
                                                                 0.3 * np.cos(2 * np.pi * x / 9.0)))]
    for U in fields:
        f = [a.copy() for a in f0]
        e0 = lat.energy_links(f, U)
        assert abs(e0[0] - e0[1]) < 1e-13 * e0[2]
        lat.step(f, th, 50, links=U)
        e1 = lat.energy_links(f, U)
        assert e1[2] < 10 * e0[2]                     # bounded: E_r is definite here
        assert abs(e1[0] - e0[0]) < 1e-13 * 50 * e0[2]
        assert abs(e1[0] - e1[1]) < 1e-13 * e0[2]
        # without the links in S_X the functional is not the conserved one
        assert abs(lat.energy(f)[0] - e0[0]) > 1e-6 * e0[2]


@pytest.mark.parametrize("dim", [2, 3])
def test_links_match_dense_from_potential(dim):
    """The oracle's link step (C,D / v rows find their link by displacement) equals
    the dense one-step matrix assembled from the vector potential itself, each
    coupling carrying exp(-i a_j(M) d) for its own midpoint M and displacement d
    (Sect. 4); the link functional equals psi^H G psi of that operator, and
    M^H G M = G."""
    g = rng(303)
    if dim == 3:
        nx, ny, nz = 4, 3, 5
        lat, cnt = oracle.Lattice3(nx, ny, nz, DT3), 8
        a_fn = smooth_potential3(lat.shape, 0.7, 11)
        D = Dense3(nx, ny, nz, DT3, a_fn=a_fn)
        U = links_from_potential3(lat.shape, a_fn)
    else:
        nx, ny = 5, 4
        lat, cnt = oracle.Lattice2(nx, ny, DT2), 4
        a_fn = lambda x, y: (0.6 * np.sin(2 * np.pi * y / ny + 0.3) + 0.2,
                             0.5 * np.cos(2 * np.pi * x / nx - 0.4) * np.cos(2 * np.pi * y / ny))
        D = Dense2(nx, ny, DT2, a_fn=a_fn)
        U = links_from_potential2(lat.shape, a_fn)
    f = rand_state(lat.shape, cnt, g)
    x0 = D.pack(f)
    x = x0.copy()
    for _ in range(3):
        th = rand_theta(lat.shape, cnt, g)
        lat.step(f, th, links=U)
        x = D.step_matrix(D.pack(th).real) @ x
    assert rel_l2([D.pack(f)], [x]) < 1e-13
    G = D.gram()
    e = lat.energy_links(f, U)
    xf = D.pack(f)
    assert abs(np.vdot(xf, G @ xf).real - e[0]) < 1e-12 * e[2]
    M = D.step_matrix(D.pack(rand_theta(lat.shape, cnt, g)).real)
    assert np.abs(M.conj().T @ G @ M - G).max() < 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_linearised_rule_is_second_order(dim):
    """Sect. 4's simplified rule for smooth potentials (a difference psi(+) -
    psi(-) becomes psi(+) - psi(-) - i a_j (psi(+) + psi(-))/2) agrees with the
    exact Peierls links to second order in a: for a uniform potential the
    one-step difference shrinks fourfold when a is halved."""
    g = rng(304)
    if dim == 3:
        nx, ny, nz = 3, 4, 4
        f = rand_state((nz, ny, nx), 8, g)
        mk = lambda fn, rule: Dense3(nx, ny, nz, DT3, a_fn=fn, rule=rule)
        n_arr = 8
        shape = (nz, ny, nx)
    else:
        nx, ny = 5, 4
        f = rand_state((ny, nx), 4, g)
        mk = lambda fn, rule: Dense2(nx, ny, DT2, a_fn=fn, rule=rule)
        n_arr = 4
        shape = (ny, nx)
    th = rand_theta(shape, n_arr, g)
    diffs = []
    for eps in (0.2, 0.1, 0.05):
        fn = (lambda x, y, z: (0.7 * eps, -0.4 * eps, 0.5 * eps)) if dim == 3 else \
             (lambda x, y: (0.7 * eps, -0.4 * eps))
        De, Dl = mk(fn, "exact"), mk(fn, "linear")
        x = De.pack(f)
        t = De.pack(th).real
        diffs.append(np.linalg.norm(De.step_matrix(t) @ x - Dl.step_matrix(t) @ x) / np.linalg.norm(x))
    assert diffs[1] > 1e-5
    for q in range(2):
        assert 3.6 < diffs[q] / diffs[q + 1] < 4.4, diffs


# --------------------------------------------------------------------------
# Observables of the plain density (its sum is the naive norm of Sect. 2.2 and
# Sect. 3; a region sum is a transmitted or reflected fraction, Sect. 5).
# Pinned against the site positions of the staggered grid (Sect. 2, Eq.
# ABCDgrid; Sect. 3 for 2D) written out here from the paper by array name, not
# from the oracle's tables: a single nonzero amplitude sits at one known site,
# and an eigen plane wave of Sect. 2.1 has a uniform density per array, so its
# first moments are the mean site coordinate of each array times its weight.
# --------------------------------------------------------------------------
#: paper positions of the amplitude stored for cell (i, j, k), by array name
GRID3 = {"A0": (0.0, 0.0, 0.0), "A1": (0.5, 0.5, 0.0), "B0": (0.5, 0.0, 0.5), "B1": (0.0, 0.5, 0.5),
         "C0": (0.0, 0.0, 0.5), "C1": (0.5, 0.5, 0.5), "D0": (0.5, 0.0, 0.0), "D1": (0.0, 0.5, 0.0)}
NAMES3 = ["A0", "A1", "B0", "B1", "C0", "C1", "D0", "D1"]
GRID2 = {"u0": (0.0, 0.0), "u1": (0.5, 0.5), "v0": (0.5, 0.0), "v1": (0.0, 0.5)}
NAMES2 = ["u0", "u1", "v0", "v1"]


def test_observables_single_site_3d():
    """One amplitude at a time: the region sum includes the site iff z_s >= z0
    (z0 on the site's own plane, and just above and below it), the moments are
    the site's position times |X|^2, and the weight lands on its component."""
    nx, ny, nz = 5, 4, 6
    lat = oracle.Lattice3(nx, ny, nz, DT3)
    for a, name in enumerate(NAMES3):
        for (i, j, k) in [(0, 0, 0), (4, 3, 5), (2, 1, 3)]:
            f = lat.zeros()
            val = 0.75 - 0.5j * (1 + a)          # dyadic: |val|^2 and its moments are exact
            w = val.real ** 2 + val.imag ** 2
            f[a][k, j, i] = val
            ox, oy, oz = GRID3[name]
            x, y, z = i + ox, j + oy, k + oz
            comp = "ABCD".index(name[0])
            out = lat.observe(f, z)
            assert out[0] == w, (name, "z0 on the site plane is inside the region")
            assert lat.observe(f, z + 1e-9)[0] == 0.0, (name, "just above the site")
            assert lat.observe(f, z - 1e-9)[0] == w, (name, "just below the site")
            assert lat.observe(f, z + 0.5)[0] == 0.0 and lat.observe(f, z - 0.5)[0] == w, name
            assert out[4] == w
            np.testing.assert_allclose(out[1:4], (x * w, y * w, z * w), rtol=1e-15, err_msg=name)
            per = [0.0] * 4
            per[comp] = w
            assert list(out[5:9]) == per, name


def test_observables_single_site_2d():
    nx, ny = 5, 3
    lat = oracle.Lattice2(nx, ny, DT2)
    for a, name in enumerate(NAMES2):
        for (i, j) in [(0, 0), (4, 2), (3, 1)]:
            f = lat.zeros()
            val = 0.25 + 1.5j * (2 + a)          # dyadic, as above
            w = val.real ** 2 + val.imag ** 2
            f[a][j, i] = val
            ox, oy = GRID2[name]
            x, y = i + ox, j + oy
            out = lat.observe(f, x)
            assert out[0] == w, name
            assert lat.observe(f, x + 1e-9)[0] == 0.0 and lat.observe(f, x - 1e-9)[0] == w, name
            assert out[3] == w
            np.testing.assert_allclose(out[1:3], (x * w, y * w), rtol=1e-15, err_msg=name)
            per = [0.0, 0.0]
            per["uv".index(name[0])] = w
            assert list(out[4:6]) == per, name


def _uniform_moments(n_cells, mean_pos, weights):
    """Sum of (position * weight) over arrays of uniform density: each array has
    n_cells sites of weight w whose coordinate averages mean_pos."""
    return sum(n_cells * w * p for w, p in zip(weights, mean_pos))


@pytest.mark.parametrize("branches", [(1,), (2,), (1, 2), (3, 4)])
def test_observables_eigen_plane_wave_3d(branches):
    """Eigenkets of Sect. 2.1 (after Eq. pwdsip) at one k, alone or superposed on
    the same energy shell: each array has the constant modulus of its spinor
    component, so the per-component sums are 2 N |psi_c|^2 in closed form, the
    first moments are the mean site coordinate times the weight, and the region
    z >= z0 holds exactly the sites on planes from z0 up.  Evolving the state
    (it is an eigenmode) leaves all of them unchanged."""
    nx, ny, nz = 6, 4, 10
    m = 0.5
    lat = oracle.Lattice3(nx, ny, nz, DT3)
    k = (2 * np.pi * 1 / nx, 2 * np.pi * 1 / ny, 2 * np.pi * 3 / nz)
    amps = np.zeros(4, complex)
    for b in branches:
        w, a4 = eigenket3(k, m, DT3, b)
        amps += np.asarray(a4, complex)
    f = plane_wave3(lat.shape, k, list(amps), w, DT3)
    ncell = nx * ny * nz
    wt = [abs(amps["ABCD".index(nm[0])]) ** 2 for nm in NAMES3]
    z0 = 4.5                     # B and C sites sit on z = 4.5; A and D on z = 5
    region = sum(wt[a] * nx * ny * sum(1 for kk in range(nz) if kk + GRID3[nm][2] >= z0)
                 for a, nm in enumerate(NAMES3))
    expect = [region]
    for ax, nn in enumerate((nx, ny, nz)):
        mean = [(nn - 1) / 2.0 + GRID3[nm][ax] for nm in NAMES3]
        expect.append(_uniform_moments(ncell, mean, wt))
    expect.append(ncell * sum(wt))
    expect += [2 * ncell * abs(amps[c]) ** 2 for c in range(4)]
    th = lat.theta(m)
    for steps in (0, 7):
        g = [a.copy() for a in f]
        lat.step(g, th, steps)
        out = lat.observe(g, z0)
        np.testing.assert_allclose(out, expect, rtol=1e-12, atol=1e-12, err_msg=str((branches, steps)))


@pytest.mark.parametrize("branch", [1, 2])
def test_observables_eigen_plane_wave_2d(branch):
    nx, ny = 8, 6
    m = 0.7
    lat = oracle.Lattice2(nx, ny, DT2)
    k = (2 * np.pi * 3 / nx, 2 * np.pi * 1 / ny)
    w, amps = eigenket2(k, m, DT2, branch)
    f = plane_wave2(lat.shape, k, amps, w, DT2)
    ncell = nx * ny
    wt = [abs(amps["uv".index(nm[0])]) ** 2 for nm in NAMES2]
    x0 = 3.5                     # u1 and v0 sit on x = 3.5
    region = sum(wt[a] * ny * sum(1 for i in range(nx) if i + GRID2[nm][0] >= x0) for a, nm in enumerate(NAMES2))
    expect = [region]
    for ax, nn in enumerate((nx, ny)):
        mean = [(nn - 1) / 2.0 + GRID2[nm][ax] for nm in NAMES2]
        expect.append(_uniform_moments(ncell, mean, wt))
    expect.append(ncell * sum(wt))
    expect += [2 * ncell * abs(amps[c]) ** 2 for c in range(2)]
    th = lat.theta(m)
    for steps in (0, 9):
        g = [a.copy() for a in f]
        lat.step(g, th, steps)
        np.testing.assert_allclose(lat.observe(g, x0), expect, rtol=1e-12, atol=1e-12, err_msg=str(steps))


def test_observables_translation_covariance_3d():
    """Moving a localised random state by one cell along x, y or z moves the
    matching first moment by the norm and leaves the rest (norm, per-component
    sums) unchanged; the region sum moves by the weight of one plane pair."""
    g = rng(77)
    nx, ny, nz = 7, 6, 9
    lat = oracle.Lattice3(nx, ny, nz, DT3)
    f = lat.zeros()
    for a in range(8):
        f[a][2:5, 1:4, 1:5] = g.standard_normal((3, 3, 4)) + 1j * g.standard_normal((3, 3, 4))
    base = lat.observe(f, 3.0)
    for ax in range(3):
        sh = [np.ascontiguousarray(np.roll(a, 1, axis=2 - ax)) for a in f]
        out = lat.observe(sh, 3.0)
        np.testing.assert_allclose(out[1 + ax], base[1 + ax] + base[4], rtol=1e-13)
        np.testing.assert_allclose(out[4:], base[4:], rtol=1e-13)


# --------------------------------------------------------------------------
# Zero values outside the lattice (a Dirichlet frame).  The Lemmas of Sect. 2
# and Sect. 3 sum by parts over the lattice; with zero ghosts, as with periodic
# wrap, no boundary terms remain, so E_r is conserved exactly.  Pinned by the
# dense matrix assembled with the outside couplings dropped, M^H G M = G, the
# reversed step, and agreement with the periodic oracle while the light cone
# of an interior state has not reached the boundary.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(3, 2, 4), (2, 3, 2), (4, 4, 3)])
def test_zero_bc_dense_matches_oracle_3d(shape):
    g = rng(201)
    nx, ny, nz = shape
    lat = oracle.Lattice3(nx, ny, nz, DT3, zero_bc=True)
    D = Dense3(nx, ny, nz, DT3, zero_bc=True)
    th = rand_theta(lat.shape, 8, g)
    f = rand_state(lat.shape, 8, g)
    x = D.pack(f)
    M = D.step_matrix(D.pack(th).real)
    lat.step(f, th, 3)
    assert rel_l2([D.pack(f)], [M @ (M @ (M @ x))]) < 1e-14
    # the periodic matrix is a different operator on these shapes
    Mp = Dense3(nx, ny, nz, DT3).step_matrix(D.pack(th).real)
    assert np.abs(Mp - M).max() > 0.1


@pytest.mark.parametrize("shape", [(4, 3), (2, 5), (1, 3)])
def test_zero_bc_dense_matches_oracle_2d(shape):
    g = rng(202)
    nx, ny = shape
    lat = oracle.Lattice2(nx, ny, DT2, zero_bc=True)
    D = Dense2(nx, ny, DT2, zero_bc=True)
    th = rand_theta(lat.shape, 4, g)
    f = rand_state(lat.shape, 4, g)
    x = D.pack(f)
    M = D.step_matrix(D.pack(th).real)
    lat.step(f, th, 3)
    assert rel_l2([D.pack(f)], [M @ (M @ (M @ x))]) < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_zero_bc_conserves_functional(dim):
    """M^H G M = G for the truncated operator (random site-dependent theta), the
    oracle's E_r equals psi^H G psi in both its forms, and a long run with
    time-dependent theta conserves it to rounding."""
    g = rng(203 + dim)
    if dim == 3:
        lat, D, cnt = oracle.Lattice3(3, 4, 2, DT3, zero_bc=True), Dense3(3, 4, 2, DT3, zero_bc=True), 8
    else:
        lat, D, cnt = oracle.Lattice2(5, 3, DT2, zero_bc=True), Dense2(5, 3, DT2, zero_bc=True), 4
    th = rand_theta(lat.shape, cnt, g)
    M = D.step_matrix(D.pack(th).real)
    G = D.gram()
    assert np.abs(M.conj().T @ G @ M - G).max() < 1e-13
    f = rand_state(lat.shape, cnt, g)
    x = D.pack(f)
    e = lat.energy(f)
    ref = float(np.real(x.conj() @ G @ x))
    assert abs(e[0] - ref) <= 1e-13 * abs(ref)
    if dim == 3:
        assert abs(e[1] - ref) <= 1e-13 * abs(ref)
    e0 = e[0]
    for _ in range(300):
        lat.step(f, rand_theta(lat.shape, cnt, g, scale=0.8))
    assert abs(lat.energy(f)[0] - e0) <= 1e-13 * abs(e0)


@pytest.mark.parametrize("dim", [2, 3])
def test_zero_bc_reverse_and_light_cone(dim):
    """The reversed step undoes the step; a state four cells from every face
    evolves for two steps exactly as on the periodic lattice (its light cone,
    one cell per step, does not reach the boundary), and differently once it
    has."""
    g = rng(205 + dim)
    if dim == 3:
        mk = lambda z: oracle.Lattice3(10, 9, 11, DT3, zero_bc=z)
        cnt, sl = 8, (slice(4, 7), slice(4, 5), slice(4, 6))
    else:
        mk = lambda z: oracle.Lattice2(10, 9, DT2, zero_bc=z)
        cnt, sl = 4, (slice(4, 5), slice(4, 6))
    zl, pl = mk(True), mk(False)
    th = rand_theta(zl.shape, cnt, g)
    f = [np.zeros(zl.shape, np.complex128) for _ in range(cnt)]
    for a in f:
        a[sl] = g.standard_normal(a[sl].shape) + 1j * g.standard_normal(a[sl].shape)
    fz, fp = [a.copy() for a in f], [a.copy() for a in f]
    zl.step(fz, th, 2)
    pl.step(fp, th, 2)
    assert all(np.array_equal(a, b) for a, b in zip(fz, fp))
    zl.step(fz, th, 6)
    pl.step(fp, th, 6)
    assert rel_l2(fz, fp) > 1e-6
    zl.reverse(fz, th, 8)
    assert rel_l2(fz, f) < 1e-13
