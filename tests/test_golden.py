"""The oracle and the workload generators against the numbers the paper prints
(tests/golden/paper_printed_values.txt, each with its caption or section).

The paper prints no numerical tables; what it fixes numerically is the
stability threshold, the parameters its figures are drawn at and the Klein-step
cases of Sect. 5.  Each test here takes those numbers from the fixture and
checks a property the paper states at them."""
import math
import os

import numpy as np
import pytest

import oracle
import workloads
from closed_form import dirac2d_transmission, eigenket2, eigenket3, omega, plane_wave2, plane_wave3, rel_l2

HERE = os.path.dirname(__file__)


def printed():
    vals = {}
    with open(os.path.join(HERE, "golden", "paper_printed_values.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            name, rhs = (s.strip() for s in line.split("=", 1))
            if "/sqrt(" in rhs:
                num, rad = rhs.split("/sqrt(")
                vals[name] = float(num) / math.sqrt(float(rad.rstrip(")")))
            else:
                xs = [float(s) for s in rhs.split()]
                vals[name] = xs[0] if len(xs) == 1 else xs
    return vals


G = printed()


@pytest.mark.parametrize("dim", [2, 3])
def test_stability_threshold_is_the_printed_one(dim):
    """Just below the printed r the plain norm of random data stays under
    E_r / (1 - sqrt(sum r^2)) for 300 steps (Sect. 2.2, Sect. 3); just above it
    the zone-corner mode grows without bound."""
    r = G["r_bound_equal_3d"] if dim == 3 else G["r_bound_equal_2d"]
    g = np.random.default_rng(30 + dim)
    for scale, stable in ((0.999, True), (1.001, False)):
        dt = scale * r
        lat = oracle.Lattice3(4, 4, 4, dt) if dim == 3 else oracle.Lattice2(4, 4, dt)
        cnt = 8 if dim == 3 else 4
        f = [g.standard_normal(lat.shape) + 1j * g.standard_normal(lat.shape) for _ in range(cnt)]
        th = lat.theta(0.0)
        e0, n0 = lat.energy(f)[0], lat.energy(f)[-1]
        lat.step(f, th, 300)
        n1 = lat.energy(f)[-1]
        if stable:
            assert n1 <= e0 / (1.0 - math.sqrt(dim) * dt) * (1.0 + 1e-12)
        else:
            assert n1 > 1e6 * n0


@pytest.mark.parametrize("kz", G["fig_dispersion3d_kz"])
def test_fig2_dispersion_panels(kz):
    """At Fig. 2's time step (m = 0) plane waves in both panels (k_z = 0 and pi)
    evolve by the dispersion's phase in the oracle, and the single cone sits at
    k = 0: omega vanishes only there, and grows along each axis to the zone edge."""
    dt, n = G["fig_dispersion3d_dt"], 8
    for kxy in ((0, 0), (1, 0), (2, 3), (3, 3)):
        k = (2 * np.pi * kxy[0] / n, 2 * np.pi * kxy[1] / n, kz)
        if kz == 0.0 and kxy == (0, 0):
            assert omega(k, 0.0, dt) == 0.0
            continue
        w = omega(k, 0.0, dt)
        assert 0.0 < w * dt / 2 < np.pi / 2
        w1, amps = eigenket3(k, 0.0, dt, 1)
        assert w1 == pytest.approx(w, rel=1e-15)
        lat = oracle.Lattice3(n, n, 2, dt)
        f = plane_wave3(lat.shape, k, amps, w, dt)
        f0 = [a.copy() for a in f]
        lat.step(f, lat.theta(0.0), 50)
        assert rel_l2(f, [np.exp(-1j * w * 50 * dt) * a for a in f0]) < 1e-13
    ws = [omega((2 * np.pi * j / 16, 0.0, kz), 0.0, dt) for j in range(9)]
    assert all(b > a for a, b in zip(ws, ws[1:]))


def test_fig5_dispersion_2d():
    """At Fig. 5's time step (m = 0): one cone at k = 0, monotonic along the axes
    and the diagonal, and the oracle moves plane waves by that phase."""
    dt, n = G["fig_dispersion2d_dt"], 16
    for d in ((1, 0), (0, 1), (1, 1)):
        ws = [omega((2 * np.pi * j * d[0] / n, 2 * np.pi * j * d[1] / n), 0.0, dt) for j in range(n // 2)]
        assert ws[0] == 0.0 and all(b > a for a, b in zip(ws, ws[1:]))
    for kxy in ((1, 0), (3, 5), (6, 2)):
        k = (2 * np.pi * kxy[0] / n, 2 * np.pi * kxy[1] / n)
        w = omega(k, 0.0, dt)
        lat = oracle.Lattice2(n, n, dt)
        f = plane_wave2(lat.shape, k, eigenket2(k, 0.0, dt, 1)[1], w, dt)
        f0 = [a.copy() for a in f]
        lat.step(f, lat.theta(0.0), 50)
        assert rel_l2(f, [np.exp(-1j * w * 50 * dt) * a for a in f0]) < 1e-13


@pytest.mark.parametrize("im_v", G["fig_absorber_im_v"])
def test_fig4_absorber_panels(im_v):
    """At Fig. 4's step (Delta_t / Delta = 0.99/sqrt(2), m = 0) and its four
    imaginary potentials the oracle's functional E_r changes monotonically
    under a constant imaginary potential: it decays for Im V < 0 and grows for
    Im V > 0 in the sign convention of the update equations."""
    dt, n = G["fig_absorber_dt"], 8
    g = np.random.default_rng(41)
    f0 = [g.standard_normal((n, n)) + 1j * g.standard_normal((n, n)) for _ in range(4)]
    rates = {}
    for sgn in (-1.0, 1.0):
        lat = oracle.Lattice2(n, n, dt)
        f = [a.copy() for a in f0]
        th = lat.theta(0.0)
        thi = [np.full((n, n), 0.5 * dt * sgn * im_v) for _ in range(4)]
        e = [lat.energy(f)[0]]
        for _ in range(5):
            lat.step(f, th, 4, thi=thi)
            e.append(lat.energy(f)[0])
        if sgn < 0:
            assert all(b < a for a, b in zip(e, e[1:]))
        else:
            assert all(b > a for a, b in zip(e, e[1:]))
        rates[sgn] = e[-1] / e[0]
    assert rates[-1.0] < 1.0 < rates[1.0]


@pytest.mark.parametrize("case", ["klein_normal", "klein_oblique"])
def test_sect5_klein_cases(case):
    """Both printed cases put the step at twice the packet energy (m = 0), so the
    hole state behind it has |q| = V - E = E: the continuum refraction angle is
    minus the incidence angle (negative refraction), transmission through a
    sharp step is cos^2 of it (complete at normal incidence), and the Klein
    workload generator uses the same ratio."""
    E, V, phi_deg = G[case]
    assert V == pytest.approx(2.0 * E)
    phi = math.radians(phi_deg)
    ky = E * math.sin(phi)
    q = V - E
    theta_t = -math.degrees(math.asin(ky / q))
    assert theta_t == pytest.approx(-phi_deg, abs=1e-9)
    T, R = dirac2d_transmission(E, ky, lambda x: 0.0 if x < 0 else V, -1.0, 1.0, slices=2)
    assert T == pytest.approx(math.cos(phi) ** 2, abs=1e-12) and T + R == pytest.approx(1.0, abs=1e-12)
    cfg = workloads.config_klein2d(phi_deg, nx=64, ny=32)
    assert cfg["V0"] == pytest.approx(2.0 * cfg["E0"]) and cfg["m"] == 0.0
