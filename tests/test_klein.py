"""Klein-step scattering (Sect. 5) against the continuum Dirac equation.

The paper shows this workload as images only, so these are physics checks of
the scheme, not parity: a massless packet at a smoothed potential step of
height twice its energy is transmitted (Klein tunnelling) and refracted to
the negative angle.  The continuum reference (closed_form.dirac2d_transmission)
is itself pinned here: a sharp step with E = V0/2 transmits cos^2(phi), flux is
conserved, and normal incidence is reflectionless for any profile.
Tolerances (0.02 in transmitted probability, 2.5 degrees in direction) cover
the lattice's dispersion error at k = 0.2 per cell, measured against the
continuum at 0, 37 and 53 degrees.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads
from closed_form import dirac2d_transmission, klein_packet_expectation

@pytest.mark.parametrize("phi_deg", [0.0, 20.0, 37.0, 53.0, 70.0])
def test_continuum_sharp_symmetric_step(phi_deg):
    """Matching (u, v) across a sharp step with E = V0/2, m = 0: the hole state
    behind it has |q| = |k| and q_x = -k_x, giving t = cos(phi) exp(i phi) and
    T = cos^2(phi)."""
    E, V0 = 0.2, 0.4
    phi = math.radians(phi_deg)
    T, R = dirac2d_transmission(E, E * math.sin(phi), lambda x: 0.0 if x < 0 else V0, -1.0, 1.0, slices=2)
    assert abs(T - math.cos(phi) ** 2) < 1e-12
    assert abs(T + R - 1.0) < 1e-12


@pytest.mark.parametrize("m", [0.0, 0.05])
def test_continuum_flux_conservation_and_normal_incidence(m):
    prof = lambda x: 0.4 * (1.0 + math.tanh(x / 3.0)) / 2.0
    for phi_deg in (0.0, 15.0, 40.0):
        phi = math.radians(phi_deg)
        E = 0.2
        k = math.sqrt(E * E - m * m)
        T, R = dirac2d_transmission(E, k * math.sin(phi), prof, -40.0, 40.0, m=m)
        assert abs(T + R - 1.0) < 1e-9
        if phi_deg == 0.0 and m == 0.0:
            assert abs(T - 1.0) < 1e-12          # Klein tunnelling: no backscattering
        if m > 0.0:
            assert T < 1.0


def _transmitted(f, xc, margin):
    """(probability at x >= xc, centroid (x, y) of the density at x > xc + margin)."""
    pt = pm = sx = sy = 0.0
    for a in range(4):
        d = np.abs(f[a]) ** 2
        ny, nx = d.shape
        X = np.arange(nx)[None, :] + workloads.OFF2[a][0]
        Y = np.arange(ny)[:, None] + workloads.OFF2[a][1]
        pt += float(d[:, X[0] >= xc].sum())
        msk = np.broadcast_to(X > xc + margin, d.shape)
        pm += float(d[msk].sum())
        sx += float((d * X)[msk].sum())
        sy += float((d * Y)[msk].sum())
    return pt, sx / pm, sy / pm


def test_oracle_klein_normal_incidence():
    """The oracle at normal incidence transmits what the continuum predicts."""
    cfg = workloads.config_klein2d(0.0, nx=768, ny=256)
    ol = oracle.Lattice2(cfg["nx"], cfg["ny"], cfg["dt"])
    th = [np.ascontiguousarray(0.5 * cfg["dt"] * cfg["v_site"][a]) for a in range(4)]
    f = [np.ascontiguousarray(t.numpy()) for t in cfg["state"]]
    ol.step(f, th, int(round(250 / cfg["dt"])))
    T, _, _ = _transmitted(f, cfg["xc"], 40.0)
    eT, _ = klein_packet_expectation(cfg["E0"], cfg["phi"], cfg["sigma"], cfg["V0"],
                                     lambda x: cfg["v_of_x"](x + cfg["xc"]))
    assert eT > 0.97
    assert abs(T - eT) < 0.02


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("phi_deg", [0.0, 37.0, 53.0])
def test_gpu_klein_step_vs_continuum(phi_deg, dtype):
    """The library on the GPU (complex64 with the absorbing frame; complex128
    without): transmitted probability and refraction angle of the transmitted
    packet against the continuum, 250 and 350 time units after the start."""
    import paper_1309_3452_amd as P
    assert torch.cuda.is_available()
    absorb = dtype == torch.complex64
    print("klein phi=%g %s" % (phi_deg, dtype), flush=True)
    cfg = workloads.config_klein2d(phi_deg, dtype=dtype, device="cuda", absorbing=absorb)
    lat = P.Lattice2D(cfg["nx"], cfg["ny"], dtype=dtype, dt=cfg["dt"])
    lat.load(cfg["state"])
    vs = [torch.from_numpy(v) for v in cfg["v_site"]]
    lat.set_fields(0.0, vs, [torch.from_numpy(w) for w in cfg["w_site"]] if absorb else None)
    out = []
    for tt in (250.0, 100.0):
        lat.step(int(round(tt / cfg["dt"])))
        f = [t.cpu().numpy().astype(np.complex128) for t in lat.state()]
        out.append(_transmitted(f, cfg["xc"], 40.0))
        obs = lat.observables(cfg["xc"])
        assert abs(obs[0] - out[-1][0]) < 1e-6       # the library's own x >= xc probability
    eT, eang = klein_packet_expectation(cfg["E0"], cfg["phi"], cfg["sigma"], cfg["V0"],
                                        lambda x: cfg["v_of_x"](x + cfg["xc"]))
    ang = math.degrees(math.atan2(out[1][2] - out[0][2], out[1][1] - out[0][1]))
    assert abs(out[0][0] - eT) < 0.02 and abs(out[1][0] - eT) < 0.02, (out, eT)
    assert abs(ang - eang) < 2.5, (ang, eang)
    if phi_deg > 0:
        assert ang < 0          # negative refraction
