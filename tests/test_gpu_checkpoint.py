"""Checkpoint/resume and the E_r watchdog on real lattices.

A lattice saved after some steps and rebuilt from the file steps to the bits of
the uninterrupted run, for V(z) tables with absorbing layers (two-step kernel),
per-site fields, gauge links, and (2+1)D.  The watchdog passes a conserving
run and stops a run whose E_r decays (an absorbing potential stands in for a
failure), restoring the last passed check bitwise (snapshot) or to rounding
(reverse step)."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1309_3452_amd as P
    assert torch.cuda.is_available(), "needs a GPU"
    P.lib()
    return P


def rand_state(shape, count, seed, dtype):
    g = np.random.default_rng(seed)
    return [torch.from_numpy(g.standard_normal(shape) + 1j * g.standard_normal(shape)).to(dtype)
            for _ in range(count)]


def build(P, case):
    g = np.random.default_rng(401)
    if case == "vz_absorber_c64":
        nx, ny, nz = 48, 16, 20
        lat = P.Lattice3D(nx, ny, nz, dtype=torch.complex64, dt=workloads.DT3)
        vi, vh = workloads.step_potential(nz, 1.5, nz / 2.0, 2.0)
        lat.set_potential_z(0.5, vi, vh)
        wi, wh = workloads.absorber(nz, 4, 0.05)
        lat.set_absorber_z(wi, wh)
        lat.load(rand_state((nz, ny, nx), 8, 402, torch.complex64))
    elif case == "site_c128":
        nx, ny, nz = 20, 12, 10
        lat = P.Lattice3D(nx, ny, nz, dtype=torch.complex128, dt=workloads.DT3)
        lat.set_fields(0.3, [torch.from_numpy(0.4 * g.standard_normal((nz, ny, nx))) for _ in range(8)])
        lat.load(rand_state((nz, ny, nx), 8, 403, torch.complex128))
    elif case == "links_c64":
        nx, ny, nz = 32, 16, 12
        lat = P.Lattice3D(nx, ny, nz, dtype=torch.complex64, dt=workloads.DT3)
        lat.set_potential_z(0.5)
        lat.set_links(workloads.peierls_links3d(nx, ny, nz, 0.3, 404, dtype=torch.complex64, device="cuda"))
        lat.load(rand_state((nz, ny, nx), 8, 405, torch.complex64))
    elif case == "site2d_c64_w":
        nx, ny = 64, 40
        lat = P.Lattice2D(nx, ny, dtype=torch.complex64, dt=workloads.DT2)
        v = [torch.from_numpy(0.3 * g.standard_normal((ny, nx))) for _ in range(4)]
        w = [torch.from_numpy(-0.02 * np.abs(g.standard_normal((ny, nx)))) for _ in range(4)]
        lat.set_fields(0.4, v, w)
        lat.load(rand_state((ny, nx), 4, 406, torch.complex64))
    else:
        lat = P.Lattice2D(48, 48, dtype=torch.complex128, dt=workloads.DT2)
        lat.set_potential_z(0.6)
        lat.load(rand_state((48, 48), 4, 407, torch.complex128))
    return lat


@pytest.mark.parametrize("case", ["vz_absorber_c64", "site_c128", "links_c64", "site2d_c64_w", "plain2d_c128"])
def test_resume_is_bitwise(P, tmp_path, case):
    print("resume %s" % case, flush=True)
    lat = build(P, case)
    lat.step(5)
    path = str(tmp_path / ("%s.safetensors" % case))
    P.save_checkpoint(lat, path, step=5)
    lat2, step, _ = P.load_checkpoint(path)
    assert step == 5
    lat.step(7)
    lat2.step(7)
    for a, b in zip(lat.state(), lat2.state()):
        assert torch.equal(a, b)


def test_watchdog_passes_a_conserving_run(P):
    print("watchdog conserving", flush=True)
    lat = build(P, "plain2d_c128")
    e0, e1, worst = P.run_watched(lat, 40, every=10, tol=1e-12)
    assert worst <= 1e-12 and abs(e1 - e0) <= 1e-12 * abs(e0)


@pytest.mark.parametrize("recover", ["snapshot", "reverse"])
def test_watchdog_stops_and_restores(P, recover):
    """E_r decays under an absorbing potential: the first check (10 steps) fails
    and the state of step 0 comes back."""
    print("watchdog %s" % recover, flush=True)
    nx, ny, nz = 32, 16, 16
    lat = P.Lattice3D(nx, ny, nz, dtype=torch.complex128, dt=workloads.DT3)
    lat.set_potential_z(0.5)
    wi, wh = workloads.absorber(nz, 4, 0.02)
    lat.set_absorber_z(wi, wh)
    f0 = rand_state((nz, ny, nx), 8, 408, torch.complex128)
    lat.load(f0)
    with pytest.raises(P.DriftError) as ei:
        P.run_watched(lat, 40, every=10, tol=1e-9, recover=recover)
    assert ei.value.step == 10 and ei.value.restored_step == 0
    for a, b in zip(lat.state(), f0):
        b = b.to(a.device)
        if recover == "snapshot":
            assert torch.equal(a, b)
        else:
            assert float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)) <= 1e-12
