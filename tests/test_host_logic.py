"""Host-side subsystems on the CPU: the E_r watchdog's control flow (against a
stand-in lattice whose E_r follows a prescribed sequence) and the checkpoint
file round trip (real Lattice objects on host memory: creating, binding and
configuring a context makes no HIP call, and nothing here steps)."""
import math

import numpy as np
import pytest
import torch

import paper_1309_3452_amd as P
from paper_1309_3452_amd import DriftError, load_checkpoint, run_watched, save_checkpoint


class StandIn:
    """E_r(t) = e(t) after t steps; the state is one tensor holding t."""
    zh = 0

    def __init__(self, e):
        self.e, self.t, self.reversed = e, 0, []
        self.buf = [torch.zeros(1, dtype=torch.float64)]

    def norm(self):
        return (self.e(self.t), 0.0, 0.0)

    def state(self):
        return self.buf

    def load(self, arrays):
        self.buf[0].copy_(arrays[0])
        self.t = int(self.buf[0].item())

    def step_norm(self, k):
        self.t += k
        self.buf[0].fill_(self.t)
        return torch.tensor([self.e(self.t), 1.0], dtype=torch.float64)

    def reverse(self, k):
        self.t -= k
        self.buf[0].fill_(self.t)
        self.reversed.append(k)


def test_watch_passes_and_reports_largest_change():
    lat = StandIn(lambda t: 1.0 + 1e-9 * t)
    e0, e1, worst = run_watched(lat, 35, every=10, tol=1e-6)
    assert lat.t == 35 and e0 == 1.0 and e1 == pytest.approx(1.0 + 35e-9)
    assert worst == pytest.approx(35e-9)


@pytest.mark.parametrize("recover,restored", [("snapshot", 20), ("reverse", 20), (None, 30)])
def test_watch_stops_at_first_failed_check(recover, restored):
    lat = StandIn(lambda t: 1.0 + (1e-3 if t >= 23 else 0.0))
    with pytest.raises(DriftError) as ei:
        run_watched(lat, 100, every=10, tol=1e-5, recover=recover)
    err = ei.value
    assert err.step == 30 and err.drift == pytest.approx(1e-3)
    assert lat.t == restored
    assert err.restored_step == (None if recover is None else 20)
    assert lat.reversed == ([10] if recover == "reverse" else [])


def test_watch_catches_non_finite_values():
    lat = StandIn(lambda t: math.nan if t >= 15 else 2.0)
    with pytest.raises(DriftError) as ei:
        run_watched(lat, 50, every=10, tol=1e-5)
    assert ei.value.step == 20 and lat.t == 10


def test_watch_rejects_slabs_and_bad_arguments():
    lat = StandIn(lambda t: 1.0)
    lat.zh = 2
    with pytest.raises(ValueError):
        run_watched(lat, 10)
    lat.zh = 0
    with pytest.raises(ValueError):
        run_watched(lat, 10, every=0)
    with pytest.raises(ValueError):
        run_watched(lat, 10, recover="retry")


def _rand(shape, dtype, g):
    a = g.standard_normal(shape) + 1j * g.standard_normal(shape)
    return torch.from_numpy(a).to(dtype)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_checkpoint_round_trip_3d(tmp_path, dtype):
    P.lib()
    g = np.random.default_rng(71)
    nx, ny, nz = 6, 4, 5
    lat = P.Lattice((nx, ny, nz), dtype=dtype, dt=0.4, d=(1.0, 1.25, 1.5), device="cpu")
    vi, vh = g.standard_normal(nz), g.standard_normal(nz)
    lat.set_potential_z(0.7, vi, vh)
    wi, wh = -np.abs(g.standard_normal(nz)), -np.abs(g.standard_normal(nz))
    lat.set_absorber_z(wi, wh)
    st = [_rand((nz, ny, nx), dtype, g) for _ in range(8)]
    lat.load(st)
    links = [torch.exp(1j * torch.from_numpy(g.uniform(-3, 3, (nz, ny, nx)))).to(dtype) for _ in range(24)]
    lat.set_links(links)
    path = str(tmp_path / "c.safetensors")
    save_checkpoint(lat, path, step=17, extra={"note": "x"})
    lat2, step, extra = load_checkpoint(path, device="cpu")
    assert step == 17 and extra == {"note": "x"}
    assert (lat2.ndim, lat2.nx, lat2.ny, lat2.nz, lat2.dtype, lat2.dt, lat2.d, lat2.zh) == \
        (3, nx, ny, nz, dtype, 0.4, (1.0, 1.25, 1.5), 0)
    for a, b in zip(lat2.state(), st):
        assert torch.equal(a, b)
    assert lat2._coef["mode"] == "vz" and lat2._coef["m"] == 0.7
    assert np.array_equal(lat2._coef["vz"][0], vi) and np.array_equal(lat2._coef["vz"][1], vh)
    assert np.array_equal(lat2._wz[0], wi) and np.array_equal(lat2._wz[1], wh)
    for a, b in zip(lat2._links, links):
        assert torch.equal(a, b)
    # per-site coefficient records instead of tables (2D and 3D alike)
    recs = [(_rand((nz, ny, nx), torch.complex64, g) if dtype == torch.complex64
             else torch.from_numpy(g.standard_normal((nz, ny, nx)))) for _ in range(8)]
    lat.set_coef_records(recs)
    lat.set_links(None)
    lat.set_absorber_z(None)
    save_checkpoint(lat, path)
    lat3, step, _ = load_checkpoint(path, device="cpu")
    assert step is None and lat3._coef["mode"] == "site" and lat3._links is None and lat3._wz is None
    for a, b in zip(lat3.theta, recs):
        assert torch.equal(a, b)


def test_checkpoint_round_trip_2d_slab_and_errors(tmp_path):
    P.lib()
    g = np.random.default_rng(72)
    lat = P.Lattice((8, 6), dtype=torch.complex64, dt=0.6, device="cpu")
    lat.set_potential_z(0.3)
    st = [_rand((6, 8), torch.complex64, g) for _ in range(4)]
    lat.load(st)
    path = str(tmp_path / "c2.safetensors")
    save_checkpoint(lat, path, step=3)
    lat2, step, _ = load_checkpoint(path, device="cpu")
    assert step == 3 and lat2.ndim == 2 and lat2._coef == {"mode": "vz", "m": 0.3, "vz": None}
    for a, b in zip(lat2.state(), st):
        assert torch.equal(a, b)
    # a z-slab keeps its halo planes and V(z) entries per stored plane
    sl = P.Lattice((4, 4, 3), dtype=torch.complex128, dt=0.5, device="cpu", slab=True)
    v = g.standard_normal(7)
    sl.set_potential_z(0.2, v, v)
    sl.load([_rand((7, 4, 4), torch.complex128, g) for _ in range(8)])
    save_checkpoint(sl, path)
    sl2, _, _ = load_checkpoint(path, device="cpu")
    assert sl2.zh == 2 and sl2.tshape == (7, 4, 4)
    for a, b in zip(sl2.state(), sl.state()):
        assert torch.equal(a, b)
    from safetensors.torch import save_file
    save_file({"x": torch.zeros(1)}, path)
    with pytest.raises(ValueError, match="not a lattice checkpoint"):
        load_checkpoint(path, device="cpu")


def test_fp32_record_on_the_host():
    """The complex64 coefficient record gamma = 1 - alpha = 2 i theta/(1 + i theta)
    of the time-averaged term (Eqs. ss1-ss4), as the host computes it for the
    V(z) tables (the device records use the same source; their bits are
    compared on the GPU): within 1e-6 of the exact value on both sides of
    |theta| = 1, |1 - gamma| = 1 to a few 1e-8, conjugate under theta -> -theta."""
    import ctypes

    import numpy as np

    from paper_1309_3452_amd import _abi
    L = _abi.lib()
    g = np.random.default_rng(11)
    th = np.ascontiguousarray(np.concatenate([g.uniform(-3.0, 3.0, 20000), [0.0, 1e-8, -1e-8, 1.0, -1.0, 0.3]]))
    out = np.empty(2 * th.size, np.float32)
    outn = np.empty_like(out)
    assert L.dirac_coef_from_theta_host(out.ctypes.data_as(ctypes.c_void_p), th.ctypes.data_as(ctypes.c_void_p),
                                        th.size) == 0
    thn = np.ascontiguousarray(-th)
    assert L.dirac_coef_from_theta_host(outn.ctypes.data_as(ctypes.c_void_p), thn.ctypes.data_as(ctypes.c_void_p),
                                        th.size) == 0
    gam = out[0::2].astype(np.float64) + 1j * out[1::2].astype(np.float64)
    exact = 2j * th / (1.0 + 1j * th)
    assert np.max(np.abs(gam - exact) / np.maximum(1.0, np.abs(exact))) <= 1.01e-6
    unit = np.abs((1.0 - gam.real) ** 2 + gam.imag ** 2 - 1.0)
    assert unit.max() <= 8e-8 and np.median(unit) <= 3e-9
    assert np.array_equal(outn[0::2], out[0::2]) and np.array_equal(outn[1::2], -out[1::2])
    assert L.dirac_coef_from_theta_host(None, th.ctypes.data_as(ctypes.c_void_p), 1) == -1
    bad = np.array([np.nan])
    assert L.dirac_coef_from_theta_host(out.ctypes.data_as(ctypes.c_void_p), bad.ctypes.data_as(ctypes.c_void_p),
                                        1) == -4
