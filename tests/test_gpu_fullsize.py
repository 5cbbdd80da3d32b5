"""GPU checks at the benchmark sizes, in the launch configuration bench.py times.

At these sizes the oracle cannot run whole: parity is checked on sampled
cells (the oracle advances a periodic sub-box around each sample whose
light cone covers the steps taken), and otherwise through properties that
hold at any size (closed-form plane waves, the conserved functional, time
reversal, finite differences, bitwise agreement between kernels).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads
from closed_form import eigenket3, plane_wave3, rel_l2

pytestmark = pytest.mark.gpu

DT3 = workloads.DT3


@pytest.fixture(scope="module")
def P():
    import paper_1309_3452_amd as P
    assert torch.cuda.is_available(), "needs a GPU"
    P.lib()
    return P


def free():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def plane_wave_gpu(n, k, amps, w, dt, dtype, t_shift=0.0):
    """Eq. (planeonlattice) on the device, built per axis (exact phases in FP64)."""
    out = []
    for a in range(8):
        ox, oy, oz = workloads.OFF3[a]
        t = (-0.5 * dt if a < 4 else 0.0) + t_shift
        ax = [torch.exp(1j * k[q] * (torch.arange(n, dtype=torch.float64, device="cuda") + o))
              for q, o in ((0, ox), (1, oy), (2, oz))]
        ph = complex(math.cos(w * t), -math.sin(w * t)) * amps[a // 2]
        out.append((ax[2][:, None, None] * ax[1][None, :, None] * (ax[0][None, None, :] * ph)).to(dtype))
    return out


def rel_l2_t(a_list, b_list):
    num = sum(float(torch.sum(torch.abs(a.to(torch.complex128) - b.to(torch.complex128)) ** 2))
              for a, b in zip(a_list, b_list))
    den = sum(float(torch.sum(torch.abs(b.to(torch.complex128)) ** 2)) for b in b_list)
    return math.sqrt(num / den)


def test_plane_wave_256_fp64(P):
    """Closed-form eigen-evolution (Eqs. planeonlattice, pwdsip) at 256^3 in FP64."""
    n, steps, m = 256, 200, 0.5
    k = (2 * math.pi * 3 / n, 2 * math.pi * 5 / n, 2 * math.pi * 46 / n)
    w, amps = eigenket3(k, m, DT3, 1)
    print("plane wave 256^3 fp64", flush=True)
    lat = P.Lattice3D(n, n, n, dtype=torch.complex128, dt=DT3)
    lat.set_potential_z(m)
    lat.load(plane_wave_gpu(n, k, amps, w, DT3, torch.complex128))
    e0 = lat.norm()
    lat.step(steps)
    expect = plane_wave_gpu(n, k, amps, w, DT3, torch.complex128, t_shift=steps * DT3)
    assert rel_l2_t(lat.state(), expect) <= steps * 1e-15
    assert abs(lat.norm()[0] - e0[0]) <= 1e-13 * e0[0]
    del lat, expect
    free()


def test_plane_wave_512_fp32_phase_error(P):
    """FP32 form: dispersion-phase error of a plane wave (k_z = 2 pi 46/512, m = 0.5,
    V = 0) after 1000 steps against Eq. (pwdsip), and the drift of E_r."""
    n, steps, m = 512, 1000, 0.5
    k = (0.0, 0.0, 2 * math.pi * 46 / n)
    w, amps = eigenket3(k, m, DT3, 1)
    print("plane wave 512^3 fp32", flush=True)
    lat = P.Lattice3D(n, n, n, dtype=torch.complex64, dt=DT3)
    lat.set_potential_z(m)
    lat.load(plane_wave_gpu(n, k, amps, w, DT3, torch.complex64))
    e0 = lat.norm()
    lat.step(steps)
    e1 = lat.norm()
    expect = plane_wave_gpu(n, k, amps, w, DT3, torch.complex128, t_shift=steps * DT3)
    inner = sum(complex(torch.sum(torch.conj(b) * a.to(torch.complex128))) for a, b in zip(lat.state(), expect))
    nrm = sum(float(torch.sum(torch.abs(b) ** 2)) for b in expect)
    phase_err = abs(math.atan2(inner.imag, inner.real))
    amp_err = abs(abs(inner) / nrm - 1.0)
    drift = abs(e1[0] - e0[0]) / abs(e0[0])
    print("fp32 plane wave: phase error %.3e rad, amplitude error %.3e, E_r drift %.3e" % (phase_err, amp_err, drift))
    assert drift <= 1e-5
    assert phase_err <= 1e-3
    del lat, expect
    free()


def test_packet_512_fp32_vs_fp64(P):
    """FP32 form against the FP64 path on the 512^3 Klein-step workload, 1000 steps:
    relative L2, global phase arg<psi64, psi32>, and E_r drift of each."""
    n, steps = 512, 1000
    print("packet 512^3 fp32 vs fp64", flush=True)
    res = {}
    for dtype in (torch.complex64, torch.complex128):
        cfg = workloads.config_step3d(n, dtype=dtype, device="cuda")
        lat = P.Lattice3D(n, n, n, dtype=dtype, dt=cfg["dt"])
        lat.set_potential_z(cfg["m"], cfg["v_int"], cfg["v_half"])
        lat.load(cfg["state"])
        del cfg
        e0 = lat.norm()
        lat.step(steps)
        e1 = lat.norm()
        res[dtype] = (lat, abs(e1[0] - e0[0]) / abs(e0[0]))
        if dtype == torch.complex64:
            s32 = [t.clone() for t in lat.state()]
            del lat
            res[dtype] = (None, res[dtype][1])
            free()
    lat64, d64 = res[torch.complex128]
    d32 = res[torch.complex64][1]
    s64 = lat64.state()
    l2 = rel_l2_t(s32, s64)
    inner = sum(complex(torch.sum(torch.conj(b) * a.to(torch.complex128))) for a, b in zip(s32, s64))
    print("fp32 vs fp64 at 512^3 after %d steps: rel L2 %.3e, phase %.3e rad; E_r drift fp32 %.3e fp64 %.3e"
          % (steps, l2, math.atan2(inner.imag, inner.real), d32, d64))
    assert d32 <= 1e-5
    assert d64 <= 1e-12
    assert l2 <= 1e-2
    del lat64, s32, s64
    free()


def test_full_oracle_parity_256_fp64(P):
    """The 256^3 complex128 Klein-step workload, 20 steps through the default
    (two steps per launch) kernel, against the oracle on every cell."""
    n, steps = 256, 20
    cfg = workloads.config_step3d(n, dtype=torch.complex128, device="cpu")
    print("full parity 256^3, %d steps" % steps, flush=True)
    lat = P.Lattice3D(n, n, n, dtype=torch.complex128, dt=cfg["dt"])
    lat.set_potential_z(cfg["m"], cfg["v_int"], cfg["v_half"])
    lat.load(cfg["state"])
    lat.step(steps)
    got = [t.cpu().numpy() for t in lat.state()]
    del lat
    free()
    ol = oracle.Lattice3(n, n, n, cfg["dt"])
    f = [np.ascontiguousarray(t.numpy()) for t in cfg["state"]]
    ol.step(f, ol.theta_vz(cfg["m"], cfg["v_int"], cfg["v_half"]), steps)
    assert rel_l2(got, f) <= 1e-13


def test_full_oracle_parity_128_fp64_1000_steps(P):
    """Long-run parity: the Klein-step workload at 128^3 (complex128, default
    two-step launches with the in-step functional every tenth step, as the
    benchmark runs it) for 1000 steps against the oracle on every cell, with E_r
    of both against its start."""
    n, steps = 128, 1000
    cfg = workloads.config_step3d(n, dtype=torch.complex128, device="cpu")
    print("full parity 128^3, %d steps" % steps, flush=True)
    lat = P.Lattice3D(n, n, n, dtype=torch.complex128, dt=cfg["dt"])
    lat.set_potential_z(cfg["m"], cfg["v_int"], cfg["v_half"])
    lat.load(cfg["state"])
    e0 = lat.norm()
    for _ in range(steps // 10):
        e = lat.step_norm(10)
    e = e.cpu().numpy()
    got = [t.cpu().numpy() for t in lat.state()]
    del lat
    free()
    ol = oracle.Lattice3(n, n, n, cfg["dt"])
    f = [np.ascontiguousarray(t.numpy()) for t in cfg["state"]]
    ol.step(f, ol.theta_vz(cfg["m"], cfg["v_int"], cfg["v_half"]), steps)
    assert rel_l2(got, f) <= 1e-13
    eo = ol.energy(f)
    assert abs(e[0] - eo[0]) <= 1e-13 * eo[2] and abs(e[0] - e0[0]) <= 1e-13 * abs(e0[0])


@pytest.mark.timeout(1200)
def test_full_oracle_parity_256_fp64_1000_steps(P, capfd):
    """The 256^3 complex128 Klein-step workload exactly as stated: 1000 steps in the
    benchmark's launch sequence (two-step launches, the in-step functional every
    tenth step) against the oracle on every cell, with E_r of both.  The oracle
    takes several minutes on the host cores; it prints its progress."""
    n, steps, chunk = 256, 1000, 100
    cfg = workloads.config_step3d(n, dtype=torch.complex128, device="cpu")
    print("full parity 256^3, %d steps" % steps, flush=True)
    lat = P.Lattice3D(n, n, n, dtype=torch.complex128, dt=cfg["dt"])
    lat.set_potential_z(cfg["m"], cfg["v_int"], cfg["v_half"])
    lat.load(cfg["state"])
    e0 = lat.norm()
    for _ in range(steps // 10):
        e = lat.step_norm(10)
    e = e.cpu().numpy()
    got = [t.cpu().numpy() for t in lat.state()]
    del lat
    free()
    ol = oracle.Lattice3(n, n, n, cfg["dt"])
    f = [np.ascontiguousarray(t.numpy()) for t in cfg["state"]]
    del cfg["state"]
    th = ol.theta_vz(cfg["m"], cfg["v_int"], cfg["v_half"])
    import time
    t0 = time.perf_counter()
    for done in range(chunk, steps + 1, chunk):
        ol.step(f, th, chunk)
        with capfd.disabled():
            print("  oracle 256^3: %d/%d steps, %.0f s" % (done, steps, time.perf_counter() - t0), flush=True)
    rel = rel_l2(got, f)
    eo = ol.energy(f)
    print("256^3 x %d: rel L2 %.3e; E_r gpu %.15e oracle %.15e start %.15e" % (steps, rel, e[0], eo[0], e0[0]))
    assert rel <= 1e-13
    assert abs(e[0] - eo[0]) <= 1e-13 * eo[2] and abs(e[0] - e0[0]) <= 1e-13 * abs(e0[0])


def test_sampled_oracle_parity_256_fp64(P):
    """Klein-step workload at 256^3 (fused kernel, bench launch configuration): after
    3 steps, sampled cells against the oracle run on a periodic sub-box of half-width
    2*3+1 around each sample (the light cone grows two cells per step)."""
    n, steps, R = 256, 3, 7
    cfg = workloads.config_step3d(n, dtype=torch.complex128, device="cuda")
    print("sampled parity 256^3", flush=True)
    lat = P.Lattice3D(n, n, n, dtype=torch.complex128, dt=cfg["dt"])
    lat.set_potential_z(cfg["m"], cfg["v_int"], cfg["v_half"])
    lat.load(cfg["state"])
    f0 = [t.cpu().numpy() for t in cfg["state"]]
    del cfg["state"]
    lat.step(steps)
    got = [t.cpu().numpy() for t in lat.state()]
    del lat
    free()
    g = np.random.default_rng(17)
    samples = [tuple(int(v) for v in g.integers(0, n, 3)) for _ in range(24)]
    samples += [(n // 2, n // 2, n // 4), (0, 0, 0), (n - 1, n - 1, n - 1), (n // 2, 0, n // 2)]
    B = 2 * R + 1
    ol = oracle.Lattice3(B, B, B, cfg["dt"])
    scale = max(float(np.abs(a).max()) for a in got)
    vz = lambda z: 1.5 * (1.0 + np.tanh((z - n / 2.0) / 4.0)) / 2.0
    for (i, j, k) in samples:
        ix = (np.arange(i - R, i + R + 1)) % n
        iy = (np.arange(j - R, j + R + 1)) % n
        iz = (np.arange(k - R, k + R + 1)) % n
        box = [np.ascontiguousarray(a[np.ix_(iz, iy, ix)]) for a in f0]
        th = []
        for a in range(8):
            oz = workloads.OFF3[a][2]
            z = (iz + oz)[:, None, None] * np.ones((1, B, B))
            sgn = 1.0 if a < 4 else -1.0
            th.append(np.ascontiguousarray(0.5 * cfg["dt"] * (sgn * cfg["m"] + vz(z))))
        ol.step(box, th, steps)
        for a in range(8):
            assert abs(box[a][R, R, R] - got[a][k, j, i]) <= 1e-13 * scale, (i, j, k, a)


def test_sampled_oracle_parity_512_fp32_headline(P):
    """The benchmark's own workload and launch sequence: 512^3 complex64, the
    Klein-step V(z) and packet, two-step launches (the second one also summing
    E_r, as the timed loop does every tenth step).  After 4 steps, cells sampled
    around the packet (where the amplitudes are not negligible), on the step and
    at random are compared with the FP64 oracle run from the same FP32 initial
    state on a periodic sub-box of half-width 2*4+1 around each; FP32 rounding
    allows about 1e-6 of the largest amplitude per step."""
    n, steps, R = 512, 4, 9
    cfg = workloads.config_step3d(n, dtype=torch.complex64, device="cuda")
    print("sampled parity 512^3 fp32 headline", flush=True)
    lat = P.Lattice3D(n, n, n, dtype=torch.complex64, dt=cfg["dt"])
    lat.set_potential_z(cfg["m"], cfg["v_int"], cfg["v_half"])
    lat.load(cfg["state"])
    del cfg["state"]
    assert lat.halo_steps == 0
    g = np.random.default_rng(29)
    c = (n // 2, n // 2, n // 4)
    samples = [tuple(int(round(c[q] + 12.0 * g.standard_normal())) % n for q in range(3)) for _ in range(20)]
    samples += [tuple(int(v) for v in g.integers(0, n, 3)) for _ in range(4)]
    samples += [(c[0], c[1], c[2]), (c[0], c[1], n // 2), (0, 0, 0), (n - 1, n - 1, n - 1)]
    B = 2 * R + 1

    def boxes(arrays):
        out = []
        for (i, j, k) in samples:
            ix = torch.arange(i - R, i + R + 1, device="cuda") % n
            iy = torch.arange(j - R, j + R + 1, device="cuda") % n
            iz = torch.arange(k - R, k + R + 1, device="cuda") % n
            out.append([a.index_select(0, iz).index_select(1, iy).index_select(2, ix).cpu().numpy().astype(np.complex128)
                        for a in arrays])
        return out

    before = boxes(lat.state())
    lat.step_norm(2)
    e = lat.step_norm(2).cpu().numpy()
    torch.cuda.synchronize()
    after = [[b[a][R, R, R] for a in range(8)] for b in boxes(lat.state())]
    ref = lat.norm()
    assert abs(e[0] - ref[0]) <= 2e-9 * ref[2]
    del lat
    free()
    ol = oracle.Lattice3(B, B, B, cfg["dt"])
    scale = max(max(abs(v) for v in row) for row in after)
    m, v_int, v_half = cfg["m"], cfg["v_int"], cfg["v_half"]
    big = 0
    for (i, j, k), box, got in zip(samples, before, after):
        iz = (np.arange(k - R, k + R + 1)) % n
        th = []
        for a in range(8):
            tab = v_int if workloads.OFF3[a][2] == 0.0 else v_half
            sgn = 1.0 if a < 4 else -1.0
            th.append(np.ascontiguousarray(0.5 * cfg["dt"] * (sgn * m + tab[iz])[:, None, None] * np.ones((1, B, B))))
        ol.step(box, th, steps)
        for a in range(8):
            assert abs(box[a][R, R, R] - got[a]) <= steps * 1e-6 * scale, (i, j, k, a)
            big += abs(got[a]) > 1e-2 * scale
    assert big >= 40       # the packet samples carry the comparison


def test_sampled_oracle_reverse_512_fp32(P):
    """The reversed step at the benchmark's size (512^3 complex64, Klein-step
    V(z)) on the march kernels: 5 reversed steps from the packet, sampled cells
    against the FP64 oracle's reversed steps from the same FP32 state on a
    periodic sub-box of half-width 2*5+1 around each; and 5 forward steps bring
    the state back."""
    n, steps, R = 512, 5, 11
    cfg = workloads.config_step3d(n, dtype=torch.complex64, device="cuda")
    print("sampled reverse 512^3 fp32", flush=True)
    lat = P.Lattice3D(n, n, n, dtype=torch.complex64, dt=cfg["dt"])
    lat.set_potential_z(cfg["m"], cfg["v_int"], cfg["v_half"])
    lat.load(cfg["state"])
    start = [t.clone() for t in cfg["state"]]
    del cfg["state"]
    g = np.random.default_rng(31)
    c = (n // 2, n // 2, n // 4)
    samples = [tuple(int(round(c[q] + 12.0 * g.standard_normal())) % n for q in range(3)) for _ in range(16)]
    samples += [tuple(int(v) for v in g.integers(0, n, 3)) for _ in range(4)]
    samples += [(c[0], c[1], c[2]), (0, 0, 0), (n - 1, n - 1, n - 1)]
    B = 2 * R + 1

    def boxes(arrays):
        out = []
        for (i, j, k) in samples:
            ix = torch.arange(i - R, i + R + 1, device="cuda") % n
            iy = torch.arange(j - R, j + R + 1, device="cuda") % n
            iz = torch.arange(k - R, k + R + 1, device="cuda") % n
            out.append([a.index_select(0, iz).index_select(1, iy).index_select(2, ix).cpu().numpy().astype(np.complex128)
                        for a in arrays])
        return out

    before = boxes(lat.state())
    lat.reverse(steps)
    after = [[b[a][R, R, R] for a in range(8)] for b in boxes(lat.state())]
    lat.step(steps)
    back = rel_l2_t(lat.state(), start)
    del lat, start
    free()
    assert back <= 2 * steps * 2e-6
    ol = oracle.Lattice3(B, B, B, cfg["dt"])
    scale = max(max(abs(v) for v in row) for row in after)
    m, v_int, v_half = cfg["m"], cfg["v_int"], cfg["v_half"]
    big = 0
    for (i, j, k), box, got in zip(samples, before, after):
        iz = (np.arange(k - R, k + R + 1)) % n
        th = []
        for a in range(8):
            tab = v_int if workloads.OFF3[a][2] == 0.0 else v_half
            sgn = 1.0 if a < 4 else -1.0
            th.append(np.ascontiguousarray(0.5 * cfg["dt"] * (sgn * m + tab[iz])[:, None, None] * np.ones((1, B, B))))
        ol.reverse(box, th, steps)
        for a in range(8):
            assert abs(box[a][R, R, R] - got[a]) <= steps * 1e-6 * scale, (i, j, k, a)
            big += abs(got[a]) > 1e-2 * scale
    assert big >= 30


def test_sampled_oracle_parity_512_fp32_site(P):
    """Per-site coefficient records at the benchmark size (512^3 complex64, the
    headline packet, V = the z-step plus 0.05 N(0, 1) per site, as `bench.py
    --workload site3d`), default two-step launches: after 4 steps, cells around
    the packet and at random against the FP64 oracle stepping sub-boxes with
    theta = (dt/2)(+-m + V) of the same (FP32) site values."""
    n, steps, R = 512, 4, 9
    cfg = workloads.config_step3d(n, dtype=torch.complex64, device="cuda")
    print("sampled parity 512^3 fp32 per-site", flush=True)
    lat = P.Lattice3D(n, n, n, dtype=torch.complex64, dt=cfg["dt"])
    lat.load(cfg["state"])
    del cfg["state"]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(13093452)
    V = []
    for a in range(8):
        z = torch.arange(n, dtype=torch.float64, device="cuda") + workloads.OFF3[a][2]
        vz = 1.5 * (1.0 + torch.tanh((z - n / 2.0) / 4.0)) / 2.0
        V.append((vz.view(n, 1, 1) + 0.05 * torch.randn((n, n, n), generator=gen, dtype=torch.float64,
                                                         device="cuda")).to(torch.float32).contiguous())
    lat.set_fields(cfg["m"], V)
    g = np.random.default_rng(31)
    c = (n // 2, n // 2, n // 4)
    samples = [tuple(int(round(c[q] + 12.0 * g.standard_normal())) % n for q in range(3)) for _ in range(20)]
    samples += [tuple(int(v) for v in g.integers(0, n, 3)) for _ in range(4)] + [c, (0, 0, 0)]
    B = 2 * R + 1

    def boxes(arrays):
        out = []
        for (i, j, k) in samples:
            ix = torch.arange(i - R, i + R + 1, device="cuda") % n
            iy = torch.arange(j - R, j + R + 1, device="cuda") % n
            iz = torch.arange(k - R, k + R + 1, device="cuda") % n
            out.append([a.index_select(0, iz).index_select(1, iy).index_select(2, ix).cpu().numpy()
                        .astype(np.complex128 if a.is_complex() else np.float64) for a in arrays])
        return out

    before, vbox = boxes(lat.state()), boxes(V)
    del V
    lat.step(steps)
    torch.cuda.synchronize()
    after = [[b[a][R, R, R] for a in range(8)] for b in boxes(lat.state())]
    del lat
    free()
    ol = oracle.Lattice3(B, B, B, cfg["dt"])
    scale = max(max(abs(v) for v in row) for row in after)
    big = 0
    for box, vb, got in zip(before, vbox, after):
        th = [np.ascontiguousarray(0.5 * cfg["dt"] * ((1.0 if a < 4 else -1.0) * cfg["m"] + vb[a])) for a in range(8)]
        ol.step(box, th, steps)
        for a in range(8):
            assert abs(box[a][R, R, R] - got[a]) <= steps * 1e-6 * scale
            big += abs(got[a]) > 1e-2 * scale
    assert big >= 40


@pytest.mark.parametrize("dtype,nz,beyond,tol", [(torch.complex64, 72, 64, 3e-6), (torch.complex128, 40, 32, 1e-13)])
def test_sampled_oracle_parity_arrays_over_4gib(P, dtype, nz, beyond, tol):
    """Arrays larger than 4 GiB (4096 x 2048 x nz cells): 64-bit addressing in the
    two-step and one-step kernels (3 steps, default launch).  The state is drawn on
    the device; sub-boxes around the samples -- including cells past the 4 GiB byte
    offset (planes >= `beyond`) and the last cell -- are cut out on the device and
    stepped by the oracle, as in the 256^3 sampled test."""
    nx, ny, steps, R = 4096, 2048, 3, 7
    print("arrays over 4 GiB: %d x %d x %d %s" % (nx, ny, nz, dtype), flush=True)
    bytes_per_array = nx * ny * nz * (8 if dtype == torch.complex64 else 16)
    assert bytes_per_array > 4 << 30 and nx * ny * beyond * (8 if dtype == torch.complex64 else 16) >= 4 << 30
    m, dt = 0.5, DT3
    v_int, v_half = workloads.step_potential(nz, 1.5, nz / 2.0, 4.0)
    lat = P.Lattice3D(nx, ny, nz, dtype=dtype, dt=dt)
    lat.set_potential_z(m, v_int, v_half)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4242)
    for t in lat.state():
        t.copy_(torch.randn(t.shape, dtype=dtype, device="cuda", generator=gen))
    g = np.random.default_rng(23)
    samples = [(int(g.integers(0, nx)), int(g.integers(0, ny)), int(g.integers(0, nz))) for _ in range(10)]
    samples += [(nx - 1, ny - 1, nz - 1), (0, 0, beyond), (nx // 2, ny - 1, beyond + 1), (17, 5, nz - 1),
                (nx - 3, 1, beyond), (0, 0, 0)]

    def boxes(arrays):
        out = []
        for (i, j, k) in samples:
            ix = torch.arange(i - R, i + R + 1, device="cuda") % nx
            iy = torch.arange(j - R, j + R + 1, device="cuda") % ny
            iz = torch.arange(k - R, k + R + 1, device="cuda") % nz
            out.append([a.index_select(0, iz).index_select(1, iy).index_select(2, ix).cpu().numpy().astype(np.complex128)
                        for a in arrays])
        return out

    before = boxes(lat.state())
    lat.step(steps)
    torch.cuda.synchronize()
    after = [[b[a][R, R, R] for a in range(8)] for b in boxes(lat.state())]
    del lat
    free()
    B = 2 * R + 1
    ol = oracle.Lattice3(B, B, B, dt)
    scale = max(max(abs(v) for v in row) for row in after)
    for (i, j, k), box, got in zip(samples, before, after):
        iz = (np.arange(k - R, k + R + 1)) % nz
        th = []
        for a in range(8):
            # V at the amplitude's own z: integer sites (A, D) take v_int, half-integer (B, C) v_half
            tab = v_int if workloads.OFF3[a][2] == 0.0 else v_half
            sgn = 1.0 if a < 4 else -1.0
            th.append(np.ascontiguousarray(0.5 * dt * (sgn * m + tab[iz])[:, None, None] * np.ones((1, B, B))))
        ol.step(box, th, steps)
        for a in range(8):
            assert abs(box[a][R, R, R] - got[a]) <= tol * scale, (i, j, k, a)


def test_sampled_oracle_parity_links_512_fp32(P):
    """The gauge-link workload bench.py times (512^3, complex64, Peierls links of a
    smooth vector potential): after 3 steps, sampled cells against the FP64 oracle
    with the same (complex64-rounded) links on periodic sub-boxes; E_r with the
    links conserved at full size."""
    n, steps, R = 512, 3, 7
    cfg = workloads.config_step3d(n, dtype=torch.complex64, device="cuda")
    print("sampled links parity 512^3 fp32", flush=True)
    lat = P.Lattice3D(n, n, n, dtype=torch.complex64, dt=cfg["dt"])
    lat.set_potential_z(cfg["m"], cfg["v_int"], cfg["v_half"])
    lat.load(cfg["state"])
    f0 = [t.clone() for t in lat.state()]
    del cfg["state"]
    U = workloads.peierls_links3d(n, n, n, 0.05, 31, dtype=torch.complex64, device="cuda")
    lat.set_links(U)
    e0 = lat.norm()
    lat.step(steps)
    e1 = lat.norm()
    assert abs(e1[0] - e0[0]) <= 1e-6 * steps * abs(e0[0])
    got = lat.state()
    g = np.random.default_rng(19)
    samples = [tuple(int(v) for v in g.integers(0, n, 3)) for _ in range(16)]
    samples += [(n // 2, n // 2, n // 4), (0, 0, 0), (n - 1, n - 1, n - 1), (n // 2, 0, n // 2)]
    B = 2 * R + 1
    ol = oracle.Lattice3(B, B, B, cfg["dt"])
    scale = max(float(t.abs().max()) for t in got)
    vz = lambda z: 1.5 * (1.0 + np.tanh((z - n / 2.0) / 4.0)) / 2.0

    def box_of(t, iz, iy, ix):
        idx = lambda v: torch.from_numpy(v).to("cuda")
        sub = t.index_select(0, idx(iz)).index_select(1, idx(iy)).index_select(2, idx(ix))
        return np.ascontiguousarray(sub.cpu().numpy().astype(np.complex128))

    for (i, j, k) in samples:
        ix = (np.arange(i - R, i + R + 1)) % n
        iy = (np.arange(j - R, j + R + 1)) % n
        iz = (np.arange(k - R, k + R + 1)) % n
        box = [box_of(a, iz, iy, ix) for a in f0]
        ubox = [box_of(u, iz, iy, ix) for u in U]
        th = []
        for a in range(8):
            z = (iz + workloads.OFF3[a][2])[:, None, None] * np.ones((1, B, B))
            sgn = 1.0 if a < 4 else -1.0
            th.append(np.ascontiguousarray(0.5 * cfg["dt"] * (sgn * cfg["m"] + vz(z))))
        ol.step(box, th, steps, links=ubox)
        for a in range(8):
            gv = complex(got[a][k, j, i].item())
            assert abs(box[a][R, R, R] - gv) <= 3e-6 * scale, (i, j, k, a)
    del lat, f0, U
    free()


def test_slabs_at_device_shape_512(P):
    """One device's share of a 512^3 lattice split over 8 devices is a 512 x 512 x 64
    slab: two such slabs (a 512 x 512 x 128 periodic lattice) with halos exchanged
    every step give the bits of the whole lattice, complex64, headline workload."""
    n, nz, steps = 512, 128, 3
    print("slabs at 512x512x64", flush=True)
    v_int, v_half = workloads.step_potential(nz, 1.5, nz / 2.0, 4.0)
    st = workloads.packet3d(n, n, nz, (n / 2.0, n / 2.0, nz / 4.0), 12.0, (0.0, 0.0, 0.56), 0.5, DT3,
                            dtype=torch.complex64, device="cuda")
    parts = P.SlabDecomposition(n, n, nz, 2, dtype=torch.complex64, dt=DT3)
    parts.set_potential_z(0.5, v_int, v_half)
    parts.load(st)
    parts.step(steps)
    got = parts.state()
    del parts
    free()
    whole = P.Lattice3D(n, n, nz, dtype=torch.complex64, dt=DT3)
    whole.set_kernel("fused")
    whole.set_potential_z(0.5, v_int, v_half)
    whole.load(st)
    whole.step(steps)
    for a, b in zip(whole.state(), got):
        assert torch.equal(a, b)
    del whole, got, st
    free()


def test_adjoint_fd_128_fp64(P):
    """The reversible adjoint's dL/dp against central finite differences (h = 1e-6)
    on the 128^3 adjoint workload (400 steps), FP64."""
    cfg = workloads.config_adjoint(128)
    n, steps = cfg["n"], cfg["steps"]
    print("adjoint fd 128^3", flush=True)
    st = workloads.packet3d(n, n, n, cfg["center"], cfg["sigma"], cfg["k0"], cfg["m"], cfg["dt"],
                            dtype=torch.complex128, device="cuda")
    lat = P.Lattice3D(n, n, n, dtype=torch.complex128, dt=cfg["dt"])
    H_int = torch.from_numpy(cfg["H_int"])
    H_half = torch.from_numpy(cfg["H_half"])
    p = torch.tensor(cfg["p"], dtype=torch.float64, requires_grad=True)
    loss = P.DiracLoss.apply(p, lat, st, cfg["m"], H_int, H_half, steps, cfg["z0"])
    loss.backward()
    grad = p.grad.numpy().copy()
    rebuilt = [t.clone() for t in lat.state()]
    assert rel_l2_t(rebuilt, st) <= 1e-12

    def L(pv):
        lat.load(st)
        lat.set_potential_z(cfg["m"], cfg["H_int"] @ pv, cfg["H_half"] @ pv)
        lat.step(steps)
        return lat.observables(cfg["z0"])[0]
    h = 1e-6
    scale = np.abs(grad).max()
    for q in (3, 15, 16, 17, 30):
        e = np.zeros_like(cfg["p"])
        e[q] = h
        fd = (L(cfg["p"] + e) - L(cfg["p"] - e)) / (2 * h)
        print("node %d: adjoint %.9e fd %.9e" % (q, grad[q], fd))
        assert abs(fd - grad[q]) <= 1e-6 * scale
    del lat
    free()


def test_adjoint_complex64_vs_complex128_128(P):
    """The adjoint workload at its stated size (128^3, 400 steps): the complex64
    gradient dL/dp against the complex128 one (itself checked against the
    oracle's adjoint and finite differences), relative to the largest
    component; and the loss and the reversal's rebuilt initial state."""
    cfg = workloads.config_adjoint(128)
    n, steps = cfg["n"], cfg["steps"]
    print("adjoint complex64 vs complex128 at 128^3", flush=True)
    H_int = torch.from_numpy(cfg["H_int"])
    H_half = torch.from_numpy(cfg["H_half"])
    res = {}
    for dtype in (torch.complex128, torch.complex64):
        st = workloads.packet3d(n, n, n, cfg["center"], cfg["sigma"], cfg["k0"], cfg["m"], cfg["dt"],
                                dtype=dtype, device="cuda")
        lat = P.Lattice3D(n, n, n, dtype=dtype, dt=cfg["dt"])
        p = torch.tensor(cfg["p"], dtype=torch.float64, requires_grad=True)
        loss = P.DiracLoss.apply(p, lat, st, cfg["m"], H_int, H_half, steps, cfg["z0"])
        loss.backward()
        res[dtype] = (float(loss), p.grad.numpy().copy(), rel_l2_t(lat.state(), st))
        del lat, st
        free()
    l64, g64, r64 = res[torch.complex128]
    l32, g32, r32 = res[torch.complex64]
    err = np.abs(g32 - g64).max() / np.abs(g64).max()
    print("loss %.9e / %.9e, grad rel err %.3e, rebuilt state %.2e / %.2e" % (l64, l32, err, r64, r32))
    assert err <= 1e-3
    assert abs(l32 - l64) <= 1e-5 * abs(l64)
    assert r64 <= 1e-12 and r32 <= 1e-3


def test_batched_full_config_matches_solo(P):
    """The 64-lattice batch (complex64, per-site theta): every lattice equals its own
    single-lattice run bitwise (the same arithmetic in any tiling), both modes."""
    lats = workloads.config_batched(device="cuda")
    print("batched full config", flush=True)
    steps = 20
    solo = []
    for L in lats:
        lat = P.Lattice2D(L["nx"], L["ny"], dtype=torch.complex64, dt=workloads.DT2)
        lat.load(L["state"])
        lat.set_fields(L["m"], L["v_site"])
        lat.step(steps)
        solo.append([t.clone() for t in lat.state()])
        del lat
    for mode in (1, 0):
        B = P.BatchedLattices(lats, dtype=torch.complex64, dt=workloads.DT2)
        B.run(steps, mode=mode, graph=True)
        for b in range(B.count):
            for x, y in zip(B.state(b), solo[b]):
                assert torch.equal(x, y), (mode, b)
        del B
    free()


@pytest.mark.parametrize("cand", [9, 12])
def test_persistent_many_items_per_workgroup(P, cand, tmp_path):
    """The 64-lattice batch in the persistent mode with 32-row chunks: several items per
    workgroup and pass, so every workgroup of the grid must be resident at once (these
    tile shapes timed out before the grid came from a census).  Bitwise equal to one
    launch per pass."""
    import json
    lats = workloads.config_batched(device="cuda")
    print("persistent many items cand=%d" % cand, flush=True)
    props = torch.cuda.get_device_properties(0)
    arch = props.gcnArchName.split(":")[0]
    cells = sum(L["nx"] * L["ny"] for L in lats)
    key = "%s/c64/n%d/cells%d/max%dx%d" % (arch, len(lats), cells, max(L["nx"] for L in lats),
                                          max(L["ny"] for L in lats))
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps({key: [cand, cand]}))
    res = []
    for mode in (1, 0):
        B = P.BatchedLattices(lats, dtype=torch.complex64, dt=workloads.DT2)
        assert B.autotune(str(cache)) == (cand, cand)
        B.run(20, mode=mode)
        res.append([t.clone() for b in range(B.count) for t in B.state(b)])
        del B
    for x, y in zip(*res):
        assert torch.equal(x, y)
    free()


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_kernels_bitwise_equal(P, dtype):
    """Split and fused kernels, and fused tilings, give identical bits (the same
    expressions evaluated in the same order; no automatic contraction)."""
    nx, ny, nz = 136, 40, 24
    print("bitwise kernels %s" % dtype, flush=True)
    g = np.random.default_rng(3)
    f0 = [g.standard_normal((nz, ny, nx)) + 1j * g.standard_normal((nz, ny, nx)) for _ in range(8)]
    v_int, v_half = workloads.step_potential(nz, 1.5, nz / 2.0, 2.0)
    outs = []
    for kernel, ty, zc in (("split", 0, 0), ("fused", 4, 0), ("fused", 8, 5), ("fused", 8, 0)):
        lat = P.Lattice3D(nx, ny, nz, dtype=dtype, dt=DT3)
        lat.set_kernel(kernel, ty, zc)
        lat.set_potential_z(0.5, v_int, v_half)
        lat.load(f0)
        lat.step(7)
        outs.append([t.clone() for t in lat.state()])
    for o in outs[1:]:
        for x, y in zip(o, outs[0]):
            assert torch.equal(x, y)


def test_graph_replay_single_lattice(P):
    """A captured graph of 100 fused steps, replayed several times with eager work and
    synchronisation in between, matches eager stepping every time."""
    nx, ny, nz = 130, 24, 32
    print("graph replay", flush=True)
    g = np.random.default_rng(4)
    f0 = [g.standard_normal((nz, ny, nx)) + 1j * g.standard_normal((nz, ny, nx)) for _ in range(8)]
    v_int, v_half = workloads.step_potential(nz, 1.5, nz / 2.0, 2.0)
    eager = P.Lattice3D(nx, ny, nz, dtype=torch.complex64, dt=DT3)
    graphed = P.Lattice3D(nx, ny, nz, dtype=torch.complex64, dt=DT3)
    for lat in (eager, graphed):
        lat.set_potential_z(0.5, v_int, v_half)
        lat.load(f0)
    graphed.step(2)                     # tables uploaded outside the capture
    eager.step(2)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    cg = torch.cuda.CUDAGraph()
    cur0 = graphed.current
    with torch.cuda.stream(s):
        with torch.cuda.graph(cg, stream=s):
            graphed.step(100)           # 50 two-step launches: an even number of buffer flips
    torch.cuda.current_stream().wait_stream(s)
    # the capture recorded launches without running them; a replayable capture
    # ends on the buffer set it started from
    assert graphed.current == cur0
    for rep in range(4):
        cg.replay()
        torch.cuda.synchronize()
        eager.step(100)
        _ = torch.ones(10, device="cuda").sum().item()      # unrelated eager work
        torch.cuda.synchronize()
        for x, y in zip(graphed.state(), eager.state()):
            assert torch.equal(x, y), rep
