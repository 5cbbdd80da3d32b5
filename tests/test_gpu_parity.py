"""GPU path vs the CPU oracle, element by element, on the same seeded inputs.

Bars: FP64 relative L2 <= 1e-13 (the stated target); reductions in FP64 to
1e-12 relative; FP32 against the FP64 oracle within a bound derived from
FP32 rounding (see each test).  Sizes span several tiles and ragged tails.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads
from closed_form import rel_l2

pytestmark = pytest.mark.gpu

DT3 = workloads.DT3
DT2 = workloads.DT2


def np_state(tensors):
    return [t.detach().cpu().numpy().astype(np.complex128) for t in tensors]


def rand_state(shape, count, seed):
    g = np.random.default_rng(seed)
    return [np.ascontiguousarray(g.standard_normal(shape) + 1j * g.standard_normal(shape)) for _ in range(count)]


@pytest.fixture(scope="module")
def P():
    import paper_1309_3452_amd as P
    assert torch.cuda.is_available(), "needs a GPU"
    P.lib()
    return P


# --------------------------------------------------------------------------
# (2+1)D, the 128x128 configuration in full
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kernel", ["split", "fused"])
def test_config1_full_parity(P, kernel):
    cfg = workloads.config1()
    print("config1 kernel=%s" % kernel, flush=True)
    lat = P.Lattice2D(128, 128, dtype=torch.complex128, dt=cfg["dt"])
    lat.set_kernel(kernel)
    lat.set_potential_z(0.0)
    lat.load(cfg["state"])
    e0 = lat.norm()
    lat.step(cfg["steps"])
    g = np_state(lat.state())
    ol = oracle.Lattice2(128, 128, cfg["dt"])
    f = [t.numpy().copy() for t in cfg["state"]]
    ol.step(f, ol.theta(0.0), cfg["steps"])
    assert rel_l2(g, f) <= 1e-13
    e1 = lat.norm()
    eo = ol.energy(f)
    assert abs(e1[0] - e0[0]) <= 1e-14 * 200 * abs(e0[0])
    assert abs(e1[0] - eo[0]) <= 1e-12 * abs(eo[0])
    assert abs(e1[2] - eo[2]) <= 1e-12 * eo[2]


@pytest.mark.parametrize("kernel", ["split", "fused"])
@pytest.mark.parametrize("shape", [(96, 70), (130, 33), (1, 5)])
def test_2d_site_fields_parity(P, kernel, shape):
    nx, ny = shape
    print("2d fields %s %s" % (shape, kernel), flush=True)
    g = np.random.default_rng(21)
    f0 = rand_state((ny, nx), 4, 22)
    V = [np.ascontiguousarray(0.6 * g.standard_normal((ny, nx))) for _ in range(4)]
    m = 0.4
    lat = P.Lattice2D(nx, ny, dtype=torch.complex128, dt=DT2)
    lat.set_kernel(kernel)
    lat.load(f0)
    lat.set_fields(m, [torch.from_numpy(v) for v in V])
    lat.step(60)
    ol = oracle.Lattice2(nx, ny, DT2)
    th = [np.ascontiguousarray(0.5 * DT2 * ((1.0 if a < 2 else -1.0) * m + V[a])) for a in range(4)]
    f = [a.copy() for a in f0]
    ol.step(f, th, 60)
    assert rel_l2(np_state(lat.state()), f) <= 1e-13


# --------------------------------------------------------------------------
# (3+1)D
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kernel,tile_y,zchunk", [("split", 0, 0), ("fused", 4, 0), ("fused", 8, 7),
                                                   ("fused", 4, 64), ("fused2", 0, 0), ("fused2", 0, 3)])
@pytest.mark.parametrize("shape", [(70, 20, 22), (64, 8, 16), (5, 3, 1)])
def test_3d_potential_z_parity(P, kernel, tile_y, zchunk, shape):
    nx, ny, nz = shape
    print("3d vz %s %s ty=%d zc=%d" % (shape, kernel, tile_y, zchunk), flush=True)
    v_int, v_half = workloads.step_potential(nz, 1.5, nz / 2.0, 2.0)
    f0 = rand_state((nz, ny, nx), 8, 31)
    lat = P.Lattice3D(nx, ny, nz, dtype=torch.complex128, dt=DT3)
    lat.set_kernel(kernel, tile_y, zchunk)
    lat.set_potential_z(0.5, v_int, v_half)
    lat.load(f0)
    lat.step(40)
    ol = oracle.Lattice3(nx, ny, nz, DT3)
    f = [a.copy() for a in f0]
    ol.step(f, ol.theta_vz(0.5, v_int, v_half), 40)
    assert rel_l2(np_state(lat.state()), f) <= 1e-13
    en = lat.norm()
    eo = ol.energy(f)
    for q in range(3):
        assert abs(en[q] - eo[q]) <= 1e-12 * abs(eo[2])
    ob = lat.observables(nz / 2.0)
    oo = ol.observe(f, nz / 2.0)
    for q in range(9):
        assert abs(ob[q] - oo[q]) <= 1e-12 * max(abs(oo[q]), oo[4])


@pytest.mark.parametrize("kernel", ["split", "fused", "fused2"])
def test_3d_site_fields_parity(P, kernel):
    nx, ny, nz = 66, 9, 12
    print("3d fields %s" % kernel, flush=True)
    g = np.random.default_rng(41)
    f0 = rand_state((nz, ny, nx), 8, 42)
    V = [np.ascontiguousarray(0.5 * g.standard_normal((nz, ny, nx))) for _ in range(8)]
    lat = P.Lattice3D(nx, ny, nz, dtype=torch.complex128, dt=DT3)
    lat.set_kernel(kernel)
    lat.load(f0)
    lat.set_fields(0.3, [torch.from_numpy(v) for v in V])
    lat.step(30)
    ol = oracle.Lattice3(nx, ny, nz, DT3)
    th = [np.ascontiguousarray(0.5 * DT3 * ((1.0 if a < 4 else -1.0) * 0.3 + V[a])) for a in range(8)]
    f = [a.copy() for a in f0]
    ol.step(f, th, 30)
    assert rel_l2(np_state(lat.state()), f) <= 1e-13


def test_3d_reverse_parity(P):
    nx, ny, nz = 40, 12, 10
    print("3d reverse", flush=True)
    v_int, v_half = workloads.step_potential(nz, 1.0, 5.0, 2.0)
    f0 = rand_state((nz, ny, nx), 8, 51)
    lat = P.Lattice3D(nx, ny, nz, dtype=torch.complex128, dt=DT3)
    lat.set_potential_z(0.5, v_int, v_half)
    lat.load(f0)
    lat.reverse(20)
    ol = oracle.Lattice3(nx, ny, nz, DT3)
    f = [a.copy() for a in f0]
    ol.reverse(f, ol.theta_vz(0.5, v_int, v_half), 20)
    assert rel_l2(np_state(lat.state()), f) <= 1e-13
    lat.step(20)
    assert rel_l2(np_state(lat.state()), f0) <= 1e-13


# --------------------------------------------------------------------------
# FP32 form.  Per step each amplitude carries a few FP32 roundings
# (relative ~6e-8 each), accumulating coherently at worst: bound 1e-6 per
# step relative L2 against the FP64 oracle.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kernel", ["split", "fused", "fused2"])
@pytest.mark.parametrize("nx,tile_y", [(70, 8), (71, 8), (262, 4)])
def test_3d_fp32_vs_oracle(P, kernel, nx, tile_y):
    ny, nz = 17, 12
    print("3d fp32 %s nx=%d ty=%d" % (kernel, nx, tile_y), flush=True)
    v_int, v_half = workloads.step_potential(nz, 1.5, 6.0, 2.0)
    f0 = rand_state((nz, ny, nx), 8, 61)
    lat = P.Lattice3D(nx, ny, nz, dtype=torch.complex64, dt=DT3)
    lat.set_kernel(kernel, tile_y if kernel == "fused" else 0)
    lat.set_potential_z(0.5, v_int, v_half)
    lat.load(f0)
    f0_32 = np_state(lat.state())
    lat.step(50)
    ol = oracle.Lattice3(nx, ny, nz, DT3)
    f = [a.copy() for a in f0_32]
    ol.step(f, ol.theta_vz(0.5, v_int, v_half), 50)
    assert rel_l2(np_state(lat.state()), f) <= 50 * 1e-6
    en = lat.norm()
    eo = ol.energy(f)
    assert abs(en[0] - eo[0]) <= 1e-5 * eo[2]


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("shape", [(37, 23), (130, 9), (1, 5)])
def test_2d_observables_vs_oracle(P, dtype, shape):
    """(2+1)D observables after some steps on a ragged lattice: region sum over
    x_s >= x0 (x0 on an integer and on a half-integer site column, and outside),
    first moments, norm and per-component sums, against the oracle's on the same
    state (complex64 amplitudes widen exactly, both sides sum in FP64: only the
    summation order differs)."""
    tol = 1e-13
    nx, ny = shape
    print("2d observables %s %s" % (shape, dtype), flush=True)
    g = np.random.default_rng(97)
    f0 = rand_state((ny, nx), 4, 98)
    lat = P.Lattice2D(nx, ny, dtype=dtype, dt=DT2)
    lat.load(f0)
    V = [np.ascontiguousarray(0.4 * g.standard_normal((ny, nx))) for _ in range(4)]
    lat.set_fields(0.3, [torch.from_numpy(v.astype(np.float32 if dtype == torch.complex64 else np.float64))
                         for v in V])
    lat.step(9)
    st = np_state(lat.state())
    ol = oracle.Lattice2(nx, ny, DT2)
    for x0 in (float(nx // 2), nx // 2 + 0.5, 0.0, nx + 1.0):
        got = lat.observables(x0)
        ref = ol.observe(st, x0)
        # out[0..5] as the oracle's; out[6..8] are zero in 2D
        for q in range(6):
            assert abs(got[q] - ref[q]) <= tol * max(1.0, abs(ref[3]) * max(nx, ny)), (q, x0, got[q], ref[q])
        assert got[6] == got[7] == got[8] == 0.0


# --------------------------------------------------------------------------
# Adjoint: GPU (reversal) vs oracle (stored states)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 1e-3)])
def test_adjoint_vs_oracle(P, dtype, tol):
    nx, ny, nz, steps = 20, 6, 16, 12
    print("adjoint %s" % dtype, flush=True)
    g = np.random.default_rng(71)
    v_int = 0.8 * g.standard_normal(nz)
    v_half = 0.8 * g.standard_normal(nz)
    f0 = rand_state((nz, ny, nx), 8, 72)
    z0 = nz / 2.0
    lat = P.Lattice3D(nx, ny, nz, dtype=dtype, dt=DT3)
    lat.load(f0)
    f0_lat = np_state(lat.state())
    loss, dvi, dvh = P.potential_gradient(lat, f0_lat, 0.5, v_int, v_half, steps, z0)
    ol = oracle.Lattice3(nx, ny, nz, DT3)
    th = ol.theta_vz(0.5, v_int, v_half)

    def seed(f):
        mask = [ol.positions(a)[2] >= z0 for a in range(8)]
        return ol.observe(f, z0)[0], [2 * f[a] * mask[a] for a in range(8)]
    oloss, _, gth, _ = oracle.run_with_adjoint3(ol, f0_lat, th, steps, seed)
    # dL/dV at integer z: A and D sites; at half-integer z: B and C sites
    gi = 0.5 * DT3 * sum(gth[a].sum(axis=(1, 2)) for a in (0, 1, 6, 7))
    gh = 0.5 * DT3 * sum(gth[a].sum(axis=(1, 2)) for a in (2, 3, 4, 5))
    scale = max(np.abs(gi).max(), np.abs(gh).max())
    ltol = 1e-12 if dtype == torch.complex128 else 1e-5
    assert abs(loss - oloss) <= ltol * max(1.0, abs(oloss))
    assert np.abs(dvi.cpu().numpy() - gi).max() <= tol * scale
    assert np.abs(dvh.cpu().numpy() - gh).max() <= tol * scale
    # the reversal rebuilt the initial state
    rtol = 1e-13 if dtype == torch.complex128 else 1e-5
    assert rel_l2(np_state(lat.state()), f0_lat) <= rtol * steps


# --------------------------------------------------------------------------
# Batched lattices: each against its own oracle run (FP64) and against the
# single-lattice kernel (bitwise: the same arithmetic)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("mode,graph", [(1, False), (1, True), (0, False), (0, True)])
def test_batched_vs_oracle(P, mode, graph):
    print("batched mode=%d graph=%s" % (mode, graph), flush=True)
    sizes = [(64, 64), (96, 130), (200, 33), (17, 250), (1, 7), (128, 96)]
    g = np.random.default_rng(81)
    lats = []
    for (nx, ny) in sizes:
        lats.append(dict(nx=nx, ny=ny, m=float(g.uniform(0, 1)),
                         v_site=[np.ascontiguousarray(0.5 * g.standard_normal((ny, nx))) for _ in range(4)],
                         state=rand_state((ny, nx), 4, int(g.integers(1 << 30)))))
    B = P.BatchedLattices(lats, dtype=torch.complex128, dt=DT2)
    steps = 25
    B.run(steps, mode=mode, graph=graph)
    if graph:
        B.run(steps, mode=mode, graph=graph)
        steps *= 2
    norms = B.norms()
    for b, L in enumerate(lats):
        ol = oracle.Lattice2(L["nx"], L["ny"], DT2)
        th = [np.ascontiguousarray(0.5 * DT2 * ((1.0 if a < 2 else -1.0) * L["m"] + L["v_site"][a]))
              for a in range(4)]
        f = [a.copy() for a in L["state"]]
        ol.step(f, th, steps)
        assert rel_l2(np_state(B.state(b)), f) <= 1e-13, b
        eo = ol.energy(f)
        assert abs(norms[b][0] - eo[0]) <= 1e-12 * eo[2]


# --------------------------------------------------------------------------
# In-step conserved functional (fused kernel) against the standalone reduction
# and the oracle: the same FP64 sums in another order.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kernel", ["fused", "fused2"])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("shape", [(70, 20, 22), (130, 9, 5)])
def test_step_norm_matches_reduction(P, dtype, shape, kernel):
    nx, ny, nz = shape
    print("step_norm %s %s %s" % (shape, dtype, kernel), flush=True)
    v_int, v_half = workloads.step_potential(nz, 1.5, nz / 2.0, 2.0)
    f0 = rand_state((nz, ny, nx), 8, 91)
    lat = P.Lattice3D(nx, ny, nz, dtype=dtype, dt=DT3)
    lat.set_kernel(kernel)
    lat.set_potential_z(0.5, v_int, v_half)
    lat.load(f0)
    out = lat.step_norm(3).cpu().numpy()
    ref = lat.norm()
    # complex128: the same FP64 sums in another order.  complex64: the in-step
    # sum uses the FP32-evaluated stencil (a few ulps, 2^-24 each, of each
    # cross term, random over the ~1e5 sites), the reduction an FP64 one.
    tol = 1e-12 if dtype == torch.complex128 else 2e-9
    assert abs(out[0] - ref[1]) <= tol * ref[2]
    assert abs(out[0] - ref[0]) <= tol * ref[2]
    assert abs(out[1] - ref[2]) <= 1e-12 * ref[2]
    if dtype == torch.complex128:
        ol = oracle.Lattice3(nx, ny, nz, DT3)
        f = [a.copy() for a in f0]
        ol.step(f, ol.theta_vz(0.5, v_int, v_half), 3)
        assert abs(out[0] - ol.energy(f)[0]) <= 1e-12 * ref[2]
    # split kernel: the fallback path gives the same values
    lat.set_kernel("split")
    out2 = lat.step_norm(1).cpu().numpy()
    ref2 = lat.norm()
    assert abs(out2[0] - ref2[1]) <= 1e-15 * ref2[2] and abs(out2[1] - ref2[2]) <= 1e-15 * ref2[2]


# --------------------------------------------------------------------------
# Two steps per launch: the same bits as one-step launches (same helpers, same
# operation order), over ragged tiles, chunk boundaries, odd step counts and
# tiny lattices whose rings wrap onto themselves.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("shape,zchunk,steps", [((70, 20, 22), 0, 6), ((64, 8, 16), 0, 7), ((130, 9, 5), 2, 5),
                                                ((2, 1, 3), 0, 4), ((6, 4, 1), 0, 3), ((36, 17, 9), 4, 8)])
def test_fused2_bitwise_equals_one_step(P, dtype, shape, zchunk, steps):
    nx, ny, nz = shape
    print("fused2 bitwise %s %s zc=%d n=%d" % (shape, dtype, zchunk, steps), flush=True)
    v_int, v_half = workloads.step_potential(nz, 1.5, nz / 2.0, 2.0)
    f0 = rand_state((nz, ny, nx), 8, 97)
    res = []
    for kernel in ("fused2", "fused"):
        lat = P.Lattice3D(nx, ny, nz, dtype=dtype, dt=DT3)
        lat.set_kernel(kernel, 0, zchunk)
        lat.set_potential_z(0.4, v_int, v_half)
        lat.load(f0)
        lat.step(steps)
        res.append([t.cpu() for t in lat.state()])
    for a, b in zip(*res):
        assert torch.equal(a, b)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("shape,zchunk,steps", [((70, 20, 22), 0, 6), ((64, 8, 16), 0, 7), ((130, 9, 5), 2, 5),
                                                ((2, 1, 3), 0, 4), ((36, 17, 9), 4, 8)])
def test_fused2_site_bitwise_equals_one_step(P, dtype, shape, zchunk, steps):
    """Per-site coefficient records (complex64: with an absorbing W, so gamma is
    complex): two steps per launch give the one-step bits, and the in-step
    functional of the two-step launch agrees with the standalone reduction."""
    nx, ny, nz = shape
    print("fused2 site bitwise %s %s zc=%d n=%d" % (shape, dtype, zchunk, steps), flush=True)
    g = np.random.default_rng(98)
    V = [torch.from_numpy(np.ascontiguousarray(0.5 * g.standard_normal((nz, ny, nx)))) for _ in range(8)]
    W = ([torch.from_numpy(np.ascontiguousarray(-0.05 * np.abs(g.standard_normal((nz, ny, nx))))) for _ in range(8)]
         if dtype == torch.complex64 else None)
    f0 = rand_state((nz, ny, nx), 8, 99)
    res = []
    for kernel in ("fused2", "fused"):
        lat = P.Lattice3D(nx, ny, nz, dtype=dtype, dt=DT3)
        lat.set_kernel(kernel, 0, zchunk)
        lat.set_fields(0.3, V, W)
        lat.load(f0)
        lat.step(steps)
        res.append([t.cpu() for t in lat.state()])
        if kernel == "fused2":
            e = lat.step_norm(2).cpu().numpy()
            ref = lat.norm()
            # as for the V(z) tables: the same FP64 sums in another order
            # (complex64: of the FP32-evaluated stencil)
            tol = 1e-12 if dtype == torch.complex128 else 2e-9
            assert abs(e[0] - ref[0]) <= tol * ref[2] and abs(e[1] - ref[2]) <= 1e-12 * ref[2]
    for a, b in zip(*res):
        assert torch.equal(a, b)


# --------------------------------------------------------------------------
# complex64 per-site coefficient records: gamma = 1 - alpha rounded once per
# site so that |1 - gamma| = 1 as closely as FP32 allows; beta = 1 - gamma/2.
# --------------------------------------------------------------------------
def test_fp32_site_coefficients(P):
    import ctypes
    g = np.random.default_rng(7)
    th = np.concatenate([g.uniform(-2.0, 2.0, 200000), [0.0, 1e-8, -1e-8, 0.3, -0.3]])
    t = torch.from_numpy(th).cuda()
    out = torch.empty(th.size, dtype=torch.complex64, device="cuda")
    out_neg = torch.empty_like(out)
    tn = (-t).contiguous()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert P.lib().dirac_coef_from_theta(ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                         th.size, s) == 0
    assert P.lib().dirac_coef_from_theta(ctypes.c_void_p(out_neg.data_ptr()), ctypes.c_void_p(tn.data_ptr()),
                                         th.size, s) == 0
    assert P.lib().dirac_coef_from_theta(None, None, 1, s) == -1
    gam = out.cpu().numpy().astype(np.complex128)
    # unit modulus of the factor multiplying X- (the paper's alpha), per site
    unit = np.abs((1.0 - gam.real) ** 2 + gam.imag ** 2 - 1.0)
    # the FP32 grid leaves a residual of at most a few 1e-8 within 1e-6 of the
    # exact value (typically ~1e-9)
    assert unit.max() <= 8e-8, unit.max()
    assert np.median(unit) <= 3e-9, np.median(unit)
    exact = 2j * th / (1.0 + 1j * th)
    # close to 2 i theta / (1 + i theta) on both sides of |theta| = 1, where the
    # real part of the Cayley factor changes sign
    assert np.max(np.abs(gam - exact) / np.maximum(1.0, np.abs(exact))) <= 1.01e-6
    # theta -> -theta gives the conjugate record exactly (the reversed step uses this)
    gn = out_neg.cpu().numpy()
    assert np.array_equal(gn.real, out.cpu().numpy().real) and np.array_equal(gn.imag, -out.cpu().numpy().imag)


def test_fp32_record_device_bits_equal_host(P):
    """The complex64 record gamma(theta) of the per-site fields (device) and of the
    V(z) tables (host) come from one source; both give the same bits over a
    sweep of theta through both sides of |theta| = 1."""
    import ctypes
    g = np.random.default_rng(9)
    th = np.ascontiguousarray(np.concatenate([np.linspace(-4.0, 4.0, 100001), g.uniform(-1.5, 1.5, 100000),
                                              [0.0, 1e-8, -1e-8, 1.0, -1.0, 5e-4]]))
    host = np.empty(2 * th.size, np.float32)
    assert P.lib().dirac_coef_from_theta_host(host.ctypes.data_as(ctypes.c_void_p),
                                              th.ctypes.data_as(ctypes.c_void_p), th.size) == 0
    t = torch.from_numpy(th).cuda()
    dev = torch.empty(th.size, dtype=torch.complex64, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert P.lib().dirac_coef_from_theta(ctypes.c_void_p(dev.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                         th.size, s) == 0
    d = torch.view_as_real(dev).cpu().numpy().reshape(-1)
    assert np.array_equal(d.view(np.uint32), host.view(np.uint32))


@pytest.mark.parametrize("kernel", ["split", "fused", "fused2"])
def test_3d_site_fields_fp32_vs_oracle(P, kernel):
    nx, ny, nz = 66, 9, 12
    print("3d fields fp32 %s" % kernel, flush=True)
    g = np.random.default_rng(43)
    f0 = rand_state((nz, ny, nx), 8, 44)
    V = [np.ascontiguousarray(0.5 * g.standard_normal((nz, ny, nx))).astype(np.float32) for _ in range(8)]
    lat = P.Lattice3D(nx, ny, nz, dtype=torch.complex64, dt=DT3)
    lat.set_kernel(kernel)
    lat.load(f0)
    f0_32 = np_state(lat.state())
    lat.set_fields(0.3, [torch.from_numpy(v) for v in V])
    lat.step(30)
    ol = oracle.Lattice3(nx, ny, nz, DT3)
    th = [np.ascontiguousarray(0.5 * DT3 * ((1.0 if a < 4 else -1.0) * 0.3 + V[a].astype(np.float64)))
          for a in range(8)]
    f = [a.copy() for a in f0_32]
    ol.step(f, th, 30)
    # a few FP32 roundings per amplitude and step (see the FP32 section above)
    assert rel_l2(np_state(lat.state()), f) <= 30 * 1e-6
    # the reversed step (conjugate records) brings the state back
    lat.reverse(30)
    assert rel_l2(np_state(lat.state()), f0_32) <= 60 * 1e-6


@pytest.mark.parametrize("mode", [1, 0])
def test_batched_per_lattice_dt_vs_oracle(P, mode):
    """Lattices with their own time steps (dirac_batch_create_dt): each against
    the oracle with its dt (FP64); the same dt everywhere gives the bits of the
    single-dt batch."""
    print("batched per-lattice dt mode=%d" % mode, flush=True)
    sizes = [(64, 64), (96, 130), (17, 250), (1, 7)]
    dts = [DT2, 0.5, 0.3, 0.61]
    g = np.random.default_rng(87)
    lats = []
    for (nx, ny) in sizes:
        lats.append(dict(nx=nx, ny=ny, m=float(g.uniform(0, 1)),
                         v_site=[np.ascontiguousarray(0.5 * g.standard_normal((ny, nx))) for _ in range(4)],
                         state=rand_state((ny, nx), 4, int(g.integers(1 << 30)))))
    B = P.BatchedLattices(lats, dtype=torch.complex128, dt=dts)
    steps = 24
    B.run(steps, mode=mode, graph=False)
    norms = B.norms()
    for b, (L, dt) in enumerate(zip(lats, dts)):
        ol = oracle.Lattice2(L["nx"], L["ny"], dt)
        th = [np.ascontiguousarray(0.5 * dt * ((1.0 if a < 2 else -1.0) * L["m"] + L["v_site"][a])) for a in range(4)]
        f = [a.copy() for a in L["state"]]
        ol.step(f, th, steps)
        assert rel_l2(np_state(B.state(b)), f) <= 1e-13, b
        eo = ol.energy(f)
        assert abs(norms[b][0] - eo[0]) <= 1e-12 * eo[2], b
    one = P.BatchedLattices(lats, dtype=torch.complex128, dt=DT2)
    same = P.BatchedLattices(lats, dtype=torch.complex128, dt=[DT2] * len(lats))
    one.run(steps, mode=mode, graph=False)
    same.run(steps, mode=mode, graph=False)
    for b in range(len(lats)):
        for x, y in zip(one.state(b), same.state(b)):
            assert torch.equal(x, y), b


def test_batched_fp32_site_vs_oracle(P):
    sizes = [(64, 64), (96, 130), (17, 250), (1, 7)]
    g = np.random.default_rng(83)
    lats = []
    for (nx, ny) in sizes:
        lats.append(dict(nx=nx, ny=ny, m=float(g.uniform(0, 1)),
                         v_site=[np.ascontiguousarray(0.5 * g.standard_normal((ny, nx))).astype(np.float32)
                                 for _ in range(4)],
                         state=rand_state((ny, nx), 4, int(g.integers(1 << 30)))))
    B = P.BatchedLattices(lats, dtype=torch.complex64, dt=DT2)
    f32 = [np_state(B.state(b)) for b in range(len(lats))]
    steps = 40
    B.run(steps, mode=1, graph=False)
    for b, L in enumerate(lats):
        ol = oracle.Lattice2(L["nx"], L["ny"], DT2)
        th = [np.ascontiguousarray(0.5 * DT2 * ((1.0 if a < 2 else -1.0) * L["m"] + L["v_site"][a].astype(np.float64)))
              for a in range(4)]
        f = [a.copy() for a in f32[b]]
        ol.step(f, th, steps)
        assert rel_l2(np_state(B.state(b)), f) <= steps * 1e-6, b


@pytest.mark.parametrize("kernel", ["split", "fused", "fused2"])
def test_3d_fp32_large_theta_vs_oracle(P, kernel):
    """|theta| > 1 on part of the lattice (strong potential step): the FP32 table
    coefficients must sit on the correct side of the unit circle there."""
    nx, ny, nz = 64, 10, 16
    print("3d fp32 large theta %s" % kernel, flush=True)
    v_int, v_half = workloads.step_potential(nz, 6.0, 8.0, 2.0)
    f0 = rand_state((nz, ny, nx), 8, 71)
    lat = P.Lattice3D(nx, ny, nz, dtype=torch.complex64, dt=DT3)
    lat.set_kernel(kernel)
    lat.set_potential_z(0.5, v_int, v_half)
    th_max = 0.5 * DT3 * (0.5 + max(np.max(v_int), np.max(v_half)))
    assert th_max > 1.2
    lat.load(f0)
    f0_32 = np_state(lat.state())
    lat.step(20)
    ol = oracle.Lattice3(nx, ny, nz, DT3)
    f = [a.copy() for a in f0_32]
    ol.step(f, ol.theta_vz(0.5, v_int, v_half), 20)
    assert rel_l2(np_state(lat.state()), f) <= 20 * 1e-6


# --------------------------------------------------------------------------
# (2+1)D two steps per launch: the same bits as one-step launches.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("site", [False, True])
@pytest.mark.parametrize("shape,steps", [((128, 128), 6), ((70, 33), 7), ((2, 5), 4), ((130, 1), 3), ((258, 40), 8)])
def test_fused2_2d_bitwise_equals_one_step(P, dtype, site, shape, steps):
    nx, ny = shape
    print("fused2 2d bitwise %s %s site=%s n=%d" % (shape, dtype, site, steps), flush=True)
    g = np.random.default_rng(101)
    f0 = rand_state((ny, nx), 4, 102)
    V = [np.ascontiguousarray(0.5 * g.standard_normal((ny, nx))) for _ in range(4)]
    res = []
    for kernel in ("fused2", "fused"):
        lat = P.Lattice2D(nx, ny, dtype=dtype, dt=DT2)
        lat.set_kernel(kernel)
        if site:
            lat.set_fields(0.4, [torch.from_numpy(v) for v in V])
        else:
            lat.set_potential_z(0.4)
        lat.load(f0)
        lat.step(steps)
        res.append([t.cpu() for t in lat.state()])
    for a, b in zip(*res):
        assert torch.equal(a, b)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("zchunk", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("shape,steps", [((130, 40), 5), ((256, 33), 6), ((64, 7), 4)])
def test_fused2_2d_short_chunks_bitwise(P, dtype, zchunk, shape, steps):
    """Two-step 2D passes over chunks of a few rows give the bits of one-step launches."""
    nx, ny = shape
    print("fused2 2d zchunk=%d %s %s" % (zchunk, shape, dtype), flush=True)
    g = np.random.default_rng(111)
    f0 = rand_state((ny, nx), 4, 112)
    V = [np.ascontiguousarray(0.5 * g.standard_normal((ny, nx))) for _ in range(4)]
    res = []
    for kernel, zc in (("fused2", zchunk), ("fused", 0)):
        lat = P.Lattice2D(nx, ny, dtype=dtype, dt=DT2)
        lat.set_kernel(kernel, 0, zc)
        lat.set_fields(0.4, [torch.from_numpy(v) for v in V])
        lat.load(f0)
        lat.step(steps)
        res.append([t.cpu() for t in lat.state()])
    for a, b in zip(*res):
        assert torch.equal(a, b)


def _batch_key(P, lats, dtype):
    props = torch.cuda.get_device_properties(0)
    arch = props.gcnArchName.split(":")[0]
    cells = sum(L["nx"] * L["ny"] for L in lats)
    mx = max(L["nx"] for L in lats)
    my = max(L["ny"] for L in lats)
    return "%s/%s/n%d/cells%d/max%dx%d" % (arch, "c64" if dtype == torch.complex64 else "c128", len(lats), cells, mx, my)


@pytest.mark.parametrize("cand", [0, 5, 7, 8, 9, 12, 14])
@pytest.mark.parametrize("mode", [1, 0])
def test_batched_candidates_vs_oracle(P, cand, mode, tmp_path):
    """Every tile shape (one- and two-step passes, strip widths 64-256), forced through
    the tuning cache, against the oracle (complex128, 1e-13)."""
    import json
    print("batched cand=%d mode=%d" % (cand, mode), flush=True)
    sizes = [(64, 64), (96, 130), (200, 33), (17, 250), (2, 7), (300, 96)]
    g = np.random.default_rng(91)
    lats = []
    for (nx, ny) in sizes:
        lats.append(dict(nx=nx, ny=ny, m=float(g.uniform(0, 1)),
                         v_site=[np.ascontiguousarray(0.5 * g.standard_normal((ny, nx))) for _ in range(4)],
                         state=rand_state((ny, nx), 4, int(g.integers(1 << 30)))))
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps({_batch_key(P, lats, torch.complex128): [cand, cand]}))
    B = P.BatchedLattices(lats, dtype=torch.complex128, dt=DT2)
    assert B.autotune(str(cache)) == (cand, cand)
    steps = 9
    B.run(steps, mode=mode, graph=(cand % 2 == 0))
    for b, L in enumerate(lats):
        ol = oracle.Lattice2(L["nx"], L["ny"], DT2)
        th = [np.ascontiguousarray(0.5 * DT2 * ((1.0 if a < 2 else -1.0) * L["m"] + L["v_site"][a]))
              for a in range(4)]
        f = [a.copy() for a in L["state"]]
        ol.step(f, th, steps)
        assert rel_l2(np_state(B.state(b)), f) <= 1e-13, b


# --------------------------------------------------------------------------
# Complex potential: absorbing layers (Im V < 0 damps in the Cayley form).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-13), (torch.complex64, 30e-6)])
@pytest.mark.parametrize("kernel", ["split", "fused", "fused2"])
def test_3d_absorbing_layers_vs_oracle(P, kernel, dtype, tol):
    nx, ny, nz = 70, 20, 22
    print("3d absorber %s %s" % (kernel, dtype), flush=True)
    v_int, v_half = workloads.step_potential(nz, 1.5, nz / 2.0, 2.0)
    w_int, w_half = workloads.absorber(nz, 5.0, 0.8)
    f0 = rand_state((nz, ny, nx), 8, 131)
    lat = P.Lattice3D(nx, ny, nz, dtype=dtype, dt=DT3)
    lat.set_kernel(kernel)
    lat.set_potential_z(0.5, v_int, v_half)
    lat.set_absorber_z(w_int, w_half)
    lat.load(f0)
    f0 = np_state(lat.state())
    e0 = lat.norm()[0]
    lat.step(30)
    ol = oracle.Lattice3(nx, ny, nz, DT3)
    th = ol.theta_vz(0.5, v_int, v_half)
    zs = [w_int, w_int, w_half, w_half, w_half, w_half, w_int, w_int]    # A,A,B,B,C,C,D,D
    thi = [np.ascontiguousarray(np.broadcast_to((0.5 * DT3 * zs[a])[:, None, None], (nz, ny, nx)))
           for a in range(8)]
    f = [a.copy() for a in f0]
    ol.step(f, th, 30, thi=thi)
    assert rel_l2(np_state(lat.state()), f) <= tol
    e1 = lat.norm()[0]
    assert e1 < e0 and abs(e1 - ol.energy(f)[0]) <= (1e-12 if dtype == torch.complex128 else 1e-5) * abs(e0)
    if dtype == torch.complex128:
        with pytest.raises(P.DiracError):
            lat.adjoint_vz(1, lat.seed_region(nz / 2.0))


@pytest.mark.parametrize("kernel", ["split", "fused", "fused2"])
def test_2d_absorbing_frame_fp32_vs_oracle(P, kernel):
    nx, ny = 96, 80
    print("2d absorbing frame %s" % kernel, flush=True)
    g = np.random.default_rng(141)
    f0 = rand_state((ny, nx), 4, 142)
    V = [np.ascontiguousarray(0.3 * g.standard_normal((ny, nx))).astype(np.float32) for _ in range(4)]
    wx = workloads.absorber(nx, 8.0, 0.6, offsets=(0.0, 0.5))
    wy = workloads.absorber(ny, 8.0, 0.6, offsets=(0.0, 0.5))
    offs = oracle.OFFSETS2
    W = [np.ascontiguousarray(wy[1 if offs[a][1] else 0][:, None] + wx[1 if offs[a][0] else 0][None, :])
         for a in range(4)]
    lat = P.Lattice2D(nx, ny, dtype=torch.complex64, dt=DT2)
    lat.set_kernel(kernel)
    lat.load(f0)
    f0_32 = np_state(lat.state())
    lat.set_fields(0.4, [torch.from_numpy(v) for v in V], [torch.from_numpy(w) for w in W])
    e0 = lat.norm()[0]
    lat.step(40)
    ol = oracle.Lattice2(nx, ny, DT2)
    th = [np.ascontiguousarray(0.5 * DT2 * ((1.0 if a < 2 else -1.0) * 0.4 + V[a].astype(np.float64)))
          for a in range(4)]
    thi = [np.ascontiguousarray(0.5 * DT2 * W[a]) for a in range(4)]
    f = [a.copy() for a in f0_32]
    ol.step(f, th, 40, thi=thi)
    assert rel_l2(np_state(lat.state()), f) <= 40e-6
    assert lat.norm()[0] < e0


def test_batched_absorbing_fp32_vs_oracle(P):
    sizes = [(64, 64), (96, 130), (32, 250)]
    g = np.random.default_rng(151)
    lats = []
    for (nx, ny) in sizes:
        wy = workloads.absorber(ny, 6.0, 0.5)
        W = [np.ascontiguousarray(np.broadcast_to(wy[1 if oracle.OFFSETS2[a][1] else 0][:, None], (ny, nx)))
             for a in range(4)]
        lats.append(dict(nx=nx, ny=ny, m=float(g.uniform(0, 1)),
                         v_site=[np.ascontiguousarray(0.5 * g.standard_normal((ny, nx))).astype(np.float32)
                                 for _ in range(4)], w_site=W,
                         state=rand_state((ny, nx), 4, int(g.integers(1 << 30)))))
    B = P.BatchedLattices(lats, dtype=torch.complex64, dt=DT2)
    f32 = [np_state(B.state(b)) for b in range(len(lats))]
    steps = 30
    B.run(steps, mode=1, graph=False)
    for b, L in enumerate(lats):
        ol = oracle.Lattice2(L["nx"], L["ny"], DT2)
        th = [np.ascontiguousarray(0.5 * DT2 * ((1.0 if a < 2 else -1.0) * L["m"] + L["v_site"][a].astype(np.float64)))
              for a in range(4)]
        thi = [np.ascontiguousarray(0.5 * DT2 * L["w_site"][a]) for a in range(4)]
        f = [a.copy() for a in f32[b]]
        ol.step(f, th, steps, thi=thi)
        assert rel_l2(np_state(B.state(b)), f) <= steps * 1e-6, b


def test_absorbing_dissipation_identity_gpu(P):
    """E_r(n+1) - E_r(n) = sum Im(theta)|X+ + X-|^2 on the GPU states (FP64)."""
    nx, ny, nz = 40, 12, 24
    v_int, v_half = workloads.step_potential(nz, 1.0, nz / 2.0, 2.0)
    w_int, w_half = workloads.absorber(nz, 6.0, 1.0)
    lat = P.Lattice3D(nx, ny, nz, dtype=torch.complex128, dt=DT3)
    lat.set_potential_z(0.5, v_int, v_half)
    lat.set_absorber_z(w_int, w_half)
    lat.load(rand_state((nz, ny, nx), 8, 161))
    zs = [w_int, w_int, w_half, w_half, w_half, w_half, w_int, w_int]
    for _ in range(3):
        pre = np_state(lat.state())
        e0 = lat.norm()[0]
        lat.step(1)
        post = np_state(lat.state())
        e1 = lat.norm()[0]
        rhs = sum(float(np.sum((0.5 * DT3 * zs[a])[:, None, None] * np.abs(post[a] + pre[a]) ** 2)) for a in range(8))
        assert abs((e1 - e0) - rhs) <= 1e-12 * abs(e0)


# --------------------------------------------------------------------------
# Vector potential by gauge links (Sect. 4, Peierls substitution)
# --------------------------------------------------------------------------
def _links_t(U):
    return [torch.from_numpy(np.ascontiguousarray(u)) for u in U]


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-13), (torch.complex64, 25e-6)])
@pytest.mark.parametrize("site", [False, True])
def test_3d_links_vs_oracle(P, dtype, tol, site):
    from closed_form import links_from_potential3, smooth_potential3
    nx, ny, nz = 70, 20, 22
    print("3d links %s site=%s" % (dtype, site), flush=True)
    shape = (nz, ny, nx)
    U = links_from_potential3(shape, smooth_potential3(shape, 0.5, 171))
    f0 = rand_state(shape, 8, 172)
    m = 0.5
    lat = P.Lattice3D(nx, ny, nz, dtype=dtype, dt=DT3)
    lat.set_kernel("fused2")          # links force the split kernels regardless
    ol = oracle.Lattice3(nx, ny, nz, DT3)
    if site:
        g = np.random.default_rng(173)
        V = [np.ascontiguousarray(0.4 * g.standard_normal(shape)) for _ in range(8)]
        if dtype == torch.complex64:
            V = [v.astype(np.float32).astype(np.float64) for v in V]
        lat.set_fields(m, [torch.from_numpy(v) for v in V])
        th = [np.ascontiguousarray(0.5 * DT3 * ((1.0 if a < 4 else -1.0) * m + V[a])) for a in range(8)]
    else:
        v_int, v_half = workloads.step_potential(nz, 1.5, nz / 2.0, 2.0)
        lat.set_potential_z(m, v_int, v_half)
        th = ol.theta_vz(m, v_int, v_half)
    lat.set_links(_links_t(U))
    lat.load(f0)
    f0 = np_state(lat.state())
    Uc = [u.astype(np.complex64).astype(np.complex128) for u in U] if dtype == torch.complex64 else U
    e0 = lat.norm()
    steps = 20
    lat.step(steps)
    f = [a.copy() for a in f0]
    ol.step(f, th, steps, links=Uc)
    assert rel_l2(np_state(lat.state()), f) <= tol
    e1 = lat.norm()
    eo = ol.energy_links(f, Uc)
    rtol = 1e-12 if dtype == torch.complex128 else 1e-5
    assert abs(e1[0] - eo[0]) <= rtol * abs(eo[0])
    assert abs(e1[1] - eo[1]) <= rtol * abs(eo[0])
    assert abs(e1[2] - eo[2]) <= rtol * eo[2]
    # conserved by the GPU steps: FP64 to rounding, FP32 within its drift bound
    assert abs(e1[0] - e0[0]) <= (1e-13 if dtype == torch.complex128 else 1e-6) * steps * abs(e0[0])
    assert e1[2] <= 20.0 * e0[2]      # bounded: E_r stays positive for this field


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-13), (torch.complex64, 25e-6)])
@pytest.mark.parametrize("site", [False, True])
@pytest.mark.parametrize("shape", [(96, 70), (130, 33)])
def test_2d_links_vs_oracle(P, dtype, tol, site, shape):
    from closed_form import links_from_potential2, links_uniform_field2
    nx, ny = shape
    print("2d links %s %s site=%s" % (shape, dtype, site), flush=True)
    tsh = (ny, nx)
    a_fn = lambda x, y: (0.3 * np.sin(2 * np.pi * y / ny) + 0.1, 0.25 * np.cos(2 * np.pi * x / nx))
    U = links_from_potential2(tsh, a_fn)
    # uniform field with a Landau gauge periodic across the y wrap (flux 4 pi / ny
    # per cell); stronger fields near the step bound make E_r indefinite
    U2 = links_uniform_field2(tsh, 4 * np.pi / ny)
    U = [u * w for u, w in zip(U, U2)]
    f0 = rand_state(tsh, 4, 181)
    m = 0.4
    lat = P.Lattice2D(nx, ny, dtype=dtype, dt=DT2)
    ol = oracle.Lattice2(nx, ny, DT2)
    if site:
        g = np.random.default_rng(182)
        V = [np.ascontiguousarray(0.5 * g.standard_normal(tsh)) for _ in range(4)]
        if dtype == torch.complex64:
            V = [v.astype(np.float32).astype(np.float64) for v in V]
        lat.set_fields(m, [torch.from_numpy(v) for v in V])
        th = [np.ascontiguousarray(0.5 * DT2 * ((1.0 if a < 2 else -1.0) * m + V[a])) for a in range(4)]
    else:
        lat.set_potential_z(m)
        th = ol.theta(m)
    lat.set_links(_links_t(U))
    lat.load(f0)
    f0 = np_state(lat.state())
    Uc = [u.astype(np.complex64).astype(np.complex128) for u in U] if dtype == torch.complex64 else U
    steps = 25
    e0 = lat.norm()
    lat.step(steps)
    f = [a.copy() for a in f0]
    ol.step(f, th, steps, links=Uc)
    assert rel_l2(np_state(lat.state()), f) <= tol
    e1 = lat.norm()
    eo = ol.energy_links(f, Uc)
    rtol = 1e-12 if dtype == torch.complex128 else 1e-5
    # GPU (u-site form, v-site form) vs oracle (v-site form, u-site form): equal up to rounding
    assert abs(e1[0] - eo[1]) <= rtol * abs(eo[0])
    assert abs(e1[1] - eo[0]) <= rtol * abs(eo[0])
    assert abs(e1[2] - eo[2]) <= rtol * eo[2]
    assert abs(e1[0] - e0[0]) <= (1e-13 if dtype == torch.complex128 else 1e-6) * steps * abs(e0[0])
    assert e1[2] <= 20.0 * e0[2]      # bounded: E_r stays positive for this field


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_unit_links_bitwise_equal_split(P, dim, dtype):
    """Unit links multiply every neighbour by exactly 1: the link kernels then
    give the bits of the plain split kernels."""
    print("unit links dim=%d %s" % (dim, dtype), flush=True)
    if dim == 3:
        nx, ny, nz = 40, 9, 13
        shape, nl, mk = (nz, ny, nx), 24, (lambda: P.Lattice3D(nx, ny, nz, dtype=dtype, dt=DT3))
        v_int, v_half = workloads.step_potential(nz, 1.0, nz / 2.0, 2.0)
    else:
        nx, ny = 70, 33
        shape, nl, mk = (ny, nx), 8, (lambda: P.Lattice2D(nx, ny, dtype=dtype, dt=DT2))
        v_int = v_half = None
    f0 = rand_state(shape, 8 if dim == 3 else 4, 191)
    out = []
    for use_links in (False, True):
        lat = mk()
        lat.set_kernel("split")
        lat.set_potential_z(0.3, v_int, v_half) if dim == 3 else lat.set_potential_z(0.3)
        if use_links:
            lat.set_links([torch.ones(shape, dtype=dtype) for _ in range(nl)])
        lat.load(f0)
        lat.step(9)
        out.append([t.clone() for t in lat.state()] + [torch.tensor(lat.norm())])
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a, b)


def test_3d_links_pure_gauge_vs_oracle(P):
    """Pure-gauge links U = exp(i (chi(Y) - chi(X))) acting on exp(-i chi) psi0
    give exp(-i chi) times the free evolution of psi0 (GPU against GPU), and
    agree with the oracle's link step."""
    from closed_form import links_from_site_phase3
    nx, ny, nz = 18, 10, 12
    shape = (nz, ny, nx)
    print("3d pure gauge", flush=True)
    g = np.random.default_rng(201)
    chi = [np.ascontiguousarray(g.uniform(-np.pi, np.pi, shape)) for _ in range(8)]
    U = links_from_site_phase3(shape, chi)
    f0 = rand_state(shape, 8, 202)
    v_int, v_half = workloads.step_potential(nz, 1.0, nz / 2.0, 2.0)
    lat = P.Lattice3D(nx, ny, nz, dtype=torch.complex128, dt=DT3)
    lat.set_potential_z(0.5, v_int, v_half)
    lat.load(f0)
    lat.step(8)
    free = np_state(lat.state())
    lat2 = P.Lattice3D(nx, ny, nz, dtype=torch.complex128, dt=DT3)
    lat2.set_potential_z(0.5, v_int, v_half)
    lat2.set_links(_links_t(U))
    lat2.load([np.exp(-1j * chi[a]) * f0[a] for a in range(8)])
    lat2.step(8)
    gauged = np_state(lat2.state())
    assert rel_l2(gauged, [np.exp(-1j * chi[a]) * free[a] for a in range(8)]) <= 1e-13
    ol = oracle.Lattice3(nx, ny, nz, DT3)
    f = [np.exp(-1j * chi[a]) * f0[a] for a in range(8)]
    ol.step(f, ol.theta_vz(0.5, v_int, v_half), 8, links=U)
    assert rel_l2(gauged, f) <= 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_links_reverse_and_step_norm(P, dim):
    """The reversed step undoes the link step; step_norm reports the link E_r."""
    from closed_form import links_from_potential2, links_from_potential3, smooth_potential3
    print("links reverse dim=%d" % dim, flush=True)
    if dim == 3:
        nx, ny, nz = 34, 12, 10
        shape = (nz, ny, nx)
        U = links_from_potential3(shape, smooth_potential3(shape, 0.6, 211))
        lat = P.Lattice3D(nx, ny, nz, dtype=torch.complex128, dt=DT3)
        narr = 8
    else:
        nx, ny = 50, 42
        shape = (ny, nx)
        U = links_from_potential2(shape, lambda x, y: (0.5 * np.sin(2 * np.pi * y / ny), 0.2))
        lat = P.Lattice2D(nx, ny, dtype=torch.complex128, dt=DT2)
        narr = 4
    lat.set_potential_z(0.7)
    lat.set_links(_links_t(U))
    f0 = rand_state(shape, narr, 212)
    lat.load(f0)
    out = lat.step_norm(12)
    torch.cuda.synchronize()
    e = lat.norm()
    assert abs(float(out[0]) - e[0]) <= 1e-13 * abs(e[0]) and float(out[1]) == e[2]
    lat.reverse(12)
    assert rel_l2(np_state(lat.state()), f0) <= 1e-12
    if dim == 3:
        with pytest.raises(P.DiracError):
            lat.adjoint_vz(1, lat.seed_region(nz / 2.0))
    lat.set_links(None)
    lat.step(1)          # plain kernels again


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("site", [False, True])
@pytest.mark.parametrize("shape,zchunk,steps", [((70, 20, 22), 0, 5), ((130, 9, 5), 2, 4), ((3, 2, 4), 0, 3),
                                                 ((64, 8, 16), 5, 4), ((1, 1, 3), 0, 2), ((65, 9, 7), 3, 3),
                                                 ((128, 64, 6), 2, 3)])
def test_fused_links_bitwise_equals_split(P, dtype, site, shape, zchunk, steps):
    """The z-march link kernel (one launch per step) gives the bits of the split
    link kernels: ragged tiles, chunk boundaries, lattices smaller than the ring;
    128 x 64 complex128 (4 x 8 tiles of 32 x 8) takes the patch order of the
    workgroups, one patch per z-chunk."""
    from closed_form import links_from_potential3, smooth_potential3
    nx, ny, nz = shape
    print("fused links %s %s site=%s zchunk=%d" % (shape, dtype, site, zchunk), flush=True)
    tsh = (nz, ny, nx)
    U = _links_t(links_from_potential3(tsh, smooth_potential3(tsh, 0.6, 221)))
    f0 = rand_state(tsh, 8, 222)
    g = np.random.default_rng(223)
    V = [torch.from_numpy(np.ascontiguousarray(0.4 * g.standard_normal(tsh))) for _ in range(8)]
    v_int, v_half = workloads.step_potential(nz, 1.5, nz / 2.0, 2.0)
    out = []
    for kind in ("split", "fused"):
        lat = P.Lattice3D(nx, ny, nz, dtype=dtype, dt=DT3)
        lat.set_kernel(kind, 0, zchunk)
        if site:
            lat.set_fields(0.3, V)
        else:
            lat.set_potential_z(0.3, v_int, v_half)
        lat.set_links(U)
        lat.load(f0)
        lat.step(steps)
        out.append([t.clone() for t in lat.state()])
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a, b)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("site", [False, True])
@pytest.mark.parametrize("shape,zchunk,steps", [((130, 40), 0, 5), ((64, 7), 0, 4), ((1, 5), 0, 3),
                                                 ((257, 33), 3, 4), ((96, 70), 8, 6), ((2, 2), 1, 3)])
def test_fused_links_2d_bitwise_equals_split(P, dtype, site, shape, zchunk, steps):
    """The (2+1)D link march (one launch per step) gives the bits of the split link
    kernels: ragged strips, chunk boundaries, lattices smaller than the ring."""
    from closed_form import links_from_potential2
    nx, ny = shape
    print("fused links 2d %s %s site=%s zchunk=%d" % (shape, dtype, site, zchunk), flush=True)
    tsh = (ny, nx)
    U = _links_t(links_from_potential2(tsh, lambda x, y: (0.4 * np.sin(2 * np.pi * y / max(ny, 2)) + 0.1,
                                                          0.3 * np.cos(2 * np.pi * x / max(nx, 2)))))
    f0 = rand_state(tsh, 4, 231)
    g = np.random.default_rng(232)
    V = [torch.from_numpy(np.ascontiguousarray(0.4 * g.standard_normal(tsh))) for _ in range(4)]
    out = []
    for kind in ("split", "fused"):
        lat = P.Lattice2D(nx, ny, dtype=dtype, dt=DT2)
        lat.set_kernel(kind, 0, zchunk)
        if site:
            lat.set_fields(0.3, V)
        else:
            lat.set_potential_z(0.3)
        lat.set_links(U)
        lat.load(f0)
        lat.step(steps)
        out.append([t.clone() for t in lat.state()])
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a, b)


def test_split_setters_and_adjoint_wrapper(P):
    """dirac_set_mass + dirac_set_potential_z give the bits of
    dirac_set_mass_potential_z; dirac_adjoint gives those of dirac_seed_region then
    dirac_adjoint_vz."""
    import ctypes
    from paper_1309_3452_amd._abi import lib, ptr_array
    print("split setters and adjoint wrapper", flush=True)
    nx, ny, nz = 40, 12, 16
    g = np.random.default_rng(811)
    f0 = [torch.from_numpy(g.standard_normal((nz, ny, nx)) + 1j * g.standard_normal((nz, ny, nx))) for _ in range(8)]
    vi, vh = 0.4 * g.standard_normal(nz), 0.4 * g.standard_normal(nz)
    outs = []
    for split in (False, True):
        lat = P.Lattice3D(nx, ny, nz, dtype=torch.complex128, dt=DT3)
        if split:
            assert lib().dirac_set_potential_z(lat._ctx, vi.ctypes.data_as(ctypes.c_void_p),
                                               vh.ctypes.data_as(ctypes.c_void_p), nz) == 0
            assert lib().dirac_set_mass(lat._ctx, 0.45) == 0
        else:
            lat.set_potential_z(0.45, vi, vh)
        lat.load(f0)
        lat.step(5)
        lam = [torch.empty((nz, ny, nx), dtype=torch.complex128, device="cuda") for _ in range(8)]
        dvi = torch.zeros(nz, dtype=torch.float64, device="cuda")
        dvh = torch.zeros(nz, dtype=torch.float64, device="cuda")
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        if split:
            assert lib().dirac_adjoint(lat._ctx, 5, ptr_array([t.data_ptr() for t in lam]), 8.0,
                                       ctypes.c_void_p(dvi.data_ptr()), ctypes.c_void_p(dvh.data_ptr()), stream) == 0
        else:
            lam = lat.seed_region(8.0)
            dvi, dvh = lat.adjoint_vz(5, lam)
        torch.cuda.synchronize()
        outs.append(([t.clone() for t in lat.state()], [t.clone() for t in lam], dvi.clone(), dvh.clone()))
    for a, b in zip(outs[0][0] + outs[0][1], outs[1][0] + outs[1][1]):
        assert torch.equal(a, b)
    assert torch.equal(outs[0][2], outs[1][2]) and torch.equal(outs[0][3], outs[1][3])


# --------------------------------------------------------------------------
# Zero values outside the lattice (DIRAC_ZERO_BC): split kernels against the
# oracle's zero-boundary mode, in both precisions, with V(z) tables and
# per-site fields; the functional (both forms) and the reversed step.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-13), (torch.complex64, 2e-5)])
@pytest.mark.parametrize("mode", ["vz", "site"])
@pytest.mark.parametrize("shape", [(70, 9, 12), (5, 130, 3), (1, 1, 4)])
def test_3d_zero_bc_vs_oracle(P, dtype, tol, mode, shape):
    nx, ny, nz = shape
    steps = 25
    print("3d zero bc %s %s %s" % (shape, mode, dtype), flush=True)
    f0 = rand_state((nz, ny, nx), 8, 501)
    lat = P.Lattice((nx, ny, nz), dtype=dtype, dt=DT3, zero_bc=True)
    lat.load(f0)
    f0_lat = np_state(lat.state())
    ol = oracle.Lattice3(nx, ny, nz, DT3, zero_bc=True)
    if mode == "vz":
        v_int, v_half = workloads.step_potential(nz, 1.5, nz / 2.0, 2.0)
        lat.set_potential_z(0.5, v_int, v_half)
        th = ol.theta_vz(0.5, v_int, v_half)
    else:
        g = np.random.default_rng(502)
        V = [np.ascontiguousarray(0.5 * g.standard_normal((nz, ny, nx))) for _ in range(8)]
        if dtype == torch.complex64:
            V = [v.astype(np.float32) for v in V]
        lat.set_fields(0.3, [torch.from_numpy(v) for v in V])
        th = [np.ascontiguousarray(0.5 * DT3 * ((1.0 if a < 4 else -1.0) * 0.3 + V[a].astype(np.float64)))
              for a in range(8)]
    e0 = lat.norm()
    eo0 = ol.energy(f0_lat)
    # complex64 lattices evaluate the functional (in FP64) with the r_j of their
    # FP32 steps, rounded to float: ~1e-8 relative to the oracle's FP64 r_j
    rtol0 = 1e-12 if dtype == torch.complex128 else 1e-8
    assert abs(e0[0] - eo0[0]) <= rtol0 * eo0[2] and abs(e0[1] - eo0[1]) <= rtol0 * eo0[2]
    lat.step(steps)
    f = [a.copy() for a in f0_lat]
    ol.step(f, th, steps)
    assert rel_l2(np_state(lat.state()), f) <= tol * (1 if dtype == torch.complex128 else steps)
    e1 = lat.norm()
    etol = 1e-13 if dtype == torch.complex128 else 1e-5
    assert abs(e1[0] - e0[0]) <= etol * abs(e0[0]) and abs(e1[1] - e1[0]) <= 1e-12 * e1[2]
    lat.reverse(steps)
    assert rel_l2(np_state(lat.state()), f0_lat) <= tol * (1 if dtype == torch.complex128 else 2 * steps)


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-13), (torch.complex64, 2e-5)])
@pytest.mark.parametrize("shape", [(130, 37), (1, 9), (64, 4)])
def test_2d_zero_bc_vs_oracle(P, dtype, tol, shape):
    nx, ny = shape
    steps = 30
    print("2d zero bc %s %s" % (shape, dtype), flush=True)
    f0 = rand_state((ny, nx), 4, 511)
    g = np.random.default_rng(512)
    V = [np.ascontiguousarray(0.5 * g.standard_normal((ny, nx))) for _ in range(4)]
    if dtype == torch.complex64:
        V = [v.astype(np.float32) for v in V]
    lat = P.Lattice((nx, ny), dtype=dtype, dt=DT2, zero_bc=True)
    lat.load(f0)
    f0_lat = np_state(lat.state())
    lat.set_fields(0.4, [torch.from_numpy(v) for v in V])
    th = [np.ascontiguousarray(0.5 * DT2 * ((1.0 if a < 2 else -1.0) * 0.4 + V[a].astype(np.float64)))
          for a in range(4)]
    ol = oracle.Lattice2(nx, ny, DT2, zero_bc=True)
    e0 = lat.norm()
    eo0 = ol.energy(f0_lat)
    rtol0 = 1e-12 if dtype == torch.complex128 else 1e-8      # r_j rounded to float (see the 3D test)
    assert abs(e0[0] - eo0[0]) <= rtol0 * eo0[2]
    buf = torch.zeros(2, dtype=torch.float64, device="cuda")
    lat.step(steps - 1)
    lat.step_norm(1, buf)
    f = [a.copy() for a in f0_lat]
    ol.step(f, th, steps)
    assert rel_l2(np_state(lat.state()), f) <= tol * (1 if dtype == torch.complex128 else steps)
    eo1 = ol.energy(f)
    etol = 1e-13 if dtype == torch.complex128 else 1e-5
    assert abs(float(buf[0]) - eo1[0]) <= etol * eo1[2] and abs(eo1[0] - eo0[0]) <= 1e-13 * eo0[2]
    lat.reverse(steps)
    assert rel_l2(np_state(lat.state()), f0_lat) <= tol * (1 if dtype == torch.complex128 else 2 * steps)


# --------------------------------------------------------------------------
# Reversed steps on the march kernels: one split reversed C,D half-step, the
# forward march with r -> -r and theta -> -theta, one split reversed A,B
# half-step.  The same helpers in the same order as the split reversed steps,
# so the same bits; V(z) tables and per-site records, both precisions, odd and
# even step counts, ragged tiles and z-chunks.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("mode", ["vz", "site"])
@pytest.mark.parametrize("shape,steps", [((70, 9, 12), 7), ((130, 20, 11), 6), ((64, 8, 5), 1), ((6, 3, 4), 2)])
def test_reverse_march_bitwise_equals_split(P, dtype, mode, shape, steps):
    nx, ny, nz = shape
    print("reverse march %s %s %s n=%d" % (shape, mode, dtype, steps), flush=True)
    f0 = rand_state((nz, ny, nx), 8, 601)
    g = np.random.default_rng(602)
    V = [np.ascontiguousarray(0.5 * g.standard_normal((nz, ny, nx))) for _ in range(8)]
    if dtype == torch.complex64:
        V = [v.astype(np.float32) for v in V]
    v_int, v_half = workloads.step_potential(nz, 1.5, nz / 2.0, 2.0)
    out = []
    for kernel in ("split", "auto", "fused"):
        lat = P.Lattice3D(nx, ny, nz, dtype=dtype, dt=DT3)
        lat.set_kernel(kernel)
        lat.load(f0)
        if mode == "vz":
            lat.set_potential_z(0.5, v_int, v_half)
        else:
            lat.set_fields(0.3, [torch.from_numpy(v) for v in V])
        lat.reverse(steps)
        out.append([t.clone() for t in lat.state()])
        if kernel == "auto":
            lat.step(steps)          # and forward again: back to the start up to rounding
            tol = 1e-13 if dtype == torch.complex128 else 2e-5 * steps
            assert rel_l2(np_state(lat.state()), np_state([torch.from_numpy(a).to(dtype) for a in f0])) <= tol
        del lat
    for kernel, st in zip(("auto", "fused"), out[1:]):
        for a, b in zip(out[0], st):
            assert torch.equal(a, b), kernel


# --------------------------------------------------------------------------
# Two-step kernel on random small shapes and z-chunk lengths: every plane count
# modulo the rotating layout's three LDS sets, chunks of one to a few planes,
# rings that wrap onto tiny lattices, odd step counts.  Bits equal the split
# kernels' (same expressions in the same order).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("site", [False, True])
def test_two_step_random_shapes_bitwise_vs_split(P, dtype, site):
    g = np.random.default_rng(4242 + (2 if site else 0) + (1 if dtype == torch.complex64 else 0))
    for case in range(10):
        nx = 2 * int(g.integers(1, 80))              # even: the complex64 two-step kernel needs it
        ny = int(g.integers(1, 28))
        nz = int(g.integers(1, 19))
        zc = int(g.integers(0, 5))                   # 0: the launcher's choice
        steps = int(g.integers(2, 8))
        print("two-step random %s site=%s case %d: %dx%dx%d zchunk %d steps %d"
              % (dtype, site, case, nx, ny, nz, zc, steps), flush=True)
        f0 = rand_state((nz, ny, nx), 8, int(g.integers(1 << 30)))
        V = [np.ascontiguousarray(0.4 * g.standard_normal((nz, ny, nx))) for _ in range(8)]
        v_int, v_half = workloads.step_potential(nz, 1.2, nz / 2.0, 2.0)
        outs = []
        for kernel in ("split", "fused2"):
            lat = P.Lattice3D(nx, ny, nz, dtype=dtype, dt=DT3)
            lat.set_kernel(kernel, 0, zc)
            if site:
                lat.set_fields(0.3, [torch.from_numpy(v.astype(np.float32 if dtype == torch.complex64 else np.float64))
                                     for v in V])
            else:
                lat.set_potential_z(0.5, v_int, v_half)
            lat.load(f0)
            lat.step(steps)
            outs.append([t.clone() for t in lat.state()])
            del lat
        for x, y in zip(outs[0], outs[1]):
            assert torch.equal(x, y), (nx, ny, nz, zc, steps)
