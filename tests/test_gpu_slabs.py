"""z-slab mode (the per-device unit of a z-decomposed multi-GPU run) on one GPU:
a periodic lattice split into slabs whose halo planes are refilled from their
neighbours after every launch (two steps with the two-step kernel, one with the
one-step kernel) gives the bits of the whole lattice stepped by the one-step
fused kernel; the slabs' functional sums add up to the whole."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

DT3 = workloads.DT3


@pytest.fixture(scope="module")
def P():
    import paper_1309_3452_amd as P
    assert torch.cuda.is_available(), "needs a GPU"
    P.lib()
    return P


def rand_state(shape, count, seed):
    g = np.random.default_rng(seed)
    return [torch.from_numpy(np.ascontiguousarray(g.standard_normal(shape) + 1j * g.standard_normal(shape)))
            for _ in range(count)]


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("mode,kernel", [("vz", "auto"), ("vz", "fused"), ("site", "auto")])
@pytest.mark.parametrize("shape,slabs", [((40, 12, 16), 1), ((40, 12, 16), 2), ((40, 12, 16), 4),
                                         ((70, 9, 16), 8), ((130, 20, 12), 3)])
def test_slabs_bitwise_equal_periodic(P, dtype, mode, kernel, shape, slabs):
    nx, ny, nz = shape
    print("slabs %s x%d %s %s %s" % (shape, slabs, mode, kernel, dtype), flush=True)
    f0 = [t.to(dtype) for t in rand_state((nz, ny, nx), 8, 301)]
    whole = P.Lattice3D(nx, ny, nz, dtype=dtype, dt=DT3)
    whole.set_kernel("fused")
    parts = P.SlabDecomposition(nx, ny, nz, slabs, dtype=dtype, dt=DT3)
    parts.set_kernel(kernel)
    if mode == "vz":
        v_int, v_half = workloads.step_potential(nz, 1.5, nz / 2.0, 2.0)
        whole.set_potential_z(0.5, v_int, v_half)
        parts.set_potential_z(0.5, v_int, v_half)
    else:
        g = np.random.default_rng(302)
        V = [torch.from_numpy(np.ascontiguousarray(0.4 * g.standard_normal((nz, ny, nx)))) for _ in range(8)]
        whole.set_fields(0.3, V)
        parts.set_fields(0.3, V)
    whole.load(f0)
    parts.load(f0)
    assert parts.halo_steps == (2 if kernel == "auto" else 1)
    e_whole, e_parts = whole.norm(), parts.norm()
    for q in range(3):
        assert abs(e_parts[q] - e_whole[q]) <= 1e-12 * abs(e_whole[2])
    whole.step(7)
    parts.step(7)
    for a, b in zip(whole.state(), parts.state()):
        assert torch.equal(a, b)
    e_whole, e_parts = whole.norm(), parts.norm()
    for q in range(3):
        assert abs(e_parts[q] - e_whole[q]) <= 1e-12 * abs(e_whole[2])


@pytest.mark.parametrize("n", [1, 2])
def test_slab_step_norm_sums(P, n):
    """The in-step functional of each slab (interior only) adds up to the whole's,
    after one step (one-step kernel) and two (two-step kernel)."""
    nx, ny, nz, slabs = 64, 16, 24, 3
    f0 = rand_state((nz, ny, nx), 8, 311)
    whole = P.Lattice3D(nx, ny, nz, dtype=torch.complex128, dt=DT3)
    whole.set_kernel("fused")
    whole.set_potential_z(0.5)
    whole.load(f0)
    parts = P.SlabDecomposition(nx, ny, nz, slabs, dtype=torch.complex128, dt=DT3)
    parts.set_potential_z(0.5)
    parts.load(f0)
    ew = whole.step_norm(n)
    es = sum(lat.step_norm(n) for lat in parts.parts)
    parts.exchange()
    torch.cuda.synchronize()
    assert abs(float(es[0]) - float(ew[0])) <= 1e-12 * float(ew[1])
    assert abs(float(es[1]) - float(ew[1])) <= 1e-12 * float(ew[1])
    for a, b in zip(whole.state(), parts.state()):
        assert torch.equal(a, b)


def test_slab_refuses_steps_past_its_halo(P):
    """A call that would step past what the two halo planes serve is refused."""
    lat = P.Lattice((40, 12, 16), dtype=torch.complex128, dt=DT3, slab=True)
    lat.set_potential_z(0.5)
    assert lat.halo_steps == 2
    with pytest.raises(P.DiracError, match="at most 2 steps"):
        lat.step(3)


def test_slab_step_norm_over_partial_cap(P):
    """A slab cross-section whose two-step launch has more workgroups (1280 x 1024
    complex128: 40 x 128 tiles of 32 x 8 cells) than the fixed partial count of
    the standalone reductions (4608 pairs): the partial area is sized from the
    lattice, so dirac_step_norm still advances both steps in one launch with the
    functional summed in-step (a reduction after the launch would read stale
    halo planes); the state stays bitwise equal to the whole periodic lattice
    and the slabs' functional sums add up to the whole's."""
    nx, ny, nz, slabs = 1280, 1024, 8, 2
    print("slab step_norm over the partial cap", flush=True)
    f0 = rand_state((nz, ny, nx), 8, 313)
    whole = P.Lattice3D(nx, ny, nz, dtype=torch.complex128, dt=DT3)
    whole.set_kernel("fused")
    whole.set_potential_z(0.5)
    whole.load(f0)
    parts = P.SlabDecomposition(nx, ny, nz, slabs, dtype=torch.complex128, dt=DT3)
    parts.set_potential_z(0.5)
    parts.load(f0)
    del f0
    assert parts.halo_steps == 2
    for _ in range(2):
        ew = whole.step_norm(2)
        es = sum(lat.step_norm(2) for lat in parts.parts)
        parts.exchange()
        torch.cuda.synchronize()
        assert abs(float(es[0]) - float(ew[0])) <= 1e-12 * float(ew[1])
        assert abs(float(es[1]) - float(ew[1])) <= 1e-12 * float(ew[1])
    for a, b in zip(whole.state(), parts.state()):
        assert torch.equal(a, b)
    del whole, parts
    torch.cuda.empty_cache()
