"""Run-to-run determinism: the step kernels have no atomics and every reduction
sums in a fixed order, so the same input gives the same bits on every run --
state, in-step functional and standalone reductions -- for the two-step and
one-step 3D kernels, the (2+1)D marches and a batch."""
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


def run(P, shape, dtype, kernel, steps):
    lat = P.Lattice(shape, dtype=dtype, dt=workloads.DT3 if len(shape) == 3 else workloads.DT2)
    lat.set_kernel(kernel)
    if len(shape) == 3:
        vi, vh = workloads.step_potential(shape[2], 1.5, shape[2] / 2.0, 2.0)
        lat.set_potential_z(0.5, vi, vh)
        f0 = rand_state((shape[2], shape[1], shape[0]), 8, 501, dtype)
    else:
        lat.set_potential_z(0.4)
        f0 = rand_state((shape[1], shape[0]), 4, 502, dtype)
    lat.load(f0)
    e_step = lat.step_norm(steps).clone()
    e = lat.norm()
    return [t.clone() for t in lat.state()], e_step, e


@pytest.mark.parametrize("shape,kernel", [((96, 40, 30), "fused2"), ((96, 40, 30), "fused"),
                                          ((300, 130), "fused2"), ((300, 130), "fused")])
@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_same_bits_every_run(P, shape, kernel, dtype):
    print("determinism %s %s %s" % (shape, kernel, dtype), flush=True)
    s1, es1, e1 = run(P, shape, dtype, kernel, 11)
    s2, es2, e2 = run(P, shape, dtype, kernel, 11)
    for a, b in zip(s1, s2):
        assert torch.equal(a, b)
    assert torch.equal(es1, es2) and e1 == e2


def test_batch_same_bits_every_run(P):
    print("determinism batch", flush=True)
    lats = workloads.config_batched(count=8, device="cuda")
    outs = []
    for graph in (False, True):
        b = P.BatchedLattices(lats, dtype=torch.complex64, dt=workloads.DT2)
        b.run(9, mode=1, graph=graph)
        outs.append(([t.clone() for i in range(b.count) for t in b.state(i)], b.norms()))
    for a, c in zip(outs[0][0], outs[1][0]):
        assert torch.equal(a, c)
    assert outs[0][1] == outs[1][1]
