"""dirac_norm_device_static (the entry point that allocates nothing: its
reduction partials live in a library-owned device array) against
dirac_norm_device (partials in the caller-bound scratch): the same kernels in
the same order, so the same bits; two calls in a row, the second on a smaller
lattice, and a context with no scratch bound at all."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


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


def _static(P, lat, out):
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = P.lib().dirac_norm_device_static(lat._ctx, ctypes.c_void_p(out.data_ptr()), s)   # through the C ABI
    assert rc == 0, P.lib().dirac_last_error(lat._ctx)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_static_scratch_norm_equals_bound_scratch(P, dtype):
    cases = [((96, 40, 24), 3), ((33, 7, 5), 2), ((130, 37), 2)]     # the second and third smaller
    for shape, ndim in ((c[0], len(c[0])) for c in cases):
        print("static-scratch norm %s %s" % (shape, dtype), flush=True)
        lat = P.Lattice(shape, dtype=dtype, dt=0.3)
        lat.set_potential_z(0.4)
        nz = shape[2] if ndim == 3 else 1
        st = rand_state((nz, shape[1], shape[0]) if ndim == 3 else (shape[1], shape[0]), 8 if ndim == 3 else 4,
                        17 + sum(shape))
        lat.load(st)
        lat.step(3)
        ref = lat.norm_device()
        got = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
        _static(P, lat, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (shape, got, ref)


def test_static_scratch_needs_no_bound_scratch(P):
    """A context that never bound scratch can still take the functional."""
    from paper_1309_3452_amd import _abi
    nx, ny, nz = 24, 16, 8
    c = ctypes.c_void_p()
    assert P.lib().dirac_create(ctypes.byref(c), 3, nx, ny, nz, _abi.DIRAC_C128, 0.3, 1.0, 1.0, 1.0, 0) == 0
    st = [t.cuda() for t in rand_state((nz, ny, nx), 8, 5)]
    pong = [torch.zeros_like(t) for t in st]
    assert P.lib().dirac_bind_state(c, _abi.ptr_array([t.data_ptr() for t in st]),
                                    _abi.ptr_array([t.data_ptr() for t in pong])) == 0
    out = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert P.lib().dirac_norm_device_static(c, ctypes.c_void_p(out.data_ptr()), s) == 0
    torch.cuda.synchronize()
    plain = sum(float(torch.sum(torch.abs(t) ** 2)) for t in st)
    assert abs(float(out[2]) - plain) <= 1e-12 * plain
    assert P.lib().dirac_norm_device_static(c, None, s) == -1
    P.lib().dirac_destroy(c)
