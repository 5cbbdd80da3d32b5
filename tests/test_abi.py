"""The C ABI without a GPU: the library loads, exports every entry point that
include/dirac.h declares, and validates arguments before any HIP call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1309_3452_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_1309_3452_amd import build
        build.build()
    return _abi.lib()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dirac.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dirac_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    from paper_1309_3452_amd import _abi
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(_abi.EXPORTS) == names


def _create(L, ndim=3, n=(8, 8, 8), dtype=2, dt=0.5, d=(1.0, 1.0, 1.0), flags=0):
    c = ctypes.c_void_p()
    rc = L.dirac_create(ctypes.byref(c), ndim, n[0], n[1], n[2], dtype, dt, d[0], d[1], d[2], flags)
    return rc, c


def test_create_validation(L):
    import math
    rc, c = _create(L)
    assert rc == 0 and c.value
    L.dirac_destroy(c)
    # stability bound sum r_j^2 <= 1 (Sect. 2.2): r = 1/sqrt(3) passes, slightly above fails
    assert _create(L, dt=1 / math.sqrt(3))[0] == 0
    assert _create(L, dt=1.001 / math.sqrt(3))[0] == -3
    assert _create(L, dt=1.001 / math.sqrt(3), flags=1)[0] == 0
    assert _create(L, ndim=2, n=(8, 8, 1), dt=1 / math.sqrt(2))[0] == 0
    assert _create(L, ndim=2, n=(8, 8, 1), dt=0.75)[0] == -3
    # anisotropic spacing enters through r_j = dt / d_j
    assert _create(L, dt=0.5, d=(1.0, 1.0, 0.5))[0] == -3
    assert _create(L, ndim=4)[0] == -1
    assert _create(L, dtype=3)[0] == -1
    assert _create(L, n=(0, 8, 8))[0] == -2
    assert _create(L, ndim=2, n=(8, 8, 2))[0] == -2
    assert _create(L, dt=float("nan"))[0] == -1
    assert _create(L, dt=-0.1)[0] == -1
    assert _create(L, flags=8)[0] == -1


def test_calls_out_of_order_are_rejected(L):
    rc, c = _create(L)
    assert rc == 0
    out = (ctypes.c_double * 3)()
    assert L.dirac_step(c, 1, None) == -6          # no state bound
    assert b"no state bound" in L.dirac_last_error(c)
    assert L.dirac_norm(c, out, None) == -6
    nb = ctypes.c_size_t()
    assert L.dirac_scratch_bytes(c, ctypes.byref(nb)) == 0 and nb.value > 0
    assert L.dirac_bind_scratch(c, ctypes.c_void_p(256), 16) == -2      # too small (checked before use)
    assert L.dirac_bind_scratch(c, ctypes.c_void_p(255), nb.value) == -1   # misaligned
    assert L.dirac_set_kernel(c, 7, 0, 0) == -1
    assert L.dirac_set_kernel(c, 3, 0, 0) == 0
    assert L.dirac_set_kernel(c, 2, 5, 0) == -1
    assert L.dirac_set_mass_potential_z(c, 0.5, None, None, 7) == -2   # nz mismatch
    # imaginary potential: validated before any HIP call
    nz = 4
    c3 = ctypes.c_void_p()
    assert L.dirac_create(ctypes.byref(c3), 3, 4, 4, nz, 2, 0.5, 1.0, 1.0, 1.0, 0) == 0
    w = (ctypes.c_double * nz)(-0.1, 0.0, 0.0, -0.1)
    bad = (ctypes.c_double * nz)(-0.1, float("nan"), 0.0, 0.0)
    assert L.dirac_set_potential_im_z(c3, w, w, nz + 1) == -2
    assert L.dirac_set_potential_im_z(c3, w, None, nz) == -1
    assert L.dirac_set_potential_im_z(c3, bad, w, nz) == -4
    assert L.dirac_set_potential_im_z(c3, w, w, nz) == 0
    assert L.dirac_set_potential_im_z(c3, None, None, nz) == 0
    assert L.dirac_coef_from_theta_c(None, None, None, 1, None) == -1
    # records from fields: validated before any launch
    assert L.dirac_coef_from_fields(None, 1, 0.5, 0.1, None, None, 4, None) == -1
    assert L.dirac_coef_from_fields(ctypes.c_void_p(256), 3, 0.5, 0.1, None, None, 4, None) == -1
    assert L.dirac_coef_from_fields(ctypes.c_void_p(256), 2, 0.5, 0.1, None, ctypes.c_void_p(256), 4, None) == -1
    assert L.dirac_coef_from_fields(ctypes.c_void_p(256), 1, float("nan"), 0.1, None, None, 4, None) == -1
    assert L.dirac_coef_from_fields(ctypes.c_void_p(256), 1, 0.5, 0.1, None, None, 0, None) == 0
    # gauge links: 24 non-null arrays in 3D (pointers only recorded, never dereferenced here)
    from paper_1309_3452_amd._abi import ptr_array
    assert L.dirac_set_links(c3, ptr_array([256] * 23 + [0])) == -1
    assert b"null link array 23" in L.dirac_last_error(c3)
    assert L.dirac_set_links(c3, ptr_array([256] * 24)) == 0
    assert L.dirac_set_links(c3, None) == 0
    L.dirac_destroy(c3)
    # z-slab mode: 3D only; tables and fields span nz + 4 planes; forward steps only
    cs = ctypes.c_void_p()
    assert L.dirac_create(ctypes.byref(cs), 2, 4, 4, 1, 2, 0.5, 1.0, 1.0, 1.0, 2) == -1
    assert L.dirac_create(ctypes.byref(cs), 3, 4, 4, nz, 2, 0.5, 1.0, 1.0, 1.0, 2) == 0
    v4 = (ctypes.c_double * (nz + 4))(*([0.1] * (nz + 4)))
    assert L.dirac_set_mass_potential_z(cs, 0.5, w, w, nz) == -2
    assert L.dirac_set_mass_potential_z(cs, 0.5, v4, v4, nz + 4) == 0
    assert L.dirac_set_potential_im_z(cs, v4, v4, nz + 4) == 0
    fake = ptr_array([256] * 8)
    assert L.dirac_bind_state(cs, fake, fake) == 0
    assert L.dirac_scratch_bytes(cs, ctypes.byref(nb)) == 0
    assert L.dirac_bind_scratch(cs, ctypes.c_void_p(256), nb.value) == 0
    assert L.dirac_reverse(cs, 1, None) == -6
    assert L.dirac_observables(cs, 0.0, (ctypes.c_double * 9)(), None) == -6
    assert L.dirac_set_links(cs, ptr_array([256] * 24)) == -6
    # steps per halo refill: two with the two-step kernel (V(z) tables or
    # per-site coefficients), one with the one-step kernel; more per call is
    # refused before any launch
    hs = ctypes.c_int(-1)
    assert L.dirac_halo_steps(cs, ctypes.byref(hs)) == 0 and hs.value == 2
    assert L.dirac_step(cs, 3, None) == -1
    assert b"at most 2 steps" in L.dirac_last_error(cs)
    assert L.dirac_step_norm(cs, 3, ctypes.c_void_p(256), None) == -1
    assert L.dirac_set_kernel(cs, 2, 0, 0) == 0
    assert L.dirac_halo_steps(cs, ctypes.byref(hs)) == 0 and hs.value == 1
    assert L.dirac_step(cs, 2, None) == -1
    assert b"1 step per call" in L.dirac_last_error(cs)
    assert L.dirac_set_kernel(cs, 0, 0, 0) == 0
    assert L.dirac_set_theta_field(cs, fake) == 0
    assert L.dirac_halo_steps(cs, ctypes.byref(hs)) == 0 and hs.value == 2
    assert L.dirac_halo_steps(cs, None) == -1
    assert L.dirac_halo_steps(c, ctypes.byref(hs)) == 0 and hs.value == 0
    L.dirac_destroy(cs)
    # complex64 slabs with odd nx have no two-step kernel
    assert L.dirac_create(ctypes.byref(cs), 3, 5, 4, nz, 1, 0.5, 1.0, 1.0, 1.0, 2) == 0
    assert L.dirac_halo_steps(cs, ctypes.byref(hs)) == 0 and hs.value == 1
    L.dirac_destroy(cs)
    L.dirac_destroy(c)
    L.dirac_destroy(None)


def test_batch_create_validation(L):
    c = ctypes.c_void_p()
    nx = (ctypes.c_int64 * 2)(64, 96)
    ny = (ctypes.c_int64 * 2)(32, 1)
    assert L.dirac_batch_create(ctypes.byref(c), 2, nx, ny, 1, 0.6, 0) == 0
    nb = ctypes.c_size_t()
    assert L.dirac_scratch_bytes(c, ctypes.byref(nb)) == 0 and nb.value > 0
    assert L.dirac_batch_run(c, 1, 0, 0, None) == -6
    L.dirac_destroy(c)
    assert L.dirac_batch_create(ctypes.byref(c), 2, nx, ny, 1, 0.75, 0) == -3
    bad = (ctypes.c_int64 * 2)(64, 0)
    assert L.dirac_batch_create(ctypes.byref(c), 2, nx, bad, 1, 0.6, 0) == -2
    assert L.dirac_batch_create(ctypes.byref(c), 0, nx, ny, 1, 0.6, 0) == -1
    # a time step per lattice, each checked against the (2+1)D bound r <= 1/sqrt(2)
    D2 = ctypes.c_double * 2
    assert L.dirac_batch_create_dt(ctypes.byref(c), 2, nx, ny, 2, D2(0.6, 0.3), 0) == 0
    L.dirac_destroy(c)
    assert L.dirac_batch_create_dt(ctypes.byref(c), 2, nx, ny, 2, D2(0.6, 0.75), 0) == -3
    assert L.dirac_batch_create_dt(ctypes.byref(c), 2, nx, ny, 2, D2(0.6, 0.75), 1) == 0
    L.dirac_destroy(c)
    assert L.dirac_batch_create_dt(ctypes.byref(c), 2, nx, ny, 2, D2(0.6, -0.1), 0) == -1
    assert L.dirac_batch_create_dt(ctypes.byref(c), 2, nx, ny, 2, D2(float("nan"), 0.1), 0) == -1
    assert L.dirac_batch_create_dt(ctypes.byref(c), 2, nx, ny, 2, None, 0) == -1
    assert L.dirac_batch_create_dt(ctypes.byref(c), 2, nx, bad, 2, D2(0.6, 0.3), 0) == -2


def test_status_strings(L):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.dirac_status_string(code)


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_1309_3452_amd import _abi
    monkeypatch.setattr(_abi, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_abi, "_lib", None)
    with pytest.raises(ImportError):
        _abi.lib()


def test_split_setters_and_wrappers_validate(L):
    """dirac_set_mass / dirac_set_potential_z / dirac_adjoint / dirac_autotune:
    argument and state checks before any HIP call."""
    assert L.dirac_set_mass(None, 0.5) == -1
    assert L.dirac_set_potential_z(None, None, None, 4) == -1
    assert L.dirac_autotune(None, None) == -1
    c = ctypes.c_void_p()
    assert L.dirac_create(ctypes.byref(c), 3, 8, 8, 4, 2, 0.5, 1.0, 1.0, 1.0, 0) == 0
    assert L.dirac_set_mass(c, float("nan")) == -1
    assert L.dirac_set_mass(c, 0.5) == 0
    v = (ctypes.c_double * 4)(0.1, 0.2, 0.3, 0.4)
    assert L.dirac_set_potential_z(c, v, v, 5) == -2
    assert L.dirac_set_potential_z(c, v, None, 4) == -1
    assert L.dirac_set_potential_z(c, v, v, 4) == 0
    assert L.dirac_set_mass(c, 0.7) == 0            # keeps the tables
    assert L.dirac_autotune(c, None) == -6          # single lattice: no tuner
    from paper_1309_3452_amd._abi import ptr_array
    lam = ptr_array([256] * 8)
    assert L.dirac_adjoint(c, 2, lam, 0.0, ctypes.c_void_p(256), ctypes.c_void_p(256), None) == -6   # no state
    L.dirac_destroy(c)


def test_zero_bc_flag_validation(L):
    """DIRAC_ZERO_BC: 2D and 3D; not with z-slab mode; links and the V(z)
    gradient are refused before any HIP call."""
    from paper_1309_3452_amd._abi import DIRAC_SLAB_Z, DIRAC_ZERO_BC, ptr_array
    assert _create(L, flags=DIRAC_ZERO_BC)[0] == 0
    assert _create(L, ndim=2, n=(8, 8, 1), flags=DIRAC_ZERO_BC)[0] == 0
    assert _create(L, flags=DIRAC_ZERO_BC | DIRAC_SLAB_Z)[0] == -1
    rc, c = _create(L, flags=DIRAC_ZERO_BC)
    assert L.dirac_set_links(c, ptr_array([256] * 24)) == -6
    assert b"DIRAC_ZERO_BC" in L.dirac_last_error(c)
    fake = ptr_array([256] * 8)
    assert L.dirac_bind_state(c, fake, fake) == 0
    nb = ctypes.c_size_t()
    assert L.dirac_scratch_bytes(c, ctypes.byref(nb)) == 0
    assert L.dirac_bind_scratch(c, ctypes.c_void_p(256), nb.value) == 0
    assert L.dirac_adjoint_vz(c, 1, fake, ctypes.c_void_p(256), ctypes.c_void_p(256), None) == -6
    L.dirac_destroy(c)


def test_stream_copy_validation(L):
    """dirac_stream_copy rejects bad arguments before any HIP call."""
    P = ctypes.c_void_p
    assert L.dirac_stream_copy(None, P(4096), 64, None) == -1
    assert L.dirac_stream_copy(P(4096), None, 64, None) == -1
    assert L.dirac_stream_copy(P(4096), P(8192), -8, None) == -1
    assert L.dirac_stream_copy(P(4096), P(8192), 12, None) == -1          # not a multiple of 8
    assert L.dirac_stream_copy(P(4100), P(8192), 64, None) == -1          # unaligned
    assert L.dirac_stream_copy(P(4096), P(4096 + 32), 64, None) == -1     # overlapping
    assert L.dirac_stream_copy(P(4096), P(8192), 0, None) == 0            # nothing to copy
