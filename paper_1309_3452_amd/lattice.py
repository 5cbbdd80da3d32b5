"""Single lattices on the GPU: torch owns the device memory and the stream,
libdirac.so does every step of the computation (argument marshalling only here).

Array convention (Sect. 2, Eq. ABCDgrid; Sect. 3): a (3+1)D state is 8 complex
tensors of shape (nz, ny, nx) -- A0, A1, B0, B1 on time sheet n-1/2 and C0, C1,
D0, D1 on sheet n; a (2+1)D state is 4 tensors of shape (ny, nx): u0, u1
(sheet n-1/2), v0, v1 (sheet n).  Site positions are in include/dirac.h.
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import torch

from . import _abi
from ._abi import check, lib, ptr_array


def _stream_handle():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(dtype):
    if dtype == torch.complex64:
        return _abi.DIRAC_C64
    if dtype == torch.complex128:
        return _abi.DIRAC_C128
    raise ValueError("dtype must be torch.complex64 or torch.complex128")


class Lattice:
    """A periodic (2+1)D or (3+1)D lattice of the staggered leap-frog scheme.

    shape: (nx, ny) or (nx, ny, nz) cells; dt: time step; d: grid spacings.
    slab: (3D) a z-slab of a larger lattice (DIRAC_SLAB_Z): nz interior planes,
    arrays of nz + 4 planes with two halo planes on each side that the caller
    fills before every step (see SlabDecomposition).
    zero_bc: zero values outside the lattice instead of periodic wrap
    (DIRAC_ZERO_BC).
    """

    def __init__(self, shape: Sequence[int], dtype=torch.complex128, dt: float = 0.5, d=None,
                 allow_unstable: bool = False, device="cuda", slab: bool = False, zero_bc: bool = False):
        if len(shape) not in (2, 3):
            raise ValueError("shape must have 2 or 3 entries")
        self.ndim = len(shape)
        self.nx, self.ny = int(shape[0]), int(shape[1])
        self.nz = int(shape[2]) if self.ndim == 3 else 1
        self.dtype = dtype
        self.real_dtype = torch.float32 if dtype == torch.complex64 else torch.float64
        self.dt = float(dt)
        d = tuple(float(x) for x in d) if d is not None else (1.0,) * self.ndim
        self.d = d
        self.allow_unstable = bool(allow_unstable)
        self.device = torch.device(device)
        self.narr = 8 if self.ndim == 3 else 4
        self.zh = 2 if slab else 0
        self.nplanes = self.nz + 2 * self.zh            # stored planes (V(z) table entries)
        self.tshape = (self.nplanes, self.ny, self.nx) if self.ndim == 3 else (self.ny, self.nx)
        ctx = ctypes.c_void_p()
        dz = d[2] if self.ndim == 3 else 1.0
        flags = ((_abi.DIRAC_ALLOW_UNSTABLE if allow_unstable else 0) | (_abi.DIRAC_SLAB_Z if slab else 0)
                 | (_abi.DIRAC_ZERO_BC if zero_bc else 0))
        self.zero_bc = bool(zero_bc)
        check(lib().dirac_create(ctypes.byref(ctx), self.ndim, self.nx, self.ny, self.nz, _dtype_code(dtype),
                                 self.dt, float(d[0]), float(d[1]), float(dz), flags))
        self._ctx = ctx
        self.bufs = [[torch.zeros(self.tshape, dtype=dtype, device=self.device) for _ in range(self.narr)]
                     for _ in range(2)]
        check(lib().dirac_bind_state(ctx, ptr_array([t.data_ptr() for t in self.bufs[0]]),
                                     ptr_array([t.data_ptr() for t in self.bufs[1]])), ctx)
        nbytes = ctypes.c_size_t()
        check(lib().dirac_scratch_bytes(ctx, ctypes.byref(nbytes)), ctx)
        self.scratch = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        base = self.scratch.data_ptr()
        aligned = (base + 255) & ~255
        check(lib().dirac_bind_scratch(ctx, ctypes.c_void_p(aligned), int(nbytes.value)), ctx)
        self.theta = None
        # what the coefficients were last set from (kept for checkpoints): V(z)
        # tables with mass m (None: V = 0), per-site records, absorbing tables
        self._coef = {"mode": "vz", "m": 0.0, "vz": None}
        self._wz = None
        self._links = None
        self._norm_out = torch.zeros(3, dtype=torch.float64, device=self.device)

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value:
            try:
                lib().dirac_destroy(ctx)
            except Exception:
                pass
            self._ctx = None

    # -- state ---------------------------------------------------------------
    @property
    def current(self) -> int:
        w = ctypes.c_int()
        check(lib().dirac_current(self._ctx, ctypes.byref(w)), self._ctx)
        return int(w.value)

    @property
    def halo_steps(self) -> int:
        """z-slab mode: the most steps one step() call may advance between halo
        refills (2 with the two-step kernel, else 1); 0 otherwise."""
        k = ctypes.c_int()
        check(lib().dirac_halo_steps(self._ctx, ctypes.byref(k)), self._ctx)
        return int(k.value)

    def state(self):
        """The tensors currently holding the state (views, not copies)."""
        return self.bufs[self.current]

    def load(self, arrays):
        """Copy a state (sequence of narr arrays/tensors) into the current buffers."""
        if len(arrays) != self.narr:
            raise ValueError("expected %d arrays" % self.narr)
        cur = self.state()
        for t, a in zip(cur, arrays):
            src = torch.as_tensor(a)
            if tuple(src.shape) != self.tshape:
                raise ValueError("array shape %s != %s" % (tuple(src.shape), self.tshape))
            t.copy_(src.to(device=self.device, dtype=self.dtype))

    # -- coefficients --------------------------------------------------------
    def set_potential_z(self, m: float, v_int=None, v_half=None):
        """Mass m and V(z) sampled at integer (v_int) and half-integer (v_half) z."""
        if v_int is None:
            check(lib().dirac_set_mass_potential_z(self._ctx, float(m), None, None, self.nplanes), self._ctx)
            self._coef = {"mode": "vz", "m": float(m), "vz": None}
            self.theta = None
            return
        import numpy as np
        vi = np.ascontiguousarray(v_int, dtype=np.float64)
        vh = np.ascontiguousarray(v_half, dtype=np.float64)
        if vi.shape != (self.nplanes,) or vh.shape != (self.nplanes,):
            raise ValueError("v_int and v_half need one entry per stored plane (%d)" % self.nplanes)
        check(lib().dirac_set_mass_potential_z(self._ctx, float(m), vi.ctypes.data_as(ctypes.c_void_p),
                                               vh.ctypes.data_as(ctypes.c_void_p), self.nplanes), self._ctx)
        self._pin = (vi, vh)
        self._coef = {"mode": "vz", "m": float(m), "vz": (vi, vh)}
        self.theta = None

    def set_absorber_z(self, w_int=None, w_half=None):
        """Imaginary part W(z) of the potential (absorbing layers where W < 0),
        sampled like V(z); None clears it (see dirac_set_potential_im_z)."""
        if w_int is None:
            check(lib().dirac_set_potential_im_z(self._ctx, None, None, self.nplanes), self._ctx)
            self._wz = None
            return
        import numpy as np
        wi = np.ascontiguousarray(w_int, dtype=np.float64)
        wh = np.ascontiguousarray(w_half, dtype=np.float64)
        if wi.shape != (self.nplanes,) or wh.shape != (self.nplanes,):
            raise ValueError("w_int and w_half need one entry per stored plane (%d)" % self.nplanes)
        check(lib().dirac_set_potential_im_z(self._ctx, wi.ctypes.data_as(ctypes.c_void_p),
                                             wh.ctypes.data_as(ctypes.c_void_p), self.nplanes), self._ctx)
        self._pin_w = (wi, wh)
        self._wz = (wi, wh)

    def set_fields(self, m: float, v_site=None, w_site=None):
        """Per-site potential: v_site[a] holds V at the sites of state array a,
        w_site[a] (optional, complex64 lattices) its imaginary part.  The
        per-site coefficient records are theta (complex128 lattices) or
        gamma = 1 - alpha (complex64 lattices), see dirac_theta_from_fields."""
        cdt = torch.complex64 if self.dtype == torch.complex64 else torch.float64
        if w_site is not None:
            if self.dtype != torch.complex64:
                raise ValueError("per-site complex potentials are supported for complex64 lattices")
            # the library forms theta = (dt/2)(+-m + V) + i (dt/2) W in FP64 and the records
            self.theta = []
            self._fields = []
            for a in range(self.narr):
                sgn = 1.0 if a < self.narr // 2 else -1.0
                v = None if v_site is None else \
                    torch.as_tensor(v_site[a]).to(device=self.device, dtype=torch.float64).contiguous()
                w = torch.as_tensor(w_site[a]).to(device=self.device, dtype=torch.float64).contiguous()
                rec = torch.empty(self.tshape, dtype=torch.complex64, device=self.device)
                check(lib().dirac_coef_from_fields(ctypes.c_void_p(rec.data_ptr()), _abi.DIRAC_C64, self.dt,
                                                   sgn * float(m), ctypes.c_void_p(v.data_ptr()) if v is not None
                                                   else None, ctypes.c_void_p(w.data_ptr()), rec.numel(),
                                                   _stream_handle()))
                self.theta.append(rec)
                self._fields.append((v, w))
            check(lib().dirac_set_theta_field(self._ctx, ptr_array([t.data_ptr() for t in self.theta])), self._ctx)
            self._coef = {"mode": "site", "m": float(m)}
            return
        self.theta = [torch.empty(self.tshape, dtype=cdt, device=self.device) for _ in range(self.narr)]
        vs = None
        if v_site is not None:
            vs = [torch.as_tensor(v).to(device=self.device, dtype=self.real_dtype).contiguous() for v in v_site]
            self._vsite = vs
        check(lib().dirac_theta_from_fields(
            self._ctx, float(m), ptr_array([v.data_ptr() for v in vs]) if vs is not None else None,
            ptr_array([t.data_ptr() for t in self.theta]), _stream_handle()), self._ctx)
        self._coef = {"mode": "site", "m": float(m)}

    @property
    def coef_dtype(self):
        """Element type of the per-site coefficient records: theta (float64) for
        complex128 lattices, gamma = 1 - alpha (complex64) for complex64 ones."""
        return torch.complex64 if self.dtype == torch.complex64 else torch.float64

    def set_coef_records(self, records):
        """Bind per-site coefficient records already in the kernels' format
        (narr tensors of the state's shape and coef_dtype; see
        dirac_set_theta_field), e.g. those of another lattice or a checkpoint."""
        if len(records) != self.narr:
            raise ValueError("expected %d record arrays" % self.narr)
        recs = [torch.as_tensor(r).to(device=self.device, dtype=self.coef_dtype).contiguous() for r in records]
        for r in recs:
            if tuple(r.shape) != self.tshape:
                raise ValueError("record shape %s != %s" % (tuple(r.shape), self.tshape))
        check(lib().dirac_set_theta_field(self._ctx, ptr_array([r.data_ptr() for r in recs])), self._ctx)
        self.theta = recs
        self._coef = {"mode": "site", "m": None}

    def set_links(self, links=None):
        """Gauge links of a vector potential (Sect. 4): 24 (3D) or 8 (2D) tensors
        of the state's shape and dtype, links[6 a + t] / links[4 a + t] for A,B /
        u array a and neighbour term t in the order +z, -z, +x, -x, +y, -y (2D:
        +x, -x, +y, -y); the C,D / v rows use the conjugates (see
        dirac_set_links).  None unbinds them."""
        if links is None:
            check(lib().dirac_set_links(self._ctx, None), self._ctx)
            self._links = None
            return
        nl = 24 if self.ndim == 3 else 8
        if len(links) != nl:
            raise ValueError("expected %d link arrays" % nl)
        lk = [torch.as_tensor(u).to(device=self.device, dtype=self.dtype).contiguous() for u in links]
        for u in lk:
            if tuple(u.shape) != self.tshape:
                raise ValueError("link shape %s != %s" % (tuple(u.shape), self.tshape))
        check(lib().dirac_set_links(self._ctx, ptr_array([u.data_ptr() for u in lk])), self._ctx)
        self._links = lk

    def set_kernel(self, kind: str = "auto", tile_y: int = 0, zchunk: int = 0):
        """kind: "auto", "split", "fused" (one step per launch) or "fused2" (two)."""
        code = {"auto": _abi.DIRAC_KERNEL_AUTO, "split": _abi.DIRAC_KERNEL_SPLIT,
                "fused": _abi.DIRAC_KERNEL_FUSED, "fused2": _abi.DIRAC_KERNEL_FUSED2}[kind]
        check(lib().dirac_set_kernel(self._ctx, code, int(tile_y), int(zchunk)), self._ctx)

    # -- time stepping -------------------------------------------------------
    def step(self, n: int = 1):
        check(lib().dirac_step(self._ctx, int(n), _stream_handle()), self._ctx)

    def step_norm(self, n: int = 1, out: torch.Tensor = None) -> torch.Tensor:
        """n steps; the last also writes (E_r, plain norm) of the new state, FP64, into
        a device tensor (asynchronous)."""
        out = torch.empty(2, dtype=torch.float64, device=self.device) if out is None else out
        check(lib().dirac_step_norm(self._ctx, int(n), ctypes.c_void_p(out.data_ptr()), _stream_handle()),
              self._ctx)
        return out

    def reverse(self, n: int = 1):
        check(lib().dirac_reverse(self._ctx, int(n), _stream_handle()), self._ctx)

    # -- reductions ----------------------------------------------------------
    def norm(self):
        """(E_r, E_r summed on the C,D / v sites, plain norm) in FP64; synchronous."""
        out = (ctypes.c_double * 3)()
        check(lib().dirac_norm(self._ctx, out, _stream_handle()), self._ctx)
        return tuple(out)

    def norm_device(self, out: torch.Tensor = None) -> torch.Tensor:
        """Asynchronous: the same three FP64 values written into a device tensor."""
        out = self._norm_out if out is None else out
        check(lib().dirac_norm_device(self._ctx, ctypes.c_void_p(out.data_ptr()), _stream_handle()), self._ctx)
        return out

    def observables(self, z0: float):
        out = (ctypes.c_double * 9)()
        check(lib().dirac_observables(self._ctx, float(z0), out, _stream_handle()), self._ctx)
        return tuple(out)

    # -- adjoint -------------------------------------------------------------
    def seed_region(self, z0: float):
        lam = [torch.empty(self.tshape, dtype=self.dtype, device=self.device) for _ in range(self.narr)]
        check(lib().dirac_seed_region(self._ctx, float(z0), ptr_array([t.data_ptr() for t in lam]),
                                      _stream_handle()), self._ctx)
        return lam

    def adjoint_vz(self, n: int, lam):
        """Backward through n steps from the current (final) state; see dirac_adjoint_vz."""
        dvi = torch.zeros(self.nz, dtype=torch.float64, device=self.device)
        dvh = torch.zeros(self.nz, dtype=torch.float64, device=self.device)
        check(lib().dirac_adjoint_vz(self._ctx, int(n), ptr_array([t.data_ptr() for t in lam]),
                                     ctypes.c_void_p(dvi.data_ptr()), ctypes.c_void_p(dvh.data_ptr()),
                                     _stream_handle()), self._ctx)
        return dvi, dvh


def stream_copy(dst: torch.Tensor, src: torch.Tensor) -> torch.Tensor:
    """dst <- src by the library's plain streaming copy (dirac_stream_copy): the
    reference for the device's copy bandwidth.  Contiguous device tensors of the
    same byte size (a multiple of 8), asynchronous on the current stream."""
    if not (dst.is_cuda and src.is_cuda and dst.is_contiguous() and src.is_contiguous()):
        raise ValueError("stream_copy takes contiguous device tensors")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("stream_copy: tensors of different byte sizes")
    check(lib().dirac_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                                  _stream_handle()))
    return dst


def Lattice3D(nx, ny, nz, **kw):
    return Lattice((nx, ny, nz), **kw)


def Lattice2D(nx, ny, **kw):
    return Lattice((nx, ny), **kw)
