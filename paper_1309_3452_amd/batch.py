"""Many independent (2+1)D lattices advanced together (dirac_batch_* calls)."""
from __future__ import annotations

import ctypes

import torch

from . import _abi
from ._abi import check, lib, ptr_array
from .lattice import _dtype_code, _stream_handle


class BatchedLattices:
    """lattices: sequence of dicts with nx, ny, m, v_site (4 real arrays or None),
    optionally w_site (4 arrays: Im V, complex64 batches) and state (4 complex
    arrays of shape (ny, nx)).  dt: one time step for all lattices, or a
    sequence with one per lattice; unit spacing."""

    def __init__(self, lattices, dtype=torch.complex64, dt=0.5, device="cuda"):
        self.device = torch.device(device)
        self.dtype = dtype
        self.real_dtype = torch.float32 if dtype == torch.complex64 else torch.float64
        self.count = len(lattices)
        per = hasattr(dt, "__len__")
        self.dts = [float(d) for d in dt] if per else [float(dt)] * self.count
        if len(self.dts) != self.count:
            raise ValueError("one dt per lattice")
        self.dt = self.dts[0]
        nx = (ctypes.c_int64 * self.count)(*[int(L["nx"]) for L in lattices])
        ny = (ctypes.c_int64 * self.count)(*[int(L["ny"]) for L in lattices])
        self.shapes = [(int(L["ny"]), int(L["nx"])) for L in lattices]
        ctx = ctypes.c_void_p()
        if per:
            dts = (ctypes.c_double * self.count)(*self.dts)
            check(lib().dirac_batch_create_dt(ctypes.byref(ctx), self.count, nx, ny, _dtype_code(dtype), dts, 0))
        else:
            check(lib().dirac_batch_create(ctypes.byref(ctx), self.count, nx, ny, _dtype_code(dtype), self.dt, 0))
        self._ctx = ctx
        self.bufs = [[], []]
        self.theta = []
        self._fields = []
        code = _dtype_code(dtype)
        for L, shp, dtb in zip(lattices, self.shapes, self.dts):
            st = [torch.as_tensor(a).to(device=self.device, dtype=dtype).contiguous().clone() for a in L["state"]]
            self.bufs[0].append(st)
            self.bufs[1].append([torch.zeros(shp, dtype=dtype, device=self.device) for _ in range(4)])
            m = float(L["m"])
            vs, ws = L.get("v_site"), L.get("w_site")
            if ws is not None and dtype != torch.complex64:
                raise ValueError("per-site complex potentials are supported for complex64 batches")
            th = []
            for a in range(4):
                # the library forms theta = (dt/2)(+-m + V) + i (dt/2) W per site (u: +m, v: -m)
                # in FP64 and writes the record (complex64: gamma, complex128: theta)
                sgn = 1.0 if a < 2 else -1.0
                v = None if vs is None else torch.as_tensor(vs[a]).to(device=self.device, dtype=torch.float64).contiguous()
                w = None if ws is None else torch.as_tensor(ws[a]).to(device=self.device, dtype=torch.float64).contiguous()
                coef = torch.empty(shp, dtype=torch.complex64 if dtype == torch.complex64 else torch.float64,
                                   device=self.device)
                check(lib().dirac_coef_from_fields(ctypes.c_void_p(coef.data_ptr()), code, dtb, sgn * m,
                                                   ctypes.c_void_p(v.data_ptr()) if v is not None else None,
                                                   ctypes.c_void_p(w.data_ptr()) if w is not None else None,
                                                   coef.numel(), _stream_handle()))
                th.append(coef)
                self._fields.append((v, w))
            self.theta.append(th)
        nbytes = ctypes.c_size_t()
        check(lib().dirac_scratch_bytes(ctx, ctypes.byref(nbytes)), ctx)
        self.scratch = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        aligned = (self.scratch.data_ptr() + 255) & ~255
        flat = lambda sets: ptr_array([t.data_ptr() for s in sets for t in s])
        check(lib().dirac_batch_bind(ctx, flat(self.bufs[0]), flat(self.bufs[1]), flat(self.theta),
                                     ctypes.c_void_p(aligned), int(nbytes.value)), ctx)

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value:
            try:
                lib().dirac_destroy(ctx)
            except Exception:
                pass
            self._ctx = None

    @property
    def current(self):
        w = ctypes.c_int()
        check(lib().dirac_current(self._ctx, ctypes.byref(w)), self._ctx)
        return int(w.value)

    def state(self, b):
        return self.bufs[self.current][b]

    def run(self, n, mode=1, graph=False):
        """mode 1: one launch per step; mode 0: one persistent launch.  graph: replay a captured HIP graph."""
        check(lib().dirac_batch_run(self._ctx, int(n), int(mode), 1 if graph else 0, _stream_handle()), self._ctx)

    def norms(self):
        out = (ctypes.c_double * (3 * self.count))()
        check(lib().dirac_batch_norms(self._ctx, out, _stream_handle()), self._ctx)
        return [tuple(out[3 * b:3 * b + 3]) for b in range(self.count)]

    def autotune(self, cache_path=None):
        """Tile choice per mode; the state is advanced by an even number of steps.
        If a persistent candidate timed out (the library then reports the bound
        state as invalid), the state from before the call is restored."""
        cur = self.current
        snap = [[t.clone() for t in self.bufs[cur][b]] for b in range(self.count)]
        ch = ctypes.c_int(-1)
        rc = lib().dirac_batch_autotune(self._ctx, cache_path.encode() if cache_path else None,
                                        ctypes.byref(ch), _stream_handle())
        if rc == _abi.DIRAC_E_STATE and ch.value >= 0:
            check(lib().dirac_set_current(self._ctx, cur), self._ctx)
            for b in range(self.count):
                for t, s0 in zip(self.bufs[cur][b], snap[b]):
                    t.copy_(s0)
        else:
            check(rc, self._ctx)
        del snap
        return int(ch.value) & 0xff, int(ch.value) >> 8
