"""CPU FP64 oracle for the single-cone staggered leap-frog Dirac scheme.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It
shares no code with the HIP library: the arithmetic lives in
``dirac_oracle.c`` (plain C, FP64, one amplitude at a time through its
physical position) and in ``dense.py`` (dense one-step matrices for tiny
lattices).  This module only marshals numpy arrays into the C functions and
builds theta sheets from (m, V) the way the paper's Eqs. ss1-ss4 sample them.

Array convention: a 3D state is a list of 8 complex128 arrays of shape
(nz, ny, nx) in the order A0, A1, B0, B1, C0, C1, D0, D1; a 2D state is 4
arrays of shape (ny, nx): u0, u1, v0, v1.  Site positions (cell units):
A0 (i,j,k), A1 (i+1/2,j+1/2,k), B0 (i+1/2,j,k+1/2), B1 (i,j+1/2,k+1/2),
C0 (i,j,k+1/2), C1 (i+1/2,j+1/2,k+1/2), D0 (i+1/2,j,k), D1 (i,j+1/2,k);
u0 (i,j), u1 (i+1/2,j+1/2), v0 (i+1/2,j), v1 (i,j+1/2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dirac_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

#: physical offsets (cell units) of each array's sites
OFFSETS3 = [(0.0, 0.0, 0.0), (0.5, 0.5, 0.0), (0.5, 0.0, 0.5), (0.0, 0.5, 0.5),
            (0.0, 0.0, 0.5), (0.5, 0.5, 0.5), (0.5, 0.0, 0.0), (0.0, 0.5, 0.0)]
OFFSETS2 = [(0.0, 0.0), (0.5, 0.5), (0.5, 0.0), (0.0, 0.5)]


def compile_source(src: str, out: str) -> str:
    """gcc, FP64, no FMA contraction, OpenMP: src (a C file) -> shared library out."""
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                           "-std=c11", src, "-o", out, "-lm"])
    return out


def build(force: bool = False) -> str:
    """Compile the C oracle."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        compile_source(_SRC, tmp)
        os.replace(tmp, _SO)
    return _SO


_lib = None


def load(path: str):
    """A ctypes handle to an oracle library at path, with the signatures set."""
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    for name in ("oracle_step3", "oracle_reverse3", "oracle_step2", "oracle_reverse2"):
        getattr(L, name).argtypes = [P, P, P, P]
    for name in ("oracle_step3c", "oracle_step2c", "oracle_step3_links", "oracle_step2_links",
                 "oracle_energy3_links", "oracle_energy2_links"):
        getattr(L, name).argtypes = [P, P, P, P, P]
    for name in ("oracle_energy3", "oracle_energy2"):
        getattr(L, name).argtypes = [P, P, P, P]
    L.oracle_observe3.argtypes = [P, P, ctypes.c_double, P]
    L.oracle_observe2.argtypes = [P, P, ctypes.c_double, P]
    L.oracle_adjoint3.argtypes = [P] * 7
    L.oracle_adjoint2.argtypes = [P] * 7
    L.oracle_threads.restype = ctypes.c_int
    L.oracle_set_threads.restype = ctypes.c_int
    L.oracle_set_threads.argtypes = [ctypes.c_int]
    L.oracle_set_zero_bc.restype = ctypes.c_int
    L.oracle_set_zero_bc.argtypes = [ctypes.c_int]
    return L


def lib():
    global _lib
    if _lib is None:
        _lib = load(build())
    return _lib


def threads() -> int:
    return int(lib().oracle_threads())


def set_threads(n: int) -> int:
    """OpenMP threads for later oracle calls; returns the count now in effect."""
    return int(lib().oracle_set_threads(int(n)))


def _ptrs(arrs, dtype):
    out = (ctypes.c_void_p * len(arrs))()
    for q, a in enumerate(arrs):
        if a.dtype != dtype or not a.flags.c_contiguous:
            raise TypeError("oracle arrays must be C-contiguous %s" % dtype)
        out[q] = a.ctypes.data
    return out


def _check(rc, what):
    if rc != 0:
        raise RuntimeError("%s failed with code %d" % (what, rc))


class _Boundary:
    """Each call into the C oracle first sets the lattice's boundary: periodic,
    or zero values outside the lattice (zero_bc)."""
    zero_bc = False

    def _bc(self):
        lib().oracle_set_zero_bc(1 if self.zero_bc else 0)
        return lib()


class Lattice3(_Boundary):
    """(3+1)D lattice of nx*ny*nz cells, periodic (or zero outside, zero_bc), r_j = dt / d_j."""

    def __init__(self, nx, ny, nz, dt, dx=1.0, dy=1.0, dz=1.0, zero_bc=False):
        self.zero_bc = bool(zero_bc)
        self.shape = (int(nz), int(ny), int(nx))
        self.n = (ctypes.c_int64 * 3)(int(nx), int(ny), int(nz))
        self.dt = float(dt)
        self.r = (ctypes.c_double * 3)(dt / dx, dt / dy, dt / dz)

    def zeros(self):
        return [np.zeros(self.shape, np.complex128) for _ in range(8)]

    def positions(self, a):
        """Physical (x, y, z) of the sites of array a, each shaped like the lattice."""
        nz, ny, nx = self.shape
        ox, oy, oz = OFFSETS3[a]
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        return i + ox, j + oy, k + oz

    def theta(self, m, V=None):
        """theta sheets of Eqs. ss1-ss4: (dt/2)(m + V) at A,B sites, (dt/2)(-m + V)
        at C,D sites.  m, V: scalars or callables f(x, y, z) of the physical position."""
        th = []
        for a in range(8):
            x, y, z = self.positions(a)
            mv = m(x, y, z) if callable(m) else np.full(self.shape, float(m))
            vv = 0.0 if V is None else (V(x, y, z) if callable(V) else np.full(self.shape, float(V)))
            sgn = 1.0 if a < 4 else -1.0
            th.append(np.ascontiguousarray(0.5 * self.dt * (sgn * mv + vv), dtype=np.float64))
        return th

    def theta_vz(self, m, v_int, v_half):
        """theta sheets for a potential that depends on z only: v_int[k] = V(z = k),
        v_half[k] = V(z = k + 1/2)."""
        nz, ny, nx = self.shape
        vi = np.broadcast_to(np.asarray(v_int, np.float64)[:, None, None], self.shape)
        vh = np.broadcast_to(np.asarray(v_half, np.float64)[:, None, None], self.shape)
        zsheet = [vi, vi, vh, vh, vh, vh, vi, vi]      # A,A,B,B,C,C,D,D
        return [np.ascontiguousarray(0.5 * self.dt * ((1.0 if a < 4 else -1.0) * m + zsheet[a]))
                for a in range(8)]

    def step(self, f, th, n=1, thi=None, links=None):
        """n steps; thi (optional): Im theta per site, (dt/2) Im V (complex potential);
        links (optional): 24 complex arrays U[6 a + t] of gauge factors (vector potential)."""
        p, t = _ptrs(f, np.complex128), _ptrs(th, np.float64)
        if links is not None:
            if thi is not None:
                raise ValueError("links with a complex theta are not combined here")
            u = _ptrs(links, np.complex128)
            for _ in range(n):
                _check(self._bc().oracle_step3_links(self.n, self.r, p, t, u), "oracle_step3_links")
            return
        if thi is not None:
            ti = _ptrs(thi, np.float64)
            for _ in range(n):
                _check(self._bc().oracle_step3c(self.n, self.r, p, t, ti), "oracle_step3c")
            return
        for _ in range(n):
            _check(self._bc().oracle_step3(self.n, self.r, p, t), "oracle_step3")

    def energy_links(self, f, links):
        """E_r with gauge links (see oracle_energy3_links)."""
        out = (ctypes.c_double * 3)()
        _check(self._bc().oracle_energy3_links(self.n, self.r, _ptrs(f, np.complex128), _ptrs(links, np.complex128),
                                          out), "oracle_energy3_links")
        return tuple(out)

    def reverse(self, f, th, n=1):
        p, t = _ptrs(f, np.complex128), _ptrs(th, np.float64)
        for _ in range(n):
            _check(self._bc().oracle_reverse3(self.n, self.r, p, t), "oracle_reverse3")

    def energy(self, f):
        """(E_r as Eq. EPM, E_r summed by parts on the C,D sites, plain norm)."""
        out = (ctypes.c_double * 3)()
        _check(self._bc().oracle_energy3(self.n, self.r, _ptrs(f, np.complex128), out), "oracle_energy3")
        return tuple(out)

    def observe(self, f, z0):
        """(P[z >= z0], sum x p, sum y p, sum z p, plain norm, |A|^2, |B|^2, |C|^2, |D|^2)."""
        out = (ctypes.c_double * 9)()
        _check(self._bc().oracle_observe3(self.n, _ptrs(f, np.complex128), float(z0), out), "oracle_observe3")
        return tuple(out)

    def adjoint(self, pre, post, lam, th, gth):
        _check(self._bc().oracle_adjoint3(self.n, self.r, _ptrs(pre, np.complex128), _ptrs(post, np.complex128),
                                     _ptrs(lam, np.complex128), _ptrs(th, np.float64),
                                     _ptrs(gth, np.float64)), "oracle_adjoint3")


class Lattice2(_Boundary):
    """(2+1)D lattice of nx*ny cells, periodic (or zero outside, zero_bc), r_j = dt / d_j."""

    def __init__(self, nx, ny, dt, dx=1.0, dy=1.0, zero_bc=False):
        self.zero_bc = bool(zero_bc)
        self.shape = (int(ny), int(nx))
        self.n = (ctypes.c_int64 * 2)(int(nx), int(ny))
        self.dt = float(dt)
        self.r = (ctypes.c_double * 3)(dt / dx, dt / dy, 0.0)

    def zeros(self):
        return [np.zeros(self.shape, np.complex128) for _ in range(4)]

    def positions(self, a):
        ny, nx = self.shape
        ox, oy = OFFSETS2[a]
        j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        return i + ox, j + oy

    def theta(self, m, V=None):
        """(dt/2)(m + V) at u sites, (dt/2)(-m + V) at v sites (Eqs. scheme2Deq-scheme4thline)."""
        th = []
        for a in range(4):
            x, y = self.positions(a)
            mv = m(x, y) if callable(m) else np.full(self.shape, float(m))
            vv = 0.0 if V is None else (V(x, y) if callable(V) else np.full(self.shape, float(V)))
            sgn = 1.0 if a < 2 else -1.0
            th.append(np.ascontiguousarray(0.5 * self.dt * (sgn * mv + vv), dtype=np.float64))
        return th

    def step(self, f, th, n=1, thi=None, links=None):
        """n steps; thi (optional): Im theta per site, (dt/2) Im V (complex potential);
        links (optional): 8 complex arrays U[4 a + t] of gauge factors (vector potential)."""
        p, t = _ptrs(f, np.complex128), _ptrs(th, np.float64)
        if links is not None:
            if thi is not None:
                raise ValueError("links with a complex theta are not combined here")
            u = _ptrs(links, np.complex128)
            for _ in range(n):
                _check(self._bc().oracle_step2_links(self.n, self.r, p, t, u), "oracle_step2_links")
            return
        if thi is not None:
            ti = _ptrs(thi, np.float64)
            for _ in range(n):
                _check(self._bc().oracle_step2c(self.n, self.r, p, t, ti), "oracle_step2c")
            return
        for _ in range(n):
            _check(self._bc().oracle_step2(self.n, self.r, p, t), "oracle_step2")

    def energy_links(self, f, links):
        """E_r with gauge links (see oracle_energy2_links)."""
        out = (ctypes.c_double * 3)()
        _check(self._bc().oracle_energy2_links(self.n, self.r, _ptrs(f, np.complex128), _ptrs(links, np.complex128),
                                          out), "oracle_energy2_links")
        return tuple(out)

    def reverse(self, f, th, n=1):
        p, t = _ptrs(f, np.complex128), _ptrs(th, np.float64)
        for _ in range(n):
            _check(self._bc().oracle_reverse2(self.n, self.r, p, t), "oracle_reverse2")

    def energy(self, f):
        """(E_r with delta_+, E_r with delta_- as printed, plain norm)."""
        out = (ctypes.c_double * 3)()
        _check(self._bc().oracle_energy2(self.n, self.r, _ptrs(f, np.complex128), out), "oracle_energy2")
        return tuple(out)

    def observe(self, f, x0):
        """(P[x >= x0], sum x p, sum y p, plain norm, |u|^2, |v|^2)."""
        out = (ctypes.c_double * 6)()
        _check(self._bc().oracle_observe2(self.n, _ptrs(f, np.complex128), float(x0), out), "oracle_observe2")
        return tuple(out)

    def adjoint(self, pre, post, lam, th, gth):
        _check(self._bc().oracle_adjoint2(self.n, self.r, _ptrs(pre, np.complex128), _ptrs(post, np.complex128),
                                     _ptrs(lam, np.complex128), _ptrs(th, np.float64),
                                     _ptrs(gth, np.float64)), "oracle_adjoint2")


def run_with_adjoint3(lat: Lattice3, f0, th, nsteps, seed_fn):
    """Forward nsteps keeping every state (checkpointing, no reversal), then the
    chain rule backwards.  seed_fn(final_state) -> (loss, lam) with
    lam = dL/dRe + i dL/dIm.  Returns (loss, final_state, gth), gth[a] = dL/dtheta
    per site summed over all steps (theta constant in time)."""
    states = [[a.copy() for a in f0]]
    for _ in range(nsteps):
        nxt = [a.copy() for a in states[-1]]
        lat.step(nxt, th)
        states.append(nxt)
    loss, lam = seed_fn(states[-1])
    lam = [np.ascontiguousarray(a, np.complex128).copy() for a in lam]
    gth = [np.zeros(lat.shape) for _ in range(8)]
    for s in range(nsteps, 0, -1):
        lat.adjoint(states[s - 1], states[s], lam, th, gth)
    return loss, states[-1], gth, lam


def run_with_adjoint2(lat: Lattice2, f0, th, nsteps, seed_fn):
    states = [[a.copy() for a in f0]]
    for _ in range(nsteps):
        nxt = [a.copy() for a in states[-1]]
        lat.step(nxt, th)
        states.append(nxt)
    loss, lam = seed_fn(states[-1])
    lam = [np.ascontiguousarray(a, np.complex128).copy() for a in lam]
    gth = [np.zeros(lat.shape) for _ in range(4)]
    for s in range(nsteps, 0, -1):
        lat.adjoint(states[s - 1], states[s], lam, th, gth)
    return loss, states[-1], gth, lam
