"""Dense one-step matrices of the scheme on tiny lattices (test infrastructure).

Independent of ``dirac_oracle.c``: the operator is assembled here in numpy
from the paper's difference equations, with sites found through a dictionary
of their physical positions, and the two half-steps are dense matrices.
Used to pin the C oracle (M^n x against stepping), the conserved functional
(M^H G M = G, Lemma of Sect. 2 / Sect. 3) and the spectrum against the
closed-form dispersion (Sect. 2.1, Eq. pwdsip).

A vector potential (Sect. 4) enters through a_fn(x, y[, z]) -> per-axis phase
per cell length (a = q A Delta / (hbar c)), positions in cell units:
  rule="exact":  the neighbour at displacement d (+-1/2 cell along axis j)
                 is multiplied by exp(-i a_j(M) d), M the half-link midpoint
                 (the Peierls substitution with the line integral by the
                 midpoint rule);
  rule="linear": the paper's simplified rule for smooth potentials, the
                 difference psi(+) - psi(-) replaced by psi(+) - psi(-)
                 - i a_j (psi(+) + psi(-))/2 with a_j taken at the row's site.

zero_bc=True drops every coupling to a position outside the lattice (zero
values there) instead of wrapping it periodically.

State vector order: the arrays of the oracle's convention concatenated,
3D: A0 A1 B0 B1 | C0 C1 D0 D1, 2D: u0 u1 | v0 v1, each flattened [k][j][i].
"""
from __future__ import annotations

import numpy as np

# doubled-coordinate parity of each array's sites (positions of Eq. ABCDgrid)
_PAR3 = [(0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1), (0, 0, 1), (1, 1, 1), (1, 0, 0), (0, 1, 0)]
_PAR2 = [(0, 0), (1, 1), (1, 0), (0, 1)]

# Eqs. ss1-ss4 read as: d/dt X + sum_j c_j * D_j Y_j, with D_j the centred
# difference over one cell along j.  Entries: (direction, coefficient
# multiplying r_direction, source component).
_RULES3 = {
    "A": [("z", 1.0, "C"), ("x", 1.0, "D"), ("y", -1j, "D")],
    "B": [("z", -1.0, "D"), ("x", 1.0, "C"), ("y", 1j, "C")],
    "C": [("z", 1.0, "A"), ("x", 1.0, "B"), ("y", -1j, "B")],
    "D": [("z", -1.0, "B"), ("x", 1.0, "A"), ("y", 1j, "A")],
}
# Eqs. scheme2Deq-scheme4thline, difference terms on the left-hand side
_RULES2 = {
    "u": [("x", 1.0, "v"), ("y", -1j, "v")],
    "v": [("x", 1.0, "u"), ("y", 1j, "u")],
}


def _factors(a_fn, rule, pos2, axis, e2):
    """(factor of the + neighbour, factor of the - neighbour) for the row at
    doubled position pos2 along axis (index), e2 the unit step in doubled units."""
    if a_fn is None:
        return 1.0, 1.0
    if rule == "linear":
        aj = a_fn(*[p / 2.0 for p in pos2])[axis]
        return 1.0 - 0.5j * aj, 1.0 + 0.5j * aj
    mp = [(p + 0.5 * e) / 2.0 for p, e in zip(pos2, e2)]
    mm = [(p - 0.5 * e) / 2.0 for p, e in zip(pos2, e2)]
    return np.exp(-0.5j * a_fn(*mp)[axis]), np.exp(0.5j * a_fn(*mm)[axis])


class Dense3:
    def __init__(self, nx, ny, nz, dt, dx=1.0, dy=1.0, dz=1.0, a_fn=None, rule="exact", zero_bc=False):
        self.a_fn, self.rule, self.zero_bc = a_fn, rule, zero_bc
        self.nx, self.ny, self.nz = nx, ny, nz
        self.dt = dt
        self.r = {"x": dt / dx, "y": dt / dy, "z": dt / dz}
        self.nc = nx * ny * nz
        self.sites = []          # (component, doubled position)
        self.index = {}
        comps = "AABBCCDD"
        for a in range(8):
            for k in range(nz):
                for j in range(ny):
                    for i in range(nx):
                        pos = (2 * i + _PAR3[a][0], 2 * j + _PAR3[a][1], 2 * k + _PAR3[a][2])
                        self.index[(comps[a], pos)] = len(self.sites)
                        self.sites.append((comps[a], pos))
        self.dim = len(self.sites)
        self.K = self._difference_operator()

    def _find(self, comp, pos):
        """Row index of the site, or None for a zero ghost outside the lattice."""
        if self.zero_bc and not all(0 <= p < 2 * n for p, n in zip(pos, (self.nx, self.ny, self.nz))):
            return None
        key = (comp, (pos[0] % (2 * self.nx), pos[1] % (2 * self.ny), pos[2] % (2 * self.nz)))
        return self.index[key]

    def _difference_operator(self):
        """K with (K psi)_s = S_X(s) for every site s (both sheets)."""
        K = np.zeros((self.dim, self.dim), np.complex128)
        unit = {"x": (1, 0, 0), "y": (0, 1, 0), "z": (0, 0, 1)}
        axis = {"x": 0, "y": 1, "z": 2}
        for s, (comp, pos) in enumerate(self.sites):
            for d, c, src in _RULES3[comp]:
                e = unit[d]
                plus = (pos[0] + e[0], pos[1] + e[1], pos[2] + e[2])
                minus = (pos[0] - e[0], pos[1] - e[1], pos[2] - e[2])
                fp, fm = _factors(self.a_fn, self.rule, pos, axis[d], e)
                ip, im = self._find(src, plus), self._find(src, minus)
                if ip is not None:
                    K[s, ip] += c * self.r[d] * fp
                if im is not None:
                    K[s, im] -= c * self.r[d] * fm
        return K

    def step_matrix(self, theta):
        """One full step for per-site theta (vector of length dim; first half on
        sheet n for A,B, second half on sheet n+1/2 for C,D); theta may be
        complex (a complex potential)."""
        theta = np.asarray(theta)
        theta = theta.astype(np.complex128) if np.iscomplexobj(theta) else theta.astype(np.float64)
        h = self.dim // 2
        alpha = (1 - 1j * theta) / (1 + 1j * theta)
        beta = 1.0 / (1 + 1j * theta)
        M1 = np.eye(self.dim, dtype=np.complex128)
        M1[:h, :h] = np.diag(alpha[:h])
        M1[:h, h:] = -beta[:h, None] * self.K[:h, h:]
        M2 = np.eye(self.dim, dtype=np.complex128)
        M2[h:, h:] = np.diag(alpha[h:])
        M2[h:, :h] = -beta[h:, None] * self.K[h:, :h]
        return M2 @ M1

    def gram(self):
        """G with E_r = psi^H G psi (Eq. EPM): identity minus half the Hermitian
        part of the A,B-rows block of K."""
        h = self.dim // 2
        G = np.eye(self.dim, dtype=np.complex128)
        K1 = self.K[:h, h:]
        G[:h, h:] -= 0.5 * K1
        G[h:, :h] -= 0.5 * K1.conj().T
        return G

    def pack(self, arrays):
        return np.concatenate([np.asarray(a).reshape(-1) for a in arrays])

    def unpack(self, vec):
        shp = (self.nz, self.ny, self.nx)
        return [vec[a * self.nc:(a + 1) * self.nc].reshape(shp).copy() for a in range(8)]


class Dense2:
    def __init__(self, nx, ny, dt, dx=1.0, dy=1.0, a_fn=None, rule="exact", zero_bc=False):
        self.a_fn, self.rule, self.zero_bc = a_fn, rule, zero_bc
        self.nx, self.ny = nx, ny
        self.dt = dt
        self.r = {"x": dt / dx, "y": dt / dy}
        self.nc = nx * ny
        self.sites = []
        self.index = {}
        comps = "uuvv"
        for a in range(4):
            for j in range(ny):
                for i in range(nx):
                    pos = (2 * i + _PAR2[a][0], 2 * j + _PAR2[a][1])
                    self.index[(comps[a], pos)] = len(self.sites)
                    self.sites.append((comps[a], pos))
        self.dim = len(self.sites)
        self.K = self._difference_operator()

    def _find(self, comp, pos):
        if self.zero_bc and not (0 <= pos[0] < 2 * self.nx and 0 <= pos[1] < 2 * self.ny):
            return None
        return self.index[(comp, (pos[0] % (2 * self.nx), pos[1] % (2 * self.ny)))]

    def _difference_operator(self):
        K = np.zeros((self.dim, self.dim), np.complex128)
        unit = {"x": (1, 0), "y": (0, 1)}
        axis = {"x": 0, "y": 1}
        for s, (comp, pos) in enumerate(self.sites):
            for d, c, src in _RULES2[comp]:
                e = unit[d]
                fp, fm = _factors(self.a_fn, self.rule, pos, axis[d], e)
                ip = self._find(src, (pos[0] + e[0], pos[1] + e[1]))
                im = self._find(src, (pos[0] - e[0], pos[1] - e[1]))
                if ip is not None:
                    K[s, ip] += c * self.r[d] * fp
                if im is not None:
                    K[s, im] -= c * self.r[d] * fm
        return K

    def step_matrix(self, theta):
        theta = np.asarray(theta)
        theta = theta.astype(np.complex128) if np.iscomplexobj(theta) else theta.astype(np.float64)
        h = self.dim // 2
        alpha = (1 - 1j * theta) / (1 + 1j * theta)
        beta = 1.0 / (1 + 1j * theta)
        M1 = np.eye(self.dim, dtype=np.complex128)
        M1[:h, :h] = np.diag(alpha[:h])
        M1[:h, h:] = -beta[:h, None] * self.K[:h, h:]
        M2 = np.eye(self.dim, dtype=np.complex128)
        M2[h:, h:] = np.diag(alpha[h:])
        M2[h:, :h] = -beta[h:, None] * self.K[h:, :h]
        return M2 @ M1

    def gram(self):
        """E_r = ||u||^2 + ||v||^2 - Re sum_u conj(u) S_u(v) as a Hermitian form."""
        h = self.dim // 2
        G = np.eye(self.dim, dtype=np.complex128)
        K1 = self.K[:h, h:]
        G[:h, h:] -= 0.5 * K1
        G[h:, :h] -= 0.5 * K1.conj().T
        return G

    def pack(self, arrays):
        return np.concatenate([np.asarray(a).reshape(-1) for a in arrays])

    def unpack(self, vec):
        shp = (self.ny, self.nx)
        return [vec[a * self.nc:(a + 1) * self.nc].reshape(shp).copy() for a in range(4)]
