"""Closed forms the paper fixes for constant coefficients (test helpers).

* Substitution rules, Sect. 2.1 (Eqs. substE, substp, substm): a discrete time
  difference becomes -(2i/dt) sin(w dt/2), a spatial one (2i/d_j) sin(k_j d_j/2),
  the time average cos(w dt/2).
* Dispersion, Eq. (pwdsip): w = +-(2/dt) arcsin X,
  X^2 = (m^2 + |P|^2) / (m^2 + (2/dt)^2), with P_j = (2/d_j) sin(k_j d_j/2).
  Sect. 3 states the same for (2+1)D; its printed denominator is garbled and is
  read as m^2 + (2/dt)^2 like the 3D one.
* Eigenkets psi^(1..4) after Eq. (pwdsip): the continuum spinors with E -> E(w),
  p -> P, m -> m cos(w dt/2).
* Plane waves on the lattice, Eq. (planeonlattice): every amplitude carries
  exp(i k.x - i w t) at its own physical position and time sheet.

hbar = c = 1 throughout.
"""
from __future__ import annotations

import math

import numpy as np

OFF3 = [(0.0, 0.0, 0.0), (0.5, 0.5, 0.0), (0.5, 0.0, 0.5), (0.0, 0.5, 0.5),
        (0.0, 0.0, 0.5), (0.5, 0.5, 0.5), (0.5, 0.0, 0.0), (0.0, 0.5, 0.0)]
OFF2 = [(0.0, 0.0), (0.5, 0.5), (0.5, 0.0), (0.0, 0.5)]


def lattice_momentum(k, d=1.0):
    return 2.0 / d * np.sin(np.asarray(k, np.float64) * d / 2.0)


def X_of(P2, m, dt):
    return np.sqrt((m * m + P2) / (m * m + (2.0 / dt) ** 2))


def omega(k, m, dt, d=(1.0, 1.0, 1.0)):
    """Positive branch of Eq. (pwdsip)."""
    P = [lattice_momentum(kj, dj) for kj, dj in zip(k, d)]
    P2 = sum(p * p for p in P)
    return 2.0 / dt * np.arcsin(X_of(P2, m, dt))


def eigenket3(k, m, dt, branch, d=(1.0, 1.0, 1.0)):
    """(w, [A, B, C, D]) of psi^(branch), branch in 1..4; 1,2 positive energy."""
    Px, Py, Pz = [lattice_momentum(kj, dj) for kj, dj in zip(k, d)]
    X = X_of(Px * Px + Py * Py + Pz * Pz, m, dt)
    E = 2.0 / dt * X                       # |E(w)|
    mk = m * np.sqrt(1.0 - X * X)          # m(w) = m cos(w dt / 2)
    den = E + mk
    w = 2.0 / dt * np.arcsin(X)
    if branch == 1:
        return w, [1.0, 0.0, Pz / den, (Px + 1j * Py) / den]
    if branch == 2:
        return w, [0.0, 1.0, (Px - 1j * Py) / den, -Pz / den]
    if branch == 3:
        return -w, [-Pz / den, -(Px + 1j * Py) / den, 1.0, 0.0]
    if branch == 4:
        return -w, [-(Px - 1j * Py) / den, Pz / den, 0.0, 1.0]
    raise ValueError(branch)


def eigenket2(k, m, dt, branch, d=(1.0, 1.0)):
    """(w, [u, v]); branch 1 positive, 2 negative energy."""
    Px, Py = [lattice_momentum(kj, dj) for kj, dj in zip(k, d)]
    X = X_of(Px * Px + Py * Py, m, dt)
    E = 2.0 / dt * X
    mk = m * np.sqrt(1.0 - X * X)
    w = 2.0 / dt * np.arcsin(X)
    if branch == 1:
        return w, [1.0, (Px + 1j * Py) / (E + mk)]
    return -w, [-(Px - 1j * Py) / (E + mk), 1.0]


def plane_wave3(shape, k, amps, w, dt, t_shift=0.0):
    """State arrays (A0..D1) of a lattice plane wave: A,B on sheet -1/2, C,D on 0
    (shifted by t_shift), cell-unit spacing, shape = (nz, ny, nx)."""
    nz, ny, nx = shape
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = []
    for a in range(8):
        ox, oy, oz = OFF3[a]
        t = (-0.5 * dt if a < 4 else 0.0) + t_shift
        ph = k[0] * (ii + ox) + k[1] * (jj + oy) + k[2] * (kk + oz) - w * t
        out.append(np.ascontiguousarray(amps[a // 2] * np.exp(1j * ph), dtype=np.complex128))
    return out


def plane_wave2(shape, k, amps, w, dt, t_shift=0.0):
    ny, nx = shape
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    out = []
    for a in range(4):
        ox, oy = OFF2[a]
        t = (-0.5 * dt if a < 2 else 0.0) + t_shift
        ph = k[0] * (ii + ox) + k[1] * (jj + oy) - w * t
        out.append(np.ascontiguousarray(amps[a // 2] * np.exp(1j * ph), dtype=np.complex128))
    return out


def growth_factor(X):
    """|lambda| per step of the growing mode when X > 1: w dt/2 = pi/2 - i acosh X."""
    return float((X + np.sqrt(X * X - 1.0)) ** 2)


def rel_l2(a_list, b_list):
    num = sum(float(np.sum(np.abs(np.asarray(a) - np.asarray(b)) ** 2)) for a, b in zip(a_list, b_list))
    den = sum(float(np.sum(np.abs(np.asarray(b)) ** 2)) for b in b_list)
    return np.sqrt(num / den)


# --------------------------------------------------------------------------
# Gauge links (vector potential): construction of link arrays from site data.
# --------------------------------------------------------------------------
#: neighbour displacements (cell units) of the link terms, in order
LINK_DIRS3 = [(0, 0, 0.5), (0, 0, -0.5), (0.5, 0, 0), (-0.5, 0, 0), (0, 0.5, 0), (0, -0.5, 0)]
LINK_DIRS2 = [(0.5, 0), (-0.5, 0), (0, 0.5), (0, -0.5)]


def _site3(shape, pos):
    """(array, k, j, i) of the 3D site at physical position pos (cell units)."""
    nz, ny, nx = shape
    x, y, z = pos
    fr = (x % 1.0, y % 1.0, z % 1.0)
    for a, o in enumerate(OFF3):
        if all(abs(f - oo) < 1e-9 for f, oo in zip(fr, o)):
            return a, int(np.floor(z)) % nz, int(np.floor(y)) % ny, int(np.floor(x)) % nx
    raise ValueError("not a site")


def _site2(shape, pos):
    ny, nx = shape
    x, y = pos
    fr = (x % 1.0, y % 1.0)
    for a, o in enumerate(OFF2):
        if all(abs(f - oo) < 1e-9 for f, oo in zip(fr, o)):
            return a, int(np.floor(y)) % ny, int(np.floor(x)) % nx
    raise ValueError("not a site")


def links_from_site_phase3(shape, chi):
    """Pure-gauge links U[6 a + t] = exp(i (chi(Y) - chi(X))) for the A,B site X
    of array a and its term-t neighbour Y; chi: 8 real arrays (one per array)."""
    nz, ny, nx = shape
    out = []
    for a in range(4):
        for d in LINK_DIRS3:
            U = np.empty(shape, np.complex128)
            for k in range(nz):
                for j in range(ny):
                    for i in range(nx):
                        pos = (i + OFF3[a][0] + d[0], j + OFF3[a][1] + d[1], k + OFF3[a][2] + d[2])
                        b, kk, jj, ii = _site3(shape, pos)
                        U[k, j, i] = np.exp(1j * (chi[b][kk, jj, ii] - chi[a][k, j, i]))
            out.append(U)
    return out


def links_from_site_phase2(shape, chi):
    ny, nx = shape
    out = []
    for a in range(2):
        for d in LINK_DIRS2:
            U = np.empty(shape, np.complex128)
            for j in range(ny):
                for i in range(nx):
                    pos = (i + OFF2[a][0] + d[0], j + OFF2[a][1] + d[1])
                    b, jj, ii = _site2(shape, pos)
                    U[j, i] = np.exp(1j * (chi[b][jj, ii] - chi[a][j, i]))
            out.append(U)
    return out


def links_uniform_field2(shape, flux):
    """Links of a static, non-pure-gauge field in 2D: every half-link along x at
    height y (cell units) carries the phase exp(-i flux y dx) (a Landau-gauge
    vector potential A_x = -B y; dx = +-1/2 the link's signed length), y links
    carry 1.  The phase around a cell is not 1: no gauge transformation removes
    it."""
    ny, nx = shape
    out = []
    for a in range(2):
        for d in LINK_DIRS2:
            jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
            y = jj + OFF2[a][1] + 0.5 * d[1]
            out.append(np.ascontiguousarray(np.exp(-1j * flux * y * d[0]) * np.ones(shape)))
    return out


def links_from_potential3(shape, a_fn):
    """Peierls links of a vector potential: U(X -> Y) = exp(-i a_j(M) d_j) with
    a = q A/(hbar c) (per cell length) evaluated at the half-link midpoint M and
    d = Y - X = +-1/2 along axis j (midpoint rule for the line integral).
    a_fn(x, y, z) -> (ax, ay, az) on arrays of physical coordinates."""
    nz, ny, nx = shape
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = []
    for a in range(4):
        for d in LINK_DIRS3:
            mx = ii + OFF3[a][0] + 0.5 * d[0]
            my = jj + OFF3[a][1] + 0.5 * d[1]
            mz = kk + OFF3[a][2] + 0.5 * d[2]
            ax, ay, az = a_fn(mx, my, mz)
            out.append(np.ascontiguousarray(np.exp(-1j * (ax * d[0] + ay * d[1] + az * d[2]))))
    return out


def links_from_potential2(shape, a_fn):
    """2D version of links_from_potential3; a_fn(x, y) -> (ax, ay)."""
    ny, nx = shape
    jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    out = []
    for a in range(2):
        for d in LINK_DIRS2:
            mx = ii + OFF2[a][0] + 0.5 * d[0]
            my = jj + OFF2[a][1] + 0.5 * d[1]
            ax, ay = a_fn(mx, my)
            out.append(np.ascontiguousarray(np.exp(-1j * (ax * d[0] + ay * d[1]))))
    return out


def smooth_potential3(shape, amp, seed):
    """A smooth periodic vector potential with nonzero curl: a few low Fourier
    modes per component with random phases."""
    nz, ny, nx = shape
    g = np.random.default_rng(seed)
    ph = g.uniform(0, 2 * np.pi, (3, 3))
    def fn(x, y, z):
        return (amp * np.sin(2 * np.pi * y / ny + ph[0, 0]) * np.cos(2 * np.pi * z / nz + ph[0, 1]),
                amp * np.sin(2 * np.pi * z / nz + ph[1, 0]) * np.cos(2 * np.pi * x / nx + ph[1, 1]),
                amp * np.sin(2 * np.pi * x / nx + ph[2, 0]) * np.cos(2 * np.pi * y / ny + ph[2, 1]))
    return fn


# --------------------------------------------------------------------------
# Continuum (2+1)D Dirac scattering at a potential step (Sect. 5)
# --------------------------------------------------------------------------
def dirac2d_transmission(E, ky, v_of_x, x0, x1, m=0.0, slices=800):
    """Flux transmission and reflection of the continuum equation of Sect. 3,
    H = sigma_x p_x + sigma_y p_y + m sigma_z + V(x), for energy E and
    conserved k_y, through the profile V(x) between x0 (incidence side) and x1.
    With psi = (u, v) exp(i k_y y), H psi = E psi is the first-order system
    (u, v)' = [[k_y, i(E + m - V)], [i(E - m - V), -k_y]] (u, v), integrated
    exactly on slices of constant V (midpoint value); the x flux is
    2 Re(conj(u) v).  E and ky may be arrays (broadcast); returns (T, R) of
    their shape (floats for scalar input)."""
    E, ky = np.broadcast_arrays(np.asarray(E, np.float64), np.asarray(ky, np.float64))
    shape = E.shape
    E, ky = E.ravel(), ky.ravel()
    N = E.size

    def mats(V):
        A = np.empty((N, 2, 2), np.complex128)
        A[:, 0, 0], A[:, 1, 1] = ky, -ky
        A[:, 0, 1] = 1j * (E + m - V)
        A[:, 1, 0] = 1j * (E - m - V)
        return A

    xs = np.linspace(x0, x1, slices + 1)
    P = np.broadcast_to(np.eye(2, dtype=np.complex128), (N, 2, 2)).copy()
    for q in range(slices):
        h = xs[q + 1] - xs[q]
        V = v_of_x(0.5 * (xs[q] + xs[q + 1]))
        A = mats(V)
        kap = np.sqrt((ky * ky - (E - V) ** 2 + m * m).astype(np.complex128))   # A^2 = kap^2 I
        small = np.abs(kap) < 1e-14
        sk = np.where(small, h, np.sinh(kap * h) / np.where(small, 1.0, kap))
        step = np.cosh(kap * h)[:, None, None] * np.eye(2) + sk[:, None, None] * A
        P = step @ P

    def modes(V):
        lam, vec = np.linalg.eig(mats(V))
        j = 2.0 * (np.conj(vec[:, 0, :]) * vec[:, 1, :]).real          # (N, 2)
        return lam, vec, j

    rows = np.arange(N)
    lamL, vecL, jL = modes(v_of_x(x0))
    inc = np.argmax(jL, axis=1)
    ref = 1 - inc
    lamR, vecR, jR = modes(v_of_x(x1))
    prop = np.all(np.abs(lamR.real) < 1e-9, axis=1)
    tr = np.where(prop, np.argmax(jR, axis=1), np.argmin(lamR.real, axis=1))
    e_in, e_ref, e_tr = vecL[rows, :, inc], vecL[rows, :, ref], vecR[rows, :, tr]
    Pe_ref = np.einsum("nij,nj->ni", P, e_ref)
    Pe_in = np.einsum("nij,nj->ni", P, e_in)
    M = np.stack([e_tr, -Pe_ref], axis=2)
    sol = np.linalg.solve(M, Pe_in[:, :, None])[:, :, 0]
    t, r = sol[:, 0], sol[:, 1]
    j_in = jL[rows, inc]
    T = np.where(prop, np.abs(t) ** 2 * jR[rows, tr] / j_in, 0.0)
    R = np.abs(r) ** 2 * np.abs(jL[rows, ref]) / j_in
    if shape == ():
        return float(T[0]), float(R[0])
    return T.reshape(shape), R.reshape(shape)


def klein_packet_expectation(E0, phi, sigma, V0, v_of_x, half_width=40.0, grid=41):
    """Transmitted probability and mean direction (degrees from +x) of the
    transmitted part for a massless packet exp(-|x-c|^2/(4 sigma^2)) exp(i k0.x)
    times the positive-energy spinor at k0 (|k0| = E0, angle phi): momentum
    weights exp(-2 sigma^2 |k - k0|^2) times the spinor's overlap cos^2(dphi/2)
    with the positive-energy state at k, energy |k|, transmission from
    dirac2d_transmission, and the transmitted group velocity (|q_x|, -k_y)/|q|
    of the hole state behind a step V0 > E.  v_of_x: the step profile with its
    centre at x = 0."""
    s = 1.0 / (2.0 * sigma)
    g = np.linspace(-5 * s, 5 * s, grid)
    dx, dy = np.meshgrid(g, g, indexing="ij")
    kx, ky = E0 * math.cos(phi) + dx, E0 * math.sin(phi) + dy
    wgt = np.exp(-2.0 * sigma ** 2 * (dx * dx + dy * dy))
    fwd = kx > 0
    k = np.hypot(kx, ky)[fwd]
    kyf = ky[fwd]
    c2 = np.cos((np.arctan2(kyf, kx[fwd]) - phi) / 2.0) ** 2
    T, _ = dirac2d_transmission(k, kyf, v_of_x, -half_width, half_width)
    wt = wgt[fwd] * c2 * T
    q = np.abs(k - V0)
    ok = q > np.abs(kyf)
    qx = np.sqrt(np.where(ok, q * q - kyf * kyf, 0.0))
    vx = float(np.sum(np.where(ok, wt * qx / q, 0.0)))
    vy = float(np.sum(np.where(ok, wt * (-kyf) / q, 0.0)))
    return float(np.sum(wt) / np.sum(wgt)), math.degrees(math.atan2(vy, vx))
