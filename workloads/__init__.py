"""Seeded synthetic inputs for the benchmark configurations and the tests.

Shared by the GPU path's tests/benchmark and the CPU oracle's tests: it holds
no arithmetic of the scheme itself.  Initial states are Gaussian packets with
the continuum Dirac spinor of the packet's central momentum (an initial
condition only), potentials are plain functions sampled at the amplitude
sites, and every random number comes from numpy's PCG64 seeded per
configuration.

Site positions (cell units) of each state array, 3D: A0 (0,0,0), A1 (1/2,1/2,0),
B0 (1/2,0,1/2), B1 (0,1/2,1/2), C0 (0,0,1/2), C1 (1/2,1/2,1/2), D0 (1/2,0,0),
D1 (0,1/2,0) added to the cell index; 2D: u0 (0,0), u1 (1/2,1/2), v0 (1/2,0),
v1 (0,1/2).  A,B (u) live on time sheet -1/2, C,D (v) on sheet 0.
"""
from __future__ import annotations

import math

import numpy as np
import torch

SEED_BASE = 13093452
OFF3 = [(0.0, 0.0, 0.0), (0.5, 0.5, 0.0), (0.5, 0.0, 0.5), (0.0, 0.5, 0.5),
        (0.0, 0.0, 0.5), (0.5, 0.5, 0.5), (0.5, 0.0, 0.0), (0.0, 0.5, 0.0)]
OFF2 = [(0.0, 0.0), (0.5, 0.5), (0.5, 0.0), (0.0, 0.5)]

DT3 = 0.9 / math.sqrt(3.0)      # 0.9 x the (3+1)D bound r <= 1/sqrt(3)
DT2 = 0.9 / math.sqrt(2.0)      # 0.9 x the (2+1)D bound r <= 1/sqrt(2)


def rng(cfg_index: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + int(cfg_index))


def _min_image(x, c, n):
    """Periodic distance x - c folded into [-n/2, n/2)."""
    return torch.remainder(x - c + n / 2.0, n) - n / 2.0


def spinor3(k0, m):
    """Positive-energy, spin-up continuum spinor (A, B, C, D) at momentum k0 and
    its energy E = sqrt(m^2 + |k0|^2)."""
    kx, ky, kz = k0
    E = math.sqrt(m * m + kx * kx + ky * ky + kz * kz)
    return E, [1.0 + 0j, 0.0 + 0j, kz / (E + m) + 0j, complex(kx, ky) / (E + m)]


def spinor2(k0, m):
    kx, ky = k0
    E = math.sqrt(m * m + kx * kx + ky * ky)
    return E, [1.0 + 0j, complex(kx, ky) / (E + m)]


def packet3d(nx, ny, nz, center, sigma, k0, m, dt, dtype=torch.complex128, device="cpu", normalize=True):
    """Gaussian packet exp(-|x - c|^2 / (4 sigma^2)) exp(i k0.x) times the spinor,
    A,B carrying the extra time phase exp(i E dt/2) of sheet -1/2.  Built as a
    product of per-axis factors (fast at 512^3).  Returns 8 tensors (nz, ny, nx)."""
    E, amps = spinor3(k0, m)
    rd = torch.float64
    out = []
    for a in range(8):
        ox, oy, oz = OFF3[a]
        fac = []
        for n, o, c, k in ((nx, ox, center[0], k0[0]), (ny, oy, center[1], k0[1]), (nz, oz, center[2], k0[2])):
            x = torch.arange(n, dtype=rd, device=device) + o
            d = _min_image(x, c, n)
            fac.append(torch.exp(-d * d / (4.0 * sigma * sigma)) * torch.exp(1j * k * x))
        t_phase = complex(math.cos(E * dt / 2), math.sin(E * dt / 2)) if a < 4 else 1.0 + 0j
        amp = amps[a // 2] * t_phase
        f = (fac[2][:, None, None] * fac[1][None, :, None]) * (fac[0][None, None, :] * amp)
        out.append(f.to(dtype))
    if normalize:
        s = sum(float(torch.sum(torch.abs(t.to(torch.complex128)) ** 2)) for t in out)
        out = [t / math.sqrt(s) for t in out]
    return out


def packet2d(nx, ny, center, sigma, k0, m, dt, noise=0.0, seed=None, dtype=torch.complex128, device="cpu"):
    """(2+1)D packet; optional phase noise psi <- psi exp(i noise xi), xi ~ N(0,1)
    iid per site in array order u0, u1, v0, v1 (row-major), seeded."""
    E, amps = spinor2(k0, m)
    rd = torch.float64
    out = []
    g = np.random.default_rng(seed) if noise else None
    for a in range(4):
        ox, oy = OFF2[a]
        x = torch.arange(nx, dtype=rd) + ox
        y = torch.arange(ny, dtype=rd) + oy
        dx = _min_image(x, center[0], nx)
        dy = _min_image(y, center[1], ny)
        gx = torch.exp(-dx * dx / (4.0 * sigma * sigma)) * torch.exp(1j * k0[0] * x)
        gy = torch.exp(-dy * dy / (4.0 * sigma * sigma)) * torch.exp(1j * k0[1] * y)
        t_phase = complex(math.cos(E * dt / 2), math.sin(E * dt / 2)) if a < 2 else 1.0 + 0j
        f = gy[:, None] * gx[None, :] * (amps[a // 2] * t_phase)
        if noise:
            xi = torch.from_numpy(g.standard_normal((ny, nx)))
            f = f * torch.exp(1j * noise * xi)
        out.append(f)
    s = sum(float(torch.sum(torch.abs(t) ** 2)) for t in out)
    return [(t / math.sqrt(s)).to(dtype=dtype, device=device) for t in out]


def step_potential(nz, V0=1.5, zc=None, w=4.0):
    """Smooth electrostatic step V(z) = V0 (1 + tanh((z - zc)/w)) / 2 at z = k and
    z = k + 1/2: returns (v_int, v_half) as float64 arrays of length nz."""
    zc = nz / 2.0 if zc is None else zc
    k = np.arange(nz, dtype=np.float64)
    f = lambda z: V0 * (1.0 + np.tanh((z - zc) / w)) / 2.0
    return f(k), f(k + 0.5)


def absorber(n, width, w0, offsets=(0.0, 0.5)):
    """Imaginary potential of absorbing layers at both ends of a periodic axis
    of n cells: W = -w0 ((width - d)/width)^2 within `width` cells of the
    boundary, d the distance to it, 0 elsewhere; sampled at each offset
    (returns one float64 array of length n per offset)."""
    out = []
    for o in offsets:
        z = np.arange(n, dtype=np.float64) + o
        d = np.minimum(z, n - z)                  # distance to the periodic boundary
        w = np.where(d < width, -w0 * ((width - d) / width) ** 2, 0.0)
        out.append(w)
    return out


def hat_basis(nz, nodes=32):
    """Periodic piecewise-linear hats h_i(z) on nodes z_i = i nz/nodes: returns
    (H_int, H_half) of shape (nz, nodes) sampled at z = k and k + 1/2."""
    spacing = nz / nodes
    zi = np.arange(nodes) * spacing

    def H(z):
        d = np.abs(((z[:, None] - zi[None, :]) + nz / 2.0) % nz - nz / 2.0)
        return np.clip(1.0 - d / spacing, 0.0, None)
    k = np.arange(nz, dtype=np.float64)
    return H(k), H(k + 0.5)


# neighbour directions of the A,B link terms, in link-array order: +z, -z, +x, -x, +y, -y
LINK_DIRS3 = [(0.0, 0.0, 0.5), (0.0, 0.0, -0.5), (0.5, 0.0, 0.0), (-0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, -0.5, 0.0)]


def peierls_links3d(nx, ny, nz, amp, seed, dtype=torch.complex64, device="cpu"):
    """Gauge links of a smooth periodic vector potential with nonzero curl,
    a(x,y,z) = amp (sin(2 pi y/ny + p0) cos(2 pi z/nz + p1), sin(2 pi z/nz + p2)
    cos(2 pi x/nx + p3), sin(2 pi x/nx + p4) cos(2 pi y/ny + p5)) in radians per
    cell, phases p from the seeded generator: for A,B array a and direction t the
    factor exp(-i a_j(M) d_j), d the displacement (+-1/2 along axis j) to the
    neighbour and M the half-link midpoint.  Returns 24 tensors (nz, ny, nx),
    index 6 a + t."""
    ph = np.random.default_rng(SEED_BASE + seed).uniform(0.0, 2.0 * math.pi, 6)
    f64 = dict(dtype=torch.float64, device=device)
    out = []
    for a in range(4):
        for d in LINK_DIRS3:
            x = (torch.arange(nx, **f64) + OFF3[a][0] + 0.5 * d[0]).view(1, 1, nx)
            y = (torch.arange(ny, **f64) + OFF3[a][1] + 0.5 * d[1]).view(1, ny, 1)
            z = (torch.arange(nz, **f64) + OFF3[a][2] + 0.5 * d[2]).view(nz, 1, 1)
            if d[0] != 0.0:
                aj = amp * torch.sin(2 * math.pi * y / ny + ph[0]) * torch.cos(2 * math.pi * z / nz + ph[1]) * d[0]
            elif d[1] != 0.0:
                aj = amp * torch.sin(2 * math.pi * z / nz + ph[2]) * torch.cos(2 * math.pi * x / nx + ph[3]) * d[1]
            else:
                aj = amp * torch.sin(2 * math.pi * x / nx + ph[4]) * torch.cos(2 * math.pi * y / ny + ph[5]) * d[2]
            u = torch.polar(torch.ones((), **f64), -aj).to(dtype)
            out.append(u.expand(nz, ny, nx).contiguous())
    return out


def landau_links2d(nx, ny, nflux, dtype=torch.complex64, device="cpu"):
    """Gauge links of a uniform magnetic field in 2D, Landau gauge a_x = b y with
    b = 4 pi nflux / ny per cell (periodic across the y wrap): for u array a and
    direction t (+x, -x, +y, -y) the factor exp(-i a_x(M) d_x), d_x = +-1/2 the
    x displacement and M the half-link midpoint; y links are 1.  Returns 8 tensors
    (ny, nx), index 4 a + t."""
    b = 4.0 * math.pi * nflux / ny
    out = []
    for a in range(2):
        for d in ((0.5, 0.0), (-0.5, 0.0), (0.0, 0.5), (0.0, -0.5)):
            y = (torch.arange(ny, dtype=torch.float64, device=device) + OFF2[a][1] + 0.5 * d[1]).view(ny, 1)
            u = torch.polar(torch.ones((), dtype=torch.float64, device=device), -(b * y) * d[0])
            out.append(u.expand(ny, nx).to(dtype).contiguous())
    return out


# --------------------------------------------------------------------------
# Configurations
# --------------------------------------------------------------------------
def config1():
    """2D 128x128, complex128, m = 0, V = 0, sigma 8, centre (64,64), k0 (0.3, 0),
    phase noise 1e-3, dt = 0.9 x bound, 200 steps."""
    return dict(nx=128, ny=128, dt=DT2, m=0.0, steps=200,
                state=packet2d(128, 128, (64.0, 64.0), 8.0, (0.3, 0.0), 0.0, DT2, noise=1e-3,
                               seed=SEED_BASE + 1))


def config_step3d(n, dtype=torch.complex128, device="cpu"):
    """3D n^3 Klein-step workload (sizes 256 and 512 of the benchmark): m = 0.5,
    V(z) = 1.5 (1 + tanh((z - n/2)/4))/2, packet sigma 12 at (n/2, n/2, n/4),
    k0 = (0, 0, 0.56), dt = 0.9 x bound."""
    v_int, v_half = step_potential(n, 1.5, n / 2.0, 4.0)
    state = packet3d(n, n, n, (n / 2.0, n / 2.0, n / 4.0), 12.0, (0.0, 0.0, 0.56), 0.5, DT3,
                     dtype=dtype, device=device)
    return dict(nx=n, ny=n, nz=n, dt=DT3, m=0.5, v_int=v_int, v_half=v_half, state=state, z0=n / 2.0)


def config_klein2d(phi_deg, nx=1024, ny=512, dtype=torch.complex128, device="cpu", absorbing=False):
    """(2+1)D Klein-step scattering (Sect. 5): m = 0, a smoothed step V(x) =
    V0 (1 + tanh((x - xc)/w))/2 with V0 = 2 E0 (the step height is twice the
    packet energy in both of the paper's figures), E0 = 0.2 per cell, w = 3
    cells, xc = 400; a packet of width sigma = 30 whose centre line meets the
    step at (xc, ny/2 + 100) at angle phi_deg from the step normal (+x),
    starting 100 cells before it.  Optional absorbing frame (imaginary
    potential) of width 32 at the x boundaries (where the periodic wrap puts
    the step back down).  Returns the state, per-array V at the sites, per-array
    W (zeros without absorber) and the parameters."""
    E0, w, xc, sigma = 0.2, 3.0, 400.0, 30.0
    V0 = 2.0 * E0
    phi = math.radians(phi_deg)
    k0 = (E0 * math.cos(phi), E0 * math.sin(phi))
    c = (xc - 100.0 * math.cos(phi), ny / 2.0 + 100.0 - 100.0 * math.sin(phi))
    state = packet2d(nx, ny, c, sigma, k0, 0.0, DT2, dtype=dtype, device=device)
    v_site, w_site = [], []
    wx = absorber(nx, 32.0, 0.5, offsets=(0.0, 0.5)) if absorbing else None
    for a in range(4):
        x = np.arange(nx, dtype=np.float64) + OFF2[a][0]
        v = V0 * (1.0 + np.tanh((x - xc) / w)) / 2.0
        v_site.append(np.ascontiguousarray(np.broadcast_to(v[None, :], (ny, nx))))
        wa = wx[1 if OFF2[a][0] else 0] if absorbing else np.zeros(nx)
        w_site.append(np.ascontiguousarray(np.broadcast_to(wa[None, :], (ny, nx))))
    return dict(nx=nx, ny=ny, dt=DT2, m=0.0, E0=E0, V0=V0, w=w, xc=xc, sigma=sigma, phi=phi, k0=k0,
                state=state, v_site=v_site, w_site=w_site,
                v_of_x=lambda x: V0 * (1.0 + math.tanh((x - xc) / w)) / 2.0)


def config_adjoint(n=128, nodes=32):
    """3D adjoint workload: V(z) = sum_i p_i h_i(z) with p_i = step(z_i) + 0.05 xi_i."""
    g = rng(5)
    H_int, H_half = hat_basis(n, nodes)
    zi = np.arange(nodes) * (n / nodes)
    p = 1.5 * (1.0 + np.tanh((zi - n / 2.0) / 4.0)) / 2.0 + 0.05 * g.standard_normal(nodes)
    return dict(n=n, dt=DT3, m=0.5, H_int=H_int, H_half=H_half, p=p, z0=n / 2.0, steps=400,
                sigma=12.0, center=(n / 2.0, n / 2.0, n / 4.0), k0=(0.0, 0.0, 0.56))


SIZES4 = list(range(64, 1025, 32))


def config_batched(count=64, device="cpu", dtype=torch.complex64):
    """64 independent 2D lattices, N_x, N_y iid uniform on {64, 96, ..., 1024};
    m ~ U[0, 1]; V = sum of 4 Gaussians a exp(-|x - c|^2/(2 s^2)), a ~ U[-1, 1],
    c ~ U(box), s ~ U[N_min/16, N_min/4] (periodic distance); packet sigma N_min/16
    at (N_x/4, N_y/2), k0 = (0.3, 0); dt = 0.9 x bound; 500 steps.
    Returns a list of dicts with nx, ny, m, v_site (4 real tensors), state (4)."""
    g = rng(4)
    lats = []
    for _ in range(count):
        nx = int(g.choice(SIZES4))
        ny = int(g.choice(SIZES4))
        m = float(g.uniform(0.0, 1.0))
        nmin = min(nx, ny)
        gauss = [(float(g.uniform(-1, 1)), float(g.uniform(0, nx)), float(g.uniform(0, ny)),
                  float(g.uniform(nmin / 16.0, nmin / 4.0))) for _ in range(4)]
        lats.append(dict(nx=nx, ny=ny, m=m, gauss=gauss, sigma=nmin / 16.0))
    real = torch.float32 if dtype == torch.complex64 else torch.float64
    for L in lats:
        nx, ny = L["nx"], L["ny"]
        vs = []
        for a in range(4):
            ox, oy = OFF2[a]
            x = torch.arange(nx, dtype=torch.float64, device=device) + ox
            y = torch.arange(ny, dtype=torch.float64, device=device) + oy
            V = torch.zeros((ny, nx), dtype=torch.float64, device=device)
            for amp, cx, cy, s in L["gauss"]:
                dx = _min_image(x, cx, nx)
                dy = _min_image(y, cy, ny)
                V = V + amp * torch.exp(-(dy[:, None] ** 2 + dx[None, :] ** 2) / (2 * s * s))
            vs.append(V.to(real))
        L["v_site"] = vs
        L["state"] = packet2d(nx, ny, (nx / 4.0, ny / 2.0), L["sigma"], (0.3, 0.0), L["m"], DT2,
                              dtype=dtype, device=device)
    return lats
