"""The (3+1)D conserved-functional reduction against the oracle's.

The reduction stages each plane of the eight arrays in LDS per x-y tile
(64 x 16 cells for complex64, 32 x 16 for complex128) and marches z in
chunks; the shapes below give ragged tiles in x and y, several z chunks, more
tiles than workgroups (several tiles per workgroup), lattices smaller than one
tile whose ring wraps onto itself, and odd row lengths (complex64 then takes
the unstaged reduction), with periodic and zero values outside the lattice.
dt = 1/4 is exact in both precisions, so both sides evaluate the same
functional of the same values and differ only in the order of the FP64 sums.
The same holds for the functional with gauge links (periodic lattices only;
tiles of 64 x 8 cells for complex64, 32 x 16 for complex128).
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

DT = 0.25

SHAPES = [(70, 20, 22), (64, 16, 7), (130, 9, 5), (2, 1, 1), (4, 3, 2), (6, 40, 1), (33, 17, 3),
          (2048, 544, 2)]


@pytest.fixture(scope="module")
def P():
    import paper_1309_3452_amd as P
    assert torch.cuda.is_available(), "needs a GPU"
    P.lib()
    return P


@pytest.mark.parametrize("zero_bc", [False, True])
@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("shape", SHAPES)
def test_3d_norm_vs_oracle(P, shape, dtype, zero_bc):
    nx, ny, nz = shape
    print("norm3 %s %s zero_bc=%s" % (shape, dtype, zero_bc), flush=True)
    g = np.random.default_rng(7000 + nx + 3 * ny + 7 * nz)
    f0 = [np.ascontiguousarray(g.standard_normal((nz, ny, nx)) + 1j * g.standard_normal((nz, ny, nx)))
          for _ in range(8)]
    lat = P.Lattice((nx, ny, nz), dtype=dtype, dt=DT, zero_bc=zero_bc)
    lat.load(f0)
    # the values the lattice holds (rounded to complex64 where it stores them so)
    f = [t.detach().cpu().numpy().astype(np.complex128) for t in lat.state()]
    e = lat.norm()
    eo = oracle.Lattice3(nx, ny, nz, DT, zero_bc=zero_bc).energy(f)
    assert abs(e[2] - eo[2]) <= 1e-13 * eo[2]
    for q in range(2):
        assert abs(e[q] - eo[q]) <= 1e-12 * eo[2], (q, e, eo)
    # the two forms of the functional agree exactly in exact arithmetic
    assert abs(e[0] - e[1]) <= 1e-12 * eo[2]


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("shape", SHAPES)
def test_3d_observables_vs_oracle(P, shape, dtype):
    """The observables reduction (region probability beyond z0, first moments,
    plain norm, per-component norms) against the oracle's on the same values;
    complex64 lattices with even rows read two cells per 16-byte load, odd rows
    one cell per load."""
    nx, ny, nz = shape
    print("obs3 %s %s" % (shape, dtype), flush=True)
    g = np.random.default_rng(7100 + nx + 3 * ny + 7 * nz)
    f0 = [np.ascontiguousarray(g.standard_normal((nz, ny, nx)) + 1j * g.standard_normal((nz, ny, nx)))
          for _ in range(8)]
    lat = P.Lattice((nx, ny, nz), dtype=dtype, dt=DT)
    lat.load(f0)
    f = [t.detach().cpu().numpy().astype(np.complex128) for t in lat.state()]
    ol = oracle.Lattice3(nx, ny, nz, DT)
    for z0 in (nz / 2.0, nz / 2.0 + 0.25, 0.0):
        ob = lat.observables(z0)
        oo = ol.observe(f, z0)
        for q in range(9):
            assert abs(ob[q] - oo[q]) <= 1e-12 * max(abs(oo[q]), oo[4]), (z0, q, ob[q], oo[q])


LINK_SHAPES = [(70, 20, 22), (64, 8, 7), (130, 9, 5), (2, 1, 1), (4, 3, 2), (6, 40, 1), (33, 17, 3),
               (96, 33, 4), (256, 24, 3)]


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("shape", LINK_SHAPES)
def test_3d_norm_links_vs_oracle(P, shape, dtype):
    """E_r with gauge links (Sect. 4) against the oracle's on the same values and
    links: random unit factors, so every link of every term is tested; odd
    complex64 rows take the unstaged reduction."""
    nx, ny, nz = shape
    print("norm3 links %s %s" % (shape, dtype), flush=True)
    g = np.random.default_rng(7200 + nx + 3 * ny + 7 * nz)
    tsh = (nz, ny, nx)
    f0 = [np.ascontiguousarray(g.standard_normal(tsh) + 1j * g.standard_normal(tsh)) for _ in range(8)]
    U = [np.ascontiguousarray(np.exp(1j * g.uniform(-np.pi, np.pi, tsh))) for _ in range(24)]
    lat = P.Lattice((nx, ny, nz), dtype=dtype, dt=DT)
    lat.load(f0)
    lat.set_links([torch.from_numpy(u) for u in U])
    f = [t.detach().cpu().numpy().astype(np.complex128) for t in lat.state()]
    Uc = [u.astype(np.complex64).astype(np.complex128) for u in U] if dtype == torch.complex64 else U
    e = lat.norm()
    eo = oracle.Lattice3(nx, ny, nz, DT).energy_links(f, Uc)
    assert abs(e[2] - eo[2]) <= 1e-13 * eo[2]
    for q in range(2):
        assert abs(e[q] - eo[q]) <= 1e-12 * eo[2], (q, e, eo)
    assert abs(e[0] - e[1]) <= 1e-12 * eo[2]
