"""Checkpoint and resume of a Lattice in one safetensors file (tensors plus a
JSON header; nothing in it is executed on load).

The file holds the state arrays of the current buffer set, the coefficients in
the form the step kernels read them (the V(z) tables and mass, or the per-site
records themselves rather than the fields they were made from), the absorbing
tables, the gauge links, and the lattice's shape, dtype, dt, spacings and mode.
A lattice rebuilt from it steps to the bits of the uninterrupted run: a step
has no atomics, its reductions run in a fixed order, and nothing the kernels
read is recomputed on resume.
"""
from __future__ import annotations

import json

import numpy as np
import torch

from .lattice import Lattice

FORMAT = "dirac-lattice-1"


def _pack(tensors):
    """Complex tensors as their real views (a trailing axis of 2): the file
    format has no complex128 type.  Returns the tensors and the complex keys."""
    out, cplx = {}, []
    for k, t in tensors.items():
        if t.is_complex():
            out[k] = torch.view_as_real(t.contiguous()).contiguous()
            cplx.append(k)
        else:
            out[k] = t.contiguous()
    return out, cplx


def _unpack(tensors, cplx):
    return {k: (torch.view_as_complex(t.contiguous()) if k in cplx else t) for k, t in tensors.items()}


def save_checkpoint(lat: Lattice, path: str, step=None, extra=None) -> None:
    """Write lat's state and configuration to path.  step and extra (JSON-able)
    are stored as given and returned by load_checkpoint."""
    from safetensors.torch import save_file
    coef = lat._coef
    meta = {"format": FORMAT, "ndim": lat.ndim,
            "shape": [lat.nx, lat.ny] + ([lat.nz] if lat.ndim == 3 else []),
            "dtype": "complex64" if lat.dtype == torch.complex64 else "complex128",
            "dt": lat.dt, "d": list(lat.d), "slab": bool(lat.zh), "allow_unstable": lat.allow_unstable,
            "coef": coef["mode"], "m": coef.get("m"), "step": step, "extra": extra}
    tensors = {"state.%d" % a: t.detach().contiguous().cpu() for a, t in enumerate(lat.state())}
    if coef["mode"] == "vz":
        if coef["vz"] is not None:
            tensors["v_int"] = torch.from_numpy(np.array(coef["vz"][0]))
            tensors["v_half"] = torch.from_numpy(np.array(coef["vz"][1]))
    else:
        for a, r in enumerate(lat.theta):
            tensors["coef.%d" % a] = r.detach().contiguous().cpu()
    if lat._wz is not None:
        tensors["w_int"] = torch.from_numpy(np.array(lat._wz[0]))
        tensors["w_half"] = torch.from_numpy(np.array(lat._wz[1]))
    if lat._links is not None:
        for q, u in enumerate(lat._links):
            tensors["link.%d" % q] = u.detach().contiguous().cpu()
    packed, meta["complex"] = _pack(tensors)
    save_file(packed, path, metadata={"dirac": json.dumps(meta)})


def load_checkpoint(path: str, device="cuda"):
    """Rebuild the lattice saved in path on device: returns (lattice, step, extra)."""
    from safetensors import safe_open
    from safetensors.torch import load_file
    with safe_open(path, framework="pt") as f:
        header = f.metadata() or {}
    if "dirac" not in header:
        raise ValueError("%s is not a lattice checkpoint" % path)
    meta = json.loads(header["dirac"])
    if meta.get("format") != FORMAT:
        raise ValueError("unknown checkpoint format %r" % meta.get("format"))
    t = _unpack(load_file(path), set(meta.get("complex", [])))
    dtype = torch.complex64 if meta["dtype"] == "complex64" else torch.complex128
    lat = Lattice(tuple(meta["shape"]), dtype=dtype, dt=meta["dt"], d=meta["d"],
                  allow_unstable=meta["allow_unstable"], device=device, slab=meta["slab"])
    if meta["coef"] == "vz":
        if "v_int" in t:
            lat.set_potential_z(meta["m"], t["v_int"].numpy(), t["v_half"].numpy())
        else:
            lat.set_potential_z(meta["m"])
    else:
        lat.set_coef_records([t["coef.%d" % a] for a in range(lat.narr)])
        lat._coef["m"] = meta["m"]
    if "w_int" in t:
        lat.set_absorber_z(t["w_int"].numpy(), t["w_half"].numpy())
    nl = 24 if lat.ndim == 3 else 8
    if "link.0" in t:
        lat.set_links([t["link.%d" % q] for q in range(nl)])
    lat.load([t["state.%d" % a] for a in range(lat.narr)])
    return lat, meta["step"], meta["extra"]
