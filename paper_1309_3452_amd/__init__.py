"""MI355X (gfx950) implementation of the single-cone staggered leap-frog scheme
for the time-dependent Dirac equation (Hammer, Poetz, Arnold, arXiv:1309.3452).

The computation runs in libdirac.so (hand-written HIP kernels behind a C ABI,
include/dirac.h); these modules marshal torch-owned device memory and streams
into it.  Importing is cheap; the library is loaded on first use and its
absence raises ImportError.
"""
from ._abi import DiracError, lib  # noqa: F401
from .lattice import Lattice, Lattice2D, Lattice3D, stream_copy  # noqa: F401
from .batch import BatchedLattices  # noqa: F401
from .autograd import DiracLoss, potential_gradient  # noqa: F401
from .slabs import SlabDecomposition  # noqa: F401
from .checkpoint import load_checkpoint, save_checkpoint  # noqa: F401
from .watch import DriftError, run_watched  # noqa: F401

__all__ = ["Lattice", "Lattice2D", "Lattice3D", "BatchedLattices", "DiracLoss", "potential_gradient",
           "SlabDecomposition", "DiracError", "lib", "save_checkpoint", "load_checkpoint", "DriftError",
           "run_watched", "stream_copy"]
