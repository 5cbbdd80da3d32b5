"""Failure detection for long runs.

With real m and V the scheme conserves the functional E_r exactly up to
rounding (Sect. 2.2 for 3D, Sect. 3 for 2D), so a change of E_r beyond the
rounding level, or a value that is no longer finite, means the run has gone
wrong: a corrupted input, an unstable time step, a fault.  run_watched checks
E_r every few steps (evaluated in the step launch itself where the kernel can
fuse it) and stops at the first check that fails, after restoring the state
of the last check that passed.  With an absorbing (complex) potential E_r
decays by design and this check does not apply.
"""
from __future__ import annotations

import math


class DriftError(RuntimeError):
    """E_r left the tolerance (or became non-finite) at a check."""

    def __init__(self, step: int, value: float, reference: float, drift: float, restored_step):
        self.step, self.value, self.reference, self.drift = step, value, reference, drift
        self.restored_step = restored_step
        where = ("state restored to step %d" % restored_step) if restored_step is not None else "state left as is"
        super().__init__("E_r = %r at step %d against %r at step 0 (relative change %.3e); %s"
                         % (value, step, reference, drift, where))


def run_watched(lat, n: int, every: int = 10, tol: float = 1e-5, recover="snapshot"):
    """Advance lat by n steps, checking E_r every `every` steps and after the
    last against its value at the start (relative change <= tol, finite).

    On a failed check the state of the last passed check is restored, then
    DriftError is raised:
      recover="snapshot"  a device copy of the state taken at every passed check
                          (one more state's memory; bitwise),
      recover="reverse"   the exact reverse step over the steps since (no extra
                          memory; the inverse up to rounding; it cannot undo a
                          non-finite value),
      recover=None        the state is left as the failed check found it.
    Returns (E_r at the start, E_r at the end, largest relative change seen).
    """
    if getattr(lat, "zh", 0):
        raise ValueError("a z-slab's E_r is not conserved on its own; watch the whole decomposition")
    if every < 1 or n < 0:
        raise ValueError("need every >= 1 and n >= 0")
    if recover not in ("snapshot", "reverse", None):
        raise ValueError("recover must be 'snapshot', 'reverse' or None")
    e0 = float(lat.norm()[0])
    snap = [t.clone() for t in lat.state()] if recover == "snapshot" else None
    done, worst, e = 0, 0.0, e0
    while done < n:
        k = min(every, n - done)
        e = float(lat.step_norm(k)[0])
        drift = abs(e - e0) / abs(e0) if e0 != 0.0 else abs(e)
        if not math.isfinite(e) or not drift <= tol:
            restored = None
            if recover == "snapshot":
                lat.load(snap)
                restored = done
            elif recover == "reverse":
                lat.reverse(k)
                restored = done
            raise DriftError(done + k, e, e0, drift, restored)
        worst = max(worst, drift)
        done += k
        if snap is not None and done < n:
            for s, t in zip(snap, lat.state()):
                s.copy_(t)
    return e0, e, worst
