"""Closeness checks shared by the GPU parity tests.

Two bars on every comparison with the oracle: the relative L2 error over all
outputs (eq. error), and, target by target, the relative error of that
target's output vector, |u_i - ref_i| / max(|ref_i|, 1e-3 median_j |ref_j|).
The floor keeps targets whose reference nearly cancels from dividing by a
value far below the scale of the sum's rounding.  The per-target bar defaults
to 100 times the L2 bar: one target may sit 100 times above the average
rounding, but one target wrong by a visible amount fails even when it is
diluted in the L2 norm over thousands of targets."""
import numpy as np


def per_target_rel(ref, got, floor_frac=1e-3):
    ref = np.asarray(ref, dtype=np.float64)
    got = np.asarray(got, dtype=np.float64)
    if ref.ndim == 1:
        ref, got = ref[None, :], got[None, :]
    if ref.shape[1] == 0:
        return 0.0
    nr = np.linalg.norm(ref, axis=0)
    ne = np.linalg.norm(got - ref, axis=0)
    den = np.maximum(nr, floor_frac * np.median(nr))
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(den > 0, ne / np.where(den > 0, den, 1.0), np.where(ne > 0, np.inf, 0.0))
    return float(r.max())


def close(orc, ref, got, l2_tol, elem_tol=None, what=""):
    """Asserts both bars; returns (relative L2, largest per-target error)."""
    l2 = orc.rel_l2(ref, got)
    et = 100.0 * l2_tol if elem_tol is None else elem_tol
    mx = per_target_rel(ref, got)
    print(f"[parity] {what} rel L2 {l2:.3e} (bar {l2_tol:.0e}), "
          f"max per-target {mx:.3e} (bar {et:.0e})", flush=True)
    assert l2 <= l2_tol, (what, "relative L2", l2, l2_tol)
    assert mx <= et, (what, "per-target relative error", mx, et)
    return l2, mx
