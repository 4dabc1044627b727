"""Parity measures shared by the GPU tests.

Relative L2 = ||X - X_ref||_2 / ||X_ref||_2 over the compared (cell, slot,
component) values, reported for E and for B separately (the larger counts).
Beside the whole-array figure every parity check bounds the largest per-cell
relative L2 (each cell's slots and components against that cell's own norm),
so that a cell far weaker than the strongest one cannot hide a large relative
error inside the global sum.

Per-cell bars: the double path's field carries a few ulps of relative error per
segment and its slot coordinates equal the oracle's bit for bit, so a cell's
error stays within a few 1e-13 of its own norm (largest seen: 6.5e-13, with the
linear hold on clipped random trajectories; 2e-13 on the default path); the bar
is 2e-12.  The single-precision paths carry ~1e-7 per segment from the field
(largest per-cell figure seen: 2.2e-6); their per-cell bar is the whole-array
bar, 1e-5.
"""
import numpy as np

TOL_FP64 = 1e-12
TOL_MIXED = 1e-5
TOLS = {"fp64": TOL_FP64, "mixed": TOL_MIXED, "mixed_twosum": TOL_MIXED}
CELL_TOL_FP64 = 2e-12
CELL_TOL_MIXED = 1e-5
CELL_TOLS = {"fp64": CELL_TOL_FP64, "mixed": CELL_TOL_MIXED, "mixed_twosum": CELL_TOL_MIXED}


def rel_l2(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / (nb if nb > 0 else 1.0)


def max_cell_rel_l2(a, b):
    """Largest over cells of ||a[c] - b[c]|| / ||b[c]|| (a cell whose reference is zero
    counts 0 if a's is zero too, else infinity).  a, b: [n_cells, ...]."""
    a = np.asarray(a, dtype=np.float64).reshape(len(a), -1)
    b = np.asarray(b, dtype=np.float64).reshape(len(b), -1)
    num = np.linalg.norm(a - b, axis=1)
    den = np.linalg.norm(b, axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num > 0, np.inf, 0.0))
    return float(r.max()) if r.size else 0.0


def check_parity(Eg, Bg, Eo, Bo, tol, what, cell_tol=None):
    """Assert the whole-array relative L2 of E and B within tol and the largest
    per-cell relative L2 within cell_tol (by default the double path's per-cell bar
    for tol <= 1e-12, else the single-precision one)."""
    if cell_tol is None:
        cell_tol = CELL_TOL_FP64 if tol <= TOL_FP64 else CELL_TOL_MIXED
    eE, eB = rel_l2(Eg, Eo), rel_l2(Bg, Bo)
    cE, cB = max_cell_rel_l2(Eg, Eo), max_cell_rel_l2(Bg, Bo)
    print(f"[parity] {what}: relL2 E={eE:.3e} B={eB:.3e}; max per cell E={cE:.3e} B={cB:.3e}",
          flush=True)
    assert max(eE, eB) <= tol, (what, eE, eB)
    assert max(cE, cB) <= cell_tol, (what, "per cell", cE, cB)
