"""Element-wise parity of a result array against the FP64 oracle's (test
infrastructure).

Three measures per array, all asserted by `check`:
- rel_L1 = sum |X - O| / sum |O|, the tolerance `tol` the test states;
- max_rel = max |X - O| / |O| over the elements with |O| > 1e-3 max |O|,
  so that a few badly wrong elements cannot hide in the sum.  Bound: 10 tol
  for the FP64 path (tol <= 1e-9); 1e-2 for the FP32 traversal, whose
  packages can still diverge from their FP64 twins after many scatterings
  (each event inherits the previous point's rounding and a density jump at
  a cell wall amplifies it), so a cell or pixel that one late leg of one
  package reaches carries that package's relative difference, and a
  gradient element, a sum of terms of both signs, carries it amplified by
  their cancellation (measured: up to 4e-4 for the spiral's absorbed tally
  at 1500 packages with rel_L1 3e-7; 3.1e-3 for the absorbed-tally gradient
  of a multiwavelength subset with rel_L1 4.5e-7).  A wrong cell, pixel,
  sign or missing term is off by O(1);
- the nonzero pattern: an element that is nonzero on one side only is
  allowed only if its value is negligible (at most 1e-3 tol max |O|) -- a
  zero-length segment that the two walks round differently at a cell
  corner, not a contribution that landed in another pixel or cell.
"""
import numpy as np


def rel_l1(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = np.abs(b).sum()
    return float(np.abs(a - b).sum() / den) if den > 0 else float(np.abs(a).sum())


def measures(got, ref):
    """(rel_L1, max_rel over the significant elements, largest one-sided
    nonzero value relative to max |O|, count of one-sided elements)."""
    g = np.asarray(got, dtype=np.float64).reshape(-1)
    o = np.asarray(ref, dtype=np.float64).reshape(-1)
    assert g.shape == o.shape, (g.shape, o.shape)
    scale = np.abs(o).max() if o.size else 0.0
    if scale == 0.0:
        return float(np.abs(g).sum()), 0.0, 0.0, int((g != 0).sum())
    big = np.abs(o) > 1e-3 * scale
    max_rel = float((np.abs(g - o)[big] / np.abs(o)[big]).max()) if big.any() else 0.0
    one = (g != 0) != (o != 0)
    worst = float((np.abs(g) + np.abs(o))[one].max() / scale) if one.any() else 0.0
    return rel_l1(g, o), max_rel, worst, int(one.sum())


def max_rel_bound(tol):
    return 10.0 * tol if tol <= 1e-9 else 1e-2


def check(got, ref, tol, what="", say=None):
    """Asserts rel_L1 < tol, max_rel below its bound and a nonzero pattern
    that differs only in negligible elements; returns the measures."""
    e, mr, worst, n_one = measures(got, ref)
    msg = "%s rel_L1 %.3e max_rel %.3e one-sided %d (largest %.1e of max)" % (what, e, mr, n_one, worst)
    if say is not None:
        say("  " + msg)
    assert e < tol, msg
    assert mr < max_rel_bound(tol), msg
    assert worst <= 1e-3 * tol, msg
    return e, mr, worst, n_one
