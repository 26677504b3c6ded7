"""Shared parity check of the GPU tests: the relative Frobenius error and the
largest element error, both against the tolerance.

  rel = ||got - ref||_F / ||ref||_F   (||got - ref||_F / ||X||_F when ref ~ 0)
  max = max |got - ref| / max |ref|   (/ max |X| when ref ~ 0)

The element bound catches one wrong tile or row that a Frobenius norm over a
large matrix would average away.  It is one order above the Frobenius gate:
an output element is a length-d FP32 inner product whose rounding scales with
||X_i|| ||p_k|| rather than with |Y_ik|, so on the 1024 x 1024 frames (row
norms about 16 times the largest output element) the worst element error is
12 times the relative Frobenius error; a wrong tile or row gives O(1)."""
import numpy as np

from oracle import metrics


def errors(got, ref, X=None):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    rel = metrics.rel_fro(got, ref, X)
    scale = float(np.max(np.abs(ref))) if ref.size else 0.0
    if scale < 1e-300 and X is not None and np.size(X):
        scale = float(np.max(np.abs(np.asarray(X, dtype=np.float64))))
    diff = float(np.max(np.abs(got - ref))) if ref.size else 0.0
    mx = diff / scale if scale > 0 else diff
    return rel, mx


ELEM_FACTOR = 10.0


def check(got, ref, tol, X=None, label=""):
    """Asserts rel <= tol and max <= ELEM_FACTOR * tol; returns (rel, max) and
    prints both."""
    rel, mx = errors(got, ref, X)
    print(f"  {label} rel_fro={rel:.3e} max_elem={mx:.3e}", flush=True)
    assert np.all(np.isfinite(np.asarray(got))), f"{label}: non-finite output"
    assert rel <= tol, (label, "rel_fro", rel)
    assert mx <= ELEM_FACTOR * tol, (label, "max_elem", mx)
    return rel, mx
