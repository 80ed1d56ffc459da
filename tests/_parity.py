"""Element-by-element comparison of GPU results with the oracle.

Every bound here is per element: for a column-major (rows, N) array whose
columns are independent instances,

    |got[i, j] - ref[i, j]| <= rtol * |ref[i, j]| + atol * rms_i(ref[:, j])

The absolute term is scaled by the column's root-mean-square entry because
the FP32 (or split-BF16) rounding error of a product with an operator row is
relative to the magnitudes that enter the dot product, i.e. to the size of
the instance's whole vector, not to the entry itself: an entry near zero
(off the support) can only be expected to sit within some ulps of that
scale.  With all |errors| below atol * rms the column's relative l2 error is
below atol too, so this bound is never more than twice as loose as the block
norm it replaces, and one bad row or a few bad entries cannot hide in it.
"""
import numpy as np


def _f64(a):
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.asarray(a, dtype=np.float64)


def col_excess(got, ref, rtol, atol, scale="rms"):
    """Largest ratio |got - ref| / bound over all elements (<= 1 passes) and
    the index where it occurs.  ``scale``: "rms" (rounding-type differences
    of iterates) or "l2" (converged solutions, whose error budget is the
    instance's relative l2 error: no element may use more than all of it)."""
    got, ref = _f64(got), _f64(ref)
    if got.shape != ref.shape:
        raise AssertionError(f"shape {got.shape} != {ref.shape}")
    if ref.ndim == 1:
        got, ref = got[:, None], ref[:, None]
    if scale == "l2":
        scale = np.sqrt(np.sum(ref * ref, axis=0, keepdims=True))
    else:
        scale = np.sqrt(np.mean(ref * ref, axis=0, keepdims=True))
    bound = rtol * np.abs(ref) + atol * scale
    err = np.abs(got - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(bound > 0, err / bound, np.where(err > 0, np.inf, 0.0))
    k = int(np.argmax(ratio))
    return float(ratio.flat[k]), np.unravel_index(k, ratio.shape), float(err.flat[k])


def assert_cols_close(got, ref, rtol, atol=None, what="result", scale="rms"):
    """Per-element bound with the column-scaled absolute term (atol defaults
    to rtol; scale "rms" or "l2", see col_excess)."""
    atol = rtol if atol is None else atol
    r, idx, e = col_excess(got, ref, rtol, atol, scale)
    assert r <= 1.0, (f"{what}: element {tuple(int(i) for i in idx)} off by {e:.3e}, "
                      f"{r:.2f}x the bound (rtol {rtol:g}, atol {atol:g} x column {scale})")


def assert_solution_close(got, ref, bound, what="solution"):
    """A converged solution against the exact optimum: the metric (relative
    l2 error of every instance, never of a block of instances) within
    ``bound``, and every element within the instance's budget."""
    err = rel_err_cols(got, ref)
    k = int(np.argmax(err))
    assert err[k] < bound, f"{what}: instance {k} rel. l2 error {err[k]:.3e} >= {bound:g}"
    assert_cols_close(got, ref, bound, what=what, scale="l2")


def assert_all_close(got, ref, rtol, atol=None, what="result"):
    """Per-element bound with one absolute term scaled by the RMS entry of
    the whole array (for arrays whose columns are not instances, such as a
    dictionary gradient)."""
    got, ref = _f64(got), _f64(ref)
    atol = rtol if atol is None else atol
    bound = rtol * np.abs(ref) + atol * np.sqrt(np.mean(ref * ref))
    err = np.abs(got - ref)
    k = int(np.argmax(err - bound))
    ok = np.all(err <= bound)
    assert ok, (f"{what}: element {np.unravel_index(k, err.shape)} off by {err.flat[k]:.3e} "
                f"(bound {bound.flat[k]:.3e}; rtol {rtol:g}, atol {atol:g} x rms)")


def oracle_pen(b, structure="cab"):
    """The oracle's default DALM penalty of every column of b, for a solve
    whose iterates are compared with the oracle's (the library's own
    default for large cross-and-bouquet batches is smaller)."""
    from oracle.dalm import default_beta
    b = np.asarray(b, np.float64)
    return np.array([default_beta(b[:, j], structure) for j in range(b.shape[1])], np.float32)


def rel_err_cols(got, ref):
    """Relative l2 error of each column (the metric's per-instance figure)."""
    got, ref = _f64(got), _f64(ref)
    if ref.ndim == 1:
        got, ref = got[:, None], ref[:, None]
    return np.linalg.norm(got - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)
