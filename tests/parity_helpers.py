"""Comparison helpers for the GPU parity tests (numpy only; nothing here
computes any step of the method)."""
import numpy as np

U64 = 2.0 ** -53   # unit roundoff, IEEE double
U32 = 2.0 ** -24   # unit roundoff, IEEE single


def rel_err(a, ref):
    """max |a - ref| relative to max(1, |ref|_inf)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if ref.size == 0:
        return 0.0
    return float(np.abs(a - ref).max() / max(1.0, float(np.abs(ref).max())))


def tol_f32(visits):
    """Tolerance of an FP32 result against the FP64 oracle after `visits`
    row visits per variable.  A visit that moves a variable rounds its
    update once (one fused multiply-add in FP32, within u32 of the value),
    and the projections do not amplify earlier errors (a projection onto a
    convex set is non-expansive in the W-norm).  With rounding errors that do
    not all share a sign the error of a variable grows as sqrt(visits) u32;
    the bound takes 2 u32 per sqrt(visit), for the update and the dual step
    that feeds it.  (Measured: 1e-6 at n = 4000 against a bound of 1.3e-5,
    2e-7 to 5e-7 at n = 130..500 against 4e-6 to 8e-6: rows that hold leave
    the variables unchanged, so fewer visits round than are counted.)"""
    return 2.0 * float(np.sqrt(max(1, visits))) * U32


def union_duals(gpos, gvals, opos, ovals):
    """Two sparse dual vectors (colex row index, value) as dense vectors over
    the union of their positions (a position missing on one side is 0
    there), and the positions nonzero on one side only."""
    gpos = np.asarray(gpos, dtype=np.int64)
    opos = np.asarray(opos, dtype=np.int64)
    union = np.union1d(gpos, opos)
    gv = np.zeros(union.size)
    ov = np.zeros(union.size)
    gv[np.searchsorted(union, gpos)] = gvals
    ov[np.searchsorted(union, opos)] = ovals
    only = np.setxor1d(gpos, opos)
    return union, gv, ov, only


def one_sided_bound(u, x_err, y_max, x_max, q_max):
    """Largest dual that may be nonzero on one side and exactly zero on the
    other.  A dual is clipped at zero: theta = max(y + delta q, 0) with
    delta = x_L - x_S1 - x_S2 and q = 1 / (g_L + g_S1 + g_S2) <= q_max.
    The two sides' values of y + delta q differ by the error the distances
    already carry (|delta| error <= 3 x_err, here taken 4 times over since
    x_err is measured at the end of the run) plus the rounding of this visit
    (a few u of |y| + 3 |x| q); only a value within that difference of zero
    can be clipped on one side and kept on the other."""
    return 4.0 * 3.0 * x_err * q_max + 8.0 * u * (y_max + 3.0 * x_max * q_max)
