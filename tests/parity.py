"""Error norms used by the parity tests.

Per variable v: ||got_v - ref_v|| / ||ref_v||.  A momentum (or any variable)
whose reference norm is below 1e-3 of the first variable's norm is measured
against the first variable's norm instead (a relative error of a field that
is nearly zero carries no information)."""
import numpy as np


def rel_errors(got, ref, order=2):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    base = np.linalg.norm(ref[0].ravel(), order)
    out = []
    for v in range(ref.shape[0]):
        d = np.linalg.norm((got[v] - ref[v]).ravel(), order)
        r = np.linalg.norm(ref[v].ravel(), order)
        out.append(d / (r if r >= 1e-3 * base else base))
    return np.array(out)


def max_rel(got, ref, order=2):
    return float(rel_errors(got, ref, order).max())


def state_rel(got, ref, order=2):
    """Relative error of the whole state vector (all variables together)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm((got - ref).ravel(), order) / np.linalg.norm(ref.ravel(), order))
