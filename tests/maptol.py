"""The parity bar of a map against a reference map: the relative L2 error (Eq. nrmsse, read
as ||a - b|| / ||b||) below `tol`, and every probe's error below `tol` times the largest
reference value, so that one bad probe cannot hide in the norm."""
import numpy as np

from oracle import metrics


def maps_close(got, ref, tol) -> bool:
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    ok_l2 = metrics.rel_l2(got, ref) < tol
    ok_max = bool(np.all(np.abs(got - ref) <= tol * np.max(np.abs(ref))))
    return bool(ok_l2 and ok_max and np.all(np.isfinite(got)))
