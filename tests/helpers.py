"""Small helpers shared by the test modules (no method arithmetic)."""
import numpy as np


def bins_np(x, lo, hi, nb):
    """Vectorised form of the binning rule: floor((x - lo) / wb) with
    wb = (hi - lo) / nb in FP64; negative -> nb (underflow); >= nb or
    NaN -> nb + 1 (overflow).  Checked against the oracle in the CPU suite."""
    x = np.asarray(x, dtype=np.float64)
    q = (x - lo) / ((hi - lo) / nb)
    inside = q < nb
    return np.where(q < 0, nb, np.where(inside, np.floor(np.where(inside, q, 0)), nb + 1)).astype(np.int32)
