"""Small helpers shared by the test modules (no method arithmetic)."""
import math

import numpy as np

# Per-event P against the oracle: the CPU-GPU residual the paper reports
# for its double-precision weights (Sec. 2.2).
P_TOL = 1e-12


def bins_np(x, lo, hi, nb):
    """Vectorised form of the binning rule: floor((x - lo) / wb) with
    wb = (hi - lo) / nb in FP64; negative -> nb (underflow); >= nb or
    NaN -> nb + 1 (overflow).  Checked against the oracle in the CPU suite."""
    x = np.asarray(x, dtype=np.float64)
    q = (x - lo) / ((hi - lo) / nb)
    inside = q < nb
    return np.where(q < 0, nb, np.where(inside, np.floor(np.where(inside, q, 0)), nb + 1)).astype(np.int32)


def hist_tolerance(w, c, bins, nbt, n, p_tol=P_TOL, contract=(64, 16, 8)):
    """Bound on |hist_gpu - hist_oracle| per bin when the two histograms
    sum different per-event P (each within p_tol of the truth) in the same
    fixed order: p_tol * sum_b |w| for the P difference, plus the rounding
    of both summations, 2 d u sum_b |c| with d = K W / A + log2(A) +
    log2(#tiles padded) + 1 additions per contribution and u = 2^-53."""
    W, K, A = contract
    ntiles = max(1, -(-n // (W * K)))
    depth = K * W // A + int(math.log2(A)) + math.ceil(math.log2(ntiles)) + 1
    sw = np.bincount(bins, weights=np.abs(w), minlength=nbt)
    sc = np.bincount(bins, weights=np.abs(c), minlength=nbt)
    return p_tol * sw + 2 * depth * 2.0 ** -53 * sc


def assert_bits_equal(got, want, what=""):
    """Bit-for-bit equality of FP64 arrays (so -0.0 differs from +0.0);
    NaN entries only have to be NaN on both sides (their sign and payload
    are not part of any result)."""
    got = np.ascontiguousarray(got, dtype=np.float64)
    want = np.ascontiguousarray(want, dtype=np.float64)
    assert got.shape == want.shape, (got.shape, want.shape)
    gn, wn = np.isnan(got), np.isnan(want)
    np.testing.assert_array_equal(gn, wn, err_msg=f"{what}: NaN positions differ")
    gb, wb = got.view(np.uint64), want.view(np.uint64)
    bad = np.nonzero((gb != wb) & ~gn)[0]
    assert bad.size == 0, (f"{what}: {bad.size} entries differ, first at {bad[:8].tolist()}: "
                           f"got {got[bad[:4]].tolist()} want {want[bad[:4]].tolist()}")


# FP32-mixed tier (FP64 eigenvalues and phase differences, FP32 sine/cosine
# and amplitude assembly): the FP32 rounding of the amplitude inputs leaves
# N_k with ~|u m| 2^-24 ~ 4e-13 eV^4 of error, which over D_k >= ~1.7e-7
# eV^4 (near the solar resonance) is ~2e-6 per projector element; the
# hardware sine/cosine add ~1e-6.  The bound doubles the sum over the
# three projector terms.
MIXED_TOL = 2e-5
