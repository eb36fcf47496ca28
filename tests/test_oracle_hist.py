"""Pins of the oracle's binning and deterministic histogram (the binned PDF
of Sec. 1.1.1 and the reweighted spectrum of Sec. 2.2).

The reduction contract: tile t holds W*K consecutive events; lane l of the
tile sums events t*W*K + m*W + l in ascending m from +0.0; the W lane sums
of a bin meet in the complete binary tree over lane index; the tile
results meet in the complete binary tree over tile index, padded with +0.0.
The tiny cases below spell that definition out with Python floats (IEEE
binary64, round to nearest even) on inputs where every other order gives
other bits, so a transposed lane assignment, a reversed lane order or a
sequential tile sum fails.
"""
import math

import numpy as np
import pytest

import oracle
from helpers import bins_np
from paper_1311_7579_amd import workload


def _seq(vals):
    s = 0.0
    for v in vals:
        s += v
    return s


# ---------------------------------------------------------------- binning
def test_bin_index_edges():
    lo, hi, nb = 0.0, 3.0, 50
    wb = (hi - lo) / nb
    assert oracle.bin_index(0.0, lo, hi, nb) == 0          # lower edge is inside
    assert oracle.bin_index(-1e-300, lo, hi, nb) == nb     # underflow
    assert oracle.bin_index(-5.0, lo, hi, nb) == nb
    assert oracle.bin_index(3.0, lo, hi, nb) == nb + 1     # upper edge is outside
    assert oracle.bin_index(1e9, lo, hi, nb) == nb + 1
    assert oracle.bin_index(float("nan"), lo, hi, nb) == nb + 1
    assert oracle.bin_index(float("inf"), lo, hi, nb) == nb + 1
    assert oracle.bin_index(float("-inf"), lo, hi, nb) == nb
    assert oracle.bin_index(wb, lo, hi, nb) == 1
    assert oracle.bin_index(np.nextafter(wb, 0.0), lo, hi, nb) == 0
    assert oracle.bin_index(2.999999, lo, hi, nb) == nb - 1
    # shifted range
    assert oracle.bin_index(0.5, 0.5, 1.5, 4) == 0
    assert oracle.bin_index(0.75, 0.5, 1.5, 4) == 1
    assert oracle.bin_index(0.4999999999, 0.5, 1.5, 4) == 4


def test_bin_index_matches_floor_of_ieee_quotient():
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.uniform(-0.5, 3.5, 4000), np.arange(51) * 0.06,
                        np.nextafter(np.arange(51) * 0.06, -1.0)])
    lo, hi, nb = 0.0, 3.0, 50
    q = (x - lo) / ((hi - lo) / nb)
    want = np.where(q < 0, nb, np.where(q < nb, np.floor(np.where(q < nb, q, 0)), nb + 1)).astype(np.int32)
    np.testing.assert_array_equal(oracle.bin_indices(x, lo, hi, nb), want)


# ---------------------------------------------------------------- contract
def test_contract_lane_order_single_tile():
    big = 2.0 ** 52
    c = [1.0, big, 3.0, big, 5.0, 5.0, 0.5, 0.5]       # W = 2, K = 4, one tile
    lane0 = _seq([c[0], c[2], c[4], c[6]])              # lane 0: m = 0..3 ascending
    lane1 = _seq([c[1], c[3], c[5], c[7]])
    want = lane0 + lane1
    transposed = _seq(c[0:4]) + _seq(c[4:8])
    reversed_m = _seq([c[6], c[4], c[2], c[0]]) + _seq([c[7], c[5], c[3], c[1]])
    naive = _seq(c)
    assert want != transposed and want != reversed_m and want != naive
    got = oracle.hist_contract(c, np.zeros(8, np.int32), 1, W=2, K=4, A=2)
    assert got[0] == want


def test_contract_shared_accumulators():
    # W = 4 lanes, K = 2, A = 2 accumulators: lanes 0 and 2 share accumulator
    # 0, lanes 1 and 3 accumulator 1; additions in ascending m, then lane
    big = 2.0 ** 53
    c = [1.0, 1.0, big, big, 1.0, 1.0, 3.0, 1.0]
    acc0 = _seq([c[0], c[2], c[4], c[6]])      # m = 0: lanes 0, 2; m = 1: lanes 0, 2
    acc1 = _seq([c[1], c[3], c[5], c[7]])
    want = acc0 + acc1
    lane_major = _seq([c[0], c[4], c[2], c[6]]) + _seq([c[1], c[5], c[3], c[7]])
    private = (_seq([c[0], c[4]]) + _seq([c[1], c[5]])) + (_seq([c[2], c[6]]) + _seq([c[3], c[7]]))
    assert want != lane_major and want != private
    got = oracle.hist_contract(c, np.zeros(8, np.int32), 1, W=4, K=2, A=2)
    assert got[0] == want
    with pytest.raises(ValueError):
        oracle.hist_contract(c, np.zeros(8, np.int32), 1, W=4, K=2, A=3)


def test_contract_tile_tree_with_padding():
    # W = K = 1: every event is its own tile, so the tile tree is visible
    c4 = [0.5, 0.75, 2.0 ** 53, 1.0]
    want4 = (c4[0] + c4[1]) + (c4[2] + c4[3])
    assert want4 != _seq(c4) and want4 != _seq(c4[::-1])
    assert oracle.hist_contract(c4, np.zeros(4, np.int32), 1, W=1, K=1, A=1)[0] == want4

    c5 = [0.75, 5.0, 2.0 ** 53, 3.0, 0.75]
    want5 = ((c5[0] + c5[1]) + (c5[2] + c5[3])) + ((c5[4] + 0.0) + (0.0 + 0.0))
    assert want5 != _seq(c5) and want5 != _seq(c5[::-1])
    assert oracle.hist_contract(c5, np.zeros(5, np.int32), 1, W=1, K=1, A=1)[0] == want5


def test_contract_lane_tree_and_bins():
    # W = 4, K = 1, two bins interleaved: each bin sees its own masked tree
    c = [0.5, 2.0 ** 53, 0.75, 1.0, 3.0, 0.5, 2.0 ** 52, 1.0]   # two tiles
    b = np.array([0, 1, 0, 1, 1, 0, 1, 0], np.int32)
    t0b0 = (c[0] + 0.0) + (c[2] + 0.0)
    t0b1 = (0.0 + c[1]) + (0.0 + c[3])
    t1b0 = (0.0 + c[5]) + (0.0 + c[7])
    t1b1 = (c[4] + 0.0) + (c[6] + 0.0)
    got = oracle.hist_contract(c, b, 2, W=4, K=1, A=4)
    assert got[0] == t0b0 + t1b0
    assert got[1] == t0b1 + t1b1


def test_contract_empty_and_ragged():
    assert (oracle.hist_contract([], np.zeros(0, np.int32), 5) == 0.0).all()
    rng = np.random.default_rng(1)
    for n in (1, 63, 64, 65, 1023, 1024, 1025, 5000):
        c = rng.uniform(0, 2, n)
        b = rng.integers(0, 7, n).astype(np.int32)
        got = oracle.hist_contract(c, b, 7)
        for k in range(7):
            assert got[k] == pytest.approx(math.fsum(c[b == k]), rel=1e-14, abs=0)


def test_contract_counts_exact_and_error_bound():
    rng = np.random.default_rng(2)
    n, nbt = 300_000, 52
    b = rng.integers(0, nbt, n).astype(np.int32)
    counts = oracle.hist_contract(np.ones(n), b, nbt)
    np.testing.assert_array_equal(counts, np.bincount(b, minlength=nbt).astype(float))
    c = rng.uniform(0.0, 1.5, n)
    got = oracle.hist_contract(c, b, nbt)
    for k in range(nbt):
        exact = math.fsum(c[b == k])
        nk = int((b == k).sum())
        # accumulator chains of <= K W / A, then trees of depth log2(A) + log2(#tiles)
        chain = oracle.CONTRACT_K * oracle.CONTRACT_W // oracle.CONTRACT_A
        depth = chain + int(math.log2(oracle.CONTRACT_A)) + math.ceil(math.log2(max(2, n / 1024)))
        assert abs(got[k] - exact) <= depth * 2.0 ** -53 * exact, (k, nk)


# ---------------------------------------------------------------- fill_pdf
def test_fill_pdf_composes_prob_bins_and_contract():
    s = workload.make_sample(20_000, 9)
    p = workload.TABLE1
    hist, P = oracle.fill_pdf(p, s.L_km, s.rho_gcc, s.Ye, s.e_true, s.flags, s.weight,
                              s.e_reco, 50, 0.0, 3.0)
    np.testing.assert_array_equal(P, oracle.prob_batch(p, s.L_km, s.rho_gcc, s.Ye, s.e_true, s.flags))
    bins = oracle.bin_indices(s.e_reco, 0.0, 3.0, 50)
    c = s.weight * P          # numpy multiply: separately rounded, as the oracle's
    np.testing.assert_array_equal(hist, oracle.hist_contract(c, bins, 52))
    # with P = 1 everywhere the PDF is the plain weighted histogram
    assert hist.sum() == pytest.approx(math.fsum(c), rel=1e-13)
    assert hist[51] > 0.2 * hist.sum()   # E_reco > 3 GeV tail of the log-uniform spectrum


def test_vectorised_bin_rule_matches_oracle():
    x = np.random.default_rng(0).uniform(-0.5, 3.5, 20_000)
    x[:3] = [0.0, 3.0, np.nan]
    np.testing.assert_array_equal(bins_np(x, 0.0, 3.0, 50), oracle.bin_indices(x, 0.0, 3.0, 50))
    x2 = np.random.default_rng(1).uniform(0.0, 10.0, 5_000)
    np.testing.assert_array_equal(bins_np(x2, 0.5, 9.5, 37), oracle.bin_indices(x2, 0.5, 9.5, 37))


def test_batched_bin_loop_equals_scalar_rule():
    """The one-call form of the bin rule gives, element by element, what
    the scalar rule gives (edges, their neighbours, NaN, infinities, -0.0,
    with and without an energy scale)."""
    lo, hi, nb = 0.0, 3.0, 50
    wb = (hi - lo) / nb
    edges = np.arange(-2, nb + 3) * wb
    x = np.concatenate([edges, np.nextafter(edges, np.inf), np.nextafter(edges, -np.inf),
                        [np.nan, np.inf, -np.inf, -0.0, 1e300, -1e300, 5e-324],
                        np.random.default_rng(3).uniform(-0.5, 3.5, 3000)])
    for es in (0.0, 0.013, -0.021):
        want = [oracle.bin_index_scaled(v, lo, hi, nb, e_scale=es) for v in x]
        np.testing.assert_array_equal(oracle.bin_indices(x, lo, hi, nb, e_scale=es), want)


# ---------------------------------------------------------------- Eq. (2)
def test_poisson_nll_matches_library_logpmf():
    import scipy.stats
    rng = np.random.default_rng(12)
    mu = rng.uniform(0.1, 300.0, 50)
    d = rng.poisson(mu).astype(float)
    want = -2.0 * scipy.stats.poisson.logpmf(d, mu).sum()
    assert oracle.poisson_nll(mu, d) == pytest.approx(want, rel=1e-13)


def test_poisson_nll_empty_bins_and_best_normalisation():
    assert oracle.poisson_nll([0.0, 2.0], [0.0, 2.0]) == pytest.approx(
        2 * (2.0 - 2.0 * math.log(2.0) + math.log(2.0)), rel=1e-15)
    assert math.isinf(oracle.poisson_nll([0.0, 1.0], [3.0, 1.0]))
    # for mu = a * m the minimum over a sits at a = sum(d) / sum(m)
    rng = np.random.default_rng(13)
    m = rng.uniform(1.0, 50.0, 40)
    d = rng.poisson(1.7 * m).astype(float)
    a0 = d.sum() / m.sum()
    f = lambda a: oracle.poisson_nll(a * m, d)
    assert f(a0) < f(a0 * 1.001) and f(a0) < f(a0 * 0.999)


# ---------------------------------------------------------------- energy scale
def test_energy_scale_binning():
    rng = np.random.default_rng(21)
    x = rng.uniform(0.0, 3.0, 3000)
    b0 = oracle.bin_indices(x, 0.0, 3.0, 50)
    np.testing.assert_array_equal(oracle.bin_indices(x, 0.0, 3.0, 50, e_scale=0.0), b0)
    # the definition: bin of fl(x * fl(1 + s)) by the unscaled rule
    for s in (0.02, -0.05, 1e-9):
        xs = x * (1.0 + s)
        np.testing.assert_array_equal(oracle.bin_indices(x, 0.0, 3.0, 50, e_scale=s),
                                      oracle.bin_indices(xs, 0.0, 3.0, 50))
    # a positive shift only moves events up (migration), never down
    up = oracle.bin_indices(x, 0.0, 3.0, 50, e_scale=0.03)
    assert (up >= b0).all() and (up > b0).any()
    # the boundary: 1.5 GeV sits on an edge; a 1e-12 shift moves it one bin down
    assert oracle.bin_index(1.5, 0.0, 3.0, 50) == 25
    assert oracle.bin_indices([1.5], 0.0, 3.0, 50, e_scale=-1e-12)[0] == 24
