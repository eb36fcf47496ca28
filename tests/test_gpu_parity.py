"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle.

Tolerances:
  * per-event P: 1e-12 absolute (the residual the paper reports between its
    CPU and GPU double-precision weights, Sec. 2.2);
  * bin indices and counts: exact;
  * histograms of given contributions (osc_fill_hist): bit-exact against
    the oracle's replay of the reduction contract on the same inputs;
  * histograms of osc_fill_pdf against the oracle's histogram: the P
    tolerance carried through the weights plus the rounding of both
    summations, |dh_b| <= 1e-12 * sum_b |w| + 2 d u sum_b |c| with
    d = K + log2(W) + log2(#tiles padded) additions per contribution and
    u = 2^-53;
  * osc_fill_pdf's histogram is bit-identical to osc_fill_hist applied to
    its own per-event P (the reduction is the same), run to run.
"""
import ctypes
import numpy as np
import pytest

import oracle
from paper_1311_7579_amd import workload
from helpers import (MIXED_TOL, MIXED_TOL_BROAD, MIXED_TOL_C3, P_TOL, assert_bits_equal,
                     bins_np, hist_tolerance)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def osc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1311_7579_amd import osc as _osc
    _osc.load()
    return _osc


@pytest.fixture(scope="module")
def ctx(osc):
    c = osc.Context(0)
    c.osc_set_params([workload.TABLE1])
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def gpu_reweight(osc, ctx, s, set_index=0):
    ds = osc.DeviceSample.from_host(s)
    p = torch.empty(s.n, dtype=torch.float64, device="cuda")
    ctx.osc_reweight(ds, set_index, p)
    return host(p)


def gpu_fill_pdf(osc, ctx, s, nbins, lo, hi, set_index=0, want_p=True):
    ds = osc.DeviceSample.from_host(s)
    h = torch.full((nbins + 2,), -1.0, dtype=torch.float64, device="cuda")
    p = torch.empty(s.n, dtype=torch.float64, device="cuda") if want_p else None
    ctx.osc_fill_pdf(ds, set_index, nbins, lo, hi, h, p)
    return host(h), (host(p) if want_p else None)


# --------------------------------------------------------------- per event
def test_c1_plain_fp64_reweight(osc, ctx):
    """1e5 events, Table 1, 295 km, 2.6 g/cm^3, seed 1."""
    s = workload.make_sample(100_000, 1)
    got = gpu_reweight(osc, ctx, s)
    want = oracle.prob_batch(workload.TABLE1, s.L_km, s.rho_gcc, s.Ye, s.e_true, s.flags)
    assert np.abs(got - want).max() <= P_TOL


@pytest.mark.parametrize("L,rho", [(295.0, 2.6), (810.0, 2.84), (1300.0, 3.0), (2500.0, 2.4),
                                   (295.0, 0.0), (0.0, 2.6)])
def test_all_channels_random_parameters(osc, ctx, L, rho):
    sets = workload.make_random_physics_sets(6, 17) + workload.make_param_sets(4, 3)
    ctx.osc_set_params(sets)
    try:
        s = workload.make_uniform_energy_sample(40_000, 23, e_max=20.0, e_min=0.05)
        s.L_km, s.rho_gcc = L, rho
        for k, p in enumerate(sets):
            got = gpu_reweight(osc, ctx, s, k)
            want = oracle.prob_batch(p, L, rho, s.Ye, s.e_true, s.flags)
            assert np.abs(got - want).max() <= P_TOL, (k, p)
    finally:
        ctx.osc_set_params([workload.TABLE1])


@pytest.mark.parametrize("rho", [0.0, 5.5])
def test_large_phases(osc, ctx, rho):
    """Phases up to ~5e4 rad (12742 km, E down to 2 MeV).  The phase
    reduction is exact, so what is left beyond 1e-12 is the FP64 rounding of
    the phase on each side: a few ulp of the eigenvalues, which the
    characteristic polynomial amplifies by (largest / smallest eigenvalue
    distance), times the phase per eV^2."""
    sets = [workload.TABLE1] + workload.make_random_physics_sets(3, 41)
    ctx.osc_set_params(sets)
    try:
        s = workload.make_uniform_energy_sample(200_000, 43, e_max=0.05, e_min=0.002)
        s.L_km, s.rho_gcc = 12742.0, rho
        for k, p in enumerate(sets):
            lam = eigenvalues(p, s, s.flags)
            gap = np.min(np.diff(lam, axis=1), axis=1)
            spread = lam[:, 2] - lam[:, 0]
            phase = oracle.k_phase() * spread * s.L_km / s.e_true   # largest phase difference
            got = gpu_reweight(osc, ctx, s, k)
            want = oracle.prob_batch(p, s.L_km, rho, s.Ye, s.e_true, s.flags)
            # an independent LAPACK route (eigh, then exp) stays within 0.04 of this bound
            tol = 1e-12 + 4 * 2.0 ** -53 * phase * (1.0 + spread / gap)
            assert float(phase.max()) > 3e4
            assert np.all(np.abs(got - want) <= tol), (k, float(np.abs(got - want).max()))
    finally:
        ctx.osc_set_params([workload.TABLE1])


def matter_term(s, flags):
    anti = (flags >> 4) & 1
    return oracle.k_matter() * s.Ye * s.rho_gcc * s.e_true * np.where(anti == 1, -1.0, 1.0)


def eigenvalues(p, s, flags):
    """Ascending eigenvalues of M = H0 + A e_e e_e^T per event (LAPACK)."""
    m2 = np.array([0.0, p["dm2_21"], p["dm2_21"] + p["dm2_32"]])
    anti = (flags >> 4) & 1
    A = matter_term(s, flags)
    out = np.empty((s.n, 3))
    for a in (0, 1):
        U = oracle.pmns(p, anti=bool(a))
        H = (U * m2) @ U.conj().T
        sel = anti == a
        M = np.broadcast_to(H, (int(sel.sum()), 3, 3)).copy()
        M[:, 0, 0] += A[sel]
        out[sel] = np.linalg.eigvalsh(M)
    return out


def large_a_conditioning(p, s, flags):
    """|A| / (smallest distance between eigenvalues of M) per event."""
    lam = eigenvalues(p, s, flags)
    return np.abs(matter_term(s, flags)) / np.min(np.diff(lam, axis=1), axis=1)


def test_matter_term_domain(osc, ctx):
    """Large matter terms within the solver's stated domain, mixed in the
    same waves with ordinary energies: |A| up to 0.8 eV^2 (E up to ~1 TeV
    through 13 g/cm^3) for Table 1 and sets around it, up to 0.03 eV^2 for
    broad random sets (any angles, both orderings).  P against the oracle
    within 1e-12 plus 64 u |A| / (smallest root distance) (u = 2^-53: both
    amplitudes lose about u |A| / distance to cancellation)."""
    n = 40_000
    rng = np.random.default_rng(8)
    ka = 1.526493e-4 * 0.5 * 13.0
    cases = [((workload.TABLE1,) + tuple(workload.make_param_sets(3, 3)), 0.8),
             (tuple(workload.make_random_physics_sets(4, 5)), 0.03)]
    for sets, a_max in cases:
        big = 10 ** rng.uniform(np.log10(0.01 * a_max / ka), np.log10(a_max / ka), n)
        small = 10 ** rng.uniform(-0.5, 1.0, n)
        E = np.where(rng.random(n) < 0.5, big, small)
        f = workload.make_flags(rng.integers(0, 3, n), rng.integers(0, 3, n), rng.random(n) < 0.5)
        s = workload.Sample(e_true=E, flags=f, weight=np.ones(n), e_reco=E, L_km=2500.0,
                            rho_gcc=13.0)
        for p in sets:
            ctx.osc_set_params([p])
            try:
                got = gpu_reweight(osc, ctx, s, 0)
            finally:
                ctx.osc_set_params([workload.TABLE1])
            want = oracle.prob_batch(p, s.L_km, s.rho_gcc, s.Ye, E, f)
            tol = 1e-12 + 64 * 2.0 ** -53 * large_a_conditioning(p, s, f)
            assert np.all(np.abs(got - want) <= tol), (a_max, p)


def test_mixed_tier_matter_term_domain(osc, ctx):
    """The FP32-mixed tier on the same large-|A| inputs: waves whose Halley
    corrections are not small relative to the root distance must still
    take the Newton step, so P stays within the tier's tolerance plus the
    FP32 share of the amplitude's cancellation (64 * 2^-24 |A| / distance);
    roots left at the Halley step there would be off by ~1e-2 of the
    distance."""
    n = 40_000
    rng = np.random.default_rng(9)
    ka = 1.526493e-4 * 0.5 * 13.0
    cases = [((workload.TABLE1,) + tuple(workload.make_param_sets(2, 3)), 0.8),
             (tuple(workload.make_random_physics_sets(3, 5)), 0.03)]
    for sets, a_max in cases:
        big = 10 ** rng.uniform(np.log10(0.01 * a_max / ka), np.log10(a_max / ka), n)
        small = 10 ** rng.uniform(-0.5, 1.0, n)
        E = np.where(rng.random(n) < 0.5, big, small)
        f = workload.make_flags(rng.integers(0, 3, n), rng.integers(0, 3, n), rng.random(n) < 0.5)
        s = workload.Sample(e_true=E, flags=f, weight=np.ones(n), e_reco=E, L_km=2500.0,
                            rho_gcc=13.0)
        ds = osc.DeviceSample.from_host(s)
        h = torch.empty(52, dtype=torch.float64, device="cuda")
        pm = torch.empty(n, dtype=torch.float64, device="cuda")
        for p in sets:
            ctx.osc_set_params([p])
            try:
                ctx.osc_fill_pdf(ds, 0, 50, 0.0, 3.0, h, pm, precision=osc.OSC_FP32_MIXED)
                got = host(pm)
            finally:
                ctx.osc_set_params([workload.TABLE1])
            want = oracle.prob_batch(p, s.L_km, s.rho_gcc, s.Ye, E, f)
            tol = MIXED_TOL_BROAD + 64 * 2.0 ** -24 * large_a_conditioning(p, s, f)
            assert np.all(np.abs(got - want) <= tol), (a_max, p, float(np.abs(got - want).max()))


def test_paper_validation_protocol(osc, ctx):
    """Sec. 2.2: 1e7 energies uniform on (0, 30] GeV, CPU vs GPU residual
    of order 1e-12 (every channel, neutrinos and antineutrinos)."""
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "validation_protocol.json")))
    s = workload.make_uniform_energy_sample(g["n_events"], 31, e_max=g["e_max_GeV"])
    got = gpu_reweight(osc, ctx, s)
    want = oracle.prob_batch(workload.TABLE1, s.L_km, s.rho_gcc, s.Ye, s.e_true, s.flags)
    assert np.abs(got - want).max() <= g["residual_abs"]


def test_invalid_flags_give_nan(osc, ctx):
    s = workload.make_sample(300, 2)
    s.flags[[0, 5, 77, 299]] = np.array([3, 3 << 2, 1 << 5, 0xFF], dtype=np.uint8)
    got = gpu_reweight(osc, ctx, s)
    assert np.isnan(got[[0, 5, 77, 299]]).all()
    ok = np.ones(300, bool)
    ok[[0, 5, 77, 299]] = False
    assert np.isfinite(got[ok]).all()


def test_every_flag_byte(osc, ctx):
    """All 256 flag byte values at 40 energies each, both tiers: the 18
    valid channels against the oracle, every other byte NaN."""
    E = np.tile(10 ** np.linspace(-1.2, 1.4, 40), 256)
    f = np.repeat(np.arange(256, dtype=np.uint8), 40)
    s = workload.Sample(e_true=E, flags=f, weight=np.ones(E.size), e_reco=E, L_km=1300.0,
                        rho_gcc=3.0)
    want = oracle.prob_batch(workload.TABLE1, s.L_km, s.rho_gcc, s.Ye, E, f)
    bad = np.isnan(want)
    assert bad.sum() == (256 - 18) * 40
    got = gpu_reweight(osc, ctx, s)
    np.testing.assert_array_equal(np.isnan(got), bad)
    assert np.abs(got[~bad] - want[~bad]).max() <= P_TOL
    ds = osc.DeviceSample.from_host(s)
    h = torch.empty(12, dtype=torch.float64, device="cuda")
    p = torch.empty(E.size, dtype=torch.float64, device="cuda")
    ctx.osc_fill_pdf(ds, 0, 10, 0.0, 30.0, h, p, precision=osc.OSC_FP32_MIXED)
    pm = host(p)
    np.testing.assert_array_equal(np.isnan(pm), bad)
    assert np.abs(pm[~bad] - want[~bad]).max() <= MIXED_TOL


def test_probabilities_bounded_and_unitary(osc, ctx):
    # sum over final flavours is 1 for every initial flavour
    n = 30_000
    rng = np.random.default_rng(4)
    E = 10 ** rng.uniform(-1, 1.3, n)
    for anti in (0, 1):
        tot = np.zeros(n)
        for a in range(3):
            tot[:] = 0
            for b in range(3):
                s = workload.Sample(e_true=E, flags=workload.make_flags(np.full(n, a), np.full(n, b),
                                                                        np.full(n, anti, bool)),
                                    weight=np.ones(n), e_reco=E, L_km=1300.0, rho_gcc=2.8)
                p = gpu_reweight(osc, ctx, s)
                assert p.min() >= -1e-15 and p.max() <= 1 + 1e-12
                tot += p
            assert np.abs(tot - 1).max() < 1e-12


# --------------------------------------------------------------- histograms
@pytest.mark.parametrize("n", [1, 63, 64, 65, 1023, 1024, 1025, 123_457, 1_000_003])
def test_fill_hist_bit_exact_vs_contract(osc, ctx, n):
    rng = np.random.default_rng(n)
    v = rng.uniform(0.0, 1.0, n)
    w = rng.uniform(0.5, 1.5, n)
    x = rng.uniform(-0.3, 3.3, n)
    h = torch.empty(52, dtype=torch.float64, device="cuda")
    ctx.osc_fill_hist(dev(v), dev(w), dev(x), 50, 0.0, 3.0, h)
    bins = oracle.bin_indices(x, 0.0, 3.0, 50) if n <= 200_000 else bins_np(x, 0.0, 3.0, 50)
    want = oracle.hist_contract(w * v, bins, 52)
    np.testing.assert_array_equal(host(h), want)


def test_fill_hist_multilevel_merge_bit_exact(osc, ctx):
    """2e7 events = 19532 tiles = 153 merge chunks: the merge needs a second
    level above the chunks; the bits must still follow the contract."""
    n = 20_000_000
    rng = np.random.default_rng(77)
    v = rng.uniform(0.0, 1.0, n)
    w = rng.uniform(0.5, 1.5, n)
    x = rng.uniform(-0.2, 3.2, n)
    h = torch.empty(52, dtype=torch.float64, device="cuda")
    ctx.osc_fill_hist(dev(v), dev(w), dev(x), 50, 0.0, 3.0, h)
    want = oracle.hist_contract(w * v, bins_np(x, 0.0, 3.0, 50), 52)
    np.testing.assert_array_equal(host(h), want)


@pytest.mark.parametrize("nbins,lo,hi", [(1, 0.0, 3.0), (7, 0.5, 2.0), (200, 0.0, 10.0)])
def test_fill_hist_counts_exact(osc, ctx, nbins, lo, hi):
    n = 200_003
    x = np.random.default_rng(nbins).uniform(lo - 0.5, hi + 0.5, n)
    x[:50] = lo
    x[50:100] = hi
    one = np.ones(n)
    h = torch.empty(nbins + 2, dtype=torch.float64, device="cuda")
    ctx.osc_fill_hist(dev(one), dev(one), dev(x), nbins, lo, hi, h)
    bins = oracle.bin_indices(x, lo, hi, nbins)
    np.testing.assert_array_equal(host(h), np.bincount(bins, minlength=nbins + 2).astype(float))


@pytest.mark.parametrize("nbins,lo,hi", [(50, 0.0, 3.0), (37, 0.5, 9.5), (316, -1.0, 0.7),
                                        (100_000, 0.0, 7.3), (100_000, -0.37, 0.91)])
def test_fill_hist_bin_edges_exact(osc, ctx, nbins, lo, hi):
    """Values on every bin edge and on the three neighbouring doubles either
    side: bin indices (hence counts) must equal the FP64 quotient rule."""
    nbins = min(nbins, ctx.max_nbins)
    wb = (hi - lo) / nbins
    x = []
    for k in range(-2, nbins + 3):
        e = lo + k * wb
        x.append(e)
        up = dn = e
        for _ in range(3):
            up, dn = np.nextafter(up, np.inf), np.nextafter(dn, -np.inf)
            x += [up, dn]
    x = np.array(x + [np.nan, np.inf, -np.inf, -0.0, 1e300, -1e300])
    one = np.ones(x.size)
    h = torch.empty(nbins + 2, dtype=torch.float64, device="cuda")
    ctx.osc_fill_hist(dev(one), dev(one), dev(x), nbins, lo, hi, h)
    bins = oracle.bin_indices(x, lo, hi, nbins)
    np.testing.assert_array_equal(host(h), np.bincount(bins, minlength=nbins + 2).astype(float))
    # weights of distinct powers of two identify which event went where
    w = 2.0 ** -np.arange(x.size % 50 + 1)[np.arange(x.size) % (x.size % 50 + 1)]
    ctx.osc_fill_hist(dev(one), dev(w), dev(x), nbins, lo, hi, h)
    np.testing.assert_array_equal(host(h), oracle.hist_contract(w, bins, nbins + 2))


def edge_contributions(seed):
    """Events (value, weight, reco energy) whose contributions c = w * v sit
    at the numeric edges of FP64, grouped by bin of 10 on [0, 10):
    bin 0 subnormal sums (products that round into the subnormal range,
    sums that cross 2^-1022 both ways), bin 1 signed normals cancelling to
    exact zero and to subnormals, bin 2 only -0.0 and +0.0 (the result
    must be +0.0), bin 3 magnitudes 2^500 and 2^-500 of both signs, bin 4
    sums that overflow to +inf, bin 5 +inf among finite values, bin 6 +inf
    and -inf (NaN), bin 7 NaN among finite values, bin 8 all of the above
    in one bin (NaN), bin 10 the finite ones of them in one bin; bin 9
    ordinary values.  The events are shuffled so the bins
    interleave across lanes, accumulators and tiles."""
    rng = np.random.default_rng(seed)
    tiny, dmin = 2.0 ** -1074, 2.0 ** -1022
    groups = {
        0: [k * tiny for k in rng.integers(-2 ** 20, 2 ** 20, 400)] + [dmin - tiny, tiny, -tiny,
                                                                     dmin, -dmin, 3 * tiny],
        1: [1e-300, -1e-300, 3.5, -3.5, dmin, -(dmin - 5 * tiny), -1.25, 1.25, 7e-310,
            -7e-310] + list(rng.uniform(-1, 1, 200)),
        2: [-0.0] * 50 + [0.0] * 3 + [-0.0] * 50,
        3: [2.0 ** 500, -(2.0 ** 500), 2.0 ** -500, -(2.0 ** -500), 3 * 2.0 ** 500, 1.0,
            -(2.0 ** -499)] * 20,
        4: [1.5 * 2.0 ** 1023, 1.5 * 2.0 ** 1023, -1.0, 2.0],
        5: [1.0, np.inf, -3.0, 2.0 ** 500],
        6: [np.inf, 1.0, -np.inf],
        7: [1.0, np.nan, -2.0],
        9: list(rng.uniform(0.5, 1.5, 300)),
    }
    finite = [g[k] for b, g in groups.items() if b in (0, 1, 2, 3, 9) for k in range(0, len(g), 5)]
    groups[8] = finite + [np.inf, -np.inf, np.nan, -0.0]
    groups[10] = finite
    c = np.concatenate([np.asarray(v, dtype=np.float64) for v in groups.values()])
    x = np.concatenate([np.full(len(v), b + 0.5) for b, v in groups.items()])
    # value x weight = c exactly: ordinary contributions as (c, 1), and every
    # third one split into a product that the multiply itself must round
    # into place (2^-600 x 2^-474 = 2^-1074, 2^-520 x (c 2^520))
    v = np.ones_like(c)
    w = c.copy()
    sel = (np.arange(c.size) % 3 == 0) & np.isfinite(c) & (np.abs(c) < 2.0 ** 400) & (c != 0)
    v[sel] = 2.0 ** -520
    w[sel] = c[sel] * 2.0 ** 520
    v[0], w[0] = 2.0 ** -600, 2.0 ** -474
    perm = rng.permutation(c.size)
    return v[perm], w[perm], x[perm]


@pytest.mark.parametrize("copies", [1, 3])
def test_fill_hist_numeric_edges_bit_exact(osc, ctx, copies):
    """The reduction at the numeric edges: subnormal, negative, +-0.0,
    +-inf, NaN and 2^+-500 contributions, alone and all in one bin, over
    one and several tiles, bit for bit against the oracle's contract replay
    (NaN only as NaN)."""
    parts = [edge_contributions(90 + k) for k in range(copies)]
    v, w, x = (np.concatenate([p[i] for p in parts]) for i in range(3))
    h = torch.empty(13, dtype=torch.float64, device="cuda")
    ctx.osc_fill_hist(dev(v), dev(w), dev(x), 11, 0.0, 11.0, h)
    bins = oracle.bin_indices(x, 0.0, 11.0, 11)
    want = oracle.hist_contract(w * v, bins, 13)
    got = host(h)
    assert_bits_equal(got, want, f"{copies} copies")
    # the expected classes of results, so that the edges really were hit
    assert np.isnan(got[[6, 7, 8]]).all() and got[4] == np.inf and got[5] == np.inf
    assert got[2] == 0.0 and not np.signbit(got[2])
    assert np.isfinite(got[[0, 1, 3, 9, 10]]).all()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fill_pdf_invalid_flags_nan_bins(osc, ctx, precision):
    """Events with invalid flag bytes have P = NaN, so the bins they fall
    into are NaN in both tiers; every bin is bit-exact against the contract
    applied to the kernel's own P, NaN in the same bins as the oracle's
    histogram, and within the tier's tolerance of it elsewhere."""
    prec = osc.OSC_FP64 if precision == "fp64" else osc.OSC_FP32_MIXED
    tol_p = P_TOL if precision == "fp64" else MIXED_TOL_C3
    s = workload.make_sample(70_001, 13)
    bad = np.array([5, 1030, 1031, 40_000, 70_000])
    s.flags[bad] = np.array([3, 0xFF, 1 << 5, 3 << 2, 35], dtype=np.uint8)
    s.e_reco[bad] = np.array([0.01, 1.21, 1.23, 2.99, 7.0])    # bins 0, 20, 20, 49, overflow
    ds = osc.DeviceSample.from_host(s)
    h = torch.empty(52, dtype=torch.float64, device="cuda")
    p = torch.empty(s.n, dtype=torch.float64, device="cuda")
    ctx.osc_fill_pdf(ds, 0, 50, 0.0, 3.0, h, p, precision=prec)
    got, P = host(h), host(p)
    assert np.isnan(P[bad]).all() and np.isfinite(np.delete(P, bad)).all()
    bins = oracle.bin_indices(s.e_reco, 0.0, 3.0, 50)
    assert_bits_equal(got, oracle.hist_contract(s.weight * P, bins, 52), precision)
    hist_o, P_o = oracle.fill_pdf(workload.TABLE1, s.L_km, s.rho_gcc, s.Ye, s.e_true, s.flags,
                                  s.weight, s.e_reco, 50, 0.0, 3.0)
    np.testing.assert_array_equal(np.isnan(got), np.isnan(hist_o))
    assert np.isnan(got[[0, 20, 49, 51]]).all()
    fin = ~np.isnan(hist_o)
    tol = hist_tolerance(s.weight, s.weight * np.nan_to_num(P_o), bins, 52, s.n, p_tol=tol_p)
    assert (np.abs(got - hist_o)[fin] <= tol[fin]).all()


def test_fill_hist_max_nbins(osc, ctx):
    nb = ctx.max_nbins
    assert nb >= 200
    n = 100_000
    rng = np.random.default_rng(5)
    v, w, x = rng.uniform(0, 1, n), rng.uniform(0.5, 1.5, n), rng.uniform(-1, 11, n)
    h = torch.empty(nb + 2, dtype=torch.float64, device="cuda")
    ctx.osc_fill_hist(dev(v), dev(w), dev(x), nb, 0.0, 10.0, h)
    want = oracle.hist_contract(w * v, oracle.bin_indices(x, 0.0, 10.0, nb), nb + 2)
    np.testing.assert_array_equal(host(h), want)
    with pytest.raises(osc.OscError):
        ctx.osc_fill_hist(dev(v), dev(w), dev(x), nb + 1, 0.0, 10.0,
                          torch.empty(nb + 3, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fill_pdf_max_nbins(osc, ctx, precision):
    """The largest bin count the context reports runs the full per-event
    kernel (histograms next to the static LDS tables)."""
    nb = ctx.max_nbins
    s = workload.make_sample(20_000, 8)
    s.e_reco = np.random.default_rng(8).uniform(-0.5, 10.5, s.n)
    prec = osc.OSC_FP64 if precision == "fp64" else osc.OSC_FP32_MIXED
    ds = osc.DeviceSample.from_host(s)
    h = torch.empty(nb + 2, dtype=torch.float64, device="cuda")
    p = torch.empty(s.n, dtype=torch.float64, device="cuda")
    ctx.osc_fill_pdf(ds, 0, nb, 0.0, 10.0, h, p, precision=prec)
    P = host(p)
    want = oracle.prob_batch(workload.TABLE1, s.L_km, s.rho_gcc, s.Ye, s.e_true, s.flags)
    assert np.abs(P - want).max() <= (P_TOL if precision == "fp64" else MIXED_TOL_C3)
    bins = oracle.bin_indices(s.e_reco, 0.0, 10.0, nb)
    np.testing.assert_array_equal(host(h), oracle.hist_contract(s.weight * P, bins, nb + 2))


def test_c2_fill_pdf_full_size(osc, ctx):
    """1e7 events, 50 bins on [0, 3] GeV: per-event P within 1e-12 of the
    oracle, histogram within the carried tolerance, and bit-identical to
    the contract applied to the GPU's own P."""
    s = workload.make_sample(10_000_000, 1)
    h, p = gpu_fill_pdf(osc, ctx, s, 50, 0.0, 3.0)
    hist_o, p_o = oracle.fill_pdf(workload.TABLE1, s.L_km, s.rho_gcc, s.Ye, s.e_true, s.flags,
                                  s.weight, s.e_reco, 50, 0.0, 3.0)
    assert np.abs(p - p_o).max() <= P_TOL
    bins = bins_np(s.e_reco, 0.0, 3.0, 50)
    tol = hist_tolerance(s.weight, s.weight * p_o, bins, 52, s.n)
    assert (np.abs(h - hist_o) <= tol).all(), np.abs(h - hist_o).max()
    # bit-exact reduction of the GPU's own contributions (same fixed order)
    hh = torch.empty(52, dtype=torch.float64, device="cuda")
    ctx.osc_fill_hist(dev(p), dev(s.weight), dev(s.e_reco), 50, 0.0, 3.0, hh)
    np.testing.assert_array_equal(host(hh), h)


def test_fill_pdf_deterministic_and_p_optional(osc, ctx):
    s = workload.make_sample(2_000_001, 7)
    ds = osc.DeviceSample.from_host(s)
    outs = []
    for k in range(3):
        h = torch.empty(52, dtype=torch.float64, device="cuda")
        if k == 2:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                ctx.osc_fill_pdf(ds, 0, 50, 0.0, 3.0, h, None)
            st.synchronize()
        else:
            p = torch.empty(s.n, dtype=torch.float64, device="cuda")
            ctx.osc_fill_pdf(ds, 0, 50, 0.0, 3.0, h, p if k == 0 else None)
        outs.append(host(h))
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])


def test_scratch_order_across_streams(osc, ctx):
    """A fresh context: back-to-back calls on one stream whose scratch slots
    grow while earlier calls still run, then calls that alternate with a
    second stream, with no host wait in between; every histogram equals the
    one-call result of the shared context bit for bit."""
    sizes = (1_025, 300_001, 2_000_001, 50_001, 2_000_001, 1_025)
    samples = {n: osc.DeviceSample.from_host(workload.make_sample(n, 900 + n))
               for n in set(sizes)}
    want = {}
    for n, ds in samples.items():
        h = torch.empty(52, dtype=torch.float64, device="cuda")
        ctx.osc_fill_pdf(ds, 0, 50, 0.0, 3.0, h, None)
        want[n] = host(h)
    c = osc.Context(0)
    try:
        c.osc_set_params([workload.TABLE1])
        a, b = torch.cuda.Stream(), torch.cuda.Stream()
        plan = [(n, a) for n in sizes] + [(n, a if k % 2 else b) for k, n in enumerate(sizes)]
        outs = []
        torch.cuda.synchronize()
        for n, st in plan:
            with torch.cuda.stream(st):
                h = torch.empty(52, dtype=torch.float64, device="cuda")
                c.osc_fill_pdf(samples[n], 0, 50, 0.0, 3.0, h, None)
            outs.append((n, h))
        torch.cuda.synchronize()
        for n, h in outs:
            np.testing.assert_array_equal(host(h), want[n])
    finally:
        c.close()


def test_fill_pdf_small_and_ragged_against_contract(osc, ctx):
    for n in (1, 65, 1025, 50_001):
        s = workload.make_sample(n, 100 + n)
        h, p = gpu_fill_pdf(osc, ctx, s, 50, 0.0, 3.0)
        hist_o, p_o = oracle.fill_pdf(workload.TABLE1, s.L_km, s.rho_gcc, s.Ye, s.e_true,
                                      s.flags, s.weight, s.e_reco, 50, 0.0, 3.0)
        assert np.abs(p - p_o).max() <= P_TOL
        bins = oracle.bin_indices(s.e_reco, 0.0, 3.0, 50)
        tol = hist_tolerance(s.weight, s.weight * p_o, bins, 52, n)
        assert (np.abs(h - hist_o) <= tol).all()
        np.testing.assert_array_equal(h, oracle.hist_contract(s.weight * p, bins, 52))


def test_empty_sample(osc, ctx):
    s = workload.make_sample(0, 1)
    h, p = gpu_fill_pdf(osc, ctx, s, 50, 0.0, 3.0)
    assert (h == 0.0).all() and p.size == 0
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    hh = torch.full((52,), 7.0, dtype=torch.float64, device="cuda")
    ctx.osc_fill_hist(e, e, e, 50, 0.0, 3.0, hh)
    assert (host(hh) == 0.0).all()


def test_invalid_arguments_raise(osc, ctx):
    s = osc.DeviceSample.from_host(workload.make_sample(100, 1))
    h = torch.empty(52, dtype=torch.float64, device="cuda")
    p = torch.empty(100, dtype=torch.float64, device="cuda")
    with pytest.raises(osc.OscError):
        ctx.osc_fill_pdf(s, 1, 50, 0.0, 3.0, h)          # no such set
    with pytest.raises(osc.OscError):
        ctx.osc_fill_pdf(s, 0, 50, 3.0, 3.0, h)          # empty range
    with pytest.raises(ValueError):
        ctx.osc_fill_pdf(s, 0, 0, 0.0, 3.0, h)           # no bins: the binding refuses
    # ... and so does the C ABI itself
    cs = s.c_struct()
    b = osc.osc_binning(0, 0.0, 3.0, 0.0)
    assert osc.load().osc_fill_pdf(ctx.handle, ctypes.byref(cs), 0, ctypes.byref(b), 0,
                                   ctypes.c_void_p(h.data_ptr()), None, None) \
        == osc.OSC_ERR_INVALID_ARG
    with pytest.raises(osc.OscError):
        ctx.osc_reweight(s, -1, p)
    bad = osc.DeviceSample(s.e_true, s.flags, s.weight, s.e_reco, L_km=-1.0)
    with pytest.raises(osc.OscError):
        ctx.osc_reweight(bad, 0, p)
    with pytest.raises(osc.OscError):
        ctx.osc_set_params([dict(workload.TABLE1, dm2_21=0.0)])
    # the context still works after rejected calls
    ctx.osc_reweight(s, 0, p)
    assert np.isfinite(host(p)).all()


# --------------------------------------------------------------- FP32-mixed tier
# FP64 eigenvalues and phase differences, FP32 sine/cosine and amplitude
# assembly; the tier's tolerances (MIXED_TOL_C3 for the C3 draw at 295 km,
# MIXED_TOL for those sets at any baseline, MIXED_TOL_BROAD for arbitrary
# angles) and their derivation are in helpers.py.


def test_mixed_tier_c3_parameter_sets(osc, ctx):
    """1e7 events x 64 parameter sets (C3 draw): mixed-tier P within
    MIXED_TOL_C3 of the FP64 tier on every event and of the oracle on a 1e5
    subsample; histograms within the carried bound; the reduction of the
    mixed tier's own P is bit-exact."""
    sets = workload.make_param_sets(64, 3)
    s = workload.make_sample(10_000_000, 1)
    ds = osc.DeviceSample.from_host(s)
    sub = slice(0, 100_000)
    ctx.osc_set_params(sets)
    try:
        h64 = torch.empty(52, dtype=torch.float64, device="cuda")
        hmx = torch.empty(52, dtype=torch.float64, device="cuda")
        p64 = torch.empty(s.n, dtype=torch.float64, device="cuda")
        pmx = torch.empty(s.n, dtype=torch.float64, device="cuda")
        worst_gpu, worst_oracle = 0.0, 0.0
        for k, p in enumerate(sets):
            ctx.osc_fill_pdf(ds, k, 50, 0.0, 3.0, h64, p64, precision=osc.OSC_FP64)
            ctx.osc_fill_pdf(ds, k, 50, 0.0, 3.0, hmx, pmx, precision=osc.OSC_FP32_MIXED)
            d = float((pmx - p64).abs().max())
            worst_gpu = max(worst_gpu, d)
            po = oracle.prob_batch(p, s.L_km, s.rho_gcc, s.Ye, s.e_true[sub], s.flags[sub])
            worst_oracle = max(worst_oracle, float(np.abs(host(pmx[sub]) - po).max()))
            assert np.abs(host(p64[sub]) - po).max() <= P_TOL
            hm = host(hmx)
            bins = bins_np(s.e_reco, 0.0, 3.0, 50)
            sw = np.bincount(bins, weights=s.weight, minlength=52)
            assert (np.abs(hm - host(h64)) <= MIXED_TOL_C3 * sw + 1e-9).all()
            if k % 16 == 0:
                hh = torch.empty(52, dtype=torch.float64, device="cuda")
                ctx.osc_fill_hist(pmx, ds.weight, ds.e_reco, 50, 0.0, 3.0, hh)
                np.testing.assert_array_equal(host(hh), hm)
        print(f"mixed tier: max |P_mixed - P_fp64| = {worst_gpu:.3g}, "
              f"max |P_mixed - P_oracle| (1e5 x 64) = {worst_oracle:.3g}")
        assert worst_gpu <= MIXED_TOL_C3
        assert worst_oracle <= MIXED_TOL_C3
    finally:
        ctx.osc_set_params([workload.TABLE1])


def test_mixed_tier_all_channels(osc, ctx):
    sets = workload.make_random_physics_sets(4, 29) + [workload.TABLE1]
    ctx.osc_set_params(sets)
    try:
        s = workload.make_uniform_energy_sample(200_000, 37, e_max=20.0, e_min=0.05)
        for L, rho in ((295.0, 2.6), (2500.0, 2.8), (810.0, 0.0)):
            s.L_km, s.rho_gcc = L, rho
            ds = osc.DeviceSample.from_host(s)
            for k, p in enumerate(sets):
                h = torch.empty(52, dtype=torch.float64, device="cuda")
                pm = torch.empty(s.n, dtype=torch.float64, device="cuda")
                ctx.osc_fill_pdf(ds, k, 50, 0.0, 3.0, h, pm, precision=osc.OSC_FP32_MIXED)
                po = oracle.prob_batch(p, L, rho, s.Ye, s.e_true, s.flags)
                tol = MIXED_TOL if p is workload.TABLE1 else MIXED_TOL_BROAD
                assert np.abs(host(pm) - po).max() <= tol, (L, rho, k)
    finally:
        ctx.osc_set_params([workload.TABLE1])


# --------------------------------------------------------------- Eq. (2)
def test_poisson_nll_against_oracle(osc, ctx):
    rng = np.random.default_rng(31)
    n_hist, n_data, nb = 12, 4, 50
    mu = rng.uniform(0.0, 400.0, (n_hist, nb + 2))
    mu[0, 3] = 0.0                                        # empty bin with empty data
    data = rng.poisson(rng.uniform(1.0, 300.0, (n_data, nb))).astype(float)
    data[0, 3] = 0.0
    out = torch.empty(n_hist, dtype=torch.float64, device="cuda")
    ctx.osc_poisson_nll(dev(mu), dev(data), out)
    got = host(out)
    for k in range(n_hist):
        want = oracle.poisson_nll(mu[k, :nb], data[k % n_data])
        assert got[k] == pytest.approx(want, rel=1e-12), k
    # an exposure scale: mu = 0.37 * hist (one rounding on both sides)
    ctx.osc_poisson_nll(dev(mu), dev(data), out, mu_scale=0.37)
    got = host(out)
    for k in range(n_hist):
        want = oracle.poisson_nll(0.37 * mu[k, :nb], data[k % n_data])
        assert got[k] == pytest.approx(want, rel=1e-12), k
    with pytest.raises(osc.OscError):
        ctx.osc_poisson_nll(dev(mu), dev(data), out, mu_scale=0.0)


def test_poisson_nll_on_fitter_loop(osc, ctx):
    """The fitter's step: PDF at a proposal, -2 ln L against fake data drawn
    at Table 1; the likelihood is smallest near the generating point."""
    s = workload.make_sample(400_000, 3)
    ds = osc.DeviceSample.from_host(s)
    sets = [workload.TABLE1, dict(workload.TABLE1, dm2_32=2.2e-3), dict(workload.TABLE1, sin2_th23=0.4)]
    ctx.osc_set_params(sets)
    try:
        h = torch.empty((3, 52), dtype=torch.float64, device="cuda")
        for k in range(3):
            ctx.osc_fill_pdf(ds, k, 50, 0.0, 3.0, h[k])
        data = np.random.default_rng(5).poisson(host(h)[0, :50]).astype(float)
        out = torch.empty(3, dtype=torch.float64, device="cuda")
        ctx.osc_poisson_nll(h, dev(data[None, :]), out)
        got = host(out)
        for k in range(3):
            assert got[k] == pytest.approx(oracle.poisson_nll(host(h)[k, :50], data), rel=1e-12)
        assert got[0] < got[1] and got[0] < got[2]
    finally:
        ctx.osc_set_params([workload.TABLE1])


# --------------------------------------------------------------- energy scale
@pytest.mark.parametrize("e_scale", [0.0, 0.013, -0.021])
def test_energy_scale_systematic(osc, ctx, e_scale):
    """Event migration under a reco-energy scale shift: bins exact, histogram
    bit-exact to the contract, P independent of the shift."""
    s = workload.make_sample(300_007, 44)
    ds = osc.DeviceSample.from_host(s)
    h = torch.empty(52, dtype=torch.float64, device="cuda")
    p = torch.empty(s.n, dtype=torch.float64, device="cuda")
    ctx.osc_fill_pdf(ds, 0, 50, 0.0, 3.0, h, p, e_scale=e_scale)
    P = host(p)
    bins = oracle.bin_indices(s.e_reco, 0.0, 3.0, 50, e_scale=e_scale)
    np.testing.assert_array_equal(host(h), oracle.hist_contract(s.weight * P, bins, 52))
    hist_o, P_o = oracle.fill_pdf(workload.TABLE1, s.L_km, s.rho_gcc, s.Ye, s.e_true, s.flags,
                                  s.weight, s.e_reco, 50, 0.0, 3.0, e_scale=e_scale)
    assert np.abs(P - P_o).max() <= P_TOL
    tol = hist_tolerance(s.weight, s.weight * P_o, bins, 52, s.n)
    assert (np.abs(host(h) - hist_o) <= tol).all()
    one = torch.ones(s.n, dtype=torch.float64, device="cuda")
    ctx.osc_fill_hist(one, one, ds.e_reco, 50, 0.0, 3.0, h, e_scale=e_scale)
    np.testing.assert_array_equal(host(h), np.bincount(bins, minlength=52).astype(float))


# --------------------------------------------------------------- domain check
@pytest.mark.parametrize("n", [0, 1, 1000, 3_000_017])
def test_validate_sample_counts(osc, ctx, n):
    rng = np.random.default_rng(n + 3)
    s = workload.make_sample(n, 5) if n else workload.make_sample(0, 5)
    if n:
        k = rng.choice(n, size=min(n, 40), replace=False)
        s.e_true[k[:10]] = np.array([0.0, -1.0, np.nan, np.inf, -np.inf, 0.0, -0.0, 1e-300,
                                     -5.0, np.nan])[:len(k[:10])]
        s.flags[k[10:25]] = np.array([3, 7, 11, 12, 13, 14, 15, 32, 64, 128, 255, 35, 48, 19, 31],
                                     np.uint8)[:len(k[10:25])]
    ds = osc.DeviceSample.from_host(s)
    be, bf = ctx.osc_validate_sample(ds)
    e, f = s.e_true, s.flags.astype(int)
    want_e = int(np.sum(~((e > 0) & np.isfinite(e))))
    valid = (f < 32) & ((f & 3) < 3) & (((f >> 2) & 3) < 3)
    assert (be, bf) == (want_e, int(np.sum(~valid)))
