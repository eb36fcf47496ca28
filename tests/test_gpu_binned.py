"""Binned samples (osc_binned_create / osc_fill_pdf_binned): the reco-energy
bins of a sample cached once, 2 bytes per event.  The histogram and P of
osc_fill_pdf_binned must equal osc_fill_pdf's bit for bit (the same
contributions reach the same accumulators in the same order), and agree
with the oracle: P within 1e-12, the histogram within the P tolerance
carried through the weights, and bit-exact against the oracle's replay of
the reduction contract on the GPU's own P with the oracle's bin rule."""
import numpy as np
import pytest

import oracle
from paper_1311_7579_amd import workload
from helpers import P_TOL, MIXED_TOL, MIXED_TOL_C3, assert_bits_equal, hist_tolerance

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
    c.osc_set_params([workload.TABLE1, dict(workload.TABLE1, sin2_th23=0.43, delta_cp=2.1,
                                            dm2_32=2.55e-3)])
    yield c
    c.close()


def run(ctx, ds, binned, set_index, nbins, lo, hi, precision, e_scale=0.0):
    n = ds.n
    h0 = torch.full((nbins + 2,), -7.0, dtype=torch.float64, device="cuda")
    p0 = torch.full((n,), -7.0, dtype=torch.float64, device="cuda")
    h1, p1 = h0.clone(), p0.clone()
    ctx.osc_fill_pdf(ds, set_index, nbins, lo, hi, h0, p0, precision=precision, e_scale=e_scale)
    ctx.osc_fill_pdf_binned(binned, set_index, h1, p1, precision=precision)
    torch.cuda.synchronize()
    return h0.cpu().numpy(), p0.cpu().numpy(), h1.cpu().numpy(), p1.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("n,nbins,lo,hi,e_scale", [
    (1, 50, 0.0, 3.0, 0.0), (1025, 50, 0.0, 3.0, 0.0), (300_007, 50, 0.0, 3.0, 0.0),
    (100_003, 7, 0.4, 2.2, 0.013), (100_003, 1000, 0.0, 10.0, -0.021)])
def test_binned_equals_fill_pdf_and_oracle(osc, ctx, precision, n, nbins, lo, hi, e_scale):
    s = workload.make_sample(n, 7000 + n + nbins)
    ds = osc.DeviceSample.from_host(s)
    with ctx.osc_binned_create(ds, nbins, lo, hi, e_scale) as b:
        for k in (0, 1):
            h0, p0, h1, p1 = run(ctx, ds, b, k, nbins, lo, hi, precision, e_scale)
            assert_bits_equal(h1, h0, f"hist set {k}")
            assert_bits_equal(p1, p0, f"P set {k}")
            pset = workload.TABLE1 if k == 0 else dict(workload.TABLE1, sin2_th23=0.43,
                                                       delta_cp=2.1, dm2_32=2.55e-3)
            hist_o, p_o = oracle.fill_pdf(pset, s.L_km, s.rho_gcc, s.Ye, s.e_true, s.flags,
                                          s.weight, s.e_reco, nbins, lo, hi, e_scale=e_scale)
            tol_p = P_TOL if precision == 0 else MIXED_TOL
            assert np.abs(p1 - p_o).max() <= tol_p
            bins = oracle.bin_indices(s.e_reco, lo, hi, nbins, e_scale)
            tol = hist_tolerance(s.weight, s.weight * p_o, bins, nbins + 2, n, p_tol=tol_p)
            assert (np.abs(h1 - hist_o) <= tol).all()
            np.testing.assert_array_equal(h1, oracle.hist_contract(s.weight * p1, bins, nbins + 2))


def test_binned_bin_edges_and_specials(osc, ctx):
    """Reco energies on every bin edge and the three doubles either side,
    plus NaN, +-inf, -0.0 and huge values: the cached slots must give the
    same histogram as the computed bins, and the oracle's bin rule."""
    nbins, lo, hi = 37, 0.5, 9.5
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
    s = workload.make_sample(x.size, 77)
    s.e_reco = x
    ds = osc.DeviceSample.from_host(s)
    with ctx.osc_binned_create(ds, nbins, lo, hi) as b:
        h0, p0, h1, p1 = run(ctx, ds, b, 0, nbins, lo, hi, 0)
    assert_bits_equal(h1, h0, "hist")
    bins = oracle.bin_indices(x, lo, hi, nbins)
    np.testing.assert_array_equal(h1, oracle.hist_contract(s.weight * p1, bins, nbins + 2))


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_binned_benchmark_workload_full_size(osc, ctx, precision):
    """The benchmark step itself: 1e7 events (seed 1), Table 1, 50 bins on
    [0, 3] GeV, P written, as bench.py launches it.  Every P against the
    oracle, the histogram within the carried tolerance, and bit-exact
    against the contract replayed on the GPU's own P."""
    s = workload.make_sample(10_000_000, 1)
    ds = osc.DeviceSample.from_host(s)
    h = torch.empty(52, dtype=torch.float64, device="cuda")
    p = torch.empty(s.n, dtype=torch.float64, device="cuda")
    with ctx.osc_binned_create(ds, 50, 0.0, 3.0) as b:
        ctx.osc_fill_pdf_binned(b, 0, h, p, precision=precision)
        torch.cuda.synchronize()
    h, p = h.cpu().numpy(), p.cpu().numpy()
    hist_o, p_o = oracle.fill_pdf(workload.TABLE1, s.L_km, s.rho_gcc, s.Ye, s.e_true, s.flags,
                                  s.weight, s.e_reco, 50, 0.0, 3.0)
    tol_p = P_TOL if precision == 0 else MIXED_TOL_C3
    assert np.abs(p - p_o).max() <= tol_p
    bins = oracle.bin_indices(s.e_reco, 0.0, 3.0, 50)
    tol = hist_tolerance(s.weight, s.weight * p_o, bins, 52, s.n, p_tol=tol_p)
    assert (np.abs(h - hist_o) <= tol).all()
    np.testing.assert_array_equal(h, oracle.hist_contract(s.weight * p, bins, 52))


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_binned_max_nbins(osc, ctx, precision):
    """The device's largest bin count: the 16-bit slots cover every row
    (rows x 8 accumulators < 2^15), and the histogram equals the computed
    bins' bit for bit."""
    nb = ctx.max_nbins
    s = workload.make_sample(50_000, 81)
    s.e_reco = np.random.default_rng(81).uniform(-0.5, 10.5, s.n)
    ds = osc.DeviceSample.from_host(s)
    with ctx.osc_binned_create(ds, nb, 0.0, 10.0) as b:
        h0, p0, h1, p1 = run(ctx, ds, b, 0, nb, 0.0, 10.0, precision)
    assert_bits_equal(h1, h0, "hist")
    assert_bits_equal(p1, p0, "P")
    bins = oracle.bin_indices(s.e_reco, 0.0, 10.0, nb)
    np.testing.assert_array_equal(h1, oracle.hist_contract(s.weight * p1, bins, nb + 2))
    assert (np.bincount(bins, minlength=nb + 2) > 0).sum() > nb // 2   # many rows used


def test_binned_invalid_flags_and_empty(osc, ctx):
    """Invalid flag bytes give NaN P and NaN bins in both paths; an empty
    sample gives an all-zero histogram."""
    s = workload.make_sample(5000, 78)
    s.flags[::97] = 0x0f                      # beta = 3: invalid
    ds = osc.DeviceSample.from_host(s)
    with ctx.osc_binned_create(ds, 50, 0.0, 3.0) as b:
        h0, p0, h1, p1 = run(ctx, ds, b, 0, 50, 0.0, 3.0, 0)
    assert np.isnan(p1[::97]).all()
    assert_bits_equal(h1, h0, "hist")
    e = workload.make_sample(0, 1)
    de = osc.DeviceSample.from_host(e)
    with ctx.osc_binned_create(de, 50, 0.0, 3.0) as b:
        h = torch.full((52,), 7.0, dtype=torch.float64, device="cuda")
        ctx.osc_fill_pdf_binned(b, 0, h)
        torch.cuda.synchronize()
        assert (h.cpu().numpy() == 0.0).all()


def test_binned_refusals(osc, ctx):
    s = workload.make_sample(100, 79)
    ds = osc.DeviceSample.from_host(s)
    h = torch.empty(52, dtype=torch.float64, device="cuda")
    with pytest.raises(osc.OscError):
        ctx.osc_binned_create(ds, 50, 3.0, 3.0)          # empty range
    with pytest.raises(ValueError):
        ctx.osc_binned_create(osc.DeviceSample(ds.e_true, ds.flags), 50, 0.0, 3.0)  # no e_reco
    with ctx.osc_binned_create(ds, 50, 0.0, 3.0) as b:
        with pytest.raises(osc.OscError):
            ctx.osc_fill_pdf_binned(b, 5, h)              # no such set
        with pytest.raises(ValueError):
            ctx.osc_fill_pdf_binned(b, 0, torch.empty(51, dtype=torch.float64, device="cuda"))
        other = osc.Context(0)
        other.osc_set_params([workload.TABLE1])
        try:
            with pytest.raises(ValueError):
                other.osc_fill_pdf_binned(b, 0, h)        # another context's binned sample
            st = osc.load().osc_fill_pdf_binned(other.handle, b.handle, 0, 0,
                                                __import__("ctypes").c_void_p(h.data_ptr()),
                                                None, None)
            assert st == osc.OSC_ERR_INVALID_ARG
        finally:
            other.close()
