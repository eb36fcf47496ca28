"""osc_fill_pdf_noalloc (the entry point that allocates no device memory)
against osc_fill_pdf through the C ABI: the same kernels on a fixed device
array instead of the context's scratch, so histograms and P must agree bit
for bit, call after call, also when a smaller call follows a larger one
(stale tile results of the first call must not leak into the second)."""
import ctypes

import numpy as np
import pytest

from paper_1311_7579_amd import workload
from helpers import assert_bits_equal

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
    c.osc_set_params([workload.TABLE1, dict(workload.TABLE1, sin2_th23=0.44, delta_cp=-1.3)])
    yield c
    c.close()


def run_both(osc, ctx, ds, set_index, nbins, lo, hi, precision):
    out = []
    for fn in (ctx.osc_fill_pdf, ctx.osc_fill_pdf_noalloc):
        h = torch.full((nbins + 2,), -7.0, dtype=torch.float64, device="cuda")
        p = torch.full((ds.n,), -7.0, dtype=torch.float64, device="cuda")
        fn(ds, set_index, nbins, lo, hi, h, p, precision=precision)
        torch.cuda.synchronize()
        out.append((h.cpu().numpy(), p.cpu().numpy()))
    return out


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
@pytest.mark.parametrize("sizes", [(3_000_017, 100_003), (20_000_000, 1_000_001)],
                         ids=["one_level", "two_levels"])
def test_noalloc_equals_fill_pdf_on_consecutive_calls(osc, ctx, precision, sizes):
    """Two calls in a row, the second on a smaller sample; 2e7 events span
    19532 tiles, so its merge takes two levels (the level buffers live in
    the fixed array too)."""
    for k, n in enumerate(sizes):
        print(f"noalloc case: n={n} precision={precision} call {k}", flush=True)
        s = workload.make_sample(n, 11 + k)
        ds = osc.DeviceSample.from_host(s)
        (h_ref, p_ref), (h_na, p_na) = run_both(osc, ctx, ds, k % 2, 50, 0.0, 3.0, precision)
        assert_bits_equal(h_na, h_ref, f"hist n={n}")
        assert_bits_equal(p_na, p_ref, f"P n={n}")
        assert np.isfinite(h_ref).all() and h_ref.sum() > 0
        del ds


def test_noalloc_small_and_empty(osc, ctx):
    """A single partial tile, then an empty sample (all-zero histogram)."""
    for n in (517, 0):
        s = workload.make_sample(n, 5)
        ds = osc.DeviceSample.from_host(s)
        (h_ref, p_ref), (h_na, p_na) = run_both(osc, ctx, ds, 0, 7, 0.2, 2.5, 0)
        assert_bits_equal(h_na, h_ref, f"hist n={n}")
        assert_bits_equal(p_na, p_ref, f"P n={n}")
    assert not h_na.any()


def test_noalloc_refuses_beyond_its_array(osc, ctx):
    """3e6 events at 1000 bins need 8 * 1002 * 2944 B = 23.6 MB of tile
    results, more than the fixed 16 MiB: OSC_ERR_BUDGET before anything is
    enqueued; the hist buffer stays untouched.  The same call through
    osc_fill_pdf works."""
    nbins = 1000
    if ctx.max_nbins < nbins:
        pytest.skip("device LDS too small for 1000 bins")
    s = workload.make_sample(3_000_000, 3)
    ds = osc.DeviceSample.from_host(s)
    h = torch.full((nbins + 2,), -7.0, dtype=torch.float64, device="cuda")
    cs = ds.c_struct()
    b = osc.osc_binning(nbins, 0.0, 3.0, 0.0)
    st = osc.load().osc_fill_pdf_noalloc(ctx.handle, ctypes.byref(cs), 0, ctypes.byref(b), 0,
                                         ctypes.c_void_p(h.data_ptr()), None, None)
    assert st == osc.OSC_ERR_BUDGET
    torch.cuda.synchronize()
    assert (h.cpu().numpy() == -7.0).all()
    with pytest.raises(osc.OscError, match="osc_fill_pdf_noalloc"):
        ctx.osc_fill_pdf_noalloc(ds, 0, nbins, 0.0, 3.0, h)
    ctx.osc_fill_pdf(ds, 0, nbins, 0.0, 3.0, h)
    torch.cuda.synchronize()
    assert np.isfinite(h.cpu().numpy()).all()
