"""Host-side checks of the Python binding's argument validation: tensors
that a kernel would read or write out of bounds (wrong dtype, wrong length,
not contiguous, not in GPU memory) are refused with ValueError before
anything reaches the library.  Runs without a GPU."""
import pytest

torch = pytest.importorskip("torch")

from paper_1311_7579_amd import osc  # noqa: E402


def f64(n):
    return torch.zeros(n, dtype=torch.float64)


def u8(n):
    return torch.zeros(n, dtype=torch.uint8)


@pytest.mark.parametrize("kw,match", [
    (dict(dtype="float64", t=torch.zeros(4, dtype=torch.float32)), "must be float64"),
    (dict(dtype="uint8", t=torch.zeros(4, dtype=torch.int32)), "must be uint8"),
    (dict(dtype="float64", t=f64(8)[::2]), "contiguous"),
    (dict(dtype="float64", t=f64(5), n=4), "must have 4 entries"),
    (dict(dtype="float64", t=f64(7), multiple_of=3), "multiple of 3"),
    (dict(dtype="float64", t=[0.0, 1.0]), "torch tensor"),
    (dict(dtype="float64", t=None), "is required"),
    (dict(dtype="float64", t=f64(4), n=4), "GPU memory"),
])
def test_device_vec_refusals(kw, match):
    t = kw.pop("t")
    with pytest.raises(ValueError, match=match):
        osc.device_vec(t, "x", **kw)


def test_device_vec_optional_none():
    assert osc.device_vec(None, "x", "float64", optional=True) is None


@pytest.mark.parametrize("args,match", [
    ((torch.zeros(4, dtype=torch.float32), u8(4)), "e_true must be float64"),
    ((f64(4), u8(3)), "flags must have 4 entries"),
    ((f64(4), torch.zeros(4, dtype=torch.int8)), "flags must be uint8"),
    ((f64(4), u8(4), f64(5)), "weight must have 4 entries"),
    ((f64(4), u8(4), f64(4), f64(8)[::2]), "e_reco must be contiguous"),
    ((f64(4), u8(4)), "GPU memory"),
])
def test_device_sample_refusals(args, match):
    with pytest.raises(ValueError, match=match):
        osc.DeviceSample(*args)


def test_context_wrappers_refuse_before_the_library():
    """Output buffers of the wrong size or dtype are refused by every
    wrapper before its C call (a context object without a device handle:
    any call that got through would fail on the NULL handle instead)."""
    ctx = object.__new__(osc.Context)
    ctx.handle, ctx.device = None, 0
    sample = object.__new__(osc.DeviceSample)
    sample.e_true, sample.flags, sample.weight, sample.e_reco = f64(4), u8(4), f64(4), f64(4)
    sample.L_km, sample.rho_gcc, sample.Ye = 295.0, 2.6, 0.5
    with pytest.raises(ValueError, match="hist_out must have 52 entries"):
        ctx.osc_fill_pdf(sample, 0, 50, 0.0, 3.0, f64(51))
    with pytest.raises(ValueError, match="hist_out must be float64"):
        ctx.osc_fill_hist(f64(4), f64(4), f64(4), 50, 0.0, 3.0, torch.zeros(52))
    with pytest.raises(ValueError, match="weight must have 4 entries"):
        ctx.osc_fill_hist(f64(4), f64(3), f64(4), 50, 0.0, 3.0, f64(52))
    with pytest.raises(ValueError, match="nll_out must have 2 entries"):
        ctx.osc_poisson_nll(f64(104), f64(50).reshape(1, 50), f64(3))
    with pytest.raises(ValueError, match="hist must have a multiple of 52"):
        ctx.osc_poisson_nll(f64(100), f64(50).reshape(1, 50), f64(1))
    with pytest.raises(ValueError, match="reads weight and e_reco"):
        sample.weight = None
        ctx.osc_fill_pdf(sample, 0, 50, 0.0, 3.0, f64(52))
