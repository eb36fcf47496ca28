"""GPU parity of the piecewise-constant (layered) matter path through the C
ABI: P within 1e-12 of the oracle's product of per-layer operators, the
histogram bit-exact against the reduction contract applied to the GPU's own
P, and argument checks."""
import numpy as np
import pytest

import oracle
from paper_1311_7579_amd import workload
from helpers import bins_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

P_TOL = 1e-12
EARTH = [(700.0, 3.3, 0.5), (3500.0, 5.0, 0.495), (3200.0, 11.5, 0.466),
         (3500.0, 5.0, 0.495), (700.0, 3.3, 0.5)]
ASYM = [(400.0, 2.6, 0.5), (1300.0, 8.0, 0.47), (250.0, 0.0, 0.5), (900.0, 4.4, 0.49)]


@pytest.fixture(scope="module")
def osc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1311_7579_amd import osc as _osc
    _osc.load()
    return _osc


SETS = [workload.TABLE1] + workload.make_random_physics_sets(3, 17)


@pytest.fixture(scope="module")
def ctx(osc):
    c = osc.Context(0)
    c.osc_set_params(SETS)
    yield c
    c.close()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def all_channel_sample(n, seed, e_min=0.1, e_max=30.0):
    rng = np.random.default_rng(seed)
    e = 10 ** rng.uniform(np.log10(e_min), np.log10(e_max), n)
    f = workload.make_flags(rng.integers(0, 3, n), rng.integers(0, 3, n), rng.random(n) < 0.4)
    w = rng.uniform(0.5, 1.5, n)
    x = np.maximum(e * rng.normal(1.0, 0.1, n), 1e-12)
    return workload.Sample(e, f, w, x)


def random_path(seed, n_layers):
    rng = np.random.default_rng(seed)
    return [(float(rng.uniform(0, 300)), float(rng.choice([0.0, rng.uniform(0.5, 13)])),
             float(rng.uniform(0.45, 0.5))) for _ in range(n_layers)]


PATHS = {"earth": EARTH, "asym": ASYM, "one": [(810.0, 2.84, 0.5)],
         "vacuum_split": [(300.0, 0.0, 0.5), (1000.0, 0.0, 0.5)],
         "zero_length": [(0.0, 5.0, 0.5), (600.0, 3.0, 0.5), (0.0, 9.0, 0.5)],
         "max_layers": random_path(5, 32)}


@pytest.mark.parametrize("name", sorted(PATHS))
def test_reweight_layered_against_oracle(osc, ctx, name):
    path = PATHS[name]
    # E >= 0.3 GeV: on the 11600 km Earth path lower energies push the
    # phases towards 1e3 rad, where FP64 rounding of the phase alone nears
    # the 1e-12 tolerance on both sides
    s = all_channel_sample(30_000 if name != "max_layers" else 4_000, 31, e_min=0.3)
    ds = osc.DeviceSample.from_host(s)
    p = torch.empty(s.n, dtype=torch.float64, device="cuda")
    for k, ps in enumerate(SETS):
        ctx.osc_reweight_layered(ds, path, k, p)
        got = host(p)
        want = oracle.prob_layered_batch(ps, path, s.e_true, s.flags)
        assert np.abs(got - want).max() <= P_TOL, (name, k)


def test_one_layer_matches_constant_density_kernel(osc, ctx):
    s = all_channel_sample(50_000, 3)
    s.L_km, s.rho_gcc, s.Ye = 1300.0, 3.0, 0.5
    ds = osc.DeviceSample.from_host(s)
    a = torch.empty(s.n, dtype=torch.float64, device="cuda")
    b = torch.empty(s.n, dtype=torch.float64, device="cuda")
    ctx.osc_reweight(ds, 0, a)
    ctx.osc_reweight_layered(ds, [(1300.0, 3.0, 0.5)], 0, b)
    assert np.abs(host(a) - host(b)).max() <= P_TOL


@pytest.mark.parametrize("n", [1, 1000, 1025, 123_457])
def test_fill_pdf_layered_histogram(osc, ctx, n):
    s = all_channel_sample(n, 7 + n, e_max=10.0)
    bad = np.random.default_rng(n).random(n) < 0.01
    s.flags[bad] = 15
    ds = osc.DeviceSample.from_host(s)
    h = torch.full((42,), -1.0, dtype=torch.float64, device="cuda")
    p = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.osc_fill_pdf_layered(ds, EARTH, 1, 40, 0.0, 10.0, h, p)
    P = host(p)
    want_P = oracle.prob_layered_batch(SETS[1], EARTH, s.e_true, s.flags)
    assert np.array_equal(np.isnan(P), np.isnan(want_P))
    ok = ~np.isnan(want_P)
    assert np.abs(P[ok] - want_P[ok]).max() <= P_TOL
    bins = bins_np(s.e_reco, 0.0, 10.0, 40)
    np.testing.assert_array_equal(host(h), oracle.hist_contract(s.weight * P, bins, 42))


def test_layered_benchmark_workload_full_size(osc, ctx):
    """The layered benchmark form as bench.py launches it: 1e7 events (E
    log-uniform on 0.5-20 GeV, every channel, 40 % antineutrinos, seed 61)
    through the five-layer Earth path, 50 bins on [0, 20] GeV, no P
    written.  Its histogram equals the P-writing call's bit for bit and
    the contract replayed on that P; P is checked against the oracle on
    every 101st event."""
    n = 10_000_000
    rng = np.random.default_rng(61)
    e = 10 ** rng.uniform(np.log10(0.5), np.log10(20.0), n)
    f = workload.make_flags(rng.integers(0, 3, n), rng.integers(0, 3, n), rng.random(n) < 0.4)
    w = rng.uniform(0.5, 1.5, n)
    x = np.maximum(e * rng.normal(1.0, 0.1, n), 1e-12)
    s = workload.Sample(e, f, w, x)
    ds = osc.DeviceSample.from_host(s)
    h0 = torch.empty(52, dtype=torch.float64, device="cuda")
    h1 = torch.empty(52, dtype=torch.float64, device="cuda")
    p = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.osc_fill_pdf_layered(ds, EARTH, 0, 50, 0.0, 20.0, h0)
    ctx.osc_fill_pdf_layered(ds, EARTH, 0, 50, 0.0, 20.0, h1, p)
    h0, h1, P = host(h0), host(h1), host(p)
    np.testing.assert_array_equal(h0, h1)
    bins = bins_np(s.e_reco, 0.0, 20.0, 50)
    np.testing.assert_array_equal(h0, oracle.hist_contract(s.weight * P, bins, 52))
    idx = np.arange(0, n, 101)
    want = oracle.prob_layered_batch(SETS[0], EARTH, s.e_true[idx], s.flags[idx])
    assert np.abs(P[idx] - want).max() <= P_TOL


def test_invalid_layers(osc, ctx):
    s = all_channel_sample(10, 1)
    ds = osc.DeviceSample.from_host(s)
    p = torch.empty(s.n, dtype=torch.float64, device="cuda")
    for path in ([], random_path(1, 33), [(-1.0, 2.0, 0.5)], [(100.0, -2.0, 0.5)],
                 [(100.0, 2.0, 1.5)], [(float("nan"), 2.0, 0.5)]):
        with pytest.raises(osc.OscError):
            ctx.osc_reweight_layered(ds, path, 0, p)
    with pytest.raises(osc.OscError):
        ctx.osc_reweight_layered(ds, EARTH, 17, p)
