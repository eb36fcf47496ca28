"""GPU parity of the bin-centre reweighting (Sec. 1.1.1) through the C ABI.

  * the migration template: bit-exact against the oracle (each cell's
    weights are added in ascending event order on both sides);
  * P at the true-bin centres: 1e-12 absolute against the oracle;
  * the PDF: bit-exact against the oracle's contraction applied to the
    GPU's own centre probabilities, and within the P tolerance carried
    through the template against the oracle's PDF;
  * the binning effect of Sec. 1.1.1 (a 25 MeV bin at 0.600-0.625 GeV):
    event-by-event against bin-centre, GPU against the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_1311_7579_amd import workload

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

P_TOL = 1e-12


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
    c.osc_set_params([workload.TABLE1] + workload.make_param_sets(3, 3))
    yield c
    c.close()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def mixed_sample(n, seed, L=810.0, rho=2.84):
    """Every channel, 3 % invalid flag bytes, energies partly outside the
    true binning, integer and fractional weights."""
    rng = np.random.default_rng(seed)
    e = 10 ** rng.uniform(-1.3, 1.1, n)
    f = workload.make_flags(rng.integers(0, 3, n), rng.integers(0, 3, n), rng.random(n) < 0.25)
    bad = rng.random(n) < 0.03
    f[bad] = rng.choice(np.array([3, 7, 13, 44, 255], np.uint8), bad.sum())
    w = rng.uniform(0.5, 1.5, n)
    x = np.maximum(e * rng.normal(1.0, 0.12, n), 1e-12)
    return workload.Sample(e, f, w, x, L_km=L, rho_gcc=rho)


def run_bincentre(osc, ctx, s, nt, lo_t, hi_t, nr, lo_r, hi_r, set_index=0, e_scale=0.0):
    ds = osc.DeviceSample.from_host(s)
    tp = osc.Template(ctx, ds, nt, lo_t, hi_t, nr, lo_r, hi_r, e_scale=e_scale)
    try:
        h = torch.full((nr + 2,), -1.0, dtype=torch.float64, device="cuda")
        P = torch.full((18, nt), -1.0, dtype=torch.float64, device="cuda")
        tp.fill_pdf(set_index, h, P)
        return tp.n_used, host(tp.copy()), host(P), host(h)
    finally:
        tp.close()


@pytest.mark.parametrize("n,nt,nr", [(0, 8, 5), (1, 8, 5), (777, 40, 20), (300_000, 100, 50)])
def test_template_and_pdf_against_oracle(osc, ctx, n, nt, nr):
    s = mixed_sample(n, 11 + n)
    lo_t, hi_t, lo_r, hi_r = 0.1, 6.1, 0.0, 5.0
    used, T, P, h = run_bincentre(osc, ctx, s, nt, lo_t, hi_t, nr, lo_r, hi_r)
    T_o, used_o = oracle.template(s.e_true, s.flags, s.weight, s.e_reco, nt, lo_t, hi_t,
                                  nr, lo_r, hi_r)
    assert used == used_o
    np.testing.assert_array_equal(T, T_o)
    P_o = oracle.centre_probs(workload.TABLE1, s.L_km, s.rho_gcc, s.Ye, nt, lo_t, hi_t)
    assert np.abs(P - P_o).max() <= P_TOL
    np.testing.assert_array_equal(h, oracle.bincentre_contract(T, P))
    h_o = oracle.bincentre_contract(T_o, P_o)
    tol = P_TOL * T_o.reshape(nr + 2, -1).sum(axis=1) + 1e-15 * np.abs(h_o)
    assert np.all(np.abs(h - h_o) <= tol)


def test_energy_scale_and_other_sets(osc, ctx):
    s = mixed_sample(50_000, 5, L=1300.0, rho=3.0)
    for k, e_scale in ((1, 0.02), (2, -0.015), (3, 0.0)):
        used, T, P, h = run_bincentre(osc, ctx, s, 64, 0.05, 12.85, 30, 0.0, 6.0, set_index=k,
                                      e_scale=e_scale)
        T_o, used_o = oracle.template(s.e_true, s.flags, s.weight, s.e_reco, 64, 0.05, 12.85,
                                      30, 0.0, 6.0, e_scale)
        np.testing.assert_array_equal(T, T_o)
        p = (workload.TABLE1 if k == 0 else workload.make_param_sets(3, 3)[k - 1])
        P_o = oracle.centre_probs(p, s.L_km, s.rho_gcc, s.Ye, 64, 0.05, 12.85)
        assert np.abs(P - P_o).max() <= P_TOL
        np.testing.assert_array_equal(h, oracle.bincentre_contract(T, P))


def test_internal_table_and_determinism(osc, ctx):
    s = mixed_sample(20_000, 9)
    ds = osc.DeviceSample.from_host(s)
    tp = osc.Template(ctx, ds, 50, 0.1, 5.1, 25, 0.0, 5.0)
    try:
        h1 = torch.empty(27, dtype=torch.float64, device="cuda")
        h2 = torch.empty(27, dtype=torch.float64, device="cuda")
        P = torch.empty((18, 50), dtype=torch.float64, device="cuda")
        tp.fill_pdf(0, h1)
        tp.fill_pdf(0, h2, P)
        a, b = host(h1), host(h2)
        np.testing.assert_array_equal(a, b)
        tp2 = osc.Template(ctx, ds, 50, 0.1, 5.1, 25, 0.0, 5.0)
        np.testing.assert_array_equal(host(tp.copy()), host(tp2.copy()))
        tp2.close()
    finally:
        tp.close()


def test_invalid_arguments(osc, ctx):
    s = mixed_sample(100, 1)
    ds = osc.DeviceSample.from_host(s)
    bad = [dict(nt=0, lo_t=0.1, hi_t=1.0), dict(nt=10, lo_t=-0.1, hi_t=1.0),
           dict(nt=10, lo_t=1.0, hi_t=1.0), dict(nt=70000, lo_t=0.1, hi_t=1.0)]
    for b in bad:
        with pytest.raises(osc.OscError):
            osc.Template(ctx, ds, b["nt"], b["lo_t"], b["hi_t"], 10, 0.0, 1.0)
    with pytest.raises(osc.OscError):
        osc.Template(ctx, ds, 10, 0.1, 1.0, 0, 0.0, 1.0)
    tp = osc.Template(ctx, ds, 10, 0.1, 1.0, 10, 0.0, 1.0)
    try:
        h = torch.empty(12, dtype=torch.float64, device="cuda")
        with pytest.raises(osc.OscError):
            tp.fill_pdf(99, h)
    finally:
        tp.close()


def test_binning_effect_against_oracle(osc, ctx):
    """Sec. 1.1.1: one 25 MeV true bin at 0.600-0.625 GeV, nu_mu -> nu_mu at
    295 km, flat flux (events at the midpoints of 200000 equal slices).
    Event-by-event: osc_fill_pdf with the reco energy equal to the true one
    and that single bin.  Bin-centre: the template path."""
    n = 200_000
    e = 0.600 + (np.arange(n) + 0.5) * (0.025 / n)
    f = workload.make_flags(np.ones(n, int), np.ones(n, int), np.zeros(n, bool))
    s = workload.Sample(e, f, np.ones(n), e.copy(), L_km=295.0, rho_gcc=2.6)
    ds = osc.DeviceSample.from_host(s)
    h = torch.empty(3, dtype=torch.float64, device="cuda")
    ctx.osc_fill_pdf(ds, 0, 1, 0.600, 0.625, h)
    ebe = host(h)[0]
    used, T, P, hb = run_bincentre(osc, ctx, s, 1, 0.600, 0.625, 1, 0.600, 0.625)
    assert used == n
    bc = hb[0]
    effect = ebe / bc - 1.0
    P_o = oracle.prob_batch(workload.TABLE1, 295.0, 2.6, 0.5, e, f)
    ebe_o = float(np.sum(P_o))
    bc_o = n * oracle.prob(workload.TABLE1, 295.0, 2.6, 0.5, 0.6125, 1, 1, 0)
    assert ebe == pytest.approx(ebe_o, rel=1e-10)
    assert bc == pytest.approx(bc_o, rel=1e-10)
    assert effect == pytest.approx(ebe_o / bc_o - 1.0, abs=1e-9)
    assert 0.02 < effect < 0.05


def test_full_size_template(osc, ctx):
    """The 1e7-event workload: 200 true bins on [0.1, 10.1] GeV, 50 reco
    bins on [0, 3] GeV."""
    s = workload.make_sample(10_000_000, 1)
    used, T, P, h = run_bincentre(osc, ctx, s, 200, 0.1, 10.1, 50, 0.0, 3.0)
    T_o, used_o = oracle.template(s.e_true, s.flags, s.weight, s.e_reco, 200, 0.1, 10.1,
                                  50, 0.0, 3.0)
    assert used == used_o
    np.testing.assert_array_equal(T, T_o)
    np.testing.assert_array_equal(h, oracle.bincentre_contract(T, P))
    P_o = oracle.centre_probs(workload.TABLE1, s.L_km, s.rho_gcc, s.Ye, 200, 0.1, 10.1)
    assert np.abs(P - P_o).max() <= P_TOL
