"""GPU tests of the serving form (osc_server_*): every served histogram
against the CPU oracle (bit for bit against the contract applied to the
request's own per-event P, and within the tier's tolerance of the oracle's
PDF), results bit-identical to osc_fill_pdf alone and in a concurrent mix,
admission by slot count and scratch budget, the queue refusing what it
cannot take."""
import numpy as np
import pytest

import oracle
from paper_1311_7579_amd import workload
from helpers import MIXED_TOL, P_TOL, assert_bits_equal, hist_tolerance

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
    yield c
    c.close()


@pytest.fixture(scope="module")
def resident(osc):
    samples = workload.make_serving_samples(sizes=(10_000, 100_003, 1_000_000, 3_000_001),
                                            seeds=(61, 62, 63, 64))
    return samples, [osc.DeviceSample.from_host(s) for s in samples]


def plain(osc, ctx, ds, params, tier, want_p=False):
    ctx.osc_set_params([params])
    h = torch.empty(52, dtype=torch.float64, device="cuda")
    p = torch.empty(ds.n, dtype=torch.float64, device="cuda") if want_p else None
    ctx.osc_fill_pdf(ds, 0, 50, 0.0, 3.0, h, p, precision=tier)
    torch.cuda.synchronize()
    return (h.cpu().numpy(), p.cpu().numpy()) if want_p else h.cpu().numpy()


class OracleCheck:
    """Compares a served histogram of (params, sample, tier) with the CPU
    oracle: bit-exact against the oracle's replay of the reduction contract
    on c = w * P, with P the per-event probabilities of a plain call of the
    same set, sample and tier; within the tier's P tolerance, carried
    through the weights, of the oracle's own PDF (its own P)."""

    def __init__(self, osc, ctx, samples, ds):
        self.osc, self.ctx, self.samples, self.ds = osc, ctx, samples, ds
        self.bins = [oracle.bin_indices(s.e_reco, 0.0, 3.0, 50) for s in samples]
        self.checked = {0: 0, 1: 0}
        self.worst = {0: 0.0, 1: 0.0}
        self.cache = {}

    def expected(self, params, sample, tier):
        key = (tuple(params[f] for f in workload.PARAM_FIELDS), sample, tier)
        if key not in self.cache:
            s, b = self.samples[sample], self.bins[sample]
            _, P = plain(self.osc, self.ctx, self.ds[sample], params, tier, want_p=True)
            h_o, P_o = oracle.fill_pdf(params, s.L_km, s.rho_gcc, s.Ye, s.e_true, s.flags,
                                       s.weight, s.e_reco, 50, 0.0, 3.0)
            p_tol = P_TOL if tier == self.osc.OSC_FP64 else MIXED_TOL
            assert np.abs(P - P_o).max() <= p_tol, key
            self.cache[key] = (oracle.hist_contract(s.weight * P, b, 52), h_o,
                               hist_tolerance(s.weight, s.weight * P_o, b, 52, s.n, p_tol=p_tol))
        return self.cache[key]

    def __call__(self, hist, params, sample, tier, what):
        replay, h_o, tol = self.expected(params, sample, tier)
        assert_bits_equal(hist, replay, what)
        dev = np.abs(hist - h_o)
        ratio = float(np.max(np.divide(dev, tol, out=np.zeros_like(dev), where=tol > 0)))
        assert (dev <= tol).all(), (what, ratio)
        self.checked[tier] += 1
        self.worst[tier] = max(self.worst[tier], ratio)


def test_server_alone_equals_mix_equals_plain(osc, ctx, resident):
    samples, ds = resident
    reqs = workload.make_proposal_stream(40, 71, len(ds))
    server = osc.Server(ctx, ds, 50, 0.0, 3.0, slots=6, scratch_budget_bytes=256 << 20)
    try:
        alone = []
        for p, s, tier in reqs:                      # one request at a time
            alone.append(server.wait(server.submit(p, s, tier))[0])
        tickets = [server.submit(p, s, tier) for p, s, tier in reqs]   # all at once
        mix = [server.wait(t)[0] for t in tickets]
        st = server.stats()
    finally:
        server.close()
    check = OracleCheck(osc, ctx, samples, ds)
    for k, (p, s, tier) in enumerate(reqs):
        check(alone[k], p, s, tier, f"request {k} alone")
        check(mix[k], p, s, tier, f"request {k} in the mix")
        np.testing.assert_array_equal(alone[k], mix[k], err_msg=f"request {k}")
        np.testing.assert_array_equal(alone[k], plain(osc, ctx, ds[s], p, tier),
                                      err_msg=f"request {k} vs plain")
    assert check.checked[0] >= 10 and check.checked[1] >= 10     # both tiers served
    print(f"served vs oracle: {check.checked} histograms, largest |dh| / tolerance "
          f"FP64 {check.worst[0]:.3g}, FP32-mixed {check.worst[1]:.3g}")
    assert st["completed"] == 80 and st["failed"] == 0
    assert st["max_in_flight"] > 1          # the mix really ran concurrently


def test_server_admission_by_budget(osc, ctx, resident):
    samples, ds = resident
    server = osc.Server(ctx, ds, 50, 0.0, 3.0, slots=8, scratch_budget_bytes=64 << 20)
    try:
        big = server.request_bytes(3)
        server.close()
        # room for exactly two of the largest requests
        server = osc.Server(ctx, ds, 50, 0.0, 3.0, slots=8,
                            scratch_budget_bytes=2 * ((big + 255) // 256 * 256))
        reqs = [(workload.TABLE1, 3, k % 2) for k in range(12)]
        tickets = [server.submit(p, s, t) for p, s, t in reqs]
        res = [server.wait(t)[0] for t in tickets]
        st = server.stats()
    finally:
        server.close()
    assert st["max_in_flight"] <= 2
    assert st["budget_waits"] >= 1
    assert st["peak_scratch_bytes"] <= 2 * ((big + 255) // 256 * 256)
    for k, (p, s, t) in enumerate(reqs):
        np.testing.assert_array_equal(res[k], plain(osc, ctx, ds[s], p, t))
    check = OracleCheck(osc, ctx, samples, ds)
    for k in (0, 1):                               # one request of each tier
        p, s, t = reqs[k]
        check(res[k], p, s, t, f"budget-bound request {k}")


def test_server_refusals(osc, ctx, resident):
    samples, ds = resident
    server = osc.Server(ctx, ds, 50, 0.0, 3.0, slots=1, scratch_budget_bytes=1 << 20,
                        queue_capacity=2)
    try:
        with pytest.raises(osc.OscError):
            server.submit(workload.TABLE1, 3, 0)        # larger than the whole budget
        with pytest.raises(osc.OscError):
            server.submit(workload.TABLE1, 9, 0)        # no such sample
        with pytest.raises(osc.OscError):
            server.submit(dict(workload.TABLE1, dm2_21=-1.0), 0, 0)
        tickets, refused = [], 0
        for _ in range(50):
            try:
                tickets.append(server.submit(workload.TABLE1, 0, 0))
            except osc.OscError:
                refused += 1
        for t in tickets:
            server.wait(t)
        st = server.stats()
        assert st["rejected"] == refused
        assert st["max_queued"] <= 2
        server.reset_stats()
        st = server.stats()
        assert st["submitted"] == st["completed"] == st["rejected"] == st["max_queued"] == 0
        server.wait(server.submit(workload.TABLE1, 0, 0))
        st = server.stats()
        assert st["submitted"] == st["completed"] == st["max_in_flight"] == 1
    finally:
        server.close()


def test_server_poisson_stream(osc, ctx, resident):
    from paper_1311_7579_amd import serving
    samples, ds = resident
    reqs = workload.make_proposal_stream(200, 72, len(ds))
    arr = workload.poisson_arrivals(200, 2000.0, 73)
    server = osc.Server(ctx, ds, 50, 0.0, 3.0, slots=8, scratch_budget_bytes=256 << 20)
    try:
        res, summ = serving.run_stream(server, reqs, arr, [s.n for s in samples])
    finally:
        server.close()
    assert summ["stats"]["completed"] == 200
    assert 0 < summ["p50_ms"] <= summ["p99_ms"]
    check = OracleCheck(osc, ctx, samples, ds)
    for k in (0, 57, 120, 199):
        p, s, t = reqs[k]
        np.testing.assert_array_equal(res[k], plain(osc, ctx, ds[s], p, t))
        check(res[k], p, s, t, f"stream request {k}")


def test_server_likelihood_and_mcmc(osc, ctx, resident):
    """Sec. 2.2's fitter loop: with data rows set, every request returns
    -2 ln L (Eq. 2) of mu_scale * hist against its sample's row, the value
    the oracle gives for the same histogram; Metropolis chains over the
    server are reproducible and move towards the generating point."""
    import oracle
    from paper_1311_7579_amd import serving
    samples, ds = resident
    truth = workload.TABLE1
    pdfs = np.array([plain(osc, ctx, d, truth, osc.OSC_FP64) for d in ds])
    rng = np.random.default_rng(71)
    mu_scale = 3000.0 / pdfs[2, :50].sum()
    data = rng.poisson(mu_scale * pdfs[:, :50]).astype(float)
    server = osc.Server(ctx, ds, 50, 0.0, 3.0, slots=4, scratch_budget_bytes=64 << 20)
    try:
        r = server.wait(server.submit(truth, 2, osc.OSC_FP64))
        assert np.isnan(r.nll)
        server.set_data(data, mu_scale)
        probe = [truth, dict(truth, sin2_th23=0.42), dict(truth, dm2_32=2.25e-3)]
        for k, p in enumerate(probe):
            for s in (1, 2):
                r = server.wait(server.submit(p, s, osc.OSC_FP64))
                want = oracle.poisson_nll(mu_scale * r.hist[:50], data[s])
                assert r.nll == pytest.approx(want, rel=1e-12), (k, s)
        kw = dict(start=dict(truth, sin2_th23=0.43, dm2_32=2.3e-3),
                  free=("sin2_th23", "dm2_32"), sigmas=(0.02, 3e-5),
                  bounds=((0.3, 0.7), (2.0e-3, 2.8e-3)), n_chains=3, n_steps=60, seed=9,
                  sample=2)
        a = serving.run_mcmc(server, **kw)
        b = serving.run_mcmc(server, **kw)
        np.testing.assert_array_equal(a["chains"], b["chains"])
        np.testing.assert_array_equal(a["nll"], b["nll"])
        assert 0.0 < a["acceptance"] < 1.0
        # the chains end closer (in -2 ln L) to the generating point than they start
        assert np.all(a["nll"][:, -1] < a["nll"][:, 0])
        server.set_data(None)
        assert np.isnan(server.wait(server.submit(truth, 0, osc.OSC_FP64)).nll)
        with pytest.raises(ValueError):
            server.set_data(data[:2], mu_scale)
        with pytest.raises(osc.OscError):
            server.set_data(data, -1.0)
    finally:
        server.close()
