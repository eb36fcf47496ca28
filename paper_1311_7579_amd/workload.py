"""Seeded synthetic inputs shared by the GPU path, the tests and the bench.

This module only draws random numbers and lays them out; it holds none of
the oscillation or histogram arithmetic.  Every draw uses numpy's PCG64
generator from an explicit seed, in a fixed order, so the same seed gives
the same bytes on every host.

Event layout (struct of arrays, one entry per Monte Carlo event):
  e_true  float64  true neutrino energy, GeV
  flags   uint8    bits 0-1 initial flavour, bits 2-3 final flavour
                   (0 = e, 1 = mu, 2 = tau), bit 4 antineutrino
  weight  float64  Monte Carlo weight
  e_reco  float64  reconstructed energy, GeV
"""
from dataclasses import dataclass, field
import math

import numpy as np

FLAV_E, FLAV_MU, FLAV_TAU = 0, 1, 2
ANTI_BIT = 1 << 4


def make_flags(alpha, beta, anti):
    """Pack flavour indices and the antineutrino flag into flag bytes."""
    a = np.asarray(alpha, dtype=np.uint8)
    b = np.asarray(beta, dtype=np.uint8)
    n = np.asarray(anti, dtype=bool).astype(np.uint8)
    return (a | (b << 2) | (n << 4)).astype(np.uint8)


# Table 1 of the paper: the oscillation parameters assumed for all studies,
# with the 295 km baseline and 2.6 g/cm^3 density.
TABLE1 = dict(sin2_th12=0.311, sin2_th23=0.5, sin2_th13=0.0251,
              dm2_32=2.4e-3, dm2_21=7.6e-5, delta_cp=0.0)
TABLE1_L_KM = 295.0
TABLE1_RHO = 2.6
YE = 0.5

PARAM_FIELDS = ("sin2_th12", "sin2_th23", "sin2_th13", "dm2_32", "dm2_21", "delta_cp")


@dataclass
class Sample:
    e_true: np.ndarray
    flags: np.ndarray
    weight: np.ndarray
    e_reco: np.ndarray
    L_km: float = TABLE1_L_KM
    rho_gcc: float = TABLE1_RHO
    Ye: float = YE
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.e_true.size)


def make_sample(n, seed, L_km=TABLE1_L_KM, rho_gcc=TABLE1_RHO, Ye=YE,
                e_range=(0.1, 10.0), p_appearance=0.5, p_anti=0.2,
                w_range=(0.5, 1.5), smear=0.1, reco_floor=1e-12) -> Sample:
    """Synthetic Monte Carlo sample of the paper's long-baseline workload.

    Draw order (one PCG64 stream): log10(E) ~ U(log10 lo, log10 hi);
    channel u ~ U(0,1) (u < p_appearance -> nu_mu -> nu_e, else
    nu_mu -> nu_mu); antineutrino u ~ U(0,1) < p_anti; weight ~ U(w_range);
    smearing factor ~ N(1, smear); e_reco = max(E * factor, reco_floor).
    """
    n = int(n)
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = e_range
    e_true = 10.0 ** rng.uniform(math.log10(lo), math.log10(hi), n)
    appear = rng.random(n) < p_appearance
    anti = rng.random(n) < p_anti
    weight = rng.uniform(w_range[0], w_range[1], n)
    factor = rng.normal(1.0, smear, n)
    e_reco = np.maximum(e_true * factor, reco_floor)
    beta = np.where(appear, FLAV_E, FLAV_MU)
    flags = make_flags(np.full(n, FLAV_MU), beta, anti)
    return Sample(e_true=e_true, flags=flags, weight=weight, e_reco=e_reco,
                  L_km=float(L_km), rho_gcc=float(rho_gcc), Ye=float(Ye), seed=seed,
                  meta=dict(kind="longbaseline", e_range=e_range))


def make_uniform_energy_sample(n, seed, e_max=30.0, e_min=1e-3, **kw) -> Sample:
    """Validation workload of Sec. 2.2: energies uniform on (0, e_max] GeV.

    Energies below e_min are redrawn from the same stream's tail (phases
    grow like 1/E, so the near-zero tail is excluded); every flavour
    channel and both neutrino kinds appear uniformly.
    """
    n = int(n)
    rng = np.random.Generator(np.random.PCG64(seed))
    e = rng.uniform(0.0, e_max, n)
    low = e < e_min
    e[low] = rng.uniform(e_min, e_max, int(low.sum()))
    alpha = rng.integers(0, 3, n)
    beta = rng.integers(0, 3, n)
    anti = rng.random(n) < 0.5
    weight = rng.uniform(0.5, 1.5, n)
    e_reco = np.maximum(e * rng.normal(1.0, 0.1, n), 1e-12)
    return Sample(e_true=e, flags=make_flags(alpha, beta, anti), weight=weight,
                  e_reco=e_reco, seed=seed, meta=dict(kind="uniform", e_max=e_max), **kw)


def make_param_sets(n_sets, seed, base=None,
                    sin2_th23=(0.4, 0.6), dm2_32=(2.2e-3, 2.6e-3),
                    delta_cp=(-math.pi, math.pi), sin2_th13=(0.02, 0.03)):
    """Random oscillation parameter sets around Table 1.

    Draw order per call: all sin^2 theta23, then all dm^2_32, then all
    delta_cp, then all sin^2 theta13 (each uniform on its range); the other
    parameters stay at ``base`` (Table 1 by default).
    """
    base = dict(TABLE1 if base is None else base)
    rng = np.random.Generator(np.random.PCG64(seed))
    s23 = rng.uniform(*sin2_th23, n_sets)
    d32 = rng.uniform(*dm2_32, n_sets)
    dcp = rng.uniform(*delta_cp, n_sets)
    s13 = rng.uniform(*sin2_th13, n_sets)
    out = []
    for k in range(n_sets):
        p = dict(base)
        p.update(sin2_th23=float(s23[k]), dm2_32=float(d32[k]),
                 delta_cp=float(dcp[k]), sin2_th13=float(s13[k]))
        out.append(p)
    return out


def make_random_physics_sets(n_sets, seed):
    """Broad random parameter sets for invariance tests: every angle in
    (0, pi/2), both mass orderings, any CP phase."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n_sets):
        s12, s23, s13 = rng.uniform(0.05, 0.95, 3)
        d21 = rng.uniform(2e-5, 2e-4)
        d32 = rng.uniform(1e-3, 4e-3) * (1 if rng.random() < 0.5 else -1)
        dcp = rng.uniform(-math.pi, math.pi)
        out.append(dict(sin2_th12=float(s12), sin2_th23=float(s23), sin2_th13=float(s13),
                        dm2_32=float(d32), dm2_21=float(d21), delta_cp=float(dcp)))
    return out


def make_batched_samples(sizes=(100_000, 500_000, 2_000_000, 5_000_000),
                         L_km=(295.0, 810.0, 1300.0, 2500.0), seeds=(41, 42, 43, 44),
                         rho_range=(2.4, 3.0), rho_seed=40):
    """Uneven samples of the batched form: one long-baseline sample per
    (size, baseline, seed); densities drawn uniformly on rho_range from
    their own PCG64 stream (one draw per sample, in order)."""
    rng = np.random.Generator(np.random.PCG64(rho_seed))
    rhos = rng.uniform(rho_range[0], rho_range[1], len(sizes))
    return [make_sample(n, seed, L_km=L, rho_gcc=float(r))
            for n, L, seed, r in zip(sizes, L_km, seeds, rhos)]


SERVING_SIZES = tuple(int(round(v)) for v in np.geomspace(1e4, 2e7, 8))


def make_serving_samples(sizes=SERVING_SIZES, seeds=tuple(range(51, 59)),
                         baselines=(295.0, 810.0, 1300.0, 2500.0), rho_range=(2.4, 3.0),
                         rho_seed=50):
    """The resident samples of the serving form: log-spaced sizes, baselines
    cycling through `baselines`, densities U(rho_range) from their own
    PCG64 stream (one draw per sample, in order)."""
    rng = np.random.Generator(np.random.PCG64(rho_seed))
    rhos = rng.uniform(rho_range[0], rho_range[1], len(sizes))
    return [make_sample(n, seed, L_km=baselines[k % len(baselines)], rho_gcc=float(rhos[k]))
            for k, (n, seed) in enumerate(zip(sizes, seeds))]


def make_proposal_stream(n, seed, n_samples, start=None, step=0.01, p_mixed=0.5):
    """Metropolis-style proposals around Table 1: a random walk where each
    proposal takes Gaussian steps of relative size `step` on the five
    positive parameters (sin^2 clipped to [0, 1]) and an additive
    step * 2 pi on delta_cp (wrapped to (-pi, pi]); every proposal becomes
    the next state.  Each request also draws a sample index uniformly and a
    precision tier (1 = FP32-mixed with probability p_mixed, else 0 = FP64).
    Draw order per request: five relative steps, the phase step, the sample
    index, the tier."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cur = dict(TABLE1 if start is None else start)
    out = []
    pos = ("sin2_th12", "sin2_th23", "sin2_th13", "dm2_32", "dm2_21")
    for _ in range(n):
        rel = rng.normal(0.0, step, 5)
        dphi = rng.normal(0.0, step * 2 * math.pi)
        sample = int(rng.integers(0, n_samples))
        tier = int(rng.random() < p_mixed)
        nxt = dict(cur)
        for k, f in enumerate(pos):
            nxt[f] = cur[f] * (1.0 + rel[k])
        for f in ("sin2_th12", "sin2_th23", "sin2_th13"):
            nxt[f] = min(max(nxt[f], 0.0), 1.0)
        d = cur["delta_cp"] + dphi
        nxt["delta_cp"] = math.remainder(d, 2 * math.pi) if abs(d) > math.pi else d
        out.append((nxt, sample, tier))
        cur = nxt
    return out


def poisson_arrivals(n, rate_hz, seed):
    """Arrival times (s) of a Poisson process: cumulative exponential gaps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate_hz, n))


# The evaluation workloads: per-event parity case, the full-size plain
# case, the precision form, the batched form and the serving form.
C1 = dict(name="plain-fp64-1e5", n=100_000, seed=1)
C2 = dict(name="plain-fp64-pdf-1e7", n=10_000_000, seed=1, nbins=50, lo=0.0, hi=3.0)
C3 = dict(name="precision-1e7x64", n=10_000_000, seed=1, n_sets=64, set_seed=3)
C4 = dict(name="batched-256x4", sizes=(100_000, 500_000, 2_000_000, 5_000_000),
          L_km=(295.0, 810.0, 1300.0, 2500.0), rho_range=(2.4, 3.0),
          seeds=(41, 42, 43, 44), n_sets=256, set_seed=4, rho_seed=40)
