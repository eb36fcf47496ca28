"""Pins of the oracle's piecewise-constant (layered) matter path: one layer
reduces to the constant-density path, a split constant layer and split
vacuum reduce to the unsplit path, unitarity, time reversal of the layer
order at delta = 0, and a brute-force product of matrix exponentials."""
import numpy as np
from scipy.linalg import expm

import oracle
from paper_1311_7579_amd import workload

P1 = workload.TABLE1
# a PREM-like five-layer path through the Earth (crust, mantle, core,
# mantle, crust), lengths in km, densities in g/cm^3
EARTH = [(700.0, 3.3, 0.5), (3500.0, 5.0, 0.495), (3200.0, 11.5, 0.466),
         (3500.0, 5.0, 0.495), (700.0, 3.3, 0.5)]
ASYM = [(400.0, 2.6, 0.5), (1300.0, 8.0, 0.47), (250.0, 0.0, 0.5), (900.0, 4.4, 0.49)]


def test_one_layer_is_constant_density():
    for (a, b, an) in ((1, 1, 0), (1, 0, 1), (0, 2, 0), (2, 0, 1)):
        for E in (0.1, 0.6, 3.0, 25.0):
            got = oracle.prob_layered(P1, [(810.0, 2.84, 0.5)], E, a, b, an)
            assert got == oracle.prob(P1, 810.0, 2.84, 0.5, E, a, b, an)


def test_split_constant_layer_and_split_vacuum():
    rng = np.random.default_rng(4)
    for _ in range(40):
        E = 10 ** rng.uniform(-1, 1.3)
        a, b, an = rng.integers(0, 3), rng.integers(0, 3), rng.integers(0, 2)
        L1, L2 = rng.uniform(10, 2000, 2)
        rho = rng.uniform(1, 12)
        whole = oracle.prob(P1, L1 + L2, rho, 0.5, E, a, b, an)
        split = oracle.prob_layered(P1, [(L1, rho, 0.5), (L2, rho, 0.5)], E, a, b, an)
        assert abs(split - whole) < 1e-12
        vac = oracle.prob_vacuum(P1, L1 + L2, E, a, b, an)
        vsplit = oracle.prob_layered(P1, [(L1, 0.0, 0.5), (L2, 0.0, 0.5)], E, a, b, an)
        assert abs(vsplit - vac) < 1e-12


def test_unitarity_through_the_earth():
    for E in (0.5, 2.0, 4.5, 7.0, 15.0):
        for an in (0, 1):
            for a in range(3):
                s = sum(oracle.prob_layered(P1, EARTH, E, a, b, an) for b in range(3))
                assert abs(s - 1.0) < 1e-13
                s = sum(oracle.prob_layered(P1, EARTH, E, b, a, an) for b in range(3))
                assert abs(s - 1.0) < 1e-13


def test_time_reversal_reverses_the_layer_order():
    # delta = 0: every layer's operator is symmetric, so the transpose of
    # the path's operator is the operator of the reversed path
    p = dict(P1, delta_cp=0.0)
    for E in (0.3, 1.1, 5.0):
        for an in (0, 1):
            for a in range(3):
                for b in range(3):
                    fwd = oracle.prob_layered(p, ASYM, E, a, b, an)
                    rev = oracle.prob_layered(p, ASYM[::-1], E, b, a, an)
                    assert abs(fwd - rev) < 1e-13
    # with CP violation and matter the asymmetric path is not T-symmetric
    q = dict(P1, delta_cp=1.2)
    d = max(abs(oracle.prob_layered(q, ASYM, 1.1, 1, 0, 0) -
                oracle.prob_layered(q, ASYM, 1.1, 0, 1, 0)), 0.0)
    assert d > 1e-4


def _brute(p, layers, E, a, b, an):
    U = oracle.pmns(p, an)
    m2 = np.array([0.0, p["dm2_21"], p["dm2_32"] + p["dm2_21"]])
    H0 = U @ np.diag(m2) @ U.conj().T
    S = np.eye(3, dtype=complex)
    for (L, rho, ye) in layers:
        A = (-1.0 if an else 1.0) * oracle.k_matter() * ye * rho * E
        M = H0 + np.diag([A, 0.0, 0.0])
        S = expm(-1j * oracle.k_phase() * L / E * M) @ S
    return abs(S[b, a]) ** 2


def test_brute_force_matrix_exponentials():
    rng = np.random.default_rng(8)
    for path in (EARTH, ASYM):
        for _ in range(25):
            E = 10 ** rng.uniform(-0.7, 1.3)
            a, b, an = rng.integers(0, 3), rng.integers(0, 3), rng.integers(0, 2)
            got = oracle.prob_layered(P1, path, E, a, b, an)
            assert abs(got - _brute(P1, path, E, a, b, an)) < 1e-11


def test_batch_and_invalid_flags():
    E = np.array([0.5, 1.0, 2.0, 4.0])
    f = np.array([0b00101, 0b00100, 3, 0b10001], np.uint8)
    got = oracle.prob_layered_batch(P1, ASYM, E, f)
    assert got[0] == oracle.prob_layered(P1, ASYM, 0.5, 1, 1, 0)
    assert got[1] == oracle.prob_layered(P1, ASYM, 1.0, 0, 1, 0)
    assert np.isnan(got[2])
    assert got[3] == oracle.prob_layered(P1, ASYM, 4.0, 1, 0, 1)
