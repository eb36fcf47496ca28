"""CPU FP64 oracle for event-by-event oscillation reweighting.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark load this package.  It wraps
``liboscoracle.so`` (plain C, see ``osc_oracle.c``) with ctypes and shares
no code with the GPU library.

Parameter sets are passed as a mapping with the keys
``sin2_th12, sin2_th23, sin2_th13, dm2_32, dm2_21, delta_cp`` or as a
sequence in that order.
"""
import ctypes
import os

import numpy as np

from .build import LIB as _LIB_PATH
from .build import NATIVE_LIB as _NATIVE_LIB_PATH

_FIELDS = ("sin2_th12", "sin2_th23", "sin2_th13", "dm2_32", "dm2_21", "delta_cp")

# tile reduction contract of the binned PDF: W lanes x K events per lane,
# A accumulators per bin (lane l adds into accumulator l mod A)
CONTRACT_W = 64
CONTRACT_K = 16
CONTRACT_A = 8


class OracleParams(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double) for f in _FIELDS]


def to_params(p) -> OracleParams:
    if isinstance(p, OracleParams):
        return p
    if hasattr(p, "keys"):
        return OracleParams(*[float(p[f]) for f in _FIELDS])
    if hasattr(p, "sin2_th12"):
        return OracleParams(*[float(getattr(p, f)) for f in _FIELDS])
    vals = [float(v) for v in p]
    if len(vals) != 6:
        raise ValueError("a parameter set has six values")
    return OracleParams(*vals)


_lib = None


def use_native_build() -> str:
    """Switch this process to the -O3 -march=native build of the same
    source (building it for this host first): CPU timing only; the tests
    use the portable build."""
    global _lib, _LIB_PATH
    from .build import build
    build(native=True)
    _LIB_PATH, _lib = _NATIVE_LIB_PATH, None
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"oracle library not built: {_LIB_PATH} "
                               "(run __graft_entry__.build() or oracle/build.py)")
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(OracleParams)
        d, i32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
        vp = ctypes.c_void_p
        L.oracle_k_phase.restype = d
        L.oracle_k_matter.restype = d
        L.oracle_pmns.argtypes = [P, ctypes.c_int, vp]
        L.oracle_prob_vacuum.argtypes = [P, d, d, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oracle_prob_vacuum.restype = d
        L.oracle_prob.argtypes = [P, d, d, d, d, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.oracle_prob.restype = d
        L.oracle_prob_batch.argtypes = [P, d, d, d, i64, vp, vp, vp]
        L.oracle_prob_batch.restype = ctypes.c_int
        L.oracle_bin_index.argtypes = [d, d, d, i32]
        L.oracle_bin_index.restype = i32
        L.oracle_hist_contract.argtypes = [vp, vp, i64, i32, i32, i32, i32, vp]
        L.oracle_fill_pdf.argtypes = [P, d, d, d, i64, vp, vp, vp, vp, i32, d, d, d, i32, i32, i32, vp,
                                      vp]
        L.oracle_bin_index_scaled.argtypes = [d, d, d, d, i32]
        L.oracle_bin_index_scaled.restype = i32
        L.oracle_bin_indices_scaled.argtypes = [i64, vp, d, d, d, i32, vp]
        L.oracle_bin_indices_scaled.restype = None
        L.oracle_fill_pdf.restype = ctypes.c_int
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_prob_layered.argtypes = [P, i32, vp, vp, vp, d, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int]
        L.oracle_prob_layered.restype = d
        L.oracle_prob_layered_batch.argtypes = [P, i32, vp, vp, vp, i64, vp, vp, vp]
        L.oracle_template.argtypes = [i64, vp, vp, vp, vp, i32, d, d, i32, d, d, d, vp, vp]
        L.oracle_bin_centre.argtypes = [d, d, i32, i32]
        L.oracle_bin_centre.restype = d
        L.oracle_centre_probs.argtypes = [P, d, d, d, i32, d, d, vp]
        L.oracle_bincentre_contract.argtypes = [vp, vp, i32, i32, vp]
        L.oracle_poisson_nll.argtypes = [vp, vp, i32]
        L.oracle_poisson_nll.restype = d
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def k_phase() -> float:
    return lib().oracle_k_phase()


def k_matter() -> float:
    return lib().oracle_k_matter()


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(n: int) -> None:
    lib().oracle_set_num_threads(int(n))


def pmns(params, anti=False) -> np.ndarray:
    out = np.zeros(18, dtype=np.float64)
    pp = to_params(params)
    lib().oracle_pmns(ctypes.byref(pp), int(bool(anti)), _ptr(out))
    return (out[0::2] + 1j * out[1::2]).reshape(3, 3)


def prob_vacuum(params, L_km, E, alpha, beta, anti=False) -> float:
    pp = to_params(params)
    return lib().oracle_prob_vacuum(ctypes.byref(pp), float(L_km), float(E),
                                    int(alpha), int(beta), int(bool(anti)))


def prob(params, L_km, rho, Ye, E, alpha, beta, anti=False) -> float:
    pp = to_params(params)
    return lib().oracle_prob(ctypes.byref(pp), float(L_km), float(rho), float(Ye),
                             float(E), int(alpha), int(beta), int(bool(anti)))


def prob_batch(params, L_km, rho, Ye, e_true, flags) -> np.ndarray:
    e = np.ascontiguousarray(e_true, dtype=np.float64)
    f = np.ascontiguousarray(flags, dtype=np.uint8)
    if e.shape != f.shape:
        raise ValueError("e_true and flags differ in length")
    out = np.empty_like(e)
    pp = to_params(params)
    lib().oracle_prob_batch(ctypes.byref(pp), float(L_km), float(rho), float(Ye),
                            e.size, _ptr(e), _ptr(f), _ptr(out))
    return out


def bin_index(x, lo, hi, nbins) -> int:
    return lib().oracle_bin_index(float(x), float(lo), float(hi), int(nbins))


def bin_indices(x, lo, hi, nbins, e_scale=0.0) -> np.ndarray:
    """oracle_bin_index_scaled of every element (one C loop)."""
    v = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
    out = np.empty(v.size, dtype=np.int32)
    lib().oracle_bin_indices_scaled(v.size, _ptr(v), float(e_scale), float(lo), float(hi),
                                    int(nbins), _ptr(out))
    return out


def bin_index_scaled(x, lo, hi, nbins, e_scale=0.0) -> int:
    return lib().oracle_bin_index_scaled(float(x), float(e_scale), float(lo), float(hi),
                                         int(nbins))


def hist_contract(c, bins, nbt, W=CONTRACT_W, K=CONTRACT_K, A=CONTRACT_A) -> np.ndarray:
    c = np.ascontiguousarray(c, dtype=np.float64)
    b = np.ascontiguousarray(bins, dtype=np.int32)
    if c.shape != b.shape:
        raise ValueError("c and bins differ in length")
    if b.size and (b.min() < 0 or b.max() >= nbt):
        raise ValueError("bin index out of range")
    if W % A or A & (A - 1) or W & (W - 1) or K & (K - 1):
        raise ValueError("W, K, A must be powers of two with A dividing W")
    out = np.zeros(int(nbt), dtype=np.float64)
    lib().oracle_hist_contract(_ptr(c), _ptr(b), c.size, int(nbt), int(W), int(K), int(A),
                               _ptr(out))
    return out


def _layers(layers):
    a = np.ascontiguousarray(np.asarray(layers, dtype=np.float64).reshape(-1, 3))
    return (np.ascontiguousarray(a[:, 0]), np.ascontiguousarray(a[:, 1]),
            np.ascontiguousarray(a[:, 2]))


def prob_layered(params, layers, E, alpha, beta, anti) -> float:
    """P through layers [(L_km, rho, Ye), ...], the first crossed first."""
    L, r, y = _layers(layers)
    pp = to_params(params)
    return lib().oracle_prob_layered(ctypes.byref(pp), L.size, _ptr(L), _ptr(r), _ptr(y),
                                     float(E), int(alpha), int(beta), int(anti))


def prob_layered_batch(params, layers, E, flags) -> np.ndarray:
    L, r, y = _layers(layers)
    e = np.ascontiguousarray(E, dtype=np.float64)
    f = np.ascontiguousarray(flags, dtype=np.uint8)
    out = np.empty_like(e)
    pp = to_params(params)
    lib().oracle_prob_layered_batch(ctypes.byref(pp), L.size, _ptr(L), _ptr(r), _ptr(y), e.size,
                                    _ptr(e), _ptr(f), _ptr(out))
    return out


N_CHANNELS = 18   # alpha + 3 beta + 9 anti


def template(e_true, flags, weight, e_reco, nt, lo_t, hi_t, nr, lo_r, hi_r, e_scale=0.0):
    """Migration template T[r][c][t] of the bin-centre method and the number
    of events it holds."""
    e = np.ascontiguousarray(e_true, dtype=np.float64)
    f = np.ascontiguousarray(flags, dtype=np.uint8)
    w = np.ascontiguousarray(weight, dtype=np.float64)
    r = np.ascontiguousarray(e_reco, dtype=np.float64)
    if not (e.shape == f.shape == w.shape == r.shape):
        raise ValueError("event arrays differ in length")
    T = np.zeros((int(nr) + 2, N_CHANNELS, int(nt)), dtype=np.float64)
    used = ctypes.c_int64()
    lib().oracle_template(e.size, _ptr(e), _ptr(f), _ptr(w), _ptr(r), int(nt), float(lo_t),
                          float(hi_t), int(nr), float(lo_r), float(hi_r), float(e_scale), _ptr(T),
                          ctypes.byref(used))
    return T, used.value


def bin_centre(lo, hi, nt, t) -> float:
    return lib().oracle_bin_centre(float(lo), float(hi), int(nt), int(t))


def centre_probs(params, L_km, rho, Ye, nt, lo_t, hi_t) -> np.ndarray:
    """P[c][t] at the true-bin centres for the 18 channels."""
    P = np.zeros((N_CHANNELS, int(nt)), dtype=np.float64)
    pp = to_params(params)
    lib().oracle_centre_probs(ctypes.byref(pp), float(L_km), float(rho), float(Ye), int(nt),
                              float(lo_t), float(hi_t), _ptr(P))
    return P


def bincentre_contract(T, P) -> np.ndarray:
    """hist[r] = sum_k fl(T[r][k] P[k]) in the lane-strided tree order."""
    T = np.ascontiguousarray(T, dtype=np.float64)
    P = np.ascontiguousarray(P, dtype=np.float64)
    nrt = T.shape[0]
    K = P.size
    if T.size != nrt * K:
        raise ValueError("template and probability table do not match")
    hist = np.zeros(nrt, dtype=np.float64)
    lib().oracle_bincentre_contract(_ptr(T), _ptr(P), int(K), int(nrt), _ptr(hist))
    return hist


def poisson_nll(mu, data) -> float:
    m = np.ascontiguousarray(mu, dtype=np.float64)
    d = np.ascontiguousarray(data, dtype=np.float64)
    if m.shape != d.shape:
        raise ValueError("mu and data differ in length")
    return lib().oracle_poisson_nll(_ptr(m), _ptr(d), m.size)


def fill_pdf(params, L_km, rho, Ye, e_true, flags, weight, e_reco, nbins, lo, hi,
             W=CONTRACT_W, K=CONTRACT_K, A=CONTRACT_A, want_p=True, e_scale=0.0):
    e = np.ascontiguousarray(e_true, dtype=np.float64)
    f = np.ascontiguousarray(flags, dtype=np.uint8)
    w = np.ascontiguousarray(weight, dtype=np.float64)
    r = np.ascontiguousarray(e_reco, dtype=np.float64)
    if not (e.shape == f.shape == w.shape == r.shape):
        raise ValueError("event arrays differ in length")
    hist = np.zeros(int(nbins) + 2, dtype=np.float64)
    p = np.empty_like(e) if want_p else None
    pp = to_params(params)
    lib().oracle_fill_pdf(ctypes.byref(pp), float(L_km), float(rho), float(Ye), e.size,
                          _ptr(e), _ptr(f), _ptr(w), _ptr(r), int(nbins), float(lo), float(hi),
                          float(e_scale), int(W), int(K), int(A), _ptr(hist), _ptr(p) if p is not None else ctypes.c_void_p(0))
    return hist, p
