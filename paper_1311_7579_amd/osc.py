"""ctypes binding of libosc (the C ABI in include/osc.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libosc.so``.  The functions keep the C names; device buffers
are torch tensors on a ROCm device (their ``data_ptr()`` is passed), and
the stream is torch's current stream unless one is given.

:func:`load` raises when the library is missing: there is no fallback.
"""
import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libosc.so")

OSC_OK = 0
OSC_ERR_INVALID_ARG = 1
OSC_ERR_OUT_OF_MEMORY = 2
OSC_ERR_DEVICE = 3
OSC_ERR_BUDGET = 4
OSC_ERR_NOT_READY = 5

OSC_FP64 = 0
OSC_FP32_MIXED = 1

PARAM_FIELDS = ("sin2_th12", "sin2_th23", "sin2_th13", "dm2_32", "dm2_21", "delta_cp")


class osc_params(ctypes.Structure):
    _fields_ = [(f, ctypes.c_double) for f in PARAM_FIELDS]


class osc_sample(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64),
                ("e_true", ctypes.c_void_p),
                ("flags", ctypes.c_void_p),
                ("weight", ctypes.c_void_p),
                ("e_reco", ctypes.c_void_p),
                ("L_km", ctypes.c_double),
                ("rho_gcc", ctypes.c_double),
                ("Ye", ctypes.c_double)]


class osc_binning(ctypes.Structure):
    _fields_ = [("nbins", ctypes.c_int32), ("lo", ctypes.c_double), ("hi", ctypes.c_double)]


class OscError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {osc_status_string(status)} (status {status})")


_lib = None


def load():
    """Open libosc.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libosc.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    st = ctypes.c_int
    L.osc_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    L.osc_create.restype = st
    L.osc_destroy.argtypes = [vp]
    L.osc_destroy.restype = st
    L.osc_validate_params.argtypes = [ctypes.POINTER(osc_params), i32]
    L.osc_validate_params.restype = st
    L.osc_set_params.argtypes = [vp, ctypes.POINTER(osc_params), i32]
    L.osc_set_params.restype = st
    L.osc_reweight.argtypes = [vp, ctypes.POINTER(osc_sample), i32, vp, vp]
    L.osc_reweight.restype = st
    L.osc_fill_pdf.argtypes = [vp, ctypes.POINTER(osc_sample), i32, ctypes.POINTER(osc_binning),
                               ctypes.c_int, vp, vp, vp]
    L.osc_fill_pdf.restype = st
    L.osc_fill_hist.argtypes = [vp, i64, vp, vp, vp, ctypes.POINTER(osc_binning), vp, vp]
    L.osc_fill_hist.restype = st
    L.osc_profile_enable.argtypes = [vp, ctypes.c_int]
    L.osc_profile_enable.restype = st
    L.osc_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    L.osc_profile_read.restype = st
    L.osc_reduction_layout.argtypes = [ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.osc_reduction_layout.restype = None
    L.osc_occupancy.argtypes = [vp, i32, ctypes.c_int, ctypes.POINTER(i32)]
    L.osc_occupancy.restype = st
    L.osc_max_nbins.argtypes = [vp]
    L.osc_max_nbins.restype = i32
    L.osc_status_string.argtypes = [ctypes.c_int]
    L.osc_status_string.restype = ctypes.c_char_p
    _lib = L
    return L


def osc_status_string(status) -> str:
    try:
        return load().osc_status_string(int(status)).decode()
    except RuntimeError:
        return "unknown"


def _check(status, what):
    if status != OSC_OK:
        raise OscError(status, what)


def to_params(p) -> osc_params:
    if isinstance(p, osc_params):
        return p
    if hasattr(p, "keys"):
        return osc_params(*[float(p[f]) for f in PARAM_FIELDS])
    return osc_params(*[float(v) for v in p])


def params_array(sets):
    sets = list(sets)
    arr = (osc_params * len(sets))()
    for k, p in enumerate(sets):
        arr[k] = to_params(p)
    return arr


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    handle = getattr(stream, "cuda_stream", stream)
    return ctypes.c_void_p(int(handle))


def osc_reduction_layout():
    w, k = ctypes.c_int32(), ctypes.c_int32()
    load().osc_reduction_layout(ctypes.byref(w), ctypes.byref(k))
    return w.value, k.value


def osc_validate_params(sets) -> int:
    arr = params_array(sets)
    return load().osc_validate_params(arr, len(arr))


@dataclass
class DeviceSample:
    """A sample resident in device memory (torch tensors, SoA)."""
    e_true: object
    flags: object
    weight: object = None
    e_reco: object = None
    L_km: float = 295.0
    rho_gcc: float = 2.6
    Ye: float = 0.5

    @property
    def n(self) -> int:
        return int(self.e_true.numel())

    def c_struct(self) -> osc_sample:
        return osc_sample(self.n, _ptr(self.e_true), _ptr(self.flags), _ptr(self.weight),
                          _ptr(self.e_reco), float(self.L_km), float(self.rho_gcc), float(self.Ye))

    @classmethod
    def from_host(cls, s, device="cuda"):
        """Upload a workload.Sample (numpy SoA) once; it stays resident."""
        import torch
        t = lambda a: torch.from_numpy(a).to(device)
        return cls(t(s.e_true), t(s.flags), t(s.weight), t(s.e_reco), s.L_km, s.rho_gcc, s.Ye)


class Context:
    """An osc_ctx on one device."""

    def __init__(self, device: int = 0):
        L = load()
        h = ctypes.c_void_p()
        _check(L.osc_create(ctypes.byref(h), int(device)), "osc_create")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            _check(load().osc_destroy(self.handle), "osc_destroy")
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def max_nbins(self) -> int:
        return load().osc_max_nbins(self.handle)

    def osc_occupancy(self, nbins=50, with_hist=True) -> int:
        w = ctypes.c_int32()
        _check(load().osc_occupancy(self.handle, int(nbins), int(bool(with_hist)), ctypes.byref(w)),
               "osc_occupancy")
        return w.value

    def osc_set_params(self, sets):
        arr = params_array(sets)
        _check(load().osc_set_params(self.handle, arr, len(arr)), "osc_set_params")

    def osc_reweight(self, sample: DeviceSample, set_index, p_out, stream=None):
        cs = sample.c_struct()
        _check(load().osc_reweight(self.handle, ctypes.byref(cs), int(set_index), _ptr(p_out),
                                   _stream(stream)), "osc_reweight")

    def osc_fill_pdf(self, sample: DeviceSample, set_index, nbins, lo, hi, hist_out,
                     p_out=None, precision=OSC_FP64, stream=None):
        cs = sample.c_struct()
        b = osc_binning(int(nbins), float(lo), float(hi))
        _check(load().osc_fill_pdf(self.handle, ctypes.byref(cs), int(set_index), ctypes.byref(b),
                                   int(precision), _ptr(hist_out), _ptr(p_out), _stream(stream)),
               "osc_fill_pdf")

    def osc_profile_enable(self, on=True):
        _check(load().osc_profile_enable(self.handle, int(bool(on))), "osc_profile_enable")

    def osc_profile_read(self):
        """Summed device time (ms) and launch counts since the last enable or
        read: (event_kernel_ms, event_launches, merge_ms, merge_launches)."""
        a, c = ctypes.c_double(), ctypes.c_double()
        b, d = ctypes.c_int64(), ctypes.c_int64()
        _check(load().osc_profile_read(self.handle, ctypes.byref(a), ctypes.byref(b),
                                       ctypes.byref(c), ctypes.byref(d)), "osc_profile_read")
        return a.value, b.value, c.value, d.value

    def osc_fill_hist(self, value, weight, e_reco, nbins, lo, hi, hist_out, stream=None):
        b = osc_binning(int(nbins), float(lo), float(hi))
        n = int(value.numel())
        _check(load().osc_fill_hist(self.handle, n, _ptr(value), _ptr(weight), _ptr(e_reco),
                                    ctypes.byref(b), _ptr(hist_out), _stream(stream)),
               "osc_fill_hist")
