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
from typing import NamedTuple

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
# device scratch of osc_fill_pdf_noalloc (include/osc.h)
OSC_NOALLOC_SCRATCH_BYTES = 16 << 20

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
    _fields_ = [("nbins", ctypes.c_int32), ("lo", ctypes.c_double), ("hi", ctypes.c_double),
                ("e_scale", ctypes.c_double)]


class osc_layer(ctypes.Structure):
    _fields_ = [("L_km", ctypes.c_double), ("rho_gcc", ctypes.c_double), ("Ye", ctypes.c_double)]


def layers_array(layers):
    """(L_km, rho_gcc, Ye) triples (or osc_layer) -> ctypes array."""
    items = [l if isinstance(l, osc_layer) else osc_layer(*map(float, l)) for l in layers]
    return (osc_layer * len(items))(*items)


class osc_batch_config(ctypes.Structure):
    _fields_ = [("sets_per_item", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("use_graph", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


SCHEDULE_DYNAMIC, SCHEDULE_STATIC, SCHEDULE_ONE_PER_BLOCK = 0, 1, 2


class osc_server_config(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("queue_capacity", ctypes.c_int32),
                ("scratch_budget_bytes", ctypes.c_int64)]


class osc_server_stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in (
        "submitted", "admitted", "completed", "failed", "rejected", "in_flight", "max_in_flight",
        "queued", "max_queued", "budget_waits", "peak_scratch_bytes", "scratch_in_use_bytes")]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


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
    L.osc_fill_pdf_noalloc.argtypes = L.osc_fill_pdf.argtypes
    L.osc_fill_pdf_noalloc.restype = st
    L.osc_binned_create.argtypes = [vp, ctypes.POINTER(osc_sample), ctypes.POINTER(osc_binning),
                                    ctypes.POINTER(vp)]
    L.osc_binned_create.restype = st
    L.osc_binned_destroy.argtypes = [vp]
    L.osc_binned_destroy.restype = st
    L.osc_fill_pdf_binned.argtypes = [vp, vp, i32, ctypes.c_int, vp, vp, vp]
    L.osc_fill_pdf_binned.restype = st
    L.osc_fill_hist.argtypes = [vp, i64, vp, vp, vp, ctypes.POINTER(osc_binning), vp, vp]
    L.osc_fill_hist.restype = st
    L.osc_profile_enable.argtypes = [vp, ctypes.c_int]
    L.osc_profile_enable.restype = st
    L.osc_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    L.osc_profile_read.restype = st
    L.osc_reduction_layout.argtypes = [ctypes.POINTER(i32)] * 3
    L.osc_reduction_layout.restype = None
    L.osc_occupancy.argtypes = [vp, i32, ctypes.c_int, ctypes.POINTER(i32)]
    L.osc_occupancy.restype = st
    L.osc_max_nbins.argtypes = [vp]
    L.osc_max_nbins.restype = i32
    L.osc_poisson_nll.argtypes = [vp, vp, i64, ctypes.c_double, vp, i64, i32, vp, vp]
    L.osc_poisson_nll.restype = st
    L.osc_batch_create.argtypes = [vp, ctypes.POINTER(osc_sample), i32, ctypes.POINTER(osc_binning),
                                   ctypes.c_int, i32, ctypes.POINTER(vp)]
    L.osc_batch_create.restype = st
    L.osc_validate_sample.argtypes = [vp, ctypes.POINTER(osc_sample), ctypes.POINTER(i64),
                                      ctypes.POINTER(i64), vp]
    L.osc_validate_sample.restype = st
    L.osc_reweight_layered.argtypes = [vp, ctypes.POINTER(osc_sample), ctypes.POINTER(osc_layer),
                                       i32, i32, vp, vp]
    L.osc_reweight_layered.restype = st
    L.osc_fill_pdf_layered.argtypes = [vp, ctypes.POINTER(osc_sample), ctypes.POINTER(osc_layer),
                                       i32, i32, ctypes.POINTER(osc_binning), vp, vp, vp]
    L.osc_fill_pdf_layered.restype = st
    L.osc_template_create.argtypes = [vp, ctypes.POINTER(osc_sample), ctypes.POINTER(osc_binning),
                                      ctypes.POINTER(osc_binning), ctypes.POINTER(vp),
                                      ctypes.POINTER(i64)]
    L.osc_template_create.restype = st
    L.osc_template_destroy.argtypes = [vp]
    L.osc_template_destroy.restype = st
    L.osc_template_copy.argtypes = [vp, vp, vp]
    L.osc_template_copy.restype = st
    L.osc_fill_pdf_bincentre.argtypes = [vp, vp, i32, vp, vp, vp]
    L.osc_fill_pdf_bincentre.restype = st
    L.osc_batch_destroy.argtypes = [vp]
    L.osc_batch_destroy.restype = st
    L.osc_batch_get_config.argtypes = [vp, ctypes.POINTER(osc_batch_config)]
    L.osc_batch_get_config.restype = st
    L.osc_batch_set_config.argtypes = [vp, ctypes.POINTER(osc_batch_config)]
    L.osc_batch_set_config.restype = st
    L.osc_batch_run.argtypes = [vp, ctypes.POINTER(osc_params), i32, vp, vp]
    L.osc_batch_run.restype = st
    L.osc_batch_tune.argtypes = [vp, ctypes.POINTER(osc_params), i32, ctypes.c_char_p,
                                 ctypes.POINTER(ctypes.c_double), vp]
    L.osc_batch_tune.restype = st
    L.osc_server_create.argtypes = [vp, ctypes.POINTER(osc_sample), i32, ctypes.POINTER(osc_binning),
                                    ctypes.POINTER(osc_server_config), ctypes.POINTER(vp)]
    L.osc_server_create.restype = st
    L.osc_server_destroy.argtypes = [vp]
    L.osc_server_destroy.restype = st
    L.osc_server_submit.argtypes = [vp, ctypes.POINTER(osc_params), i32, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_uint64)]
    L.osc_server_submit.restype = st
    for name in ("osc_server_poll", "osc_server_wait"):
        fn = getattr(L, name)
        fn.argtypes = [vp, ctypes.c_uint64, vp, ctypes.POINTER(ctypes.c_double),
                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        fn.restype = st
    L.osc_server_set_data.argtypes = [vp, vp, ctypes.c_double]
    L.osc_server_set_data.restype = st
    L.osc_server_get_stats.argtypes = [vp, ctypes.POINTER(osc_server_stats)]
    L.osc_server_get_stats.restype = st
    L.osc_server_reset_stats.argtypes = [vp]
    L.osc_server_reset_stats.restype = st
    L.osc_server_request_bytes.argtypes = [vp, i32, ctypes.POINTER(i64)]
    L.osc_server_request_bytes.restype = st
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


def _vec_layout(t, name, dtype, n=None, multiple_of=None, optional=False):
    if t is None:
        if optional:
            return
        raise ValueError(f"{name} is required")
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor, not {type(t).__name__}")
    if t.dtype != getattr(torch, dtype):
        raise ValueError(f"{name} must be {dtype}, not {str(t.dtype).replace('torch.', '')}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} entries, not {t.numel()}")
    if multiple_of is not None and t.numel() % multiple_of:
        raise ValueError(f"{name} must have a multiple of {multiple_of} entries, not {t.numel()}")


def _vec_device(t, name, device):
    if t is None:
        return None
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be in GPU memory, not on {t.device}")
    if device is not None and t.device.index not in (None, device):
        raise ValueError(f"{name} is on GPU {t.device.index}, the context on GPU {device}")
    return ctypes.c_void_p(t.data_ptr()) if t.numel() else None


def device_vecs(*specs, device=None):
    """Check the tensors a kernel will read or write through their data
    pointers.  Each spec is (tensor, name, dtype, {n, multiple_of,
    optional}): a contiguous torch tensor of `dtype` (``"float64"`` or
    ``"uint8"``) with exactly `n` entries (or a multiple of `multiple_of`);
    None only when optional.  Then every tensor must be in GPU memory, on
    device index `device` when given.  Raises ValueError before anything
    reaches the library; returns the data pointers (None for absent or
    empty tensors)."""
    for t, name, dtype, *kw in specs:
        _vec_layout(t, name, dtype, **(kw[0] if kw else {}))
    ptrs = [_vec_device(t, name, device) for t, name, *_ in specs]
    return ptrs if len(ptrs) != 1 else ptrs[0]


def device_vec(t, name, dtype, device=None, **kw):
    """device_vecs for one tensor."""
    return device_vecs((t, name, dtype, kw), device=device)


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    handle = getattr(stream, "cuda_stream", stream)
    return ctypes.c_void_p(int(handle))


def osc_reduction_layout():
    w, k, a = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    load().osc_reduction_layout(ctypes.byref(w), ctypes.byref(k), ctypes.byref(a))
    return w.value, k.value, a.value


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

    def __post_init__(self):
        _vec_layout(self.e_true, "e_true", "float64")
        n = self.n
        device_vecs((self.e_true, "e_true", "float64"), (self.flags, "flags", "uint8", dict(n=n)),
                    (self.weight, "weight", "float64", dict(n=n, optional=True)),
                    (self.e_reco, "e_reco", "float64", dict(n=n, optional=True)),
                    device=self.e_true.device.index)

    @property
    def n(self) -> int:
        return int(self.e_true.numel())

    @property
    def device(self):
        return self.e_true.device.index

    def c_struct(self) -> osc_sample:
        return osc_sample(self.n, _ptr(self.e_true), _ptr(self.flags), _ptr(self.weight),
                          _ptr(self.e_reco), float(self.L_km), float(self.rho_gcc), float(self.Ye))

    def require_hist_inputs(self):
        if self.weight is None or self.e_reco is None:
            raise ValueError("this call reads weight and e_reco; the sample has none")

    @classmethod
    def from_host(cls, s, device="cuda"):
        """Upload a workload.Sample (numpy SoA) once; it stays resident."""
        import torch
        t = lambda a: torch.from_numpy(a).to(device)
        return cls(t(s.e_true), t(s.flags), t(s.weight), t(s.e_reco), s.L_km, s.rho_gcc, s.Ye)


class BinnedSample:
    """An osc_binned: a resident sample with its histogram slots cached for
    one binning (Context.osc_binned_create)."""

    def __init__(self, handle, ctx, sample, nbins):
        self.handle, self.ctx, self.sample, self.nbins = handle, ctx, sample, nbins

    def close(self):
        if self.handle:
            _check(load().osc_binned_destroy(self.handle), "osc_binned_destroy")
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

    def _sample(self, sample, hist_inputs):
        if not isinstance(sample, DeviceSample):
            raise ValueError("sample must be a DeviceSample")
        if sample.device not in (None, self.device):
            raise ValueError(f"the sample is on GPU {sample.device}, the context on "
                             f"GPU {self.device}")
        if hist_inputs:
            sample.require_hist_inputs()
        return sample.c_struct()

    @staticmethod
    def _hist(hist_out, nbins):
        if int(nbins) < 1:
            raise ValueError("nbins must be at least 1")
        return (hist_out, "hist_out", "float64", dict(n=int(nbins) + 2))

    def osc_reweight(self, sample: DeviceSample, set_index, p_out, stream=None):
        cs = self._sample(sample, False)
        pp = device_vec(p_out, "p_out", "float64", n=sample.n, device=self.device)
        _check(load().osc_reweight(self.handle, ctypes.byref(cs), int(set_index), pp,
                                   _stream(stream)), "osc_reweight")

    def osc_fill_pdf(self, sample: DeviceSample, set_index, nbins, lo, hi, hist_out,
                     p_out=None, precision=OSC_FP64, stream=None, e_scale=0.0):
        cs = self._sample(sample, True)
        hp, pp = device_vecs(self._hist(hist_out, nbins),
                             (p_out, "p_out", "float64", dict(n=sample.n, optional=True)),
                             device=self.device)
        b = osc_binning(int(nbins), float(lo), float(hi), float(e_scale))
        _check(load().osc_fill_pdf(self.handle, ctypes.byref(cs), int(set_index), ctypes.byref(b),
                                   int(precision), hp, pp, _stream(stream)),
               "osc_fill_pdf")

    def osc_fill_pdf_noalloc(self, sample: DeviceSample, set_index, nbins, lo, hi, hist_out,
                             p_out=None, precision=OSC_FP64, stream=None, e_scale=0.0):
        """osc_fill_pdf without device allocation: the library's fixed
        scratch array (OSC_NOALLOC_SCRATCH_BYTES per GPU) holds the tile
        results; calls that overlap on one GPU race."""
        cs = self._sample(sample, True)
        hp, pp = device_vecs(self._hist(hist_out, nbins),
                             (p_out, "p_out", "float64", dict(n=sample.n, optional=True)),
                             device=self.device)
        b = osc_binning(int(nbins), float(lo), float(hi), float(e_scale))
        _check(load().osc_fill_pdf_noalloc(self.handle, ctypes.byref(cs), int(set_index),
                                           ctypes.byref(b), int(precision), hp, pp,
                                           _stream(stream)),
               "osc_fill_pdf_noalloc")

    def osc_binned_create(self, sample: DeviceSample, nbins, lo, hi, e_scale=0.0):
        """Cache the histogram slot of every event of `sample` for this
        binning (2 bytes per event); returns a BinnedSample that keeps the
        sample alive."""
        cs = self._sample(sample, True)
        b = osc_binning(int(nbins), float(lo), float(hi), float(e_scale))
        h = ctypes.c_void_p()
        _check(load().osc_binned_create(self.handle, ctypes.byref(cs), ctypes.byref(b),
                                        ctypes.byref(h)), "osc_binned_create")
        return BinnedSample(h, self, sample, int(nbins))

    def osc_fill_pdf_binned(self, binned, set_index, hist_out, p_out=None, precision=OSC_FP64,
                            stream=None):
        if not isinstance(binned, BinnedSample) or binned.ctx is not self or not binned.handle:
            raise ValueError("binned must be a live BinnedSample of this context")
        hp, pp = device_vecs(self._hist(hist_out, binned.nbins),
                             (p_out, "p_out", "float64", dict(n=binned.sample.n, optional=True)),
                             device=self.device)
        _check(load().osc_fill_pdf_binned(self.handle, binned.handle, int(set_index),
                                          int(precision), hp, pp, _stream(stream)),
               "osc_fill_pdf_binned")

    def osc_validate_sample(self, sample: DeviceSample, stream=None):
        """(events with a true energy that is not finite and > 0, events with
        an invalid flag byte)."""
        cs = self._sample(sample, False)
        be, bf = ctypes.c_int64(), ctypes.c_int64()
        _check(load().osc_validate_sample(self.handle, ctypes.byref(cs), ctypes.byref(be),
                                          ctypes.byref(bf), _stream(stream)),
               "osc_validate_sample")
        return be.value, bf.value

    def osc_reweight_layered(self, sample: DeviceSample, layers, set_index, p_out, stream=None):
        cs = self._sample(sample, False)
        pp = device_vec(p_out, "p_out", "float64", n=sample.n, device=self.device)
        arr = layers_array(layers)
        _check(load().osc_reweight_layered(self.handle, ctypes.byref(cs), arr, len(arr),
                                           int(set_index), pp, _stream(stream)),
               "osc_reweight_layered")

    def osc_fill_pdf_layered(self, sample: DeviceSample, layers, set_index, nbins, lo, hi,
                             hist_out, p_out=None, stream=None, e_scale=0.0):
        cs = self._sample(sample, True)
        hp, pp = device_vecs(self._hist(hist_out, nbins),
                             (p_out, "p_out", "float64", dict(n=sample.n, optional=True)),
                             device=self.device)
        arr = layers_array(layers)
        b = osc_binning(int(nbins), float(lo), float(hi), float(e_scale))
        _check(load().osc_fill_pdf_layered(self.handle, ctypes.byref(cs), arr, len(arr),
                                           int(set_index), ctypes.byref(b), hp, pp,
                                           _stream(stream)), "osc_fill_pdf_layered")

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

    def osc_poisson_nll(self, hist, data, nll_out, stream=None, mu_scale=1.0):
        """-2 ln L of every histogram in `hist` (..., nbins + 2), scaled by
        mu_scale, against the rows of `data` (n_data, nbins); histogram k
        uses row k % n_data."""
        nbins = int(data.shape[-1])
        if nbins < 1:
            raise ValueError("data must have at least one bin")
        _vec_layout(hist, "hist", "float64", multiple_of=nbins + 2)
        _vec_layout(data, "data", "float64", multiple_of=nbins)
        n_hist = int(hist.numel() // (nbins + 2))
        n_data = int(data.numel() // nbins)
        if n_data < 1:
            raise ValueError("data must hold at least one row")
        hp, dp, op = device_vecs((hist, "hist", "float64"), (data, "data", "float64"),
                                 (nll_out, "nll_out", "float64", dict(n=n_hist)),
                                 device=self.device)
        _check(load().osc_poisson_nll(self.handle, hp, n_hist, float(mu_scale), dp,
                                      n_data, nbins, op, _stream(stream)),
               "osc_poisson_nll")

    def osc_fill_hist(self, value, weight, e_reco, nbins, lo, hi, hist_out, stream=None,
                      e_scale=0.0):
        b = osc_binning(int(nbins), float(lo), float(hi), float(e_scale))
        _vec_layout(value, "value", "float64")
        n = int(value.numel())
        vp, wp, xp, hp = device_vecs((value, "value", "float64"),
                                     (weight, "weight", "float64", dict(n=n)),
                                     (e_reco, "e_reco", "float64", dict(n=n)),
                                     self._hist(hist_out, nbins), device=self.device)
        _check(load().osc_fill_hist(self.handle, n, vp, wp, xp, ctypes.byref(b), hp,
                                    _stream(stream)), "osc_fill_hist")


N_CHANNELS = 18   # alpha + 3 beta + 9 anti


class Template:
    """osc_template: the migration template of the bin-centre method
    (Sec. 1.1.1) and its per-call PDF."""

    def __init__(self, ctx: Context, sample: "DeviceSample", nt, lo_t, hi_t, nr, lo_r, hi_r,
                 e_scale=0.0):
        self.ctx = ctx
        self.nt, self.nr = int(nt), int(nr)
        cs = ctx._sample(sample, True)
        tb = osc_binning(self.nt, float(lo_t), float(hi_t), 0.0)
        rb = osc_binning(self.nr, float(lo_r), float(hi_r), float(e_scale))
        h = ctypes.c_void_p()
        used = ctypes.c_int64()
        _check(load().osc_template_create(ctx.handle, ctypes.byref(cs), ctypes.byref(tb),
                                          ctypes.byref(rb), ctypes.byref(h), ctypes.byref(used)),
               "osc_template_create")
        self.handle = h
        self.n_used = used.value

    def close(self):
        if getattr(self, "handle", None):
            _check(load().osc_template_destroy(self.handle), "osc_template_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def copy(self, stream=None):
        """The template (nr + 2, 18, nt) on the device."""
        import torch
        out = torch.empty((self.nr + 2, N_CHANNELS, self.nt), dtype=torch.float64, device="cuda")
        _check(load().osc_template_copy(self.handle, _ptr(out), _stream(stream)),
               "osc_template_copy")
        return out

    def fill_pdf(self, set_index, hist_out, p_centre_out=None, stream=None):
        hp, cp = device_vecs(self.ctx._hist(hist_out, self.nr),
                             (p_centre_out, "p_centre_out", "float64",
                              dict(n=N_CHANNELS * self.nt, optional=True)),
                             device=self.ctx.device)
        _check(load().osc_fill_pdf_bincentre(self.ctx.handle, self.handle, int(set_index), hp, cp,
                                             _stream(stream)), "osc_fill_pdf_bincentre")


class Batch:
    """osc_batch: every parameter set x every sample in one persistent launch.

    The DeviceSample tensors are kept referenced for the life of the batch
    (the captured graph holds their addresses)."""

    def __init__(self, ctx: Context, samples, nbins, lo, hi, precision=OSC_FP32_MIXED,
                 max_sets=256, e_scale=0.0):
        self.ctx = ctx
        self.samples = list(samples)
        self.nbins = int(nbins)
        self.max_sets = int(max_sets)
        arr = (osc_sample * len(self.samples))(*[ctx._sample(s, True) for s in self.samples])
        b = osc_binning(self.nbins, float(lo), float(hi), float(e_scale))
        h = ctypes.c_void_p()
        _check(load().osc_batch_create(ctx.handle, arr, len(self.samples), ctypes.byref(b),
                                       int(precision), self.max_sets, ctypes.byref(h)),
               "osc_batch_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _check(load().osc_batch_destroy(self.handle), "osc_batch_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def config(self) -> osc_batch_config:
        c = osc_batch_config()
        _check(load().osc_batch_get_config(self.handle, ctypes.byref(c)), "osc_batch_get_config")
        return c

    @config.setter
    def config(self, c):
        if isinstance(c, dict):
            cur = self.config
            for k, v in c.items():
                setattr(cur, k, int(v))
            c = cur
        _check(load().osc_batch_set_config(self.handle, ctypes.byref(c)), "osc_batch_set_config")

    def run(self, sets, hist_out=None, stream=None):
        """Histograms (n_sets, n_samples, nbins + 2) on the device."""
        import torch
        arr = params_array(sets)
        if hist_out is None:
            hist_out = torch.empty((len(arr), len(self.samples), self.nbins + 2),
                                   dtype=torch.float64, device=self.samples[0].e_true.device)
        hp = device_vec(hist_out, "hist_out", "float64",
                        n=len(arr) * len(self.samples) * (self.nbins + 2), device=self.ctx.device)
        _check(load().osc_batch_run(self.handle, arr, len(arr), hp, _stream(stream)),
               "osc_batch_run")
        return hist_out

    def tune(self, sets, cache_path=None, stream=None) -> float:
        arr = params_array(sets)
        ms = ctypes.c_double()
        path = cache_path.encode() if cache_path else None
        _check(load().osc_batch_tune(self.handle, arr, len(arr), path, ctypes.byref(ms),
                                     _stream(stream)), "osc_batch_tune")
        return ms.value


class ServerResult(NamedTuple):
    hist: object        # numpy, nbins + 2
    latency_s: float
    queue_s: float
    nll: float          # -2 ln L, NaN when the server has no data


class Server:
    """osc_server: FIFO request loop with slot- and memory-bound admission.

    Results come back as numpy arrays (nbins + 2 bins, host memory)."""

    def __init__(self, ctx: Context, samples, nbins, lo, hi, slots=8, scratch_budget_bytes=1 << 30,
                 queue_capacity=1 << 20, e_scale=0.0):
        self.ctx = ctx
        self.samples = list(samples)
        self.nbins = int(nbins)
        arr = (osc_sample * len(self.samples))(*[ctx._sample(s, True) for s in self.samples])
        b = osc_binning(self.nbins, float(lo), float(hi), float(e_scale))
        cfg = osc_server_config(int(slots), int(queue_capacity), int(scratch_budget_bytes))
        h = ctypes.c_void_p()
        _check(load().osc_server_create(ctx.handle, arr, len(self.samples), ctypes.byref(b),
                                        ctypes.byref(cfg), ctypes.byref(h)), "osc_server_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _check(load().osc_server_destroy(self.handle), "osc_server_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, params, sample, precision=OSC_FP64) -> int:
        t = ctypes.c_uint64()
        p = to_params(params)
        _check(load().osc_server_submit(self.handle, ctypes.byref(p), int(sample), int(precision),
                                        ctypes.byref(t)), "osc_server_submit")
        return t.value

    def set_data(self, data, mu_scale=1.0):
        """Observed counts, one row of nbins per sample (or None to clear):
        requests admitted afterwards also return -2 ln L of mu_scale * hist
        against their sample's row."""
        import numpy as np
        if data is None:
            _check(load().osc_server_set_data(self.handle, None, float(mu_scale)),
                   "osc_server_set_data")
            return
        d = np.ascontiguousarray(data, dtype=np.float64)
        if d.shape != (len(self.samples), self.nbins):
            raise ValueError("data must have one row of nbins counts per sample")
        _check(load().osc_server_set_data(self.handle, ctypes.c_void_p(d.ctypes.data),
                                          float(mu_scale)), "osc_server_set_data")

    def _result(self, fn, ticket):
        import numpy as np
        h = np.empty(self.nbins + 2, dtype=np.float64)
        nll, lat, q = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        st = fn(self.handle, ctypes.c_uint64(ticket), ctypes.c_void_p(h.ctypes.data),
                ctypes.byref(nll), ctypes.byref(lat), ctypes.byref(q))
        return st, ServerResult(h, lat.value, q.value, nll.value)

    def poll(self, ticket):
        """ServerResult(hist, latency_s, queue_s, nll) once done, else None."""
        st, r = self._result(load().osc_server_poll, ticket)
        if st == OSC_ERR_NOT_READY:
            return None
        _check(st, "osc_server_poll")
        return r

    def wait(self, ticket):
        st, r = self._result(load().osc_server_wait, ticket)
        _check(st, "osc_server_wait")
        return r

    def stats(self) -> dict:
        s = osc_server_stats()
        _check(load().osc_server_get_stats(self.handle, ctypes.byref(s)), "osc_server_get_stats")
        return s.as_dict()

    def reset_stats(self):
        """Start a new statistics window (counters from zero, maxima from
        the current state)."""
        _check(load().osc_server_reset_stats(self.handle), "osc_server_reset_stats")

    def request_bytes(self, sample) -> int:
        b = ctypes.c_int64()
        _check(load().osc_server_request_bytes(self.handle, int(sample), ctypes.byref(b)),
               "osc_server_request_bytes")
        return b.value
