"""Host-side checks of the C ABI: the library loads, exports every entry
point include/osc.h declares, validates arguments without a device, and
reports the same reduction contract the oracle replays."""
import ctypes
import math
import os
import re

import pytest

import oracle
from paper_1311_7579_amd import osc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "osc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(osc_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(osc.LIB_PATH):
        from paper_1311_7579_amd.build import build
        build()
    return osc.load()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for want in ("osc_create", "osc_destroy", "osc_set_params", "osc_reweight", "osc_fill_pdf",
                 "osc_fill_hist", "osc_validate_params", "osc_reduction_layout",
                 "osc_max_nbins", "osc_status_string", "osc_occupancy", "osc_profile_enable",
                 "osc_profile_read", "osc_poisson_nll", "osc_batch_create", "osc_batch_run",
                 "osc_batch_tune", "osc_server_create", "osc_server_submit", "osc_server_wait",
                 "osc_server_set_data", "osc_server_poll", "osc_reweight_layered",
                 "osc_fill_pdf_layered", "osc_template_create", "osc_template_copy",
                 "osc_template_destroy", "osc_fill_pdf_bincentre", "osc_validate_sample",
                 "osc_binned_create", "osc_binned_destroy", "osc_fill_pdf_binned",
                 "osc_fill_pdf_noalloc"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_reduction_layout_matches_oracle_contract(lib):
    assert osc.osc_reduction_layout() == (oracle.CONTRACT_W, oracle.CONTRACT_K, oracle.CONTRACT_A)


def test_status_strings(lib):
    for code in range(6):
        assert osc.osc_status_string(code) not in ("", "unknown status")


def test_create_without_gpu_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.osc_create(ctypes.byref(h), 0) == osc.OSC_ERR_DEVICE
    assert not h.value
    assert lib.osc_create(None, 0) == osc.OSC_ERR_INVALID_ARG
    assert lib.osc_destroy(None) == osc.OSC_OK


def test_null_context_is_rejected(lib):
    s = osc.osc_sample()
    b = osc.osc_binning(50, 0.0, 3.0)
    assert lib.osc_reweight(None, ctypes.byref(s), 0, None, None) == osc.OSC_ERR_INVALID_ARG
    assert lib.osc_fill_pdf(None, ctypes.byref(s), 0, ctypes.byref(b), 0, None, None, None) \
        == osc.OSC_ERR_INVALID_ARG
    assert lib.osc_set_params(None, None, 1) == osc.OSC_ERR_INVALID_ARG
    assert lib.osc_max_nbins(None) == 0


TABLE1 = dict(sin2_th12=0.311, sin2_th23=0.5, sin2_th13=0.0251,
              dm2_32=2.4e-3, dm2_21=7.6e-5, delta_cp=0.0)


@pytest.mark.parametrize("bad", [
    dict(sin2_th12=-0.01), dict(sin2_th23=1.01), dict(sin2_th13=math.nan),
    dict(dm2_21=0.0), dict(dm2_21=-7.6e-5), dict(dm2_32=0.0), dict(dm2_32=-7.6e-5),
    dict(delta_cp=math.inf), dict(dm2_32=math.nan),
])
def test_invalid_parameters_are_rejected(lib, bad):
    assert osc.osc_validate_params([dict(TABLE1, **bad)]) == osc.OSC_ERR_INVALID_ARG
    # an invalid set anywhere in the array rejects the call
    assert osc.osc_validate_params([TABLE1, dict(TABLE1, **bad)]) == osc.OSC_ERR_INVALID_ARG


def test_valid_parameters_are_accepted(lib):
    assert osc.osc_validate_params([TABLE1]) == osc.OSC_OK
    inverted = dict(TABLE1, dm2_32=-2.5e-3)
    edges = dict(TABLE1, sin2_th12=0.0, sin2_th23=1.0, sin2_th13=0.0)
    assert osc.osc_validate_params([inverted, edges]) == osc.OSC_OK
    assert lib.osc_validate_params(None, 1) == osc.OSC_ERR_INVALID_ARG
    arr = osc.params_array([TABLE1])
    assert lib.osc_validate_params(arr, 0) == osc.OSC_ERR_INVALID_ARG
