"""Host-side checks of osc_fill_pdf_noalloc (no GPU needed): the size of
the fixed array in the header and in the binding agree, and the argument
checks run before any device work."""
import ctypes
import os
import re

from paper_1311_7579_amd import osc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_and_binding_agree_on_the_array_size():
    text = open(os.path.join(ROOT, "include", "osc.h")).read()
    m = re.search(r"#define OSC_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m, "OSC_NOALLOC_SCRATCH_BYTES not found"
    assert int(m.group(1)) << int(m.group(2)) == osc.OSC_NOALLOC_SCRATCH_BYTES


def test_null_arguments_are_rejected():
    lib = osc.load()
    s = osc.osc_sample()
    b = osc.osc_binning(50, 0.0, 3.0, 0.0)
    assert lib.osc_fill_pdf_noalloc(None, ctypes.byref(s), 0, ctypes.byref(b), 0, None, None,
                                    None) == osc.OSC_ERR_INVALID_ARG
