"""Event-by-event neutrino-oscillation reweighting on AMD MI355X (gfx950).

Per Monte Carlo event: the three-flavour oscillation probability through
constant-density matter, then weight x probability into a binned
reconstructed-energy PDF (arXiv:1311.7579).  The arithmetic runs in HIP
kernels inside ``libosc.so`` behind the C ABI declared in
``include/osc.h``; :mod:`paper_1311_7579_amd.osc` is the ctypes binding.

Importing this package loads nothing; :func:`paper_1311_7579_amd.osc.load`
opens the library and raises if it is missing.
"""

__all__ = ["osc", "workload"]
