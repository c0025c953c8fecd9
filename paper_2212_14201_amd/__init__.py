"""MI355X (gfx950) full-amplitude state-vector library.

The compute path is the HIP library ``libqvm.so`` (sources in ``csrc/``,
C ABI in ``include/qvm.h``); ``qvm`` is its thin Python binding.
"""
from . import qvm  # noqa: F401
from .qvm import StateVector, GateArray, QvmError, gate_matrix, workspace_bytes  # noqa: F401
