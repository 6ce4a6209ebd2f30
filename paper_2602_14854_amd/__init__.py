"""MI355X-native DD-DLRA time-step engine (HIP for gfx950 behind a C ABI).

The compute path is the shared library ``libdd_dlra.so`` built from
``csrc/`` (see ``build.py``); this package only marshals arguments to it
with ctypes.  There is no CPU fallback: if the library is missing the
import of :class:`DDDLRA` raises.
"""
from ._native import (  # noqa: F401
    DD_OK, DD_EINVAL, DD_ENOMEM, DD_EHIP, DD_ERANK, DD_ENUMERIC, DD_ESTATE,
    DD_PREC_FP64, DD_PREC_MIXED_FP32, DD_PREC_MIXED_BF16, DD_RANK_FIXED, DD_RANK_ADAPTIVE,
    DD_EXEC_PER_SUBDOMAIN, DD_EXEC_BATCHED, DD_EXEC_BATCHED_GRAPH, DD_INT_EULER, DD_INT_RK4,
    DD_BC_VACUUM, DD_BC_INFLOW_LOWRANK, DD_PROBE_VHAT, DD_PROBE_K1, DD_PROBE_U1, DD_PROBE_S2, DD_PROBE_L1,
    DDError, DDDLRA, Config, load_library, library_path, workspace_size, EXPORTS,
)
