"""Exact closeness centrality for homogeneous multilayer networks on AMD
MI355X (gfx950): a C-ABI HIP library (``libhln.so``, declared in
``include/hln.h``) and this thin Python binding."""
from ._lib import (  # noqa: F401
    EXPORTS, Graph, HlnError, check, device_status, hln_closeness_layer, lib, workspace,
    closeness_workspace_size,
)
