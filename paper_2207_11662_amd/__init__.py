"""Exact closeness centrality for homogeneous multilayer networks on AMD
MI355X (gfx950): a C-ABI HIP library (``libhln.so``, declared in
``include/hln.h``) and this thin Python binding."""
from ._lib import (  # noqa: F401
    EXPORTS, Graph, HlnError, check, device_status, lib, workspace,
    HLN_RANK_WF, HLN_RANK_CC2, HLN_RANK_NAIVE, HLN_FLAG_PER_VERTEX,
    closeness_workspace_size, compose_workspace_size,
    hln_closeness_layer, hln_closeness_estimate, hln_csr_from_edges, hln_csr_from_edges_batch, csr_from_edges_batch_workspace_size,
    hln_csr_validate, hln_compose_and, hln_compose_or, hln_compose_and_batch, AndBatch,
    hln_compose_cc_topk, hln_compose_cc_topk_batch, TopkBatch, hln_compose_cc1, Plan,
    mlp_param_count, hln_proposer_features, hln_mlp_init, hln_mlp_forward, hln_mlp_train_step, hln_topk,
    hln_rank_labels, closeness_kernel_residency, last_launch_path, HLN_TOPK_SET,
)
