"""MI355X (gfx950) Barnes-Hut tree-code: hand-written HIP kernels behind a C
ABI (include/bh.h), with a ctypes binding.  Method: Bedorf et al., SC14
(arXiv:1412.0659)."""
from .binding import (BhError, Tree, bh_boundary, bh_create, bh_decompose,
                      bh_decompose_sampled, bh_destroy,
                      bh_diagnostics, bh_domain_extract, bh_export, bh_export_keys, bh_export_tree,
                      bh_get_state, bh_let_build,
                      bh_set_box, bh_set_state, bh_stats_get, bh_sync, leapfrog_step,
                      leapfrog_vjp_drift, leapfrog_vjp_segment, load, tree_build, tree_direct, tree_force,
                      tree_force_add, tree_force_let, tree_force_vjp)
from .domains import Domains

__all__ = ["BhError", "Domains", "Tree", "bh_boundary", "bh_create", "bh_decompose", "bh_decompose_sampled",
           "bh_destroy", "bh_diagnostics", "bh_domain_extract", "bh_export", "bh_export_keys",
           "bh_export_tree", "bh_get_state",
           "bh_let_build", "bh_set_box", "bh_set_state", "bh_stats_get", "bh_sync",
           "leapfrog_step", "leapfrog_vjp_drift", "leapfrog_vjp_segment", "load", "tree_build", "tree_direct",
           "tree_force", "tree_force_add", "tree_force_let", "tree_force_vjp"]
