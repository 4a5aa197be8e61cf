"""MI355X (gfx950) Barnes-Hut tree-code: hand-written HIP kernels behind a C
ABI (include/bh.h), with a ctypes binding.  Method: Bedorf et al., SC14
(arXiv:1412.0659)."""
from .binding import (BhError, Tree, bh_create, bh_destroy, bh_export, bh_get_state,
                      bh_set_state, bh_stats_get, bh_sync, leapfrog_step, load, tree_build,
                      tree_force)

__all__ = ["BhError", "Tree", "bh_create", "bh_destroy", "bh_export", "bh_get_state",
           "bh_set_state", "bh_stats_get", "bh_sync", "leapfrog_step", "load", "tree_build",
           "tree_force"]
