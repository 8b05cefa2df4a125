"""MI355X Torontonian library: Python binding of the C ABI in include/tor.h.

The numerical work runs in HIP kernels (libtor_hip.so, built in-tree for
gfx950); this package only marshals arguments.  Importing it does not load
the library; the first call does, and raises if it is missing.
"""
from ._lib import TorError, TOR_FP64, TOR_DD, TOR_QD, TOR_AUTO  # noqa: F401
from .api import (  # noqa: F401
    TorResult, Batch, tor_eval_batched, tor_version, tor_init, tor_shutdown, tor_eval, tor_debug_level_sums,
    tor_debug_sampled_terms, tor_debug_phase_clocks, tor_last_kernel_ms, tor_next_mask, tor_kth_mask, tor_plan_items,
    tor_features, tor_mlp_forward, tor_mlp_grad, tor_mlp_adam, tor_selector_set, tor_selector_get,
    tor_selector_save, tor_selector_load, tor_fallback_bits, tor_select_tiers, tor_last_select_stats,
    tor_autotune, tor_autotune_save, tor_autotune_load, tor_mcmc, results_of, tier_id,
    tor_eval_part, tor_combine_parts, tor_workspace_bytes,
    tor_batch_workspace_bytes, tor_eval_noalloc, tor_noalloc_nmax, tor_mlp_grad_quantile,
    tor_selector_label, tor_selector_train, train_options,
)
