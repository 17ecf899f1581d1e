"""RapidPT permutation testing on MI355X (gfx950).

The compute lives in librpt.so (hand-written HIP kernels behind a C ABI, see
include/rpt.h); this package is a thin torch binding.  Importing it loads the
library and fails loudly if it has not been built
(``python paper_1703_01506_amd/build.py``).
"""
from . import _lib
from .api import (  # noqa: F401
    autotune_clear,
    autotune_count,
    autotune_load,
    autotune_naive,
    autotune_recover,
    autotune_save,
    complete,
    corrected_pvalues,
    fwer_threshold,
    masked_loss_bwd,
    gen_relabellings,
    gen_sampled_sets,
    gen_start_basis,
    masked_loss_fwd,
    naive_maxnull,
    observed_tstat,
    rapidpt_maxnull,
    rapidpt_maxnull_seeded,
    recover_maxnull,
    recover_maxnull_batched,
    recover_studies_launch,
    recover_studies_prepare,
    rejection_counts,
    reorth,
    sample_count,
    sampled_tstat,
    sigma_mu_heldout,
    train_subspace,
)
from .autograd import MaskedSubspaceLoss, masked_subspace_loss  # noqa: F401

_lib.load()

__all__ = [
    "naive_maxnull", "sampled_tstat", "complete", "reorth", "train_subspace", "sigma_mu_heldout", "recover_maxnull",
    "rapidpt_maxnull", "recover_maxnull_batched", "recover_studies_prepare", "recover_studies_launch",
    "observed_tstat", "fwer_threshold", "corrected_pvalues", "rejection_counts", "masked_loss_fwd", "masked_loss_bwd",
    "MaskedSubspaceLoss", "masked_subspace_loss", "autotune_naive", "autotune_recover", "autotune_save",
    "autotune_load", "autotune_clear", "autotune_count", "rapidpt_maxnull_seeded", "sample_count",
    "gen_relabellings", "gen_sampled_sets", "gen_start_basis",
]
