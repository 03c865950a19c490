"""MI355X (gfx950) signature-kernel solvers: finite-difference, polynomial
approximation and polynomial interpolation schemes for the Goursat PDE of
the signature kernel, batched over path pairs, forward and adjoint."""
from .api import (PairsPlan, SigKernelGram, SigKernelPairs, cell_constants, device_status, gram,
                  gram_algo,
                  gram_backward, gram_backward_saved, gram_save, gram_state_size, mmd2,
                  gram_tuned, mmd_permutation_test, pairs, pairs_backward, sig_gram, sig_pairs,
                  tune_gram)
from ._lib import SigKernelError, tune_cache_clear, tune_cache_load, tune_cache_save

__all__ = ["gram", "gram_algo", "pairs", "gram_backward", "pairs_backward", "cell_constants", "gram_save",
           "gram_backward_saved", "gram_state_size",
           "PairsPlan", "SigKernelGram", "sig_gram", "SigKernelPairs", "sig_pairs", "mmd2", "mmd_permutation_test",
           "SigKernelError", "device_status", "tune_gram", "gram_tuned", "tune_cache_save",
           "tune_cache_load", "tune_cache_clear"]
