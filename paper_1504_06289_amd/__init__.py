"""MI355X (gfx950) library for the grid-based Newton-kernel convolution and
two-electron-integral Gram assembly of Khoromskaia & Khoromskij
(arXiv:1504.06289).  The C ABI is include/tc.h; this package is its thin
Python binding (see api.py) plus the seeded synthetic workloads."""
from .api import (TeiGram, TeiGramGraph, autotune, autotune_batched,  # noqa: F401
                  batch_tune_get, batch_tune_set,
                  canonical_to_tucker, convolve,
                  coulomb, density_fit, lattice_energy, lattice_sum, make_instance,
                  newton_kernel, nuclear,
                  profile_enable, profile_read,
                  tei_cholesky, tei_gram, tei_gram_backward, tei_gram_batched,
                  tei_gram_noalloc, term_classes,
                  tune_get, tune_set)
