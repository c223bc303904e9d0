"""FP64 CPU oracle for the spectral-fit likelihood -- TEST INFRASTRUCTURE.

Plain, slow, obviously correct definitions of what the GPU library computes.
Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
use it; the library never calls it and shares no code with it.

Every function follows a passage of Ding et al., "Speeding up complex
multivariate data analysis in Borexino with parallel computing based on GPU"
(arXiv:1805.11125):

* response convolution of each species' deposited spectrum (Sec. 3, Eq. 1);
* pile-up convolution with the random-trigger spectrum (Sec. 3, Eq. 2);
* TFC-vetoed + TFC-tagged joint likelihood (Sec. 3, Eq. 3);
* radial and pulse-shape terms added to it (Sec. 3, Eq. 4);
* the minimiser varying the parameters to find the likelihood optimum
  (Sec. 4, workflow steps 5-6).

Where the paper is silent the readings are the ones listed in the design
notes (response forms, discretisation, Poisson NLL without the data-only
constant, pile-up as a (1-p) delta + p g mixture, ...).

Parity status: every function here is pinned by tests against closed forms,
library routines, brute-force quadrature or invariants, except the physical
realism of the synthetic inputs (parity unpinned: no detector data exist here).
"""
from .model import (DomainError, column_params, edge_tails, response_matrix,
                    response_derivs, contraction, pileup, expected, nll, nll_terms,
                    grad, nll_grad, grad_scale, grad_scale_abs, lnfact, per_species_expected,
                    support_cells, support_edges)
from .fit import fit

__all__ = ["DomainError", "column_params", "edge_tails", "response_matrix",
           "response_derivs", "contraction", "pileup", "expected", "nll",
           "nll_terms", "grad", "nll_grad", "grad_scale", "grad_scale_abs", "lnfact", "per_species_expected",
           "support_cells", "support_edges", "fit"]
