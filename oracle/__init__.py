"""CPU oracle of the multi-axis Kronecker-sum Gaussian graphical model's hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package; the
product path never does, and it shares no code with the GPU library.

Everything here is plain NumPy in float64, written from the paper (arXiv
2407.19892): the per-axis Gram / covariance matrices (Notation section), their
partial eigendecomposition and the cell-axis factor (Algorithm 1, Theorem 1),
the eigenvalue maximum-likelihood estimate (model equation, eigenvalue-gradient
Proposition, Existence lemma), the eigen-recomposition with per-row top-k
thresholding (Algorithm 1's final loop and the complexity appendix), the
significance threshold of Theorem 3 and the thresholded graph it defines, the
Nonparanormal Skeptic kept sparse (input-sparsity appendix), the eigenvalue
estimate for modalities of three or more axes (tensor-variate data), and the
learned warm start's multilayer perceptron.

Readings of passages that are silent or ambiguous are stated in the docstring
of the function that takes them.
"""
from .gram import gram_dense, gram_csr
from .spectral import eigh_desc, numerical_rank, cell_factor
from .solver import Problem, nll, grad, solve_eigs, projected_gradient, default_eps
from .recompose import psi_dense, psi_rows, psi_blockwise
from .topk import topk_row, topk_csr, near_tie_rows
from . import warmstart
from . import range_finder
from . import significance
from . import skeptic
from . import solver_tensor

__all__ = [
    "gram_dense", "gram_csr", "eigh_desc", "numerical_rank", "cell_factor",
    "Problem", "nll", "grad", "solve_eigs", "projected_gradient", "default_eps",
    "psi_dense", "psi_rows", "psi_blockwise", "topk_row", "topk_csr", "near_tie_rows",
    "warmstart", "range_finder", "significance", "skeptic", "solver_tensor",
]
