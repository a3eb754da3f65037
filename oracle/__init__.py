"""Plain FP64 CPU oracle for the CVA / PCA enhancement hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the
package entry file and the CPU-baseline leg of the benchmark may import or
run anything in this package; the library path never does, and this package
imports nothing from it.

What it computes, and where the paper defines it:

* CVA (Section 2, the canonical variates paragraph; Section 4, the GSL
  implementation and its generalized symmetric-definite eigensolver): class
  counts and means, within-class and between-class scatter, the generalized
  eigenproblem S_b w = lambda S_w w, projection of every page pixel onto the
  canonical vectors and the rescale of each projection to 0..255 (Section 2,
  the paragraphs on regression coefficients and rescaling).
* PCA (Section 2, the PCA paragraph and its list of stages; the unsupervised
  whole-page variant): mean, covariance, eigen-decomposition, projection.
* Soft-label CVA: the Fisher criterion J = sum of the canonical eigenvalues
  with real-valued per-pixel class weights, and its closed-form gradient with
  respect to those weights.  This extension is not in the paper; its
  definition reduces to the paper's CVA when the weights are one-hot.

Everything is float64 NumPy/SciPy, written as the definitions read, with no
blocking or fusion beyond chunking over pixels to bound memory.

Parity status of each function is listed in its docstring: "pinned" names
the tests/ checks that tie it to something other than itself.  The
components beyond C = K-1 of the CVA eigenbasis span the null space of S_b,
are not unique, and are not produced (parity unpinned by construction).
"""
from .cva import (class_counts, class_index_lists, class_moments, within_scatter,
                  between_scatter, total_scatter, generalized_eig, sign_rule,
                  cva_fit, cva_fit_points, project, cva_project)
from .stretch import compose_rgb, stretch_minmax, stretch_training_range, stretch_percentile
from .pca import pca_fit, pca_project
from .soft import soft_moments, soft_fit, soft_grad, soft_delta_J, simplex_projection, soft_update
from .cluster import cluster_indices

__all__ = [
    "class_counts", "class_index_lists", "class_moments", "within_scatter",
    "between_scatter", "total_scatter", "generalized_eig", "sign_rule",
    "cva_fit", "cva_fit_points", "project", "cva_project", "stretch_minmax",
    "stretch_training_range", "stretch_percentile", "compose_rgb", "pca_fit", "pca_project",
    "soft_moments", "soft_fit", "soft_grad", "soft_delta_J", "simplex_projection", "soft_update",
    "cluster_indices",
]
