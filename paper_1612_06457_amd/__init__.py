"""cvamx: canonical variates analysis and PCA enhancement of multispectral
page images on AMD Instinct MI355X (gfx950).

The computation lives in libcvamx.so (hand-written HIP kernels plus an FP64
host finisher behind a C ABI, declared in include/cvamx.h); this package is
a thin ctypes binding over torch tensors.
"""
from .api import (ClusterIndices, CvaFit, SoftFit, SoftCVA, bands_to_cube, cluster_indices, compose_rgb,
                  cva_fit, cva_fit_points, cva_fit_project, cva_pca, cva_project, cva_project_noalloc,
                  cva_soft_backward, cva_soft_forward, cva_soft_update, cva_solve_moments, label_index,
                  pca_fit, pca_project, profile_enable, profile_report, project_float, refine_weights,
                  run_pages, set_plain_fp32, set_schedule, stream_mix, stream_read, stretch, sym_eig,
                  sym_eig_top)
from ._lib import CvamxError, LIB_PATH

__all__ = ["ClusterIndices", "CvaFit", "SoftFit", "SoftCVA", "bands_to_cube", "cluster_indices", "compose_rgb",
           "cva_fit", "cva_fit_points", "cva_fit_project", "cva_pca", "cva_project", "cva_project_noalloc",
           "cva_soft_backward", "cva_soft_forward", "cva_soft_update", "cva_solve_moments", "label_index",
           "pca_fit", "pca_project", "profile_enable", "profile_report", "project_float", "refine_weights",
           "run_pages", "set_plain_fp32", "set_schedule", "stream_mix", "stream_read", "stretch", "sym_eig",
           "sym_eig_top",
           "CvamxError", "LIB_PATH"]
