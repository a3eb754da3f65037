"""The Python binding refuses bad tensors before any pointer reaches the
library: wrong dtype, shape, layout or device raises ValueError (no GPU is
needed, nothing is launched)."""
import numpy as np
import pytest
import torch

import paper_1612_06457_amd as cx
from paper_1612_06457_amd.api import SoftFit


def _fit(K=4, B=6):
    C = min(K - 1, B)
    return SoftFit(J=1.0, W=np.zeros((B, C)), eigvals=np.ones(C), mean=np.zeros(B), class_means=np.zeros((K, B)))


def test_soft_backward_checks():
    X = torch.zeros((10, 6), dtype=torch.float32)
    fit = _fit()
    with pytest.raises(ValueError, match="float32"):
        cx.cva_soft_backward(X.double(), fit, 1.0, 4)
    with pytest.raises(ValueError, match="contiguous"):
        cx.cva_soft_backward(torch.zeros((6, 10)).t(), fit, 1.0, 4)
    with pytest.raises(ValueError, match="fit does not belong"):
        cx.cva_soft_backward(X, fit, 1.0, 5)                       # K differs from the fit's
    with pytest.raises(ValueError, match="fit does not belong"):
        cx.cva_soft_backward(torch.zeros((10, 7)), fit, 1.0, 4)    # B differs from the fit's
    with pytest.raises(ValueError, match="out must be"):
        cx.cva_soft_backward(X, fit, 1.0, 4, out=torch.zeros((10, 3)))
    with pytest.raises(ValueError, match="out must be"):
        cx.cva_soft_backward(X, fit, 1.0, 4, out=torch.zeros((10, 4), dtype=torch.float64))
    with pytest.raises(ValueError, match="device"):
        cx.cva_soft_backward(X, fit, 1.0, 4)                       # a host tensor
    with pytest.raises(ValueError, match="device"):
        cx.cva_soft_backward(X, fit, 1.0, 4, out=torch.zeros((10, 4)))


def test_soft_forward_checks():
    with pytest.raises(ValueError, match="float32"):
        cx.cva_soft_forward(torch.zeros((10, 6), dtype=torch.float64), torch.zeros((10, 3)))
    with pytest.raises(ValueError, match="N x B"):
        cx.cva_soft_forward(torch.zeros((10, 6)), torch.zeros((9, 3)))
    with pytest.raises(ValueError, match="device"):
        cx.cva_soft_forward(torch.zeros((10, 6)), torch.zeros((10, 3)))


def test_projection_checks():
    cube = torch.zeros((4, 5, 3), dtype=torch.uint16)
    W = np.zeros((3, 2))
    with pytest.raises(ValueError, match="cube must be H x W x B"):
        cx.cva_project(cube[0], W, np.zeros(3))
    with pytest.raises(ValueError, match="W must be B x n"):
        cx.cva_project(cube, np.zeros((4, 2)), np.zeros(3))
    with pytest.raises(ValueError, match="wrong size"):
        cx.cva_project(cube, W, np.zeros(4))
    with pytest.raises(ValueError, match="out must be"):
        cx.cva_project(cube, W, np.zeros(3), out=torch.zeros((2, 4, 5), dtype=torch.int16))
    with pytest.raises(ValueError, match="device"):
        cx.cva_project(cube, W, np.zeros(3))
    lab = torch.zeros((4, 5), dtype=torch.int8)
    with pytest.raises(ValueError, match="labels must be int8"):
        cx.cva_fit_project(cube, lab.to(torch.int16), 3)
    with pytest.raises(ValueError, match="out must be"):
        cx.cva_fit_project(cube, lab, 3, out=torch.zeros((2, 4, 4), dtype=torch.uint8))
    with pytest.raises(ValueError, match="device"):
        cx.cva_fit_project(cube, lab, 3)
    with pytest.raises(ValueError, match="labels must be int8"):
        cx.cva_pca(cube, lab.to(torch.int16), 3)
    with pytest.raises(ValueError, match="mask must be uint8"):
        cx.cva_pca(cube, lab, 3, mask=torch.zeros((4, 5), dtype=torch.int8))
    with pytest.raises(ValueError, match="cva_out must be"):
        cx.cva_pca(cube, lab, 3, cva_out=torch.zeros((3, 4, 5), dtype=torch.uint8))
    with pytest.raises(ValueError, match="pca_out must be"):
        cx.cva_pca(cube, lab, 3, n_pca=2, pca_out=torch.zeros((3, 4, 5), dtype=torch.uint8))
    with pytest.raises(ValueError, match="device"):
        cx.cva_pca(cube, lab, 3)
