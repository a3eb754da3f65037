"""Python binding of the cvamx C ABI: torch tensors in, argument marshalling
only.  Every step of the computation runs in the HIP library; this module
checks shapes and devices, passes pointers and the current torch stream,
and wraps host outputs as NumPy float64 arrays.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import Cube, check, context, lib

_DTYPES = {torch.uint16: _lib.DT_U16, torch.float32: _lib.DT_F32,
           torch.bfloat16: _lib.DT_BF16, torch.float16: _lib.DT_F16}


def _ptr(a) -> ctypes.c_void_p:
    if a is None:
        return ctypes.c_void_p(0)
    if isinstance(a, np.ndarray):
        return ctypes.c_void_p(a.ctypes.data)
    return ctypes.c_void_p(a.data_ptr())


def _stream(dev: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _dev_index(t: torch.Tensor) -> int:
    if t.device.type != "cuda":
        raise ValueError("tensor must be on a HIP (cuda) device")
    return t.device.index if t.device.index is not None else torch.cuda.current_device()


def _cube(cube: torch.Tensor) -> Cube:
    if cube.dim() != 3:
        raise ValueError("cube must be H x W x B (band-interleaved by pixel)")
    if not cube.is_contiguous():
        raise ValueError("cube must be contiguous")
    if cube.dtype not in _DTYPES:
        raise ValueError(f"unsupported cube dtype {cube.dtype}")
    H, W, B = cube.shape
    return Cube(cube.data_ptr(), H, W, B, _DTYPES[cube.dtype])


def _f64(a, n=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if n is not None and a.size != n:
        raise ValueError("wrong size")
    return a


@dataclass
class CvaFit:
    W: np.ndarray            # B x n_comp
    eigvals: np.ndarray      # n_comp
    mean: np.ndarray         # B
    counts: np.ndarray       # K (int64)
    class_means: Optional[np.ndarray]  # K x B
    Sw: Optional[np.ndarray]           # B x B
    Sb: Optional[np.ndarray]           # B x B


def cva_fit(cube: torch.Tensor, labels: torch.Tensor, K: int, precision: str = "fp32",
            ridge: float = 0.0, n_comp: Optional[int] = None) -> CvaFit:
    """CVA fit on the labelled pixels (labels: int8 H x W, -1 = none)."""
    c = _cube(cube)
    if labels.dtype != torch.int8 or tuple(labels.shape) != tuple(cube.shape[:2]):
        raise ValueError("labels must be int8 with the page's H x W shape")
    if labels.device != cube.device or not labels.is_contiguous():
        raise ValueError("labels must be contiguous and on the cube's device")
    B = c.bands
    C = min(K - 1, B)
    n_comp = C if n_comp is None else int(n_comp)
    W = np.empty((B, n_comp))
    lam = np.empty(n_comp)
    mean = np.empty(B)
    counts = np.empty(K, dtype=np.int64)
    cm = np.empty((K, B))
    Sw = np.empty((B, B))
    Sb = np.empty((B, B))
    dev = _dev_index(cube)
    ctx = context(dev)
    st = lib().cva_fit(ctx, ctypes.byref(c), _ptr(labels), K, _lib.PREC[precision], float(ridge),
                       n_comp, _ptr(W), _ptr(lam), _ptr(mean), _ptr(counts), _ptr(cm), _ptr(Sw),
                       _ptr(Sb), _stream(cube.device))
    check(st, ctx)
    return CvaFit(W, lam, mean, counts, cm, Sw, Sb)


def _image_out(out, n, cube, name):
    H, Wd = cube.shape[0], cube.shape[1]
    if out is None:
        return torch.empty((n, H, Wd), dtype=torch.uint8, device=cube.device)
    if out.dtype != torch.uint8 or tuple(out.shape) != (n, H, Wd) or not out.is_contiguous() \
            or out.device != cube.device:
        raise ValueError(f"{name} must be a contiguous uint8 {n} x H x W tensor on the cube's device")
    return out


def cva_pca(cube: torch.Tensor, labels: torch.Tensor, K: int, mask: Optional[torch.Tensor] = None,
            n_pca: int = 3, precision: str = "fp32", ridge: float = 0.0, n_cva: Optional[int] = None,
            cva_out: Optional[torch.Tensor] = None, pca_out: Optional[torch.Tensor] = None,
            standardize: bool = False):
    """CVA and PCA of one page in one library call (cvamx_cva_pca): the same
    results as cva_fit_project, pca_fit (standardize as there) and
    pca_project, with each host finish overlapping GPU work.  Returns
    (cva_images, fit, pca_images, (V, eigvals, mean)); fit as for
    cva_fit_project."""
    c = _cube(cube)
    if labels.dtype != torch.int8 or tuple(labels.shape) != tuple(cube.shape[:2]):
        raise ValueError("labels must be int8 with the page's H x W shape")
    if labels.device != cube.device or not labels.is_contiguous():
        raise ValueError("labels must be contiguous and on the cube's device")
    if mask is not None:
        if mask.dtype != torch.uint8 or tuple(mask.shape) != tuple(cube.shape[:2]):
            raise ValueError("mask must be uint8 with the page's H x W shape")
        if mask.device != cube.device or not mask.is_contiguous():
            raise ValueError("mask must be contiguous and on the cube's device")
    B = c.bands
    n_cva = min(K - 1, B) if n_cva is None else int(n_cva)
    n_pca = int(n_pca)
    cva_out = _image_out(cva_out, n_cva, cube, "cva_out")
    pca_out = _image_out(pca_out, n_pca, cube, "pca_out")
    W = np.empty((B, n_cva))
    lam = np.empty(n_cva)
    mean = np.empty(B)
    counts = np.empty(K, dtype=np.int64)
    V = np.empty((B, n_pca))
    plam = np.empty(n_pca)
    pmean = np.empty(B)
    dev = _dev_index(cube)
    ctx = context(dev)
    check(lib().cvamx_set_pca_standardize(ctx, 1 if standardize else 0), ctx)
    try:
        st = lib().cvamx_cva_pca(ctx, ctypes.byref(c), _ptr(labels), K, _lib.PREC[precision], float(ridge), n_cva,
                                 _ptr(W), _ptr(lam), _ptr(mean), _ptr(counts), _ptr(cva_out), _ptr(mask), n_pca,
                                 _ptr(V), _ptr(plam), _ptr(pmean), _ptr(pca_out), _stream(cube.device))
    finally:
        lib().cvamx_set_pca_standardize(ctx, 0)
    check(st, ctx)
    return cva_out, CvaFit(W, lam, mean, counts, None, None, None), pca_out, (V, plam, pmean)


def cva_fit_points(cube: torch.Tensor, pixels: torch.Tensor, classes: torch.Tensor, K: int,
                   precision: str = "fp32", ridge: float = 0.0, n_comp: Optional[int] = None) -> CvaFit:
    """CVA fit on a list of training points: pixels (int64 N, y * W + x) and
    classes (int8 N, -1 = skip), both on the cube's device."""
    c = _cube(cube)
    if pixels.dtype != torch.int64 or classes.dtype != torch.int8 or pixels.dim() != 1 \
            or tuple(classes.shape) != tuple(pixels.shape):
        raise ValueError("pixels must be int64 N and classes int8 N")
    for t in (pixels, classes):
        if t.device != cube.device or not t.is_contiguous():
            raise ValueError("pixels and classes must be contiguous and on the cube's device")
    B = c.bands
    C = min(K - 1, B)
    n_comp = C if n_comp is None else int(n_comp)
    W = np.empty((B, n_comp))
    lam = np.empty(n_comp)
    mean = np.empty(B)
    counts = np.empty(K, dtype=np.int64)
    cm = np.empty((K, B))
    Sw = np.empty((B, B))
    Sb = np.empty((B, B))
    dev = _dev_index(cube)
    ctx = context(dev)
    st = lib().cva_fit_points(ctx, ctypes.byref(c), _ptr(pixels), _ptr(classes), int(pixels.numel()), K,
                              _lib.PREC[precision], float(ridge), n_comp, _ptr(W), _ptr(lam), _ptr(mean),
                              _ptr(counts), _ptr(cm), _ptr(Sw), _ptr(Sb), _stream(cube.device))
    check(st, ctx)
    return CvaFit(W, lam, mean, counts, cm, Sw, Sb)


def label_index(labels: torch.Tensor, K: int):
    """The training pixels of each class, as the fits gather them: returns
    (idx, counts, offsets) with idx an int32 device tensor holding, for
    k = 0..K-1 in turn, the flat positions of the entries equal to k in
    increasing order (class k at idx[offsets[k]:offsets[k + 1]]), counts
    int64 K and offsets int32 K + 1 (NumPy).  labels: int8, any shape,
    contiguous, on a GPU (-1 = no class)."""
    if labels.dtype != torch.int8 or not labels.is_contiguous() or labels.device.type != "cuda":
        raise ValueError("labels must be a contiguous int8 tensor on the GPU")
    n = int(labels.numel())
    idx = torch.empty(max(n, 1), dtype=torch.int32, device=labels.device)
    counts = np.empty(K, dtype=np.int64)
    offsets = np.empty(K + 1, dtype=np.int32)
    ctx = context(_dev_index(labels))
    st = lib().cvamx_label_index(ctx, _ptr(labels), n, int(K), _ptr(idx), _ptr(counts), _ptr(offsets),
                                 _stream(labels.device))
    check(st, ctx)
    return idx[: int(offsets[K])], counts, offsets


def cva_fit_project(cube: torch.Tensor, labels: torch.Tensor, K: int, precision: str = "fp32",
                    ridge: float = 0.0, n_comp: Optional[int] = None, out: Optional[torch.Tensor] = None,
                    return_range: bool = False):
    """cva_fit then cva_project with the fitted vectors, in one library call
    (no return to Python between the fit's host finish and the projection).
    Returns (images, fit) or (images, fit, range); fit carries W, eigvals,
    mean and counts (class_means, Sw, Sb are None)."""
    c = _cube(cube)
    if labels.dtype != torch.int8 or tuple(labels.shape) != tuple(cube.shape[:2]):
        raise ValueError("labels must be int8 with the page's H x W shape")
    if labels.device != cube.device or not labels.is_contiguous():
        raise ValueError("labels must be contiguous and on the cube's device")
    B = c.bands
    n_comp = min(K - 1, B) if n_comp is None else int(n_comp)
    H, Wd = cube.shape[0], cube.shape[1]
    if out is None:
        out = torch.empty((n_comp, H, Wd), dtype=torch.uint8, device=cube.device)
    elif out.dtype != torch.uint8 or tuple(out.shape) != (n_comp, H, Wd) or not out.is_contiguous() \
            or out.device != cube.device:
        raise ValueError("out must be a contiguous uint8 n_comp x H x W tensor on the cube's device")
    W = np.empty((B, n_comp))
    lam = np.empty(n_comp)
    mean = np.empty(B)
    counts = np.empty(K, dtype=np.int64)
    rng = np.empty((n_comp, 2), dtype=np.float32) if return_range else None
    dev = _dev_index(cube)
    ctx = context(dev)
    st = lib().cva_fit_project(ctx, ctypes.byref(c), _ptr(labels), K, _lib.PREC[precision], float(ridge), n_comp,
                               _ptr(W), _ptr(lam), _ptr(mean), _ptr(counts), _ptr(out), _ptr(rng),
                               _stream(cube.device))
    check(st, ctx)
    fit = CvaFit(W, lam, mean, counts, None, None, None)
    return (out, fit, rng) if return_range else (out, fit)


def cva_project(cube: torch.Tensor, W, center, out: Optional[torch.Tensor] = None,
                return_range: bool = False):
    """Project every pixel on the columns of W (B x n) about `center` and
    stretch each component to uint8 by its page-wide min/max.  Returns an
    n x H x W uint8 tensor (and the n x 2 float32 (min, max) when asked)."""
    c = _cube(cube)
    B = c.bands
    W = _f64(W)
    if W.ndim != 2 or W.shape[0] != B:
        raise ValueError("W must be B x n")
    n = W.shape[1]
    center = _f64(center, B)
    H, Wd = cube.shape[0], cube.shape[1]
    if out is None:
        out = torch.empty((n, H, Wd), dtype=torch.uint8, device=cube.device)
    elif out.dtype != torch.uint8 or tuple(out.shape) != (n, H, Wd) or not out.is_contiguous() \
            or out.device != cube.device:
        raise ValueError("out must be a contiguous uint8 n x H x W tensor on the cube's device")
    rng = np.empty((n, 2), dtype=np.float32) if return_range else None
    dev = _dev_index(cube)
    ctx = context(dev)
    st = lib().cva_project(ctx, ctypes.byref(c), _ptr(W), _ptr(center), n, _ptr(out), _ptr(rng),
                           _stream(cube.device))
    check(st, ctx)
    return (out, rng) if return_range else out


def cva_project_noalloc(cube: torch.Tensor, W, center, out: torch.Tensor, return_range: bool = False):
    """cva_project through the library's allocation-free entry point: the
    caller passes the n x H x W uint8 output, and the library's device
    scratch is a fixed array per GPU (calls overlapping on one GPU race)."""
    c = _cube(cube)
    B = c.bands
    W = _f64(W)
    if W.ndim != 2 or W.shape[0] != B:
        raise ValueError("W must be B x n")
    n = W.shape[1]
    center = _f64(center, B)
    H, Wd = cube.shape[0], cube.shape[1]
    if out is None or out.dtype != torch.uint8 or tuple(out.shape) != (n, H, Wd) or not out.is_contiguous() \
            or out.device != cube.device:
        raise ValueError("out must be a contiguous uint8 n x H x W tensor on the cube's device")
    rng = np.empty((n, 2), dtype=np.float32) if return_range else None
    dev = _dev_index(cube)
    ctx = context(dev)
    st = lib().cva_project_noalloc(ctx, ctypes.byref(c), _ptr(W), _ptr(center), n, _ptr(out), _ptr(rng),
                                   _stream(cube.device))
    check(st, ctx)
    return (out, rng) if return_range else out


def project_float(cube: torch.Tensor, W, center, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """The float images y_j = w_j^T (x - center) of every pixel (the (W, mean)
    of a CVA fit or the (V, mean) of a PCA fit) as an n x H x W float32
    tensor: the values whose min/max and stretch cva_project takes."""
    c = _cube(cube)
    B = c.bands
    W = _f64(W)
    if W.ndim != 2 or W.shape[0] != B:
        raise ValueError("W must be B x n")
    n = W.shape[1]
    center = _f64(center, B)
    H, Wd = cube.shape[0], cube.shape[1]
    if out is None:
        out = torch.empty((n, H, Wd), dtype=torch.float32, device=cube.device)
    elif out.dtype != torch.float32 or tuple(out.shape) != (n, H, Wd) or not out.is_contiguous() \
            or out.device != cube.device:
        raise ValueError("out must be a contiguous float32 n x H x W tensor on the cube's device")
    dev = _dev_index(cube)
    ctx = context(dev)
    st = lib().cvamx_project_float(ctx, ctypes.byref(c), _ptr(W), _ptr(center), n, _ptr(out),
                                   _stream(cube.device))
    check(st, ctx)
    return out


STRETCH_MODES = {"minmax": 1, "training": 2, "percentile": 3}


def stretch(y: torch.Tensor, mode: str = "minmax", pct: float = 1.0, train_pixels: Optional[torch.Tensor] = None,
            bits: int = 8, out: Optional[torch.Tensor] = None, return_range: bool = False):
    """Stretch planar float images (n x ... float32, e.g. from project_float)
    to uint8 (bits=8) or uint16 (bits=16) planes of the same shape.
    mode "minmax": each plane's own min/max; "training": the min/max over
    train_pixels (int64 flat pixel indices on the same device); "percentile":
    the pct-th and (100 - pct)-th percentiles, values beyond them clamped.
    With return_range, also the n x 2 float64 (a_j, b_j)."""
    if y.dtype != torch.float32 or y.dim() < 2 or not y.is_contiguous():
        raise ValueError("y must be a contiguous float32 n x ... tensor")
    if mode not in STRETCH_MODES:
        raise ValueError(f"mode must be one of {sorted(STRETCH_MODES)}")
    if bits not in (8, 16):
        raise ValueError("bits must be 8 or 16")
    n = y.shape[0]
    P = y[0].numel()
    odt = torch.uint8 if bits == 8 else torch.uint16
    if out is None:
        out = torch.empty(y.shape, dtype=odt, device=y.device)
    elif out.dtype != odt or tuple(out.shape) != tuple(y.shape) or not out.is_contiguous() or out.device != y.device:
        raise ValueError("out must be a contiguous tensor of y's shape, uint8 or uint16 per bits, on y's device")
    n_train = 0
    if mode == "training":
        if train_pixels is None or train_pixels.dtype != torch.int64 or train_pixels.dim() != 1:
            raise ValueError("mode 'training' needs train_pixels, an int64 vector")
        if train_pixels.device != y.device or not train_pixels.is_contiguous():
            raise ValueError("train_pixels must be contiguous and on y's device")
        n_train = int(train_pixels.numel())
    else:
        train_pixels = None
    rng = np.empty((n, 2)) if return_range else None
    dev = _dev_index(y)
    ctx = context(dev)
    st = lib().cvamx_stretch(ctx, _ptr(y), P, n, STRETCH_MODES[mode], float(pct), _ptr(train_pixels), n_train,
                             bits, _ptr(out), _ptr(rng), _stream(y.device))
    check(st, ctx)
    return (out, rng) if return_range else out


def compose_rgb(r: Optional[torch.Tensor], g: Optional[torch.Tensor], b: Optional[torch.Tensor]) -> torch.Tensor:
    """Interleave three uint8 planes of one shape (None = an all-zero channel)
    into a ... x 3 uint8 RGB image."""
    planes = [t for t in (r, g, b) if t is not None]
    if not planes:
        raise ValueError("at least one channel must be given")
    ref = planes[0]
    for t in planes:
        if t.dtype != torch.uint8 or t.shape != ref.shape or t.device != ref.device or not t.is_contiguous():
            raise ValueError("channels must be contiguous uint8 tensors of one shape on one device")
    rgb = torch.empty(tuple(ref.shape) + (3,), dtype=torch.uint8, device=ref.device)
    dev = _dev_index(ref)
    ctx = context(dev)
    st = lib().cvamx_compose_rgb(ctx, _ptr(r), _ptr(g), _ptr(b), int(ref.numel()), _ptr(rgb), _stream(ref.device))
    check(st, ctx)
    return rgb


_BAND_DTYPES = {torch.uint8: _lib.DT_U8, torch.uint16: _lib.DT_U16, torch.float32: _lib.DT_F32}


def bands_to_cube(bands: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """A page's band images, band-sequential B x H x W (uint8, uint16 or
    float32, on the device), as the band-interleaved H x W x B page
    (uint16 for 8/16-bit bands, float32 for float bands)."""
    if bands.dtype not in _BAND_DTYPES or bands.dim() != 3 or not bands.is_contiguous():
        raise ValueError("bands must be a contiguous B x H x W uint8, uint16 or float32 tensor")
    B, H, W = bands.shape
    odt = torch.float32 if bands.dtype == torch.float32 else torch.uint16
    if out is None:
        out = torch.empty((H, W, B), dtype=odt, device=bands.device)
    elif out.dtype != odt or tuple(out.shape) != (H, W, B) or not out.is_contiguous() or out.device != bands.device:
        raise ValueError("out must be a contiguous H x W x B tensor of the page type on the bands' device")
    dev = _dev_index(bands)
    ctx = context(dev)
    st = lib().cvamx_bands_to_cube(ctx, _ptr(bands), _BAND_DTYPES[bands.dtype], B, H * W, _ptr(out),
                                   _stream(bands.device))
    check(st, ctx)
    return out


def run_pages(pages, K: int, n_comp: Optional[int] = None, precision: str = "fp32", ridge: float = 0.0,
              mode: str = "minmax", pct: float = 1.0, bits: int = 8, device: int = 0):
    """CVA enhancement of many pages of one geometry, copies overlapped with
    compute.  pages: a list of dicts with host tensors 'bands' (B x H x W
    uint8 / uint16 / float32; page-locked memory, e.g. pin_memory=True,
    for the overlap), 'pixels' (int64 N) and 'classes' (int8 N).  Returns
    one dict per page: 'images' (n_comp x H x W, uint8 or uint16, in
    page-locked host memory), 'W', 'eigvals', 'range' and 'status' (0 = ok;
    a page whose fit failed keeps its error code and no images)."""
    if not pages:
        raise ValueError("no pages")
    b0 = pages[0]["bands"]
    if b0.dtype not in _BAND_DTYPES or b0.dim() != 3:
        raise ValueError("bands must be B x H x W uint8, uint16 or float32")
    B, H, W = b0.shape
    C = min(K - 1, B)
    n_comp = C if n_comp is None else int(n_comp)
    odt = torch.uint8 if bits == 8 else torch.uint16
    arr = (_lib.Page * len(pages))()
    keep, outs = [], []
    for i, pg in enumerate(pages):
        bands, pix, cls = pg["bands"], pg["pixels"], pg["classes"]
        if bands.dtype != b0.dtype or tuple(bands.shape) != (B, H, W) or bands.device.type != "cpu" \
                or not bands.is_contiguous():
            raise ValueError(f"page {i}: bands must be a contiguous host tensor like page 0's")
        if pix.dtype != torch.int64 or cls.dtype != torch.int8 or pix.dim() != 1 \
                or tuple(cls.shape) != tuple(pix.shape) or pix.device.type != "cpu" or cls.device.type != "cpu":
            raise ValueError(f"page {i}: pixels must be host int64 N and classes host int8 N")
        pix, cls = pix.contiguous(), cls.contiguous()
        images = torch.empty((n_comp, H, W), dtype=odt, pin_memory=True)
        o = {"images": images, "W": np.empty((B, n_comp)), "eigvals": np.empty(n_comp),
             "range": np.empty((n_comp, 2))}
        arr[i] = _lib.Page(bands.data_ptr(), pix.data_ptr(), cls.data_ptr(), int(pix.numel()), images.data_ptr(),
                           o["W"].ctypes.data, o["eigvals"].ctypes.data, o["range"].ctypes.data, 0)
        keep += [bands, pix, cls]
        outs.append(o)
    ctx = context(device)
    st = lib().cvamx_run_pages(ctx, _BAND_DTYPES[b0.dtype], B, H, W, K, n_comp, _lib.PREC[precision],
                               float(ridge), STRETCH_MODES[mode], float(pct), bits, arr, len(pages),
                               _stream(torch.device("cuda", device)))
    check(st, ctx)
    for i, o in enumerate(outs):
        o["status"] = int(arr[i].status)
    return outs


@dataclass
class ClusterIndices:
    centroids: np.ndarray   # K x n
    scatter: np.ndarray     # K   (S_k, the mean distance to the centroid)
    dist: np.ndarray        # K x K (M_ij, centroid distances)
    dbi_pairs: np.ndarray   # K x K (R_ij)
    dunn_pairs: np.ndarray  # K x K (D_ij)
    dbi: float
    dunn: float


_IMG_DTYPES = {torch.uint8: _lib.DT_U8, **_DTYPES}


def cluster_indices(images: torch.Tensor, pixels: torch.Tensor, classes: torch.Tensor, K: int,
                    p: float = 2.0) -> ClusterIndices:
    """Davies-Bouldin and Dunn indices of labelled points on images
    (n x ... planes, or one H x W image): pixels int64 N flat indices,
    classes int8 N (-1 = skip), all on one device."""
    if images.dtype not in _IMG_DTYPES or not images.is_contiguous():
        raise ValueError("images must be a contiguous uint8, uint16, float32, bfloat16 or float16 tensor")
    if images.dim() == 2:
        images = images.unsqueeze(0)
    if pixels.dtype != torch.int64 or classes.dtype != torch.int8 or pixels.dim() != 1 \
            or tuple(classes.shape) != tuple(pixels.shape):
        raise ValueError("pixels must be int64 N and classes int8 N")
    for t in (pixels, classes):
        if t.device != images.device or not t.is_contiguous():
            raise ValueError("pixels and classes must be contiguous and on the images' device")
    n = images.shape[0]
    P = images[0].numel()
    A = np.empty((K, n))
    S = np.empty(K)
    M = np.empty((K, K))
    R = np.empty((K, K))
    D = np.empty((K, K))
    sc = np.empty(2)
    dev = _dev_index(images)
    ctx = context(dev)
    st = lib().cvamx_cluster_indices(ctx, _ptr(images), _IMG_DTYPES[images.dtype], P, n, _ptr(pixels),
                                     _ptr(classes), int(pixels.numel()), K, float(p), _ptr(A), _ptr(S),
                                     _ptr(M), _ptr(R), _ptr(D), _ptr(sc), _stream(images.device))
    check(st, ctx)
    return ClusterIndices(A, S, M, R, D, float(sc[0]), float(sc[1]))


def pca_fit(cube: torch.Tensor, mask: Optional[torch.Tensor] = None, n_comp: int = 3,
            precision: str = "fp32", standardize: bool = False):
    """Covariance PCA of the page (or of the pixels where mask != 0); with
    standardize=True, PCA of the bands scaled to unit variance (correlation
    matrix), V then holding the projection vectors D^-1/2 u.
    Returns (V B x n, eigvals n, mean B, cov B x B)."""
    c = _cube(cube)
    B = c.bands
    if mask is not None:
        if mask.dtype != torch.uint8 or tuple(mask.shape) != tuple(cube.shape[:2]):
            raise ValueError("mask must be uint8 with the page's H x W shape")
        if mask.device != cube.device or not mask.is_contiguous():
            raise ValueError("mask must be contiguous and on the cube's device")
    V = np.empty((B, n_comp))
    lam = np.empty(n_comp)
    mean = np.empty(B)
    cov = np.empty((B, B))
    dev = _dev_index(cube)
    ctx = context(dev)
    check(lib().cvamx_set_pca_standardize(ctx, 1 if standardize else 0), ctx)
    try:
        st = lib().pca_fit(ctx, ctypes.byref(c), _ptr(mask), n_comp, _lib.PREC[precision], _ptr(V),
                           _ptr(lam), _ptr(mean), _ptr(cov), _stream(cube.device))
    finally:
        lib().cvamx_set_pca_standardize(ctx, 0)
    check(st, ctx)
    return V, lam, mean, cov


def pca_project(cube: torch.Tensor, V, mean, out=None, return_range: bool = False):
    return cva_project(cube, V, mean, out=out, return_range=return_range)


@dataclass
class SoftFit:
    J: float
    W: np.ndarray            # B x C
    eigvals: np.ndarray      # C
    mean: np.ndarray         # B
    class_means: np.ndarray  # K x B


def _soft_inputs(X: torch.Tensor, w: torch.Tensor):
    if X.dtype != torch.float32 or w.dtype != torch.float32:
        raise ValueError("X and w must be float32")
    if X.dim() != 2 or w.dim() != 2 or X.shape[0] != w.shape[0]:
        raise ValueError("X must be N x B and w N x K")
    if not (X.is_contiguous() and w.is_contiguous()) or X.device != w.device:
        raise ValueError("X and w must be contiguous and on one device")
    return X.shape[0], X.shape[1], w.shape[1]


def cva_soft_forward(X: torch.Tensor, w: torch.Tensor, precision: str = "fp32",
                     ridge: float = 0.0) -> SoftFit:
    N, B, K = _soft_inputs(X, w)
    C = min(K - 1, B)
    J = np.empty(1)
    W = np.empty((B, C))
    lam = np.empty(C)
    mean = np.empty(B)
    cm = np.empty((K, B))
    dev = _dev_index(X)
    ctx = context(dev)
    st = lib().cva_soft_forward(ctx, _ptr(X), _ptr(w), N, B, K, _lib.PREC[precision], float(ridge),
                                _ptr(J), _ptr(W), _ptr(lam), _ptr(mean), _ptr(cm), _stream(X.device))
    check(st, ctx)
    return SoftFit(float(J[0]), W, lam, mean, cm)


def cva_soft_backward(X: torch.Tensor, fit: SoftFit, dJ: float, K: int,
                      out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """dJ * dJ/dw for the training pixels X (N x B float32, contiguous, on the
    GPU) of a soft-label fit with K classes; out (N x K float32, contiguous,
    on X's device) receives it, or a new tensor does."""
    if X.dtype != torch.float32 or X.dim() != 2 or not X.is_contiguous():
        raise ValueError("X must be a contiguous N x B float32 tensor")
    N, B = X.shape
    C = min(int(K) - 1, B)
    if np.shape(fit.class_means) != (K, B) or np.shape(fit.W) != (B, C) or np.size(fit.eigvals) != C \
            or np.size(fit.mean) != B:
        raise ValueError("fit does not belong to K classes of X's bands: class_means must be K x B, "
                         "W B x min(K-1, B), eigvals min(K-1, B) and mean B")
    if out is not None and (out.dtype != torch.float32 or tuple(out.shape) != (N, K) or not out.is_contiguous()
                            or out.device != X.device):
        raise ValueError("out must be a contiguous float32 N x K tensor on X's device")
    dev = _dev_index(X)
    if out is None:
        out = torch.empty((N, K), dtype=torch.float32, device=X.device)
    W = _f64(fit.W)
    lam = _f64(fit.eigvals)
    mean = _f64(fit.mean)
    cm = _f64(fit.class_means)
    ctx = context(dev)
    st = lib().cva_soft_backward(ctx, _ptr(X), _ptr(W), _ptr(lam), _ptr(mean), _ptr(cm), N, B, K,
                                 float(dJ), _ptr(out), _stream(X.device))
    check(st, ctx)
    return out


class SoftCVA(torch.autograd.Function):
    """J = sum of the canonical eigenvalues of the soft-label problem, with
    the hand-written backward kernel for dJ/dw.  X carries no gradient."""

    @staticmethod
    def forward(ctx, X, w, precision="fp32", ridge=0.0):
        fit = cva_soft_forward(X.detach(), w.detach(), precision, ridge)
        ctx.fit = fit
        ctx.K = w.shape[1]
        ctx.save_for_backward(X)
        return torch.tensor(fit.J, dtype=torch.float64, device=w.device)

    @staticmethod
    def backward(ctx, gJ):
        (X,) = ctx.saved_tensors
        dJ = float(gJ.item())
        dw = cva_soft_backward(X.detach(), ctx.fit, dJ, ctx.K)
        return None, dw, None, None


def cva_soft_update(w: torch.Tensor, grad: torch.Tensor, step: float) -> torch.Tensor:
    """One refinement step of the class weights w (N x K float32, updated in
    place) along grad (N x K float32, e.g. cva_soft_backward with dJ = 1):
    the mean-free gradient, scaled to `step` at its largest entry, then the
    projection of each row onto the probability simplex.  Returns w."""
    for name, t in (("w", w), ("grad", grad)):
        if t.dtype != torch.float32 or t.dim() != 2 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous N x K float32 tensor")
    if grad.shape != w.shape or grad.device != w.device:
        raise ValueError("grad must have w's shape and device")
    dev = _dev_index(w)
    ctx = context(dev)
    N, K = w.shape
    check(lib().cva_soft_update(ctx, _ptr(grad), _ptr(w), N, K, float(step), _stream(w.device)), ctx)
    return w


def refine_weights(X: torch.Tensor, w: torch.Tensor, steps: int = 3, step: float = 0.5,
                   precision: str = "fp32") -> SoftFit:
    """Refine an analyst's class weights (N x K float32 on the GPU, updated
    in place) by `steps` gradient steps on the Fisher criterion: soft-label
    forward, hand-written backward, cva_soft_update.  Returns the fit of the
    refined weights."""
    g = torch.empty_like(w)
    for _ in range(int(steps)):
        fit = cva_soft_forward(X, w, precision)
        cva_soft_backward(X, fit, 1.0, w.shape[1], out=g)
        cva_soft_update(w, g, step)
    return cva_soft_forward(X, w, precision)


# ------------------------------------------------------------ host-only calls

def cva_solve_moments(counts, class_means, Sw, ridge: float = 0.0, n_comp: Optional[int] = None):
    """FP64 CVA solve from class counts, class means and S_w (no GPU)."""
    counts = np.ascontiguousarray(np.asarray(counts, dtype=np.int64))
    cm = _f64(class_means)
    Sw = _f64(Sw)
    K, B = cm.shape
    n_comp = min(K - 1, B) if n_comp is None else n_comp
    W = np.empty((B, n_comp))
    lam = np.empty(n_comp)
    mean = np.empty(B)
    st = lib().cva_solve_moments(_ptr(counts), _ptr(cm), _ptr(Sw), K, B, float(ridge), n_comp,
                                 _ptr(W), _ptr(lam), _ptr(mean))
    check(st)
    return W, lam, mean


def sym_eig(A):
    """Descending symmetric eigendecomposition (no GPU)."""
    A = _f64(A)
    n = A.shape[0]
    w = np.empty(n)
    V = np.empty((n, n))
    check(lib().cvamx_sym_eig(n, _ptr(A), _ptr(w), _ptr(V)))
    return w, V


def sym_eig_top(A, k: int):
    """All eigenvalues (descending) and the k leading eigenvectors (no GPU)."""
    A = _f64(A)
    n = A.shape[0]
    w = np.empty(n)
    V = np.empty((n, int(k)))
    check(lib().cvamx_sym_eig_top(n, _ptr(A), int(k), _ptr(w), _ptr(V)))
    return w, V


# ------------------------------------------------------------ kernel timing

def set_plain_fp32(enable: bool = True, device: int = 0) -> None:
    """Run every FP32 request on `device` on the plain FP32 vector-ALU kernels
    (fit moments, PCA covariance, projections) instead of the matrix-core
    paths; False restores the default.  The reference for the speed-ups."""
    ctx = context(device)
    check(lib().cvamx_set_plain_fp32(ctx, 1 if enable else 0), ctx)


def stream_read(buf: torch.Tensor, sink: Optional[torch.Tensor] = None) -> None:
    """Read every byte of a contiguous device tensor once (the reference
    read stream of the page passes), asynchronously on torch's current
    stream; for timing the device's read ceiling."""
    if buf.device.type != "cuda" or not buf.is_contiguous():
        raise ValueError("buf must be a contiguous device tensor")
    nbytes = buf.numel() * buf.element_size()
    if nbytes < 16 or nbytes % 16 != 0:
        raise ValueError("buf must hold a positive multiple of 16 bytes")
    if sink is None:
        sink = torch.zeros(1, dtype=torch.int32, device=buf.device)
    elif sink.device != buf.device or sink.dtype != torch.int32 or sink.numel() < 1:
        raise ValueError("sink must be an int32 tensor on buf's device")
    ctx = context(_dev_index(buf))
    check(lib().cvamx_stream_read(ctx, _ptr(buf), nbytes, _ptr(sink), _stream(buf.device)), ctx)


def stream_mix(src: torch.Tensor, dst: torch.Tensor, sink: Optional[torch.Tensor] = None) -> None:
    """Read every byte of src once and write every byte of dst once, the
    writes spread evenly over the reads (the ceiling of a pass that writes
    as it reads in that proportion); dst's contents afterwards are
    unspecified.  Asynchronous on torch's current stream."""
    for name, t in (("src", src), ("dst", dst)):
        if t.device.type != "cuda" or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous device tensor")
    if dst.device != src.device:
        raise ValueError("dst must be on src's device")
    nr, nw = src.numel() * src.element_size(), dst.numel() * dst.element_size()
    if nr < 16 or nr % 16 != 0 or nw < 16 or nw % 16 != 0 or nw > nr:
        raise ValueError("src and dst must hold positive multiples of 16 bytes, dst no more than src")
    if sink is None:
        sink = torch.zeros(1, dtype=torch.int32, device=src.device)
    elif sink.device != src.device or sink.dtype != torch.int32 or sink.numel() < 1:
        raise ValueError("sink must be an int32 tensor on src's device")
    ctx = context(_dev_index(src))
    check(lib().cvamx_stream_mix(ctx, _ptr(src), nr, _ptr(dst), nw, _ptr(sink), _stream(src.device)), ctx)


_SCHEDULES = {"auto": 0, "two_reads": 1, "force_reread": 2}


def set_schedule(schedule: str = "auto", device: int = 0) -> None:
    """How the projections read the page on `device`: "auto" (once, with an
    fp16 intermediate whose error bound is checked on the device, on every
    page type), "two_reads", or "force_reread" (the one-read pass 1, then
    its page re-reading fallback; for tests)."""
    if schedule not in _SCHEDULES:
        raise ValueError(f"schedule must be one of {sorted(_SCHEDULES)}")
    ctx = context(device)
    check(lib().cvamx_set_schedule(ctx, _SCHEDULES[schedule]), ctx)


def profile_enable(enable=True, device: int = 0) -> None:
    """Bracket every kernel the library launches on `device` with HIP events
    (on the stream it is launched on); enable="projection" brackets only the
    page-streaming projection passes; clears earlier totals."""
    ctx = context(device)
    mode = 2 if enable == "projection" else (1 if enable else 0)
    check(lib().cvamx_profile_enable(ctx, mode), ctx)


def profile_report(device: int = 0) -> dict:
    """{kernel name: (launches, total milliseconds)} since profile_enable."""
    ctx = context(device)
    need = lib().cvamx_profile_report(ctx, None, 0)
    if need < 0:
        check(int(need), ctx)
    buf = ctypes.create_string_buffer(int(need))
    lib().cvamx_profile_report(ctx, buf, need)
    out = {}
    for line in buf.value.decode().splitlines():
        name, n, ms = line.split()
        out[name] = (int(n), float(ms))
    return out
