"""Seeded synthetic multispectral pages.

The paper's workload is a page of a palimpsest imaged under 23 illuminations,
8-bit, with an analyst picking 50 training pixels in each of four classes
(parchment, overwriting, underwriting, both) and optionally an "outside the
folio" class (Section 2, data description and choice of input points).  The
page images themselves are not available, so these generators stand in for
them with the same structure:

* a per-pixel class map built from stroke masks: quadratic Bezier strokes
  2-6 px thick and 10-60 px long scattered along text lines; the under-text
  lines are offset and turned against the over-text lines; where over- and
  under-text overlap the pixel belongs to the "both" class when that class
  exists; the full-page layout adds an outside-the-folio border, stains,
  ruling lines and bleed-through strokes;
* per-class spectra: mean spectra drawn U[800, 3500] per band (12-bit
  detector range), and either a shared covariance 60^2 (0.7 I + 0.3 11^T) or
  per-class covariances Q diag(10^U[2,4]) Q^T with Q Haar-random;
* pixel values x = mu_k + L_k z with z standard normal, rounded to the
  nearest integer and clipped to [0, 4095] for uint16 pages, or kept as
  float32 digital numbers;
* a sparse label map (int8, -1 = not a training pixel) holding n training
  pixels per class drawn without replacement from each class mask;
* for the soft-label variant, per-pixel class weights drawn Dirichlet(0.5)
  for training pixels within 2 px of a class boundary and one-hot inside.

Nothing here computes moments, scatter matrices, eigenvectors or
projections: this module only draws inputs.
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# Class-map layouts by number of classes.
#   text3: parchment, overtext, undertext (overlap -> overtext)
#   text4: parchment, overtext, undertext, both
#   text5: parchment, overtext, undertext, both, outside
#   page8: parchment, overtext, undertext, both, outside, stain, ruling, bleed
CLASS_NAMES = {
    "text3": ["parchment", "overtext", "undertext"],
    "text4": ["parchment", "overtext", "undertext", "both"],
    "text5": ["parchment", "overtext", "undertext", "both", "outside"],
    "page8": ["parchment", "overtext", "undertext", "both", "outside",
              "stain", "ruling", "bleed"],
}

WORKLOADS = {
    1: dict(workload="cva_512x512x16_u16_k3", H=512, W=512, B=16, dtype="u16",
            K=3, n_per_class=2000, cov="shared", layout="text3", seed=1,
            text_spacing=30.0, pca_comps=0),
    2: dict(workload="cva_pca_4096x4096x23_u16_k4", H=4096, W=4096, B=23,
            dtype="u16", K=4, n_per_class=50000, cov="per_class",
            layout="text4", seed=2, text_spacing=28.0, pca_comps=3),
    3: dict(workload="cva_mixed_4096x4096x23_half_k4", H=4096, W=4096, B=23,
            dtype="u16", K=4, n_per_class=50000, cov="per_class",
            layout="text4", seed=2, text_spacing=28.0, pca_comps=3,
            half=("bf16", "f16")),
    4: dict(workload="soft_cva_8192x6144x23_f32_k5", H=8192, W=6144, B=23,
            dtype="f32", K=5, n_per_class=200000, cov="per_class",
            layout="text5", seed=4, text_spacing=26.0, pca_comps=0),
    5: dict(workload="cva_pca_page_7216x5412x33_u16_k8", H=7216, W=5412, B=33,
            dtype="u16", K=8, n_per_class=200000, cov="per_class",
            layout="page8", seed=5, text_spacing=26.0, pca_comps=3),
}


@dataclass
class Case:
    """One synthetic page and its training pixels."""
    config: int
    workload: str
    H: int
    W: int
    B: int
    K: int
    dtype: str                      # "u16" or "f32" (half cubes via to_half_cube)
    cube: Optional[np.ndarray]      # H x W x B, band-interleaved-by-pixel
    labels: np.ndarray              # H x W int8, -1 = not a training pixel
    class_map: np.ndarray           # H x W int8, class of every pixel
    mu: np.ndarray                  # K x B class mean spectra used to draw
    chol: np.ndarray                # K x B x B lower Cholesky factors used to draw
    class_names: list = field(default_factory=list)
    n_per_class: int = 0
    seed: int = 0


# ---------------------------------------------------------------------------
# geometry
# ---------------------------------------------------------------------------

def _disk_offsets(r: float):
    ri = int(math.ceil(r))
    dy, dx = np.mgrid[-ri:ri + 1, -ri:ri + 1]
    keep = dx * dx + dy * dy <= r * r + 1e-9
    return dy[keep].astype(np.int64), dx[keep].astype(np.int64)


def _stamp(mask: np.ndarray, y: np.ndarray, x: np.ndarray, r: np.ndarray):
    """Set mask pixels within radius r of each (y, x) sample point."""
    H, W = mask.shape
    flat = mask.reshape(-1)
    yi = np.rint(y).astype(np.int64)
    xi = np.rint(x).astype(np.int64)
    for rv in np.unique(r):
        sel = r == rv
        oy, ox = _disk_offsets(float(rv))
        ys, xs = yi[sel], xi[sel]
        step = max(1, 4_000_000 // max(1, oy.size))
        for s in range(0, ys.size, step):
            yy = (ys[s:s + step, None] + oy[None, :]).ravel()
            xx = (xs[s:s + step, None] + ox[None, :]).ravel()
            ok = (yy >= 0) & (yy < H) & (xx >= 0) & (xx < W)
            flat[yy[ok] * W + xx[ok]] = True


def _bezier_strokes(mask, rng, cx, cy, ux, uy, L, bend, thick):
    """Rasterise quadratic Bezier strokes centred at (cx, cy), chord
    direction (ux, uy), chord length L, control-point bend along the normal,
    integer thickness."""
    n = cx.size
    if n == 0:
        return
    m = np.ceil(L).astype(np.int64) + 1
    sid = np.repeat(np.arange(n), m)
    start = np.concatenate([[0], np.cumsum(m)[:-1]])
    t = (np.arange(sid.size) - start[sid]) / (m[sid] - 1)
    p0x = cx - 0.5 * L * ux
    p0y = cy - 0.5 * L * uy
    p2x = cx + 0.5 * L * ux
    p2y = cy + 0.5 * L * uy
    p1x = cx - bend * uy
    p1y = cy + bend * ux
    a = (1 - t) ** 2
    b = 2 * (1 - t) * t
    c = t * t
    x = a * p0x[sid] + b * p1x[sid] + c * p2x[sid]
    y = a * p0y[sid] + b * p1y[sid] + c * p2y[sid]
    r = (thick[sid] / 2.0)
    _stamp(mask, y, x, r)


def _text_layer(H, W, rng, spacing, angle_deg, pitch=(22.0, 44.0)):
    """Strokes scattered along parallel text lines at the given angle."""
    mask = np.zeros((H, W), dtype=bool)
    ang = math.radians(angle_deg)
    dx, dy = math.cos(ang), math.sin(ang)          # along the line
    nx, ny = -dy, dx                               # across the line
    diag = math.hypot(H, W)
    cx0, cy0 = W / 2.0, H / 2.0
    offs = np.arange(-diag / 2, diag / 2, spacing) + rng.uniform(0, spacing)
    xh = 0.45 * spacing                            # text band height
    for o in offs:
        nst = int(diag / pitch[0]) + 2
        gaps = rng.uniform(pitch[0], pitch[1], nst)
        s = -diag / 2 + np.cumsum(gaps)
        s = s[s < diag / 2]
        k = s.size
        jit = rng.uniform(-xh / 2, xh / 2, k)
        cx = cx0 + o * nx + s * dx + jit * nx
        cy = cy0 + o * ny + s * dy + jit * ny
        inside = (cx > -40) & (cx < W + 40) & (cy > -40) & (cy < H + 40)
        if not inside.any():
            continue
        cx, cy = cx[inside], cy[inside]
        k = cx.size
        th = ang + rng.uniform(-math.pi / 2, math.pi / 2, k)
        L = rng.uniform(10.0, 60.0, k)
        bend = rng.uniform(-0.25, 0.25, k) * L
        thick = rng.integers(2, 7, k).astype(np.float64)
        _bezier_strokes(mask, rng, cx, cy, np.cos(th), np.sin(th), L, bend, thick)
    return mask


def _blobs(H, W, rng, target_px, rmin, rmax, region=None):
    """Irregular elliptical blobs until about target_px pixels are covered."""
    mask = np.zeros((H, W), dtype=bool)
    covered = 0
    tries = 0
    while covered < target_px and tries < 10000:
        tries += 1
        a = rng.uniform(rmin, rmax)
        b = a * rng.uniform(0.4, 1.0)
        cy = rng.uniform(0, H)
        cx = rng.uniform(0, W)
        rot = rng.uniform(0, math.pi)
        y0, y1 = int(max(0, cy - a - 2)), int(min(H, cy + a + 3))
        x0, x1 = int(max(0, cx - a - 2)), int(min(W, cx + a + 3))
        if y1 <= y0 or x1 <= x0:
            continue
        yy, xx = np.mgrid[y0:y1, x0:x1]
        u = (xx - cx) * math.cos(rot) + (yy - cy) * math.sin(rot)
        v = -(xx - cx) * math.sin(rot) + (yy - cy) * math.cos(rot)
        phi = np.arctan2(v, u)
        wob = 1.0 + 0.15 * np.sin(3 * phi + rng.uniform(0, 6.3)) \
            + 0.08 * np.sin(5 * phi + rng.uniform(0, 6.3))
        inside = (u / a) ** 2 + (v / b) ** 2 <= wob ** 2
        if region is not None:
            inside &= region[y0:y1, x0:x1]
        before = mask[y0:y1, x0:x1].sum()
        mask[y0:y1, x0:x1] |= inside
        covered += int(mask[y0:y1, x0:x1].sum() - before)
    return mask


def _ruling(H, W, rng, spacing, angle_deg):
    mask = np.zeros((H, W), dtype=bool)
    ang = math.radians(angle_deg)
    dx, dy = math.cos(ang), math.sin(ang)
    nx, ny = -dy, dx
    diag = math.hypot(H, W)
    offs = np.arange(-diag / 2, diag / 2, spacing) + rng.uniform(0, spacing)
    s = np.arange(-diag / 2, diag / 2, 1.0)
    for o in offs:
        th = float(rng.integers(2, 4))
        x = W / 2 + o * nx + s * dx
        y = H / 2 + o * ny + s * dy
        ok = (x > -5) & (x < W + 5) & (y > -5) & (y < H + 5)
        if ok.any():
            _stamp(mask, y[ok], x[ok], np.full(int(ok.sum()), th / 2.0))
    return mask


def make_class_map(H: int, W: int, layout: str, rng: np.random.Generator,
                   text_spacing: float = 28.0) -> np.ndarray:
    """Per-pixel class ids (int8) for the given layout."""
    over_ang = rng.uniform(-3.0, 3.0)
    under_ang = over_ang + 90.0 + rng.uniform(-10.0, 10.0)
    over = _text_layer(H, W, rng, text_spacing, over_ang)
    under = _text_layer(H, W, rng, text_spacing * rng.uniform(0.9, 1.1), under_ang)
    cm = np.zeros((H, W), dtype=np.int8)
    if layout == "text3":
        cm[under] = 2
        cm[over] = 1
        return cm
    extra = {}
    folio = np.ones((H, W), dtype=bool)
    if layout in ("text5", "page8"):
        my, mx = int(0.06 * H), int(0.06 * W)
        folio[:] = False
        folio[my:H - my, mx:W - mx] = True
    if layout == "page8":
        area = H * W
        extra[5] = _blobs(H, W, rng, 0.04 * area, 0.02 * min(H, W), 0.06 * min(H, W), folio)
        extra[6] = _ruling(H, W, rng, text_spacing * 3.5, over_ang)
        bleed = _text_layer(H, W, rng, text_spacing * 1.6, -over_ang + rng.uniform(-2, 2),
                            pitch=(40.0, 80.0))
        extra[7] = bleed
    for k in (5, 6, 7):
        if k in extra:
            cm[extra[k]] = k
    cm[under] = 2
    cm[over] = 1
    cm[over & under] = 3
    if layout in ("text5", "page8"):
        cm[~folio] = 4
    return cm


# ---------------------------------------------------------------------------
# spectra
# ---------------------------------------------------------------------------

def class_params(B: int, K: int, cov: str, rng: np.random.Generator):
    """Class mean spectra (K x B) and lower Cholesky factors (K x B x B)."""
    mu = rng.uniform(800.0, 3500.0, size=(K, B))
    chol = np.empty((K, B, B))
    if cov == "shared":
        S = 60.0 ** 2 * (0.7 * np.eye(B) + 0.3 * np.ones((B, B)))
        L = np.linalg.cholesky(S)
        chol[:] = L
    elif cov == "per_class":
        for k in range(K):
            G = rng.standard_normal((B, B))
            Q, R = np.linalg.qr(G)
            Q = Q * np.sign(np.diag(R))[None, :]
            ev = 10.0 ** rng.uniform(2.0, 4.0, size=B)
            S = (Q * ev[None, :]) @ Q.T
            S = 0.5 * (S + S.T)
            chol[k] = np.linalg.cholesky(S)
    else:
        raise ValueError(cov)
    return mu, chol


def _draw_pixels(rng, cls, mu, chol, B, out_dtype):
    out = np.empty((cls.size, B), dtype=np.float64)
    for k in np.unique(cls):
        sel = np.flatnonzero(cls == k)
        z = rng.standard_normal((sel.size, B))
        out[sel] = z @ chol[k].T + mu[k]
    if out_dtype == "u16":
        return np.clip(np.rint(out), 0, 4095).astype(np.uint16)
    return out.astype(np.float32)


def render_cube(class_map: np.ndarray, mu: np.ndarray, chol: np.ndarray,
                dtype: str, seed: int, chunk_rows: int = 64,
                threads: int = 8) -> np.ndarray:
    """Draw every pixel of the page from its class distribution.

    Row chunks use independent child streams of ``seed`` so the result does
    not depend on the thread count."""
    H, W = class_map.shape
    B = mu.shape[1]
    npd = np.uint16 if dtype == "u16" else np.float32
    cube = np.empty((H, W, B), dtype=npd)
    nch = (H + chunk_rows - 1) // chunk_rows
    seqs = np.random.SeedSequence([seed, 0xC0BE]).spawn(nch)

    def work(i):
        r0, r1 = i * chunk_rows, min(H, (i + 1) * chunk_rows)
        rng = np.random.default_rng(seqs[i])
        cls = class_map[r0:r1].reshape(-1)
        cube[r0:r1] = _draw_pixels(rng, cls, mu, chol, B, dtype).reshape(r1 - r0, W, B)

    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        list(ex.map(work, range(nch)))
    return cube


def sample_labels(class_map: np.ndarray, K: int, n_per_class: int,
                  rng: np.random.Generator, min_pool_factor: float = 2.0):
    """Label map with n_per_class training pixels per class, drawn without
    replacement from each class mask; -1 elsewhere."""
    flat = class_map.reshape(-1)
    labels = np.full(flat.size, -1, dtype=np.int8)
    for k in range(K):
        pool = np.flatnonzero(flat == k)
        if pool.size < min_pool_factor * n_per_class:
            raise ValueError(f"class {k} has {pool.size} pixels, fewer than "
                             f"{min_pool_factor} x {n_per_class}")
        pick = rng.choice(pool, size=n_per_class, replace=False)
        labels[pick] = k
    return labels.reshape(class_map.shape)


def border_map(class_map: np.ndarray, radius: int = 2) -> np.ndarray:
    """True where some pixel within Chebyshev distance ``radius`` has another
    class."""
    from scipy.ndimage import maximum_filter, minimum_filter
    size = 2 * radius + 1
    return maximum_filter(class_map, size=size) != minimum_filter(class_map, size=size)


def soft_weights(classes: np.ndarray, near_border: np.ndarray, K: int,
                 rng: np.random.Generator, alpha: float = 0.5) -> np.ndarray:
    """Per-pixel class weights: Dirichlet(alpha) near a boundary, one-hot
    inside (float32, N x K)."""
    N = classes.size
    w = np.zeros((N, K), dtype=np.float64)
    w[np.arange(N), classes.astype(np.int64)] = 1.0
    nb = np.flatnonzero(near_border)
    if nb.size:
        w[nb] = rng.dirichlet(np.full(K, alpha), size=nb.size)
    return w.astype(np.float32)


def _scaled(cfg: dict, scale: float):
    H = max(48, int(round(cfg["H"] * scale)))
    W = max(48, int(round(cfg["W"] * scale)))
    n = max(8, int(round(cfg["n_per_class"] * (H * W) / (cfg["H"] * cfg["W"]))))
    return H, W, n


def make_case(config: int, seed: Optional[int] = None, scale: float = 1.0,
              n_per_class: Optional[int] = None, render: bool = True,
              threads: int = 8) -> Case:
    """Synthetic page for one of the workload configurations.

    ``scale`` shrinks both page sides (the training-pixel count shrinks with
    the page area) so the same structure can be drawn at test sizes."""
    cfg = WORKLOADS[config]
    seed = cfg["seed"] if seed is None else seed
    H, W, n = _scaled(cfg, scale)
    if n_per_class is not None:
        n = n_per_class
    rng = np.random.default_rng([seed, 0x5EED])
    cm = make_class_map(H, W, cfg["layout"], rng, cfg["text_spacing"])
    mu, chol = class_params(cfg["B"], cfg["K"], cfg["cov"], rng)
    labels = sample_labels(cm, cfg["K"], n, rng)
    cube = render_cube(cm, mu, chol, cfg["dtype"], seed, threads=threads) if render else None
    return Case(config=config, workload=cfg["workload"], H=H, W=W, B=cfg["B"],
                K=cfg["K"], dtype=cfg["dtype"], cube=cube, labels=labels,
                class_map=cm, mu=mu, chol=chol,
                class_names=CLASS_NAMES[cfg["layout"]], n_per_class=n, seed=seed)


def make_soft_case(config: int = 4, seed: Optional[int] = None, scale: float = 1.0,
                   n_per_class: Optional[int] = None, case: Optional[Case] = None):
    """Training pixels X (N x B float32), soft weights (N x K float32) and
    their hard classes.

    Without ``case`` the page is not rendered: the training pixels are drawn
    directly from their class distributions, which gives the same joint law as
    rendering the page and gathering them.  With ``case`` the pixels are
    gathered from its rendered cube."""
    if case is None:
        case = make_case(config, seed=seed, scale=scale, n_per_class=n_per_class,
                         render=False)
    rng = np.random.default_rng([case.seed, 0x50F7])
    flat = case.labels.reshape(-1)
    idx = np.flatnonzero(flat >= 0)
    cls = flat[idx].astype(np.int64)
    if case.cube is not None:
        X = case.cube.reshape(-1, case.B)[idx].astype(np.float32)
    else:
        X = _draw_pixels(rng, cls, case.mu, case.chol, case.B, "f32")
    nb = border_map(case.class_map)[np.unravel_index(idx, case.labels.shape)]
    w = soft_weights(cls, nb, case.K, rng)
    return X, w, cls, idx, case


def to_half_cube(cube_u16: np.ndarray, kind: str):
    """The uint16 page scaled to [0, 1] and rounded to nearest-even bf16 or
    fp16 (returned as a CPU torch tensor, since numpy has no bf16)."""
    import torch
    x = torch.from_numpy(cube_u16.astype(np.float32) / np.float32(4095.0))
    if kind == "bf16":
        return x.to(torch.bfloat16)
    if kind == "f16":
        return x.to(torch.float16)
    raise ValueError(kind)
