"""Benchmark of the CVA / PCA page-enhancement hot path on one MI355X.

Workload: a synthetic 7216 x 5412 x 33-band uint16 page (2.58 GB, resident
in HBM before timing), 8 classes with 200,000 training pixels each.  One
step is one pass of the whole hot path over that page:

  CVA fit + project in one library call (labels -> counts, class moments,
  S_w, S_b, FP64 eigensolve; 7 canonical variates, min-max stretch to 8 bits)
  PCA fit (whole-page covariance) and PCA project (3 components)
  soft-label CVA forward + backward on the 1.6M training pixels

The headline value is CVA fit + project throughput in Gpix*band/s
(page pixels x bands / t_fit+project); ms_per_step is the whole step.
`vs_plain_fp32` times the same calls on the plain FP32 vector-ALU kernels
and with the bf16x3 split, beside the default path.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0



# The sources the stretch kernel is compiled from: a recorded traffic figure
# holds only while all of them are unchanged.
STRETCH_SOURCES = ("k_project_u16.hip", "k_tile.hpp", "k_common.hpp")


def stretch_source_digest() -> str:
    import hashlib
    h = hashlib.sha1()
    for name in STRETCH_SOURCES:
        with open(os.path.join(ROOT, "paper_1612_06457_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()

def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case, min_seconds: float = 10.0):
    """The FP64 oracle, as it stands, on the whole page: CVA fit on all its
    training pixels, then projection + min-max stretch of every pixel,
    repeated until at least `min_seconds` of CPU work; then one page on a
    single thread.  Returns (Gpix*band/s, seconds per page, threads, sample,
    single-thread seconds per page)."""
    import oracle

    def one_page():
        fit = oracle.cva_fit(case.cube, case.labels, case.K)
        oracle.cva_project(case.cube, fit["W"], fit["mean"])

    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count() or 1
    reps, t0 = 0, time.perf_counter()
    while True:
        one_page()
        reps += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds or reps >= 10:
            break
    per = dt / reps
    per1 = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            one_page()
            per1 = time.perf_counter() - t1
    pixbands = case.H * case.W * case.B
    sample = (f"whole {case.H}x{case.W}x{case.B} page, {reps} repetition(s) of CVA fit on "
              f"{int((case.labels >= 0).sum())} training pixels + projection + stretch of every pixel, "
              f"on {_cpu_model()}")
    return pixbands / per / 1e9, per, threads, sample, per1


def fit_last(cx, cube, labels, K):
    return cx.cva_fit(cube, labels, K)


def _timed(torch, fn, reps=5):
    """Median milliseconds of fn() over reps runs, HIP events on torch's
    current stream (the one the library launches on)."""
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def vs_plain(cx, torch, cube, labels, K, img, pimg, fit_proj_bytes, per, mean_fp, P, B):
    """The headline call and the PCA calls on the plain FP32 reference path
    (the FP32 vector-ALU kernels for the class moments, the covariance and
    the projections), and the headline call with the bf16x3 split asked
    for, beside the default path; all three meet the same FP32 tolerances
    against the oracle (the GPU tests check each).  The soft-label passes
    have one path, FP32 products on the FP32 matrix instruction."""
    reps = 10
    t_mixed = _timed(torch, lambda: cx.cva_fit_project(cube, labels, K, precision="bf16x3", out=img), reps)
    cx.set_plain_fp32(True)
    try:
        t_plain = _timed(torch, lambda: cx.cva_fit_project(cube, labels, K, precision="fp32", out=img), reps)
        V, _, mean, _ = cx.pca_fit(cube, n_comp=3)
        t_pfit = _timed(torch, lambda: cx.pca_fit(cube, n_comp=3))
        t_pproj = _timed(torch, lambda: cx.pca_project(cube, V, mean, out=pimg))
    finally:
        cx.set_plain_fp32(False)

    def rate(ms):
        return {"ms": round(ms, 4), "Gpix_band_per_s": round(P * B / (ms * 1e-3) / 1e9, 1),
                "frac_of_8TBps": round(fit_proj_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    return {
        "cva_fit_project": {"default": rate(mean_fp), "plain_fp32": rate(t_plain), "bf16x3": rate(t_mixed),
                            "speedup_default_vs_plain": round(t_plain / mean_fp, 3),
                            "speedup_bf16x3_vs_plain": round(t_plain / t_mixed, 3)},
        "pca_fit": {"default_ms": round(per["pca_fit"], 4), "plain_fp32_ms": round(t_pfit, 4),
                    "speedup": round(t_pfit / per["pca_fit"], 3)},
        "pca_project": {"default_ms": round(per["pca_project"], 4), "plain_fp32_ms": round(t_pproj, 4),
                        "speedup": round(t_pproj / per["pca_project"], 3)},
        "soft_fwd_bwd_ms": round(per["soft_fwd"] + per["soft_bwd"], 4),
    }


def copy_bandwidth(torch, gib: int = 1) -> float:
    """GB/s of a plain device-to-device copy (bytes read + bytes written
    over the median time of 5), the measured roof beside the nominal one."""
    src = torch.ones(gib << 30, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    ms = _timed(torch, lambda: dst.copy_(src))
    del src, dst
    return 2 * (gib << 30) / (ms * 1e-3) / 1e9


def mixed_half_pages(cx, torch, dev):
    """The 4096 x 4096 x 23 page (4 classes, 200,000 training pixels) as bf16
    and as fp16 values: CVA fit + project and PCA fit with the FP32 request
    (vector-ALU moments; exact split projection on the matrix cores), with
    the bf16x3 / f16x3 split (moments on the matrix cores too) and on the
    plain FP32 path; every variant meets the FP32 tolerances against the
    oracle (GPU tests)."""
    from synth import make_case, to_half_cube
    c = make_case(3, threads=16)
    P, B, K = c.H * c.W, c.B, c.K
    labels = torch.from_numpy(c.labels).to(dev)
    img = torch.empty((K - 1, c.H, c.W), dtype=torch.uint8, device=dev)
    nbytes = 2 * P * B * 2 + P * (K - 1) + c.labels.size + int((c.labels >= 0).sum()) * B * 2
    res = {"workload": c.workload, "algorithmic_MB": round(nbytes / 1e6, 1)}
    for kind, split in (("bf16", "bf16x3"), ("f16", "f16x3")):
        cube = to_half_cube(c.cube, kind).to(dev)
        r = {}
        for name, prec, plain in (("fp32", "fp32", False), (split, split, False), ("plain_fp32", "fp32", True)):
            cx.set_plain_fp32(plain)
            try:
                t = _timed(torch, lambda: cx.cva_fit_project(cube, labels, K, precision=prec, out=img))
                tp = _timed(torch, lambda: cx.pca_fit(cube, n_comp=3, precision=prec))
            finally:
                cx.set_plain_fp32(False)
            r[name] = {"cva_fit_project_ms": round(t, 4), "Gpix_band_per_s": round(P * B / (t * 1e-3) / 1e9, 1),
                       "frac_of_8TBps": round(nbytes / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "pca_fit_ms": round(tp, 4)}
        r["speedup_vs_plain"] = {k: round(r["plain_fp32"]["cva_fit_project_ms"] / r[k]["cva_fit_project_ms"], 3)
                                 for k in ("fp32", split)}
        r["pca_speedup_vs_plain"] = {k: round(r["plain_fp32"]["pca_fit_ms"] / r[k]["pca_fit_ms"], 3)
                                     for k in ("fp32", split)}
        res[kind] = r
        del cube
    return res


def extras(cx, torch, case, cube, fit, dev, labels=None):
    """Timings of the calls beyond the headline path on the same page:
    float images, the three rescaling modes, 16-bit output, the RGB
    composite, the cluster indices, the band-sequential import and the
    many-page pipeline (host-resident pages, so its rate includes PCIe)."""
    H, W, B, K = case.H, case.W, case.B, case.K
    P, C = H * W, K - 1
    res = {}

    def rec(name, ms, nbytes):
        res[name] = {"ms": round(ms, 4), "algorithmic_MB": round(nbytes / 1e6, 1),
                     "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1)}

    # the two halves of the headline call, each on its own
    if labels is not None:
        res["cva_fit_alone_ms"] = round(_timed(torch, lambda: cx.cva_fit(cube, labels, K)), 4)
        img = torch.empty((C, H, W), dtype=torch.uint8, device=dev)
        res["cva_project_alone_ms"] = round(_timed(torch, lambda: cx.cva_project(cube, fit.W, fit.mean, out=img)), 4)
    y = torch.empty((C, H, W), dtype=torch.float32, device=dev)
    rec("project_float", _timed(torch, lambda: cx.project_float(cube, fit.W, fit.mean, out=y)),
        P * B * 2 + P * C * 4)
    q8 = torch.empty((C, H, W), dtype=torch.uint8, device=dev)
    q16 = torch.empty((C, H, W), dtype=torch.uint16, device=dev)
    rec("stretch_minmax_8bit", _timed(torch, lambda: cx.stretch(y, "minmax", out=q8)), 2 * P * C * 4 + P * C)
    flat = case.labels.reshape(-1)
    train = torch.from_numpy(np.flatnonzero(flat >= 0).astype(np.int64)).to(dev)
    rec("stretch_training_8bit", _timed(torch, lambda: cx.stretch(y, "training", train_pixels=train, out=q8)),
        P * C * 4 + P * C + train.numel() * (8 + 4 * C))
    # three radix passes read every value once each, then the stretch pass
    rec("stretch_percentile_16bit", _timed(torch, lambda: cx.stretch(y, "percentile", pct=1.0, bits=16, out=q16)),
        4 * P * C * 4 + P * C * 2)
    rec("compose_rgb", _timed(torch, lambda: cx.compose_rgb(q8[0], q8[1], q8[2])), 6 * P)
    cls = torch.from_numpy(flat[flat >= 0].astype(np.int8)).to(dev)
    rec("cluster_indices_7x8bit", _timed(torch, lambda: cx.cluster_indices(q8, train, cls, K)),
        train.numel() * (8 + 1 + 2 * C))
    bands8 = torch.from_numpy(np.ascontiguousarray(np.moveaxis((case.cube >> 4).astype(np.uint8), -1, 0)))
    b8 = bands8.to(dev)
    page = torch.empty((H, W, B), dtype=torch.uint16, device=dev)
    rec("bands_to_cube_8bit", _timed(torch, lambda: cx.bands_to_cube(b8, out=page)), P * B * 3)
    del b8, page, y, q16
    # many pages: three host-resident 8-bit pages, batched (copies overlapped)
    # against one call per page
    pinned = bands8.pin_memory()
    del bands8
    pix = torch.from_numpy(np.flatnonzero(flat >= 0).astype(np.int64))
    pcls = torch.from_numpy(flat[flat >= 0].astype(np.int8))
    pages = [{"bands": pinned, "pixels": pix, "classes": pcls} for _ in range(3)]
    cx.run_pages(pages[:1], K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outp = cx.run_pages(pages, K)
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    for pg in pages:
        cx.run_pages([pg], K)
    t_single = time.perf_counter() - t0
    assert all(o["status"] == 0 for o in outp)
    res["run_pages_3x8bit"] = {
        "batched_ms_per_page": round(t_batch * 1e3 / 3, 2),
        "one_call_per_page_ms": round(t_single * 1e3 / 3, 2),
        "pcie_inclusive_Gpix_band_per_s": round(P * B / (t_batch / 3) / 1e9, 2),
        "host_to_device_MB_per_page": round(P * B / 1e6, 1),
        "device_to_host_MB_per_page": round(P * C / 1e6, 1)}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3", "f16x3"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the timings of the rescaling, colour, assessment and many-page calls "
                         "and of the plain FP32 path")
    ap.add_argument("--copy-gib", type=int, default=0,
                    help="after the timed steps, copy this many GiB device to device (a plain copy of "
                         "known size, to calibrate hardware byte counters against)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path has no multi-GPU "
              "launch: pages are independent, so several GPUs run several pages.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1612_06457_amd as cx
    from synth import make_case, soft_weights, border_map

    dev = torch.device("cuda:0")
    t0 = time.time()
    case = make_case(5, threads=16)
    log(f"page generated in {time.time() - t0:.1f}s: {case.H}x{case.W}x{case.B} u16, K={case.K}")
    H, W, B, K = case.H, case.W, case.B, case.K
    P = H * W
    cube = torch.from_numpy(case.cube).to(dev)
    labels = torch.from_numpy(case.labels).to(dev)
    # soft-label inputs: the training pixels, gathered once (outside the timed region)
    flat = case.labels.reshape(-1)
    idx = np.flatnonzero(flat >= 0)
    cls = flat[idx].astype(np.int64)
    rng = np.random.default_rng([case.seed, 0x50F7])
    nb = border_map(case.class_map)[np.unravel_index(idx, case.labels.shape)]
    wts = soft_weights(cls, nb, K, rng)
    X = torch.from_numpy(case.cube.reshape(-1, B)[idx].astype(np.float32)).to(dev)
    w = torch.from_numpy(wts).to(dev)
    N = X.shape[0]
    C = K - 1
    img = torch.empty((C, H, W), dtype=torch.uint8, device=dev)
    pimg = torch.empty((3, H, W), dtype=torch.uint8, device=dev)
    dw = torch.empty((N, K), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    phases = ["cva_fit_project", "pca_fit", "pca_project", "soft_fwd", "soft_bwd"]

    def step(ev=None):
        def mark(i):
            if ev is not None:
                ev[i].record()
        mark(0)
        _, fit = cx.cva_fit_project(cube, labels, K, precision=args.precision, out=img)
        mark(1)
        V, lam, mean, _ = cx.pca_fit(cube, n_comp=3, precision=args.precision)
        mark(2)
        cx.pca_project(cube, V, mean, out=pimg)
        mark(3)
        sf = cx.cva_soft_forward(X, w, precision="fp32")
        mark(4)
        cx.cva_soft_backward(X, sf, 1.0, K, out=dw)
        mark(5)
        return fit

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: HIP event pairs around the page-streaming projection
    # passes only (the roofline's kernel), none around the fit's short
    # kernels, whose per-launch times come from the untimed steps below
    cx.profile_enable("projection")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(phases) + 1)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = cx.profile_report()
    cx.profile_enable(True)
    for _ in range(3):
        step()
    torch.cuda.synchronize()
    prof_all = cx.profile_report()
    cx.profile_enable(False)
    prof_all.update(prof)

    ms_step = (t1 - t0) * 1e3 / args.steps
    per = {p: float(np.median([evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(args.steps)]))
           for i, p in enumerate(phases)}
    fp = [evs[k][0].elapsed_time(evs[k][1]) for k in range(args.steps)]
    mean_fp = float(np.mean(fp))
    median_fp = float(np.median(fp))
    value = P * B / (mean_fp * 1e-3) / 1e9

    # roofline of the dominant kernel (the projection pass that writes the
    # images): algorithmic bytes = page read once + the planar bytes written
    cube_bytes = P * B * 2
    n_str, ms_str = prof.get(f"project_stretch_nc{C}", (0, 0.0))
    n_rng, ms_rng = prof.get(f"project_range_nc{C}", (0, 0.0))
    # per launch of the CVA stretch pass: the page read once + C planes written
    str_bytes = cube_bytes + P * C
    avg_str = ms_str / max(n_str, 1)
    achieved = str_bytes / (avg_str * 1e-3) / 1e9
    avg_rng = ms_rng / max(n_rng, 1)
    fit_proj_bytes = 2 * cube_bytes + P * C + (labels.numel() + N * B * 2)
    roof = {
        "kernel": f"k_stretch_u16 (CVA stretch pass, {C} components)",
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": None,
        "avg_launch_ms": round(avg_str, 4),
        "range_pass": {"avg_launch_ms": round(avg_rng, 4),
                       "achieved_GBps": round(cube_bytes / (avg_rng * 1e-3) / 1e9, 1)},
        "fit_plus_project": {"algorithmic_MB": round(fit_proj_bytes / 1e6, 1),
                             "ms": round(mean_fp, 4), "median_ms": round(median_fp, 4),
                             "frac_of_8TBps": round(fit_proj_bytes / (mean_fp * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
    }
    traffic_file = os.path.join(ROOT, "profiles", "traffic_project_stretch.json")
    if os.path.exists(traffic_file):
        try:
            tr = json.load(open(traffic_file))
            if tr.get("source_sha1") == stretch_source_digest():
                roof["traffic"] = tr.get("bytes_per_launch")
        except Exception:
            pass

    out = {
        "metric": "CVA fit+project Gpix*band/s (7216x5412x33 u16 page, K=8)",
        "value": round(value, 2),
        "unit": "Gpix*band/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "cva_pca_page_7216x5412x33_u16_k8", "H": H, "W": W, "B": B, "K": K,
                   "train_pixels": int(N), "cva_components": C, "pca_components": 3,
                   "precision": args.precision,
                   "arithmetic": "u16 page; exact fp16 split products on the matrix cores (projection, class "
                                 "scatter) with FP32 accumulation, exact int8 digit products (PCA covariance), "
                                 "FP64 combine and eigensolve"},
        "phases_ms": {k: round(v, 4) for k, v in per.items()},
        "soft_fwd_bwd_ms": round(per["soft_fwd"] + per["soft_bwd"], 4),
        "kernels_ms_per_launch": {k: round(v[1] / max(v[0], 1), 4) for k, v in sorted(prof_all.items())},
        "roofline": roof,
    }
    copy_gbs = copy_bandwidth(torch)
    roof["measured_copy_GBps"] = round(copy_gbs, 1)
    roof["frac_of_measured_copy"] = round(achieved / copy_gbs, 4)
    roof["fit_plus_project"]["frac_of_measured_copy"] = round(fit_proj_bytes / (mean_fp * 1e-3) / 1e9 / copy_gbs, 4)
    if not args.no_extras:
        out["vs_plain_fp32"] = vs_plain(cx, torch, cube, labels, K, img, pimg, fit_proj_bytes, per, mean_fp, P, B)
        out["vs_plain_fp32"]["half_pages"] = mixed_half_pages(cx, torch, dev)
    if not args.no_extras:
        out["extras"] = extras(cx, torch, case, cube, fit_last(cx, cube, labels, K), dev, labels)
    if args.copy_gib > 0:
        src = torch.ones(args.copy_gib << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu:
        gbs, dt, threads, sample, dt1 = cpu_baseline(case, args.cpu_seconds)
        out["cpu_baseline"] = {"value": round(gbs, 4), "unit": "Gpix*band/s", "cores": threads,
                               "kind": "oracle", "sample": sample, "seconds_per_page": round(dt, 2)}
        if dt1 is not None:
            out["cpu_baseline"]["single_thread_seconds_per_page"] = round(dt1, 2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
