"""The allocation-free projection entry point (cva_project_noalloc) against
cva_project, through the C ABI, on two calls in a row (the second on a
smaller page), and both against the FP64 oracle.

Bar: the ranges of the two entry points equal bit for bit when they run the
same passes; every byte within one grey level of cva_project's and of the
oracle's; ranges within 1e-4 of b - a of the oracle's.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import make_case

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1612_06457_amd  # noqa: F401  (raises if the library is missing)
    return torch.device("cuda:0")


def _one(case, dev, n_comp):
    import torch

    import paper_1612_06457_amd as cx
    ref = oracle.cva_fit(case.cube, case.labels, case.K)
    W = np.ascontiguousarray(ref["W"][:, :n_comp])
    cube = torch.from_numpy(case.cube).to(dev)
    H, Wd, _ = case.cube.shape
    out_a = torch.full((n_comp, H, Wd), 7, dtype=torch.uint8, device=dev)
    out_b = torch.full((n_comp, H, Wd), 7, dtype=torch.uint8, device=dev)
    q_a, ab_a = cx.cva_project(cube, W, ref["mean"], out=out_a, return_range=True)
    q_b, ab_b = cx.cva_project_noalloc(cube, W, ref["mean"], out_b, return_range=True)
    torch.cuda.synchronize()
    q_a = q_a.cpu().numpy().astype(np.int32)
    q_b = q_b.cpu().numpy().astype(np.int32)
    q_ref, ab_ref = oracle.cva_project(case.cube, W, ref["mean"])
    span = ab_ref[:, 1] - ab_ref[:, 0]
    assert np.max(np.abs(ab_b - ab_ref) / span[:, None]) <= 1e-4
    assert np.array_equal(ab_a, ab_b)
    assert np.max(np.abs(q_b - q_a)) <= 1
    assert np.max(np.abs(q_b - q_ref.astype(np.int32))) <= 1
    frac = float(np.mean(q_b != q_a))
    say(f"  {H}x{Wd}x{case.cube.shape[2]} n_comp={n_comp}: bytes differing from cva_project {frac:.2e}")
    return q_b


def test_noalloc_matches_cva_project_twice_second_smaller(dev):
    say("cva_project_noalloc: 1024x1024x16 u16 (3 classes), then 512x512x16 with 1 component")
    big = make_case(1, scale=2.0)
    small = make_case(1)
    _one(big, dev, 2)
    _one(small, dev, 1)


def test_noalloc_float_page(dev):
    say("cva_project_noalloc: float32 page (vector-ALU passes)")
    c = make_case(1, scale=0.5)
    c.cube = c.cube.astype(np.float32)
    _one(c, dev, 2)
