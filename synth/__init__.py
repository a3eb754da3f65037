"""Seeded synthetic multispectral pages (inputs only).

This package draws the inputs that both the HIP path and the CPU oracle
consume: a band-interleaved cube, a per-pixel class map, a sparse label map
of analyst-chosen training pixels and, for the soft-label variant, per-pixel
class weights.  It holds none of the method's arithmetic (no moments, no
scatter matrices, no eigenproblems, no projection).
"""
from .cubes import (WORKLOADS, Case, make_case, make_class_map, class_params,
                    render_cube, sample_labels, soft_weights, border_map,
                    make_soft_case, to_half_cube)

__all__ = ["WORKLOADS", "Case", "make_case", "make_class_map", "class_params",
           "render_cube", "sample_labels", "soft_weights", "border_map",
           "make_soft_case", "to_half_cube"]
