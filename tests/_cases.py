"""Shared synthetic cases for the GPU tests (built once per test session)."""
import functools

from synth import make_case


@functools.lru_cache(maxsize=1)
def full_page():
    """The 7216 x 5412 x 33 uint16 page with 8 classes (about 2.6 GB)."""
    return make_case(5, threads=16)
