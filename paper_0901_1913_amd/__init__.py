"""MI355X (gfx950) implementation of the fast chi-squared period search.

The search itself runs in the HIP kernels of ``libfchi2.so`` behind the C ABI
declared in ``include/fchi2.h``; :mod:`paper_0901_1913_amd.fchi2` is the thin
Python binding and :mod:`paper_0901_1913_amd.synth` draws seeded inputs.
"""
from .fchi2 import (FChi2Error, Plan, fchi2_fn, lib, search)  # noqa: F401

__all__ = ["Plan", "search", "fchi2_fn", "lib", "FChi2Error"]
