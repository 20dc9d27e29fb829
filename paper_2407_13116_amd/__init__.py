"""MI355X (gfx950) implementation of the enhanced Kogbetliantz SVD of order two
(V. Novakovic, arXiv 2407.13116), batched, with its adjoint and a batched
two-sided Kogbetliantz sweep.

The compute lives in libksvd2.so (hand-written HIP, C ABI in include/ksvd2.h);
this package is the thin Python binding.  Build with
``python -m paper_2407_13116_amd.build``.
"""
import importlib

from ._lib import KSVD2Error, LIB_PATH  # noqa: F401

_SUBMODULES = ("api", "sweep", "inputs", "build", "autotune")


def __getattr__(name):
    # submodules and the torch-facing API load lazily, so that `inputs` and
    # `build` work without initialising torch
    if name in _SUBMODULES:
        return importlib.import_module("." + name, __name__)
    api = importlib.import_module(".api", __name__)
    if hasattr(api, name):
        return getattr(api, name)
    sweep = importlib.import_module(".sweep", __name__)
    if hasattr(sweep, name):
        return getattr(sweep, name)
    raise AttributeError(name)
