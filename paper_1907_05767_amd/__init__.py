"""EbV LU on MI355X (gfx950): no-pivot Doolittle LU + triangular solves for
diagonally dominant systems, after Hashemi, Lahooti and Shirani,
"Equal bi-Vectorized (EbV) method to high performance on GPU" (arXiv:1907.05767).

The compute path is the HIP library ``libebv.so`` behind the C ABI declared in
``include/ebv.h``; ``paper_1907_05767_amd.ebv`` binds it (argument marshalling
only).  Importing this package does not load the library; the binding loads it
on first use and raises if it is missing.
"""
import importlib

__all__ = ["ebv", "inputs"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
