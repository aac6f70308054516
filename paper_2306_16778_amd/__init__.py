"""expm-pfd for MI355X: exp(tA)V for Hermitian A by the partial-fraction form of
R_d(z) = 1/exp_d(-z) (Hecht, Kaber, Perrin, Plagne, Salomon, arXiv 2306.16778).

The compute path is the HIP library ``libexpm_pfd.so`` (C ABI, ``include/expm_pfd.h``).
``paper_2306_16778_amd.expm_pfd`` is its Python binding; it is imported on first
use so that modules without GPU work (``workloads``) import on any machine.
"""

import importlib

__all__ = ["expm_pfd", "workloads", "serving"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
