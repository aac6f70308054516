"""expm-pfd for MI355X: exp(tA)V for Hermitian A by the partial-fraction form of
R_d(z) = 1/exp_d(-z) (Hecht, Kaber, Perrin, Plagne, Salomon, arXiv 2306.16778).

The compute path is the HIP library ``libexpm_pfd.so`` (C ABI, ``include/expm_pfd.h``).
``paper_2306_16778_amd.expm_pfd`` is its Python binding; it is imported lazily so
that modules without GPU work (``workloads``) import on any machine.
"""

__all__ = ["expm_pfd", "workloads"]


def __getattr__(name):
    if name == "expm_pfd":
        from . import expm_pfd as m
        return m
    raise AttributeError(name)
