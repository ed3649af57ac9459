"""Batched Lorentz-vector kernels for AMD Instinct MI355X (gfx950).

The data-parallel hot path of GenVectorX (arXiv 2312.02756): pair invariant
masses and Lorentz boosts over millions of independent items, a one-launch
per-event reduction over jagged events, and the reverse mode of each, as
hand-written HIP kernels behind the C ABI of include/glv.h.

``glv``       binding of every C entry point (same names), torch tensors in/out
``autograd``  torch.autograd.Function wrappers (invariant_mass, boost, event_reduce)
``build``     the hipcc build step
"""

from . import build  # noqa: F401


def __getattr__(name):
    # the binding loads libglv.so (and torch) lazily, on first use
    if name in ("glv", "autograd", "_lib"):
        import importlib
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
