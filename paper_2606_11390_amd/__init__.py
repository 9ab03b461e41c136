"""MI355X-native Gaussian-splatting hot path (gfx950, HIP).

One GPU's share of a Gaussian-splatting training step: per-Gaussian EWA
projection with spherical-harmonic colour, tile binning by a stable radix sort
on a (tile id | depth) key, front-to-back alpha compositing, an L2 image loss,
and the backward passes of all of them.  Every step runs in hand-written HIP
kernels behind the C ABI declared in ``include/gs.h``; this package only
marshals arguments (``binding``), wraps the differentiable calls in a
``torch.autograd.Function`` (``render``) and draws seeded synthetic inputs
(``scenes``).

Submodules are imported lazily so that ``scenes`` can be used without
loading the HIP library.
"""

__all__ = ["scenes", "binding", "render"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
