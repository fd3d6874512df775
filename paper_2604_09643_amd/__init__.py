"""MI355X-native differentiable acoustic radiation (PA-SFM, arxiv 2604.09643).

The model and its adjoints run in the gfx950 HIP library ``libradiate.so`` behind
the C ABI of ``include/radiate.h``; ``paper_2604_09643_amd._lib`` is its ctypes
binding.  Importing this package does not load the library; the first call does,
and fails loudly if it has not been built.
"""

__all__ = ["Grid", "Sampling", "radiate_forward", "radiate_adjoint", "loss_and_grad",
           "pose_from_axis_angle", "pose_grad_axis_angle", "count_updates", "Context"]


def __getattr__(name):
    if name in __all__:
        from . import _lib
        return getattr(_lib, name)
    raise AttributeError(name)
