"""MI355X (gfx950) search over an augmented neighborhood graph (arXiv 1312.3062).

The compute path is the HIP library libann.so behind the C ABI in
include/ann.h; this package only marshals arguments.  It raises on import
of the binding when the library has not been built.
"""
from . import synth  # noqa: F401  (seeded synthetic workloads; no method arithmetic)

__all__ = ["synth", "Index", "knn_device", "recall_at"]


def __getattr__(name):
    if name in ("Index", "knn_device", "recall_at", "search_params"):
        from . import index
        return getattr(index, name)
    raise AttributeError(name)
