"""emrt: gfx950 (MI355X) dynamic EM ray tracer for large urban scenes.

Hot path (HIP, ``csrc/``) behind the C ABI of ``include/emrt.h``; this
package is the thin Python binding.  Importing it does not touch the GPU;
``Tracer`` loads ``libemrt.so`` and fails loudly when it is missing.
"""
from ._abi import LIB_PATH, load  # noqa: F401


def __getattr__(name):
    if name in ("Tracer", "Batch", "EmrtError"):
        from . import tracer

        return getattr(tracer, name)
    raise AttributeError(name)
