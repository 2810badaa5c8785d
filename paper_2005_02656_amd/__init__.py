"""MI355X-native SPH time step (arXiv 2005.02656): Python binding of libsph.

The compute path lives in the HIP library ``libsph.so`` (see ``include/sph.h``);
this package only marshals arguments.  The library is loaded on first use and
its absence raises: there is no CPU fallback.
"""
from . import inputs  # noqa: F401  (seeded workloads; no method arithmetic)


def __getattr__(name):
    # the binding is imported lazily so that ``inputs`` stays usable without a build
    if name in ("sph", "lib"):
        from . import sph as _sph
        return _sph if name == "sph" else _sph.lib()
    raise AttributeError(name)
