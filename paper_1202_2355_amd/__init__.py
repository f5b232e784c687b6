"""MI355X-native chi^2 made-to-measure (M2M) step with moving-prior
regularization (Morganti & Gerhard 2012).

The computation lives in the HIP library ``libm2m.so`` (C ABI in
``include/m2m.h``); this package is its Python binding:

* ``_abi``  -- ctypes declarations and the C-named wrappers,
* ``fit``   -- ``Fit``: one fit over device-resident particles,
* ``batch`` -- ``Batch``: many fits stepping in one launch,
* ``serve`` -- a continuous-batching server of fit requests,
* ``autotune`` -- launch-shape search for the fused step kernel,
* ``build`` -- in-tree hipcc build of the library.
"""

from .build import build  # noqa: F401

__all__ = ["build", "Fit", "Batch"]


def __getattr__(name):
    # import lazily so that building does not need torch or the library
    if name == "Fit":
        from .fit import Fit
        return Fit
    if name == "Batch":
        from .batch import Batch
        return Batch
    raise AttributeError(name)
