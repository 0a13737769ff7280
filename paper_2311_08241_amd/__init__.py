"""MI355X-native split-explicit barotropic subcycle (arXiv 2311.08241).

The compute path is the HIP library libsesub.so (gfx950) behind the C ABI of
include/sesub.h; this package marshals arguments to it.  Importing the
package does not load the library; the first call does, and fails with
ImportError if it has not been built.
"""
from .api import Batch, Mesh, Params, batch_inputs, device_inputs  # noqa: F401


def subcycle_autograd(*args, **kw):
    """Differentiable subcycle (see autograd.subcycle)."""
    from .autograd import subcycle
    return subcycle(*args, **kw)
