"""MI355X (gfx950) implementation of the coupled guiding-center / Boris
particle pusher of Bacchini et al. (arXiv:2007.14401).

The compute path is libgcb.so (HIP kernels behind the C ABI of include/gcb.h);
`gcb` is its ctypes binding, `state` moves particle ensembles to and from
device tensors, and `autograd` wraps the push and its hand-written adjoint in
a torch.autograd.Function.  Importing the package loads libgcb.so and fails
if it has not been built.
"""
from . import gcb  # noqa: F401  (loads libgcb.so)
from .gcb import GcbError  # noqa: F401
