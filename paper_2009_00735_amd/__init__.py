"""MI355X (gfx950) implementation of the real-space signature + orientation
indexing hot path of Kuehbach et al., arXiv 2009.00735.

The compute path lives in libaraullo.so (HIP kernels behind the C ABI of
include/araullo.h); `native` is its ctypes binding, `synth` the seeded input
generator, `refine` the torch.autograd wrapper of the structure-factor
adjoint.
"""
__all__ = ["native", "synth"]
