"""MI355X (gfx950) scattering-state solver of the IOBM transport method with
FFT-applied jellium self-energies and preconditioned COCG (arXiv:1009.5300).

The compute path is the HIP library libiobm.so (C ABI in include/iobm.h);
`paper_1009_5300_amd.iobm` is its ctypes binding and
`paper_1009_5300_amd.autograd` the torch.autograd wrapper of the adjoint
gradient.  Importing the binding fails if the library is not built.
"""
__all__ = ["iobm"]
