"""MI355X (gfx950) NUFFT with the exponential-of-semicircle kernel.

The compute path is the HIP library ``libesnufft.so`` behind the C ABI in
``include/esnufft.h``; ``binding`` marshals arguments to it.  Submodules load
lazily so that ``inputs`` can be imported without the GPU library.
"""
__all__ = ["binding", "inputs"]
