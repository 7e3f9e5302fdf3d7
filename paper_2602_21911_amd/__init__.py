"""GRPrec finite-volume hot path for MI355X (gfx950): HIP kernels behind a C ABI.

The compiled library ``libgrprec.so`` holds every step of the method; this
package only marshals arguments to it (``grprec``) and generates seeded inputs
(``inputs``).  Submodules are imported lazily so that ``inputs`` can be used
without loading the GPU library.
"""
__all__ = ["grprec", "inputs", "learn"]
