"""MI355X (gfx950) hot path of the randomised primal-dual RI imaging solver.

The arithmetic lives in libri.so (HIP kernels behind the C ABI of include/ri.h); this
package is its Python binding.  Importing the package loads nothing; the first use of
an operator loads the library and fails loudly if it has not been built.
"""
__version__ = "1.0.0"

__all__ = ["Plan", "Sara", "PD", "probabilities", "residual_energy"]


def __getattr__(name):
    if name in __all__:
        from . import ops

        return getattr(ops, name)
    raise AttributeError(name)
