"""MI355X-native D3Q19 lattice Boltzmann step for VANSE with Carreau-Yasuda
rheology (arXiv:2402.10809): HIP kernels behind the C ABI of include/lbm.h.

``lbm`` is the ctypes binding (``Solver`` and the ABI's functions);
``autograd`` wraps the adjoint as a ``torch.autograd.Function``
(``sac_kinetic_energy``).  The shared library is loaded on first use; a
missing build raises ImportError naming the build step.
"""

from .lbm import Solver, LBMError, lib  # noqa: F401
