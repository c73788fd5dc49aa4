"""MI355X (gfx950) library for the non-LTE line radiative-transfer hot path of
De Ceuster et al. (Magritte I): ray walk, ray-pair Feautrier formal solve, J / L* /
Jeff accumulation and statistical equilibrium inside an accelerated Lambda iteration.

The compute path is the HIP library libnlte.so (C ABI in include/nlte.h); the Python
binding in ``binding`` only marshals arguments.
"""
__all__ = ["binding", "build"]


def Solver(device: int = 0):
    from .binding import Solver as _S
    return _S(device)
