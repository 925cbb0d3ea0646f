"""MI355X-native block-MPS Trotter evolution of the periodic 2D transverse-field
Ising model with fidelity-rescaled estimators (arXiv:2511.23438).

The compute path is the HIP library ``libmpsim.so`` (sources in ``csrc/``,
C-ABI in ``include/mpsim.h``); ``mpsim`` is its thin ctypes binding.
"""
__all__ = ["mpsim", "workloads"]
