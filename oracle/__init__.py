"""Plain, slow CPU reference ("oracle") for the block-MPS Trotter evolution of
the periodic 2D transverse-field Ising model (arXiv:2511.23438).

This package is TEST INFRASTRUCTURE. Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the product path (the HIP
library and its Python binding) never does. It shares no code with the HIP
path: its lattice geometry, gate tables, schedule, truncation and measurement
are all written here, in float64 / complex128 numpy, each function citing the
passage of the paper it follows.

Modules
-------
lattice      grid, blocks (half rows), snake order, ZZ bonds, gate tables
schedule     the step schedule (which block pairs are updated, in which order)
mps          block MPS with two-site updates, SVD truncation, fidelity, measurement
statevector  exact Trotterised state-vector evolution for at most 20 qubits
estimators   fidelity-rescaled estimators and the gamma_fit table

Parity status: every function here is pinned by a CPU test against closed
forms, an independent dense-Hamiltonian construction, or exact state-vector
evolution (see the test docstrings), except where a docstring says
"parity unpinned".
"""
