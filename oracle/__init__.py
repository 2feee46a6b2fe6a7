"""FP64 CPU oracle for trajectory-parallel Krotov optimisation.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
restatement of what the paper computes (Goerz & Jacobs, "Efficient
optimization of state preparation in quantum networks using quantum
trajectories"): the Monte-Carlo wave-function (quantum jump) algorithm of
Sec. 2.1, the trajectory functional and independent-trajectory Krotov update of
Sec. 2.3, and the Lindblad master equation of Sec. 2.1 used to check the
trajectory ensemble.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product library never does, and it
shares no code, table or helper with the GPU path.

Everything is complex128 and uses dense matrices: exact step propagators come
from ``scipy.linalg.expm``; jump times come from plain bisection on the exact
propagator.  Random numbers come from a Philox4x64-10 generator written here
from its published definition (Salmon et al., SC'11).

Modules:
  philox   -- the counter-based generator and the stream layout
  mcwf     -- effective Hamiltonian, exact step propagators, MCWF passes
  krotov   -- trajectory functional, costates, sequential Krotov update
  lindblad -- dense density-matrix propagation (ensemble check)
  gradient -- pathwise dJ_T/du with the jump record fixed: replay, adjoint
              sweep with Van Loan's block exponential, finite differences
"""
