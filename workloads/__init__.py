"""Seeded synthetic inputs for trajectory-parallel Krotov optimisation.

This package only *builds inputs*: the Hamiltonian pieces H0, H_ctrl[i] and the
Lindblad operators L_l of a cascaded quantum network (as sparse matrices), the
initial and target states, and the guess pulses.  It holds none of the method's
arithmetic (no effective Hamiltonian, propagation, jumps or pulse updates), so
both the CPU oracle and the GPU library can consume the same inputs without
sharing any computation.
"""

from .cascade import (  # noqa: F401
    CascadeSpec,
    Workload,
    build_cascade,
    build_paper_model,
    guess_pulses,
    config_workload,
    batch_instances,
    CONFIGS,
)
