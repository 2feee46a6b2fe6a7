"""Monte-Carlo wave-function (quantum jump) trajectories, FP64 reference.

Follows the MCWF algorithm of Sec. 2.1 of the paper, steps 1 to 6, with
precise jump times inside a time step (Sec. 2.1, the paragraph after the
algorithm: jump times located inside a step by bisection, several jumps per
step allowed).

Readings of the paper taken here (each also listed in the design notes):

* Step 1 prints H_eff = H + sum_l L_l^+ L_l; the anti-Hermitian factor is
  missing.  We use H_eff = H - (i/2) sum_l L_l^+ L_l, the standard quantum-jump
  effective Hamiltonian; only this form makes the norm of a single decaying
  cavity fall as exp(-kappa t).
* Step 4 prints p(L_l) = <Psi|L_l^+ L_l|Psi> without normalisation; we use
  p_l = ||L_l Psi||^2 / sum_l' ||L_l' Psi||^2 and pick the smallest l whose
  cumulative weight exceeds x * total for the stream's variate x.
* Step 3 ("propagate until ||Psi||^2 = r"): the unnormalised state is the
  clock.  A jump happens inside a step when the norm at the end of the step
  is strictly below r; the jump time tau* is the crossing of the (monotonically
  non-increasing) norm, found by bisection on the exact sub-step propagator
  until the bracket cannot shrink further, taking the upper end.
* Step 6: every *use* of the state normalises it; the propagated state stays
  unnormalised between jumps.
* Backward (costate) trajectories run the same algorithm in reverse time with
  the adjoint propagator exp(+i H_eff^+ tau), the same jump operators and an
  independent random stream (direction 1).

Pulses are piecewise constant: u_ij is the value of control i on the interval
(t_{j-1}, t_j] (Sec. 2.2); here j is 0-based, interval j = (j dt, (j+1) dt].
"""

from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence

import numpy as np
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg

from .philox import TrajectoryStream


def dense(m) -> np.ndarray:
    return np.asarray(m.toarray() if hasattr(m, "toarray") else m, dtype=np.complex128)


@dataclasses.dataclass
class System:
    """Dense copy of the problem statement of Sec. 2.1: H = H0 + sum_i u_i H_i, {L_l}."""

    H0: np.ndarray
    H_ctrl: List[np.ndarray]
    L_jump: List[np.ndarray]

    @classmethod
    def from_sparse(cls, H0, H_ctrl, L_jump) -> "System":
        return cls(dense(H0), [dense(h) for h in H_ctrl], [dense(L) for L in L_jump])

    @property
    def dim(self) -> int:
        return self.H0.shape[0]

    def effective_hamiltonian(self, u_j: Sequence[float]) -> np.ndarray:
        """MCWF step 1: H_eff = H0 + sum_i u_i H_i - (i/2) sum_l L_l^+ L_l."""
        H = self.H0.copy()
        for ui, Hi in zip(u_j, self.H_ctrl):
            H = H + ui * Hi
        for L in self.L_jump:
            H = H - 0.5j * (L.conj().T @ L)
        return H


def propagator(H_eff: np.ndarray, tau: float, direction: int) -> np.ndarray:
    """Exact step propagator: exp(-i H_eff tau) forward, exp(+i H_eff^+ tau) backward."""
    if direction == 0:
        return scipy.linalg.expm(-1j * tau * H_eff)
    return scipy.linalg.expm(1j * tau * H_eff.conj().T)


# Above this dimension the propagator is never formed: its action on states
# comes from scipy's expm_multiply (Al-Mohy & Higham's truncated Taylor series
# with norm-based scaling), which is the same exp(-i H_eff tau) applied to a
# vector without the d x d matrix.
DENSE_MAX_DIM = 256


def step_operator(H_eff: np.ndarray):
    """H_eff as the propagator routines take it: dense up to DENSE_MAX_DIM, else sparse."""
    if H_eff.shape[0] <= DENSE_MAX_DIM:
        return H_eff
    return scipy.sparse.csr_matrix(H_eff)


def apply_propagator(H_op, tau: float, direction: int, psi: np.ndarray) -> np.ndarray:
    """U(tau) psi: exp(-i H_eff tau) psi forward, exp(+i H_eff^+ tau) psi backward."""
    if not scipy.sparse.issparse(H_op):
        return propagator(H_op, tau, direction) @ psi
    A = -1j * tau * H_op if direction == 0 else 1j * tau * H_op.conj().T.tocsr()
    return scipy.sparse.linalg.expm_multiply(A, psi)


def norm2(psi: np.ndarray) -> float:
    return float(np.vdot(psi, psi).real)


@dataclasses.dataclass(frozen=True)
class Jump:
    """One quantum jump: trajectory, 0-based step, operator, ordinal, direction, time.

    ``rate`` is a diagnostic beside the record: the relative rate at which the
    norm falls at the crossing, sum_l ||L_l psi||^2 / ||psi||^2.  A relative
    error e in the propagated state moves the crossing by about e / rate, so
    comparisons of jump times use it to scale their bar.
    """

    traj: int
    step: int
    op: int
    ordinal: int
    direction: int
    t: float
    rate: float = float("nan")


def jump_time(H_eff, psi: np.ndarray, tau_rem: float, r: float, direction: int) -> float:
    """First tau in (0, tau_rem] with ||U(tau) psi||^2 < r, by bisection.

    The norm is non-increasing in tau (d/dtau ||psi||^2 = -sum_l ||L_l psi||^2),
    so bisection on [lo, hi] with ||U(lo) psi||^2 >= r > ||U(hi) psi||^2
    converges to the crossing; we halve until the midpoint equals an end point
    and return the upper end.
    """
    lo, hi = 0.0, tau_rem
    while True:
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            return hi
        if norm2(apply_propagator(H_eff, mid, direction, psi)) < r:
            hi = mid
        else:
            lo = mid


def choose_operator(psi: np.ndarray, L_jump: List[np.ndarray], x: float) -> int:
    """MCWF step 4: pick l with probability ||L_l psi||^2 / sum_l' ||L_l' psi||^2."""
    weights = [norm2(L @ psi) for L in L_jump]
    total = sum(weights)
    if not total > 0.0:
        raise FloatingPointError("all jump operators annihilate the state")
    target = x * total
    acc = 0.0
    for l, w in enumerate(weights):
        acc += w
        if target < acc:
            return l
    return len(weights) - 1


class Ensemble:
    """M trajectories advanced through piecewise-constant steps by the MCWF rules."""

    def __init__(self, system: System, psi_start: np.ndarray, M: int, seed: int,
                 iteration: int, direction: int, instance: int = 0):
        self.sys = system
        d = system.dim
        psi_start = np.asarray(psi_start, dtype=np.complex128)
        if psi_start.ndim == 1:
            psi_start = np.broadcast_to(psi_start, (M, d))
        self.psi = np.array(psi_start, dtype=np.complex128)  # [M, d], unnormalised
        self.M = M
        self.direction = direction
        self.streams = [TrajectoryStream(seed, k, iteration, direction, instance)
                        for k in range(M)]
        self.ordinal = np.zeros(M, dtype=np.int64)
        self.r = np.array([s.threshold(0) for s in self.streams])
        self.records: List[Jump] = []

    def normalised(self) -> np.ndarray:
        """MCWF step 6: the normalised states Psi / ||Psi|| (rows)."""
        n = np.sqrt(np.einsum("kd,kd->k", self.psi.conj(), self.psi).real)
        return self.psi / n[:, None]

    def advance(self, step: int, u_j: Sequence[float], dt: float, t_start: float) -> None:
        """Advance every trajectory across one time step of length dt.

        ``t_start`` is the time at which the step begins in the direction of
        propagation (t_{j-1} forward, t_j backward); recorded jump times are
        t_start + elapsed forward and t_start - elapsed backward.
        """
        H_eff = step_operator(self.sys.effective_hamiltonian(u_j))
        dense = not scipy.sparse.issparse(H_eff)
        U = propagator(H_eff, dt, self.direction) if dense else None
        sign = 1.0 if self.direction == 0 else -1.0
        for k in range(self.M):
            psi = self.psi[k]
            tau_rem = dt
            U_rem = U
            while True:
                phi = U_rem @ psi if dense else apply_propagator(H_eff, tau_rem,
                                                                  self.direction, psi)
                if norm2(phi) >= self.r[k]:
                    self.psi[k] = phi
                    break
                # MCWF step 3: the norm reaches r inside this step
                tau = jump_time(H_eff, psi, tau_rem, self.r[k], self.direction)
                psi = apply_propagator(H_eff, tau, self.direction, psi)
                n = int(self.ordinal[k])
                stream = self.streams[k]
                # MCWF step 4: instantaneous jump with operator l
                l = choose_operator(psi, self.sys.L_jump, stream.choice(n))
                elapsed = (dt - tau_rem) + tau
                rate = sum(norm2(L @ psi) for L in self.sys.L_jump) / norm2(psi)
                self.records.append(Jump(k, step, l, n, self.direction,
                                         t_start + sign * elapsed, rate))
                psi = self.sys.L_jump[l] @ psi
                psi = psi / np.sqrt(norm2(psi))
                # MCWF step 5: new random number, continue within the step
                self.ordinal[k] = n + 1
                self.r[k] = stream.threshold(n + 1)
                tau_rem = tau_rem - tau
                U_rem = propagator(H_eff, tau_rem, self.direction) if dense else None


def forward_pass(system: System, psi0: np.ndarray, u: np.ndarray, T: float, M: int,
                 seed: int, iteration: int, instance: int = 0,
                 pulse_hook: Optional[Callable[[int, "Ensemble"], np.ndarray]] = None,
                 keep_states: bool = False):
    """Propagate M trajectories from psi0 over [0, T] with pulses u [n_ctrl, nt].

    ``pulse_hook(j, ens)`` may return the pulse values to use on interval j
    (Krotov's sequential update); otherwise u[:, j] is used.  Returns the
    ensemble (unnormalised final states, records) and, if requested, the
    normalised states at every t_j ([nt+1, M, d]).
    """
    nt = u.shape[1]
    dt = T / nt
    ens = Ensemble(system, psi0, M, seed, iteration, 0, instance)
    states = [ens.normalised()] if keep_states else None
    for j in range(nt):
        u_j = u[:, j] if pulse_hook is None else pulse_hook(j, ens)
        ens.advance(j, u_j, dt, j * dt)
        if keep_states:
            states.append(ens.normalised())
    return ens, (np.array(states) if keep_states else None)


def backward_pass(system: System, chi_T: np.ndarray, u: np.ndarray, T: float, M: int,
                  seed: int, iteration: int, instance: int = 0):
    """Propagate M costate trajectories from chi_T (rows, unnormalised) back to t=0.

    Returns the ensemble and the normalised backward states chi_hat(t_j) for
    j = 0 .. nt-1, array [nt, M, d] (index j holds the state at t_j).
    """
    nt = u.shape[1]
    dt = T / nt
    ens = Ensemble(system, chi_T, M, seed, iteration, 1, instance)
    out = np.zeros((nt, M, system.dim), dtype=np.complex128)
    for j in range(nt - 1, -1, -1):
        ens.advance(j, u[:, j], dt, (j + 1) * dt)
        out[j] = ens.normalised()
    return ens, out
