"""Trajectory functional and independent-trajectory Krotov optimisation, FP64.

Sec. 2.3 of the paper:

* functional  J_T = 1 - (1/M) sum_k |tau_k|^2 with tau_k the overlap of the
  trajectory's normalised final state with the target
  (the trajectory functional of Sec. 2.3);
* costate boundary chi_k(T) = -dJ_T/d<Psi_k| ;
* update  Delta u_i(t) = S_i(t) / (M lambda_i) sum_k Im <chi_k(t)| H_i |Psi_k(t)>
  (the independent-trajectory update of Sec. 2.3), evaluated sequentially:
  the forward states already carry the updated pulses (Sec. 2.2, "sequential").

Readings taken here:

* tau_k.  The paper defines tau_k = <Psi_k(T)|Psi_tgt> but then writes the
  boundary condition as tau_k |Psi_tgt>.  Differentiating J_T with respect to
  <Psi_k| gives <Psi_tgt|Psi_k(T)> |Psi_tgt> (up to the 1/M that the update
  carries), so we take tau_k = <Psi_tgt|Psi_hat_k(T)> and
  chi_k(T) = tau_k Psi_tgt.  J_T only needs |tau_k|, which both conventions
  share.
* Costate normalisation.  The backward trajectory starts from the normalised
  target and evolves by the MCWF rules in reverse time; the costate used in the
  update is chi_k(t) = tau_k chi_hat_k(t), with chi_hat the normalised backward
  state.
* Time grid.  The update of interval j (0-based, (t_j, t_{j+1}]) uses the
  costate at t_j from the previous iteration and the forward state at t_j
  propagated with the pulses already updated on intervals 0..j-1.
* Iterations: iteration 0 is a forward pass with the guess; iteration n >= 1 is
  a backward pass with u^(n-1) (random stream iteration n, direction 1)
  followed by the sequential forward pass (iteration n, direction 0).

The cross-trajectory update of Sec. 2.3 (eq. cross_traj_update) is here too:
  Delta u_i(t) = S_i(t) / (M^2 lambda_i)
                 sum_{k,k'} Im[<xi_k(t)| H_i |Psi_k'(t)> <Psi_k'(t)|xi_k(t)>]
with xi_k propagated backward from xi_k(T) = Psi_tgt.  Readings: xi_k runs
the same reverse-time MCWF rules and streams as the costates above, and enters
normalised (like the forward states), so that (1/M) sum_k |xi_k><xi_k| is the
trajectory estimate of the backward-propagated target projector; the sums
over k and k' are taken as printed, as two M x M overlap matrices per control.
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from .mcwf import Ensemble, Jump, System, backward_pass, forward_pass


def overlaps(psi_hat_T: np.ndarray, psi_tgt: np.ndarray) -> np.ndarray:
    """tau_k = <Psi_tgt | Psi_hat_k(T)> for rows of psi_hat_T."""
    return psi_hat_T @ psi_tgt.conj()


def functional(tau: np.ndarray) -> float:
    """J_T = 1 - (1/M) sum_k |tau_k|^2 (trajectory functional, Sec. 2.3)."""
    return float(1.0 - np.mean(np.abs(tau) ** 2))


@dataclasses.dataclass
class PassResult:
    psi_hat_T: np.ndarray
    tau: np.ndarray
    J_T: float
    records: List[Jump]
    u: np.ndarray


def plain_forward(system: System, psi0, psi_tgt, u, T, M, seed, iteration=0,
                  instance=0) -> PassResult:
    ens, _ = forward_pass(system, psi0, u, T, M, seed, iteration, instance)
    psi_hat = ens.normalised()
    tau = overlaps(psi_hat, psi_tgt)
    return PassResult(psi_hat, tau, functional(tau), ens.records, u.copy())


def costates(system: System, psi_tgt, tau, u, T, M, seed, iteration, instance=0):
    """Backward pass: chi_k(t_j) = tau_k chi_hat_k(t_j), array [nt, M, d]."""
    chi_T = np.broadcast_to(psi_tgt / np.linalg.norm(psi_tgt), (M, psi_tgt.shape[0]))
    ens, chi_hat = backward_pass(system, chi_T, u, T, M, seed, iteration, instance)
    return chi_hat * tau[None, :, None], ens.records


def krotov_update_term(system: System, chi_j: np.ndarray, psi_hat_j: np.ndarray) -> np.ndarray:
    """s_i = sum_k Im <chi_k| H_i |Psi_hat_k> for every control i."""
    s = np.zeros(len(system.H_ctrl))
    for i, Hi in enumerate(system.H_ctrl):
        s[i] = np.sum(np.imag(np.einsum("kd,kd->k", chi_j.conj(), psi_hat_j @ Hi.T)))
    return s


def sequential_forward(system: System, psi0, psi_tgt, u_old, chi, S, lam, T, M, seed,
                       iteration, instance=0) -> PassResult:
    """Forward pass with the sequential independent-trajectory Krotov update."""
    u_new = np.array(u_old, dtype=np.float64, copy=True)

    def hook(j: int, ens: Ensemble) -> np.ndarray:
        s = krotov_update_term(system, chi[j], ens.normalised())
        u_new[:, j] = u_old[:, j] + S[:, j] * s / (lam * M)
        return u_new[:, j]

    ens, _ = forward_pass(system, psi0, u_new, T, M, seed, iteration, instance,
                          pulse_hook=hook)
    psi_hat = ens.normalised()
    tau = overlaps(psi_hat, psi_tgt)
    return PassResult(psi_hat, tau, functional(tau), ens.records, u_new)


@dataclasses.dataclass
class OptimisationResult:
    J_T: List[float]
    u: List[np.ndarray]  # pulses after each iteration (index 0 = guess)
    passes: List[PassResult]
    backward_records: List[List[Jump]]
    chi: Optional[List[np.ndarray]] = None


def optimise(system: System, psi0, psi_tgt, u0, S, lam, T, M, seed, n_iter,
             instance=0, keep_chi=False) -> OptimisationResult:
    """Iteration 0 = guess forward pass; then n_iter Krotov iterations."""
    first = plain_forward(system, psi0, psi_tgt, u0, T, M, seed, 0, instance)
    res = OptimisationResult([first.J_T], [first.u], [first], [], [] if keep_chi else None)
    u, tau = first.u, first.tau
    for n in range(1, n_iter + 1):
        chi, brec = costates(system, psi_tgt, tau, u, T, M, seed, n, instance)
        p = sequential_forward(system, psi0, psi_tgt, u, chi, S, lam, T, M, seed, n,
                               instance)
        res.J_T.append(p.J_T)
        res.u.append(p.u)
        res.passes.append(p)
        res.backward_records.append(brec)
        if keep_chi:
            res.chi.append(chi)
        u, tau = p.u, p.tau
    return res


# ---------------------------------------------------------------------------
# cross-trajectory update (Sec. 2.3, eq. cross_traj_update)
# ---------------------------------------------------------------------------

def cross_costates(system: System, psi_tgt, u, T, M, seed, iteration, instance=0):
    """Backward trajectories from xi_k(T) = Psi_tgt: normalised xi_k(t_j), [nt, M, d]."""
    xi_T = np.broadcast_to(psi_tgt / np.linalg.norm(psi_tgt), (M, psi_tgt.shape[0]))
    ens, xi_hat = backward_pass(system, xi_T, u, T, M, seed, iteration, instance)
    return xi_hat, ens.records


def cross_update_term(system: System, xi_j: np.ndarray, psi_hat_j: np.ndarray) -> np.ndarray:
    """s_i = sum_{k,k'} Im[<xi_k|H_i|Psi_k'> <Psi_k'|xi_k>] for every control i."""
    B = psi_hat_j.conj() @ xi_j.T  # B[k', k] = <Psi_k'|xi_k>
    s = np.zeros(len(system.H_ctrl))
    for i, Hi in enumerate(system.H_ctrl):
        A = xi_j.conj() @ (psi_hat_j @ Hi.T).T  # A[k, k'] = <xi_k|H_i|Psi_k'>
        s[i] = float(np.sum(np.imag(A * B.T)))
    return s


def sequential_forward_cross(system: System, psi0, psi_tgt, u_old, xi, S, lam, T, M, seed,
                             iteration, instance=0) -> PassResult:
    """Forward pass with the sequential cross-trajectory Krotov update."""
    u_new = np.array(u_old, dtype=np.float64, copy=True)

    def hook(j: int, ens: Ensemble) -> np.ndarray:
        s = cross_update_term(system, xi[j], ens.normalised())
        u_new[:, j] = u_old[:, j] + S[:, j] * s / (lam * M * M)
        return u_new[:, j]

    ens, _ = forward_pass(system, psi0, u_new, T, M, seed, iteration, instance,
                          pulse_hook=hook)
    psi_hat = ens.normalised()
    tau = overlaps(psi_hat, psi_tgt)
    return PassResult(psi_hat, tau, functional(tau), ens.records, u_new)


def optimise_cross(system: System, psi0, psi_tgt, u0, S, lam, T, M, seed, n_iter,
                   instance=0) -> OptimisationResult:
    """Iteration 0 = guess forward pass; then n_iter cross-trajectory iterations."""
    first = plain_forward(system, psi0, psi_tgt, u0, T, M, seed, 0, instance)
    res = OptimisationResult([first.J_T], [first.u], [first], [])
    u = first.u
    for n in range(1, n_iter + 1):
        xi, brec = cross_costates(system, psi_tgt, u, T, M, seed, n, instance)
        p = sequential_forward_cross(system, psi0, psi_tgt, u, xi, S, lam, T, M, seed, n,
                                     instance)
        res.J_T.append(p.J_T)
        res.u.append(p.u)
        res.passes.append(p)
        res.backward_records.append(brec)
        u = p.u
    return res
