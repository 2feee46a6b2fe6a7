"""Density-matrix optimisation of Sec. 2.2 (Liouville space), FP64.

TEST INFRASTRUCTURE ONLY (see the package header).

* Functional (eq. functional): J_T = 1 - <<rho(T)|P_tgt>> = 1 - <tgt|rho(T)|tgt>
  with <<a|b>> = tr(a^+ b) and P_tgt = |tgt><tgt|.
* Forward: the master equation of Sec. 2.1, d rho/dt = L(rho),
  L(rho) = -i [H, rho] + sum_l (L_l rho L_l^+ - 1/2 {L_l^+ L_l, rho}),
  piecewise constant in time; rho(0) = |psi0><psi0|.
* Backward (eq. bwprop): P(t_j) = D_{j+1}^+ ... D_nt^+ P_tgt with the adjoint
  ("conjugate") map of each step, i.e. P propagated from P(T) = P_tgt
  (eq. krotov_boundary) with the adjoint Liouvillian
  L^+(P) = +i [H, P] + sum_l (L_l^+ P L_l - 1/2 {L_l^+ L_l, P}).
* Krotov update (eq. krotovupdate) with dL/du_i rho = [H_i, rho] as the paper
  prints it: Delta u_i(t) = S_i(t)/lambda_i Im <<P^(0)(t)| [H_i, rho^(1)(t)]>>,
  sequential (rho^(1) carries the pulses already updated).

Readings taken here:

* Time grid as for the trajectories: the update of interval j uses P(t_j) of
  the previous pulses and rho^(1)(t_j) at the interval's left end.
* The factor of the update is taken as printed (no -i from dL/du, whose
  imaginary part would flip; the weight lambda absorbs the scale).  For pure
  states and kappa = 0 this makes the density-matrix update exactly twice the
  cross-trajectory update with one trajectory, which a pin checks.

Each interval is applied with scipy's expm_multiply on the row-major
vectorised operator (vec(A X B) = (A kron B^T) vec(X)).
"""

from __future__ import annotations

import dataclasses
from typing import List

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg

from .lindblad import liouvillian
from .mcwf import System


def adjoint_liouvillian(system: System, u_j) -> sp.csr_matrix:
    """L^+ as a matrix on row-major vec(P): the Hilbert-Schmidt adjoint of L."""
    return liouvillian(system, u_j).conj().T.tocsr()


def rho_functional(rho_T: np.ndarray, psi_tgt: np.ndarray) -> float:
    """J_T = 1 - <tgt|rho(T)|tgt> (eq. functional) for a normalised target."""
    t = np.asarray(psi_tgt, dtype=np.complex128)
    t = t / np.linalg.norm(t)
    return float(1.0 - np.real(np.vdot(t, rho_T @ t)))


def forward_rho(system: System, psi0, u: np.ndarray, T: float, keep: bool = False):
    """rho(T) (or every rho(t_j), j = 0 .. nt) from |psi0><psi0|."""
    nt = u.shape[1]
    dt = T / nt
    d = system.dim
    v = np.outer(psi0, np.conj(psi0)).reshape(-1)
    out = [v.reshape(d, d)] if keep else None
    for j in range(nt):
        v = scipy.sparse.linalg.expm_multiply(dt * liouvillian(system, u[:, j]), v)
        if keep:
            out.append(v.reshape(d, d))
    return np.array(out) if keep else v.reshape(d, d)


def backward_P(system: System, psi_tgt, u: np.ndarray, T: float) -> np.ndarray:
    """P(t_j) for j = 0 .. nt - 1 from P(T) = P_tgt with the adjoint steps, [nt, d, d]."""
    nt = u.shape[1]
    dt = T / nt
    d = system.dim
    t = np.asarray(psi_tgt, dtype=np.complex128)
    t = t / np.linalg.norm(t)
    v = np.outer(t, t.conj()).reshape(-1)
    out = np.zeros((nt, d, d), dtype=np.complex128)
    for j in range(nt - 1, -1, -1):
        v = scipy.sparse.linalg.expm_multiply(dt * adjoint_liouvillian(system, u[:, j]), v)
        out[j] = v.reshape(d, d)
    return out


def update_term(system: System, P_j: np.ndarray, rho_j: np.ndarray) -> np.ndarray:
    """Im <<P_j| [H_i, rho_j]>> for every control i."""
    return np.array([float(np.imag(np.trace(P_j.conj().T @ (Hi @ rho_j - rho_j @ Hi))))
                     for Hi in system.H_ctrl])


@dataclasses.dataclass
class RhoOptimisation:
    J_T: List[float]
    u: List[np.ndarray]


def optimise_rho(system: System, psi0, psi_tgt, u0, S, lam, T, n_iter) -> RhoOptimisation:
    """Density-matrix Krotov: iteration 0 evaluates the guess; iteration n
    propagates P backward with u^(n-1), then rho forward with the sequential
    update of every interval."""
    nt = u0.shape[1]
    dt = T / nt
    d = system.dim
    u = np.array(u0, dtype=np.float64, copy=True)
    res = RhoOptimisation([rho_functional(forward_rho(system, psi0, u, T), psi_tgt)], [u.copy()])
    for _ in range(n_iter):
        P = backward_P(system, psi_tgt, u, T)
        u_new = u.copy()
        v = np.outer(psi0, np.conj(psi0)).reshape(-1)
        for j in range(nt):
            s = update_term(system, P[j], v.reshape(d, d))
            u_new[:, j] = u[:, j] + S[:, j] * s / lam
            v = scipy.sparse.linalg.expm_multiply(dt * liouvillian(system, u_new[:, j]), v)
        res.J_T.append(rho_functional(v.reshape(d, d), psi_tgt))
        res.u.append(u_new.copy())
        u = u_new
    return res
