"""Pathwise gradient of the trajectory functional with the jump record fixed, FP64.

TEST INFRASTRUCTURE ONLY (see the package header).

A forward MCWF pass (Sec. 2.1) leaves, per trajectory, the list of its jumps:
step, time and operator.  Holding that list fixed turns every trajectory into
a fixed composition of linear maps -- the piecewise-constant propagators
exp(-i H_eff(u_j) tau) between consecutive jump times and the jump operators
L_l -- and the trajectory functional of Sec. 2.3,
J_T(u) = 1 - (1/M) sum_k |<tgt|psi_hat_k(T)>|^2, into a smooth function of
the pulse values u_ij.  This module evaluates that function ("replay") and
its gradient dJ_T/du_ij in two independent ways:

* central finite differences of the replayed functional;
* the adjoint (reverse) sweep, with the exact derivative of each propagator
  piece from the block exponential of Van Loan (1978):
      exp(tau [[A, E], [0, A]]) = [[e^{tau A}, D], [0, e^{tau A}]],
      D = int_0^tau e^{(tau-s) A} E e^{s A} ds,
  with A = -i H_eff and E = -i H_i, so D = d exp(-i H_eff tau) / du_i.

Readings taken here:

* The renormalisation after a jump (MCWF step 4) multiplies the state by a
  positive number; psi_hat_k(T) and hence J_T do not change if those numbers
  are held constant, so the pathwise derivative treats them as constants.
* A jump time is used exactly as recorded: a jump recorded at t in step j
  splits interval j at t; the pieces before and after use the same u_j.
"""

from __future__ import annotations

from typing import Dict, Iterable, List, Sequence, Tuple

import numpy as np
import scipy.linalg

import scipy.sparse
import scipy.sparse.linalg

from .mcwf import Jump, System, apply_propagator, norm2, step_operator

Path = List[Tuple[int, float, int]]  # (step, time, operator) in time order


def paths_from_records(records: Iterable[Jump], M: int) -> List[Path]:
    """Per-trajectory jump lists (forward records only), ordered by ordinal."""
    by_k: Dict[int, List[Jump]] = {k: [] for k in range(M)}
    for r in records:
        if r.direction == 0 and 0 <= r.traj < M:
            by_k[r.traj].append(r)
    out = []
    for k in range(M):
        rs = sorted(by_k[k], key=lambda r: r.ordinal)
        out.append([(r.step, r.t, r.op) for r in rs])
    return out


def _pieces(path: Path, nt: int, dt: float):
    """The trajectory as a list of (step j, piece length tau, jump op after or None)."""
    out = []
    q = 0
    for j in range(nt):
        t_cur = j * dt
        while q < len(path) and path[q][0] == j:
            _, t_star, l = path[q]
            out.append((j, t_star - t_cur, l))
            t_cur = t_star
            q += 1
        out.append((j, (j + 1) * dt - t_cur, None))
    if q != len(path):
        raise ValueError("jump record with a step outside the pulse grid")
    return out


def replay_states(system: System, psi0, u: np.ndarray, T: float, paths: Sequence[Path]):
    """Final unnormalised states phi_k(T) of the replayed trajectories, [M, d]."""
    nt = u.shape[1]
    dt = T / nt
    H = [step_operator(system.effective_hamiltonian(u[:, j])) for j in range(nt)]
    out = []
    for path in paths:
        phi = np.array(psi0, dtype=np.complex128)
        for j, tau, l in _pieces(path, nt, dt):
            phi = apply_propagator(H[j], tau, 0, phi)
            if l is not None:
                phi = system.L_jump[l] @ phi
                phi = phi / np.sqrt(norm2(phi))
        out.append(phi)
    return np.array(out)


def replay_functional(system: System, psi0, psi_tgt, u, T, paths) -> Tuple[float, np.ndarray]:
    """J_T of the replayed trajectories and their overlaps tau_k = <tgt|phi_hat_k(T)>."""
    phi = replay_states(system, psi0, u, T, paths)
    phi_hat = phi / np.sqrt(np.einsum("kd,kd->k", phi.conj(), phi).real)[:, None]
    tau = phi_hat @ np.asarray(psi_tgt).conj()
    return float(1.0 - np.mean(np.abs(tau) ** 2)), tau


def propagator_derivative(H_eff, H_i: np.ndarray, tau: float, x: np.ndarray) -> np.ndarray:
    """(d exp(-i (H_eff + u H_i) tau) / du at u = 0) x, by Van Loan's block
    exponential: the top half of exp(tau [[-iH, -iH_i], [0, -iH]]) [0; x]."""
    d = H_eff.shape[0]
    if not scipy.sparse.issparse(H_eff):
        blk = np.zeros((2 * d, 2 * d), dtype=np.complex128)
        blk[:d, :d] = -1j * tau * H_eff
        blk[d:, d:] = -1j * tau * H_eff
        blk[:d, d:] = -1j * tau * H_i
        return scipy.linalg.expm(blk)[:d, d:] @ x
    A = -1j * tau * H_eff
    blk = scipy.sparse.bmat([[A, -1j * tau * scipy.sparse.csr_matrix(H_i)], [None, A]]).tocsr()
    z = np.concatenate([np.zeros(d, dtype=np.complex128), x])
    return scipy.sparse.linalg.expm_multiply(blk, z)[:d]


def gradient_adjoint(system: System, psi0, psi_tgt, u: np.ndarray, T: float,
                     paths: Sequence[Path]) -> np.ndarray:
    """dJ_T/du_ij for all i, j by the reverse sweep, array [n_ctrl, nt]."""
    nt = u.shape[1]
    dt = T / nt
    M = len(paths)
    n_ctrl = len(system.H_ctrl)
    H = [step_operator(system.effective_hamiltonian(u[:, j])) for j in range(nt)]
    tgt = np.asarray(psi_tgt, dtype=np.complex128)
    grad = np.zeros((n_ctrl, nt))
    for path in paths:
        pieces = _pieces(path, nt, dt)
        # forward: state at the start of every piece, renormalisation constants
        starts, consts = [], []
        phi = np.array(psi0, dtype=np.complex128)
        for j, tau, l in pieces:
            starts.append(phi)
            phi = apply_propagator(H[j], tau, 0, phi)
            c = None
            if l is not None:
                phi = system.L_jump[l] @ phi
                c = 1.0 / np.sqrt(norm2(phi))
                phi = c * phi
            consts.append(c)
        # F = |<tgt|phi>|^2 / <phi|phi>;  dF = 2 Re <lam|dphi>
        nrm = np.sqrt(norm2(phi))
        phi_hat = phi / nrm
        t_k = np.vdot(tgt, phi_hat)
        lam = (t_k * tgt - abs(t_k) ** 2 * phi_hat) / nrm
        for (j, tau, l), start, c in zip(reversed(pieces), reversed(starts), reversed(consts)):
            if l is not None:  # adjoint of the (constant-scaled) jump map
                lam = c * (system.L_jump[l].conj().T @ lam)
            for i, Hi in enumerate(system.H_ctrl):
                grad[i, j] += 2.0 * np.real(np.vdot(lam, propagator_derivative(H[j], Hi, tau, start)))
            # adjoint of the piece: exp(-i H tau)^+ = exp(+i H^+ tau)
            lam = apply_propagator(H[j], tau, 1, lam)
    return -grad / M


def gradient_fd(system: System, psi0, psi_tgt, u: np.ndarray, T: float,
                paths: Sequence[Path], entries: Sequence[Tuple[int, int]],
                h: float = 1e-4) -> np.ndarray:
    """Central differences (J(u + h e_ij) - J(u - h e_ij)) / 2h for the given (i, j)."""
    out = []
    for i, j in entries:
        up = np.array(u, dtype=np.float64, copy=True)
        dn = np.array(u, dtype=np.float64, copy=True)
        up[i, j] += h
        dn[i, j] -= h
        Jp, _ = replay_functional(system, psi0, psi_tgt, up, T, paths)
        Jm, _ = replay_functional(system, psi0, psi_tgt, dn, T, paths)
        out.append((Jp - Jm) / (2.0 * h))
    return np.array(out)
