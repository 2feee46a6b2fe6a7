"""Dense density-matrix propagation under the Lindblad master equation.

Sec. 2.1, the master equation: d rho/dt = -i [H(u(t)), rho] + L_D rho with the
dissipator L_D rho = sum_l (L_l rho L_l^+ - 1/2 {L_l^+ L_l, rho}).  The
trajectory average (1/M) sum_k |Psi_k><Psi_k| converges to rho(t) as M grows
(Sec. 2.1, the trajectory expansion of rho), which is how the MCWF oracle is
checked.  Liouville space uses row-major vectorisation, vec(A X B) =
(A kron B^T) vec(X); each piecewise-constant interval is applied with
``scipy.sparse.linalg.expm_multiply``.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg

from .mcwf import System


def liouvillian(system: System, u_j) -> sp.csr_matrix:
    d = system.dim
    I = sp.identity(d, dtype=np.complex128, format="csr")
    H = sp.csr_matrix(system.H0)
    for ui, Hi in zip(u_j, system.H_ctrl):
        H = H + ui * sp.csr_matrix(Hi)
    # -i [H, rho] = -i H rho + i rho H
    Lv = -1j * sp.kron(H, I) + 1j * sp.kron(I, H.T)
    for L in system.L_jump:
        Ls = sp.csr_matrix(L)
        LdL = (Ls.conj().T @ Ls).tocsr()
        Lv = Lv + sp.kron(Ls, Ls.conj()) - 0.5 * sp.kron(LdL, I) - 0.5 * sp.kron(I, LdL.T)
    return Lv.tocsr()


def propagate_rho(system: System, rho0: np.ndarray, u: np.ndarray, T: float,
                  keep: bool = False):
    """rho(T) (or all rho(t_j)) from rho0 under piecewise-constant pulses u [n_ctrl, nt]."""
    nt = u.shape[1]
    dt = T / nt
    v = np.asarray(rho0, dtype=np.complex128).reshape(-1)
    out = [v.reshape(rho0.shape)] if keep else None
    for j in range(nt):
        v = scipy.sparse.linalg.expm_multiply(dt * liouvillian(system, u[:, j]), v)
        if keep:
            out.append(v.reshape(rho0.shape))
    return np.array(out) if keep else v.reshape(rho0.shape)
