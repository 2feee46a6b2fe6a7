"""Cascaded quantum-network workloads (inputs only).

Two models are built here, both as complex128 ``scipy.sparse.csr_matrix``:

* ``build_cascade`` -- the explicit model: N nodes, each a three-level atom
  {g, e, r} in a cavity truncated at ``n_fock`` photon levels, coupled in a
  unidirectional (cascade) chain by a travelling field (paper Sec. 3.1,
  eqs. ``ham`` and ``ham_interaction``).  Node basis |atom, n>, index
  ``atom * n_fock + n`` with atom order (g, e, r); global basis is the Kronecker
  product node 1 (x) node 2 (x) ..., node 1 most significant, so
  d = (3 n_fock)^N.

  Node Hamiltonian (hbar = 1, energies in units of the atom-cavity coupling)::

      H^(i) = Delta Pi_e + g (sigma_er a_i + sigma_re a_i^+)
              + Omega_i(t) * 1/2 (sigma_eg + sigma_ge)

  The drive couples g <-> e (detuning Delta), the cavity couples e <-> r.
  Cascade interaction between nodes i < j, for node jump operators
  L_i = sqrt(kappa) a_i, is the series-product term
  (i kappa / 2)(a_i^+ a_j - a_j^+ a_i), and the single collective jump operator
  is L = sqrt(kappa) sum_i a_i (paper Sec. 3.1: the total Lindblad operator is
  the sum of the node operators).  With L_i = sqrt(2 kappa) a_i the same
  construction gives the paper's i kappa a_i^+ a_j + h.c.

* ``build_paper_model`` -- the paper's own effective single-excitation model of
  Sec. 3.1/3.2 (auxiliary level adiabatically eliminated; d = 2N + 1).

Guess pulses: a Gaussian of amplitude 0.5 centred at T/2 with width T/6,
sampled at interval midpoints, plus normal noise of standard deviation 0.01.
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

# atom level indices
G_LEVEL, E_LEVEL, R_LEVEL = 0, 1, 2


@dataclasses.dataclass(frozen=True)
class CascadeSpec:
    n_nodes: int
    n_fock: int
    delta: float = 1.0
    g: float = 1.0
    kappa: float = 1.0

    @property
    def local_dim(self) -> int:
        return 3 * self.n_fock

    @property
    def dim(self) -> int:
        return self.local_dim ** self.n_nodes


@dataclasses.dataclass
class Workload:
    """Everything a trajectory-Krotov run consumes (all FP64 / complex128)."""

    name: str
    H0: sp.csr_matrix
    H_ctrl: List[sp.csr_matrix]
    L_jump: List[sp.csr_matrix]
    psi0: np.ndarray
    psi_tgt: np.ndarray
    T: float
    nt: int
    u0: np.ndarray  # [n_ctrl, nt] guess pulses (piecewise constant)
    S: np.ndarray  # [n_ctrl, nt] update shape, in [0, 1]
    lam: np.ndarray  # [n_ctrl] Krotov step weights lambda_i
    M: int
    seed: int
    n_iter: int
    precision: str = "fp64"
    instance: int = 0

    @property
    def dim(self) -> int:
        return self.psi0.shape[0]

    @property
    def n_ctrl(self) -> int:
        return len(self.H_ctrl)

    @property
    def dt(self) -> float:
        return self.T / self.nt

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def _local_ops(n_fock: int):
    a_f = sp.diags(np.sqrt(np.arange(1, n_fock, dtype=np.float64)), 1,
                   shape=(n_fock, n_fock), format="csr")
    i_f = sp.identity(n_fock, format="csr")

    def proj(p, q):  # |p><q| on the atom
        m = sp.lil_matrix((3, 3))
        m[p, q] = 1.0
        return m.tocsr()

    i_a = sp.identity(3, format="csr")
    ops = {
        "a": sp.kron(i_a, a_f, format="csr"),
        "Pi_e": sp.kron(proj(E_LEVEL, E_LEVEL), i_f, format="csr"),
        "s_er": sp.kron(proj(E_LEVEL, R_LEVEL), i_f, format="csr"),
        "s_re": sp.kron(proj(R_LEVEL, E_LEVEL), i_f, format="csr"),
        "s_eg": sp.kron(proj(E_LEVEL, G_LEVEL), i_f, format="csr"),
        "s_ge": sp.kron(proj(G_LEVEL, E_LEVEL), i_f, format="csr"),
    }
    return {k: v.astype(np.complex128) for k, v in ops.items()}


def _embed(op: sp.csr_matrix, node: int, n_nodes: int, local_dim: int) -> sp.csr_matrix:
    left = sp.identity(local_dim ** node, format="csr", dtype=np.complex128)
    right = sp.identity(local_dim ** (n_nodes - node - 1), format="csr",
                        dtype=np.complex128)
    return sp.kron(sp.kron(left, op, format="csr"), right, format="csr")


def basis_index(spec: CascadeSpec, atoms, photons) -> int:
    """Global index of |atom_1, n_1; atom_2, n_2; ...> (node 1 most significant)."""
    idx = 0
    for a, n in zip(atoms, photons):
        idx = idx * spec.local_dim + a * spec.n_fock + n
    return idx


def build_cascade(spec: CascadeSpec):
    """Return (H0, [H_ctrl_i], [L]) for the explicit cascade chain."""
    N, dl = spec.n_nodes, spec.local_dim
    ops = _local_ops(spec.n_fock)
    d = spec.dim
    H0 = sp.csr_matrix((d, d), dtype=np.complex128)
    a_g = [_embed(ops["a"], i, N, dl) for i in range(N)]
    for i in range(N):
        h_node = spec.delta * ops["Pi_e"] + spec.g * (
            ops["s_er"] @ ops["a"] + ops["s_re"] @ ops["a"].conj().T)
        H0 = H0 + _embed(h_node.tocsr(), i, N, dl)
    for i in range(N):
        for j in range(i + 1, N):
            H0 = H0 + (0.5j * spec.kappa) * (a_g[i].conj().T @ a_g[j]
                                             - a_g[j].conj().T @ a_g[i])
    H_ctrl = [
        _embed((0.5 * (ops["s_eg"] + ops["s_ge"])).tocsr(), i, N, dl)
        for i in range(N)
    ]
    L = sum(a_g[1:], a_g[0]) * np.sqrt(spec.kappa)
    clean = lambda m: _clean(m)
    return clean(H0), [clean(h) for h in H_ctrl], [clean(L)]


def _clean(m: sp.spmatrix) -> sp.csr_matrix:
    m = sp.csr_matrix(m, dtype=np.complex128)
    m.eliminate_zeros()
    m.sum_duplicates()
    m.sort_indices()
    return m


def initial_state(spec: CascadeSpec) -> np.ndarray:
    psi = np.zeros(spec.dim, dtype=np.complex128)
    psi[basis_index(spec, [G_LEVEL] * spec.n_nodes, [0] * spec.n_nodes)] = 1.0
    return psi


def w_target(spec: CascadeSpec) -> np.ndarray:
    """(1/sqrt N) sum_i |r on node i, g elsewhere, all cavities empty>."""
    N = spec.n_nodes
    psi = np.zeros(spec.dim, dtype=np.complex128)
    for i in range(N):
        atoms = [G_LEVEL] * N
        atoms[i] = R_LEVEL
        psi[basis_index(spec, atoms, [0] * N)] = 1.0
    return psi / np.linalg.norm(psi)


def random_gr_target(spec: CascadeSpec, rng: np.random.Generator) -> np.ndarray:
    """Normalised complex Gaussian vector in the {g, r}^N subspace, cavities empty."""
    N = spec.n_nodes
    psi = np.zeros(spec.dim, dtype=np.complex128)
    for bits in range(2 ** N):
        atoms = [R_LEVEL if (bits >> (N - 1 - i)) & 1 else G_LEVEL for i in range(N)]
        psi[basis_index(spec, atoms, [0] * N)] = rng.normal() + 1j * rng.normal()
    return psi / np.linalg.norm(psi)


def guess_pulses(n_ctrl: int, nt: int, T: float, rng: np.random.Generator,
                 amplitude: float = 0.5, noise: float = 0.01) -> np.ndarray:
    dt = T / nt
    tmid = (np.arange(nt) + 0.5) * dt
    sigma = T / 6.0
    shape = amplitude * np.exp(-((tmid - T / 2) ** 2) / (2 * sigma ** 2))
    return shape[None, :] + rng.normal(0.0, noise, size=(n_ctrl, nt))


def build_paper_model(n_nodes: int, delta: float = 100.0, g: float = 1.0,
                      kappa: float = 1.0):
    """The paper's effective single-excitation network (d = 2N + 1).

    Basis: 0 = all atoms in g and all cavities empty; 1 + 2i = atom i excited
    (|e_i>); 2 + 2i = one photon in cavity i (|1_i>).  H0 of each node vanishes
    in this space; the drive term -(i Omega g / 2 Delta)(sigma_eg a - h.c.)
    couples |1_i> and |e_i>; the cascade term i kappa a_i^+ a_j + h.c. (i < j);
    L = sqrt(2 kappa) sum_i a_i.
    Returns (H0, H_ctrl, L, psi0 = |e_1>, target = (1/sqrt N) sum |e_i>).
    """
    N = n_nodes
    d = 2 * N + 1
    e = lambda i: 1 + 2 * i
    one = lambda i: 2 + 2 * i
    H0 = sp.lil_matrix((d, d), dtype=np.complex128)
    for i in range(N):
        for j in range(i + 1, N):
            H0[one(i), one(j)] += 1j * kappa
            H0[one(j), one(i)] += -1j * kappa
    H_ctrl = []
    for i in range(N):
        h = sp.lil_matrix((d, d), dtype=np.complex128)
        h[e(i), one(i)] = -1j * g / (2 * delta)
        h[one(i), e(i)] = 1j * g / (2 * delta)
        H_ctrl.append(_clean(h))
    L = sp.lil_matrix((d, d), dtype=np.complex128)
    for i in range(N):
        L[0, one(i)] = np.sqrt(2 * kappa)
    psi0 = np.zeros(d, dtype=np.complex128)
    psi0[e(0)] = 1.0
    tgt = np.zeros(d, dtype=np.complex128)
    for i in range(N):
        tgt[e(i)] = 1.0
    tgt /= np.linalg.norm(tgt)
    return _clean(H0), H_ctrl, [_clean(L)], psi0, tgt


# ---------------------------------------------------------------------------
# named synthetic workloads
# ---------------------------------------------------------------------------

CONFIGS = {
    # chain of 2 nodes, cavity at 2 levels (d = 36); M = 8, nt = 500, 10 its
    "chain2_fock2": dict(n_nodes=2, n_fock=2, M=8, nt=500, n_iter=10,
                         precision="fp64"),
    # chain of 2 nodes, cavity at 3 levels (d = 81); M = 1024, nt = 2000, 20 its
    "chain2_fock3": dict(n_nodes=2, n_fock=3, M=1024, nt=2000, n_iter=20,
                         precision="fp64"),
    # chain of 3 nodes, cavity at 2 levels (d = 216); M = 4096, nt = 4000
    "chain3_fock2": dict(n_nodes=3, n_fock=2, M=4096, nt=4000, n_iter=10,
                         precision="fp32"),
    # chain of 4 nodes, cavity at 2 levels (d = 1296); M = 2048, nt = 4000
    "chain4_fock2": dict(n_nodes=4, n_fock=2, M=2048, nt=4000, n_iter=1,
                         precision="fp32"),
}


def config_workload(name: str, *, M: Optional[int] = None, nt: Optional[int] = None,
                    T: float = 50.0, seed: int = 0, lam: float = 5.0,
                    n_iter: Optional[int] = None, delta: float = 1.0) -> Workload:
    c = dict(CONFIGS[name])
    spec = CascadeSpec(n_nodes=c["n_nodes"], n_fock=c["n_fock"], delta=delta)
    H0, Hc, L = build_cascade(spec)
    M = c["M"] if M is None else M
    nt = c["nt"] if nt is None else nt
    rng = np.random.default_rng(seed)
    u0 = guess_pulses(spec.n_nodes, nt, T, rng)
    return Workload(
        name=name, H0=H0, H_ctrl=Hc, L_jump=L, psi0=initial_state(spec),
        psi_tgt=w_target(spec), T=T, nt=nt, u0=u0,
        S=np.ones((spec.n_nodes, nt)), lam=np.full(spec.n_nodes, lam),
        M=M, seed=seed, n_iter=c["n_iter"] if n_iter is None else n_iter,
        precision=c["precision"])


def batch_instances(n_instances: int = 64, seed: int = 0, T: float = 50.0,
                    lam: float = 5.0, delta: float = 1.0,
                    m_range=(64, 2048), nt_range=(500, 4000),
                    nodes=(2, 3, 4)) -> List[Workload]:
    """Independent optimisation instances of uneven size (cavity at 2 levels).

    The instance shape (chain length, M, nt) comes from ``default_rng(seed)``;
    each instance's target and guess pulses come from
    ``default_rng(seed + instance)``; targets are random in the atoms' {g, r}
    subspace with the cavities empty.
    """
    shape_rng = np.random.default_rng(seed)
    out = []
    cache = {}
    for inst in range(n_instances):
        N = int(shape_rng.choice(nodes))
        M = int(shape_rng.integers(m_range[0], m_range[1] + 1))
        nt = int(shape_rng.integers(nt_range[0], nt_range[1] + 1))
        spec = CascadeSpec(n_nodes=N, n_fock=2, delta=delta)
        if N not in cache:
            cache[N] = build_cascade(spec)
        H0, Hc, L = cache[N]
        rng = np.random.default_rng(seed + inst)
        tgt = random_gr_target(spec, rng)
        u0 = guess_pulses(N, nt, T, rng)
        out.append(Workload(
            name=f"batch{inst}", H0=H0, H_ctrl=Hc, L_jump=L,
            psi0=initial_state(spec), psi_tgt=tgt, T=T, nt=nt, u0=u0,
            S=np.ones((N, nt)), lam=np.full(N, lam), M=M, seed=seed,
            n_iter=1, precision="fp32", instance=inst))
    return out
