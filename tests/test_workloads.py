"""Input generators: model structure (Hermiticity, excitation conservation)."""

import numpy as np
import pytest
import scipy.sparse as sp

from workloads import CONFIGS, batch_instances, build_paper_model, config_workload
from workloads.cascade import (CascadeSpec, E_LEVEL, G_LEVEL, R_LEVEL, basis_index,
                               build_cascade, initial_state, w_target)


def _q_operator(spec: CascadeSpec) -> np.ndarray:
    """Q = sum_i (n_i - Pi_r^(i)), diagonal in the product basis."""
    N, nf = spec.n_nodes, spec.n_fock
    q = np.zeros(spec.dim)
    for idx in range(spec.dim):
        rest = idx
        val = 0
        for _ in range(N):
            loc = rest % spec.local_dim
            rest //= spec.local_dim
            atom, n = divmod(loc, nf)
            val += n - (1 if atom == R_LEVEL else 0)
        q[idx] = val
    return np.diag(q)


@pytest.mark.parametrize("n_nodes,n_fock", [(1, 2), (2, 2), (2, 3), (3, 2)])
def test_cascade_structure(n_nodes, n_fock):
    spec = CascadeSpec(n_nodes, n_fock)
    H0, Hc, L = build_cascade(spec)
    d = spec.dim
    assert H0.shape == (d, d) and d == (3 * n_fock) ** n_nodes
    for H in [H0] + Hc:
        assert abs(H - H.conj().T).max() < 1e-15
    Q = _q_operator(spec)
    Heff = (H0 + sum(0.7 * h for h in Hc)
            - 0.5j * sum(l.conj().T @ l for l in L)).toarray()
    # the drive moves g <-> e (Q unchanged), the cavity e <-> r with a photon
    assert np.abs(Heff @ Q - Q @ Heff).max() < 1e-13
    for l in L:
        ld = l.toarray()
        assert np.abs(Q @ ld - ld @ Q + ld).max() < 1e-13  # each jump lowers Q by one


def test_cascade_direction():
    """H_eff moves a photon from node 1 to node 2 only (cascade, Sec. 3.1)."""
    spec = CascadeSpec(2, 2)
    H0, _, L = build_cascade(spec)
    Heff = (H0 - 0.5j * L[0].conj().T @ L[0]).toarray()
    one0 = basis_index(spec, [G_LEVEL, G_LEVEL], [1, 0])
    zero1 = basis_index(spec, [G_LEVEL, G_LEVEL], [0, 1])
    assert abs(Heff[zero1, one0] - (-1j)) < 1e-15
    assert abs(Heff[one0, zero1]) < 1e-15


def test_states_and_pulses():
    w = config_workload("chain2_fock2")
    assert w.dim == 36 and w.u0.shape == (2, 500) and w.M == 8
    assert abs(np.linalg.norm(w.psi_tgt) - 1) < 1e-15
    assert abs(np.vdot(w.psi0, w.psi_tgt)) == 0
    assert abs(w.u0.max() - 0.5) < 0.05 and abs(w.u0[:, 0]).max() < 0.05
    w2 = config_workload("chain2_fock2")
    assert np.array_equal(w.u0, w2.u0)
    spec = CascadeSpec(3, 2)
    t = w_target(spec)
    assert np.count_nonzero(t) == 3


def test_config_sizes():
    dims = {"chain2_fock2": 36, "chain2_fock3": 81, "chain3_fock2": 216,
            "chain4_fock2": 1296}
    for name, d in dims.items():
        c = CONFIGS[name]
        assert (3 * c["n_fock"]) ** c["n_nodes"] == d


def test_batch_instances():
    inst = batch_instances(8, seed=0)
    assert len(inst) == 8
    for k, w in enumerate(inst):
        assert 64 <= w.M <= 2048 and 500 <= w.nt <= 4000
        assert w.instance == k and abs(np.linalg.norm(w.psi_tgt) - 1) < 1e-14
    assert inst[0].psi_tgt is not inst[1].psi_tgt


def test_paper_model():
    H0, Hc, L, psi0, tgt = build_paper_model(2)
    assert H0.shape == (5, 5)
    for H in [H0] + Hc:
        assert abs(H - H.conj().T).max() < 1e-15
    # the target (two excited atoms in superposition, cavities empty) is dark
    assert np.linalg.norm(L[0] @ tgt) == 0
