"""Pins of the oracle's pathwise gradient (jump record fixed).

The adjoint sweep is checked against a closed form, against central finite
differences of the replayed functional (a separate computation: only plain
propagators, no derivative formula), and against a structural zero; the replay
is checked against the independent MCWF pass that produced the record.
"""

import math

import numpy as np

from oracle import krotov
from oracle.gradient import (gradient_adjoint, gradient_fd, paths_from_records,
                             replay_functional)
from oracle.mcwf import Jump, System, forward_pass
from workloads import config_workload

SX = np.array([[0, 1], [1, 0]], complex)
SY = np.array([[0, -1j], [1j, 0]])


def test_two_level_closed_form():
    """H = u(t) sigma_x / 2 from |0> to |1>: J = 1 - sin^2(theta/2), theta = sum u_j dt,
    so dJ/du_j = -sin(theta) dt / 2 for every j."""
    sysd = System(np.zeros((2, 2), complex), [0.5 * SX], [])
    rng = np.random.default_rng(4)
    nt, T = 12, 3.0
    dt = T / nt
    u = rng.uniform(0.1, 0.6, size=(1, nt))
    psi0 = np.array([1, 0], complex)
    tgt = np.array([0, 1], complex)
    paths = [[]]
    J, _ = replay_functional(sysd, psi0, tgt, u, T, paths)
    theta = float(np.sum(u) * dt)
    assert abs(J - (1 - math.sin(theta / 2) ** 2)) < 1e-13
    g = gradient_adjoint(sysd, psi0, tgt, u, T, paths)
    assert np.max(np.abs(g - (-math.sin(theta) * dt / 2))) < 1e-13


def test_gradient_vanishes_before_rank_one_jump():
    """A jump with L = sqrt(kappa)|g><e| maps every state onto |g>: the replayed
    functional cannot depend on the pulses before it."""
    kappa = 0.7
    L = math.sqrt(kappa) * np.array([[0, 1], [0, 0]], complex)
    sysd = System(0.3 * np.diag([0.0, 1.0]).astype(complex), [0.5 * SX, 0.5 * SY], [L])
    nt, T = 10, 5.0
    dt = T / nt
    u = np.random.default_rng(1).uniform(-0.5, 0.8, size=(2, nt))
    psi0 = np.array([0, 1], complex)
    tgt = np.array([1, 1j], complex) / math.sqrt(2)
    j_jump = 4
    paths = [[(j_jump, (j_jump + 0.37) * dt, 0)]]
    g = gradient_adjoint(sysd, psi0, tgt, u, T, paths)
    assert np.max(np.abs(g[:, :j_jump])) < 1e-14
    assert np.max(np.abs(g[:, j_jump + 1:])) > 1e-3
    entries = [(0, 1), (1, 3), (0, j_jump), (1, j_jump), (0, 7), (1, 9)]
    fd = gradient_fd(sysd, psi0, tgt, u, T, paths, entries)
    ad = np.array([g[i, j] for i, j in entries])
    assert np.max(np.abs(ad - fd)) < 1e-9


def _cascade_case(M=3, nt=30, seed=2):
    w = config_workload("chain2_fock2", M=M, nt=nt, seed=seed)
    sysd = System.from_sparse(w.H0, w.H_ctrl, w.L_jump)
    return w, sysd


def test_replay_reproduces_mcwf_pass():
    w, sysd = _cascade_case()
    res = krotov.plain_forward(sysd, w.psi0, w.psi_tgt, w.u0, w.T, w.M, w.seed, 0)
    assert len(res.records) > 0
    paths = paths_from_records(res.records, w.M)
    J, tau = replay_functional(sysd, w.psi0, w.psi_tgt, w.u0, w.T, paths)
    assert abs(J - res.J_T) < 1e-9
    assert np.max(np.abs(tau - res.tau)) < 1e-9


def test_adjoint_matches_finite_differences_on_cascade():
    w, sysd = _cascade_case()
    res = krotov.plain_forward(sysd, w.psi0, w.psi_tgt, w.u0, w.T, w.M, w.seed, 0)
    paths = paths_from_records(res.records, w.M)
    assert sum(len(p) for p in paths) > 0
    g = gradient_adjoint(sysd, w.psi0, w.psi_tgt, w.u0, w.T, paths)
    # entries in steps that hold a jump, and plain ones
    jump_steps = sorted({s for p in paths for s, _, _ in p})
    entries = [(i, j) for i in range(2) for j in jump_steps[:3]] + [(0, 0), (1, 5), (0, 29)]
    fd = gradient_fd(sysd, w.psi0, w.psi_tgt, w.u0, w.T, paths, entries)
    ad = np.array([g[i, j] for i, j in entries])
    scale = np.max(np.abs(g))
    assert scale > 1e-4
    assert np.max(np.abs(ad - fd)) <= 1e-7 * scale


def test_paths_from_records_orders_by_ordinal():
    recs = [Jump(1, 5, 0, 1, 0, 2.6), Jump(1, 2, 0, 0, 0, 1.1), Jump(0, 3, 1, 0, 0, 1.7),
            Jump(1, 2, 0, 0, 1, 9.9)]
    paths = paths_from_records(recs, 2)
    assert paths == [[(3, 1.7, 1)], [(2, 1.1, 0), (5, 2.6, 0)]]


def test_replay_with_several_jumps_in_one_step():
    """Long driven steps with several jumps each: the replay splits a step at every
    recorded time and must land on the MCWF pass's final states."""
    from workloads.cascade import CascadeSpec, G_LEVEL, basis_index, build_cascade
    spec = CascadeSpec(1, 3)
    H0, Hc, L = build_cascade(spec)
    sysd = System.from_sparse(H0, Hc, L)
    psi0 = np.zeros(spec.dim, complex)
    psi0[basis_index(spec, [G_LEVEL], [2])] = 1.0
    u = np.array([[0.9, 0.4]])
    T, M, seed = 16.0, 10, 7
    ens, _ = forward_pass(sysd, psi0, u, T, M, seed, 0)
    multi = {(r.traj, r.step) for r in ens.records
             if sum(1 for q in ens.records if (q.traj, q.step) == (r.traj, r.step)) > 1}
    assert len(multi) >= 2
    paths = paths_from_records(ens.records, M)
    tgt = ens.normalised()[0]
    _, tau = replay_functional(sysd, psi0, tgt, u, T, paths)
    ref = ens.normalised() @ tgt.conj()
    assert np.max(np.abs(tau - ref)) < 1e-9


def test_sparse_propagator_action_matches_dense():
    """The large-d route (expm_multiply on a sparse H_eff, and on Van Loan's block
    applied to [0; x]) agrees with the dense matrix exponential."""
    import scipy.sparse
    from oracle.gradient import propagator_derivative
    from oracle.mcwf import apply_propagator
    w = config_workload("chain2_fock2", M=1, nt=10, seed=3)
    sysd = System.from_sparse(w.H0, w.H_ctrl, w.L_jump)
    H = sysd.effective_hamiltonian([0.7, -0.4])
    x = np.random.default_rng(0).normal(size=w.dim) + 1j * np.random.default_rng(1).normal(size=w.dim)
    for direction in (0, 1):
        for tau in (0.05, 1.3):
            dense = apply_propagator(H, tau, direction, x)
            sparse = apply_propagator(scipy.sparse.csr_matrix(H), tau, direction, x)
            assert np.max(np.abs(dense - sparse)) < 1e-12 * np.max(np.abs(dense))
    for i in range(2):
        a = propagator_derivative(H, sysd.H_ctrl[i], 0.8, x)
        b = propagator_derivative(scipy.sparse.csr_matrix(H), sysd.H_ctrl[i], 0.8, x)
        assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_large_system_norm_conserved_without_dissipation():
    """Chain of 4 nodes (d = 1296, sparse route): no Lindblad operators, so the
    norm stays 1 through driven steps."""
    from oracle.mcwf import Ensemble
    w = config_workload("chain4_fock2", M=2, nt=4)
    sysd = System.from_sparse(w.H0, w.H_ctrl, [])
    assert w.dim == 1296
    ens = Ensemble(sysd, w.psi0, 2, 0, 0, 0)
    for j in range(3):
        ens.advance(j, 3.0 * w.u0[:, j] + 0.5, 0.4, 0.4 * j)
    n = np.einsum("kd,kd->k", ens.psi.conj(), ens.psi).real
    assert np.max(np.abs(n - 1.0)) < 1e-12
    assert abs(ens.psi[0] - w.psi0).max() > 1e-3  # the drive moved the state
