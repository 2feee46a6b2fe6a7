"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars (FP64 GPU form): discrete jump records identical (trajectory, step,
operator, ordinal, direction) with jump times within 1e-10 dt; states, overlaps,
costates, J_T and pulses within 1e-10 (absolute, states normalised).
FP32 form: records identical on these seeds, states within 1e-5, |dJ_T| <= 1e-4.
"""

import numpy as np
import pytest

from oracle import krotov as okrotov
from oracle.mcwf import System, backward_pass
from parity import (compare_records, gpu_records, max_abs, oracle_records, oracle_system,
                    say)
from workloads import build_paper_model, config_workload
from workloads.cascade import CascadeSpec, Workload, build_cascade, guess_pulses, initial_state

pytestmark = pytest.mark.gpu

T_TOL_DT = 1e-10  # jump times: within 1e-10 of the step length
STATE_TOL = 1e-10


def t_tol(w):
    return T_TOL_DT * w.T / w.nt


@pytest.fixture(scope="module")
def tk():
    from paper_1801_04382_amd import trajkrotov
    return trajkrotov


def small_workload(M=8, nt=500, seed=0):
    return config_workload("chain2_fock2", M=M, nt=nt, seed=seed)


def paper_workload(M=6, nt=200, T=5.0, seed=3):
    H0, Hc, L, psi0, tgt = build_paper_model(2, delta=2.0)
    rng = np.random.default_rng(seed)
    u0 = guess_pulses(2, nt, T, rng, amplitude=3.0)
    return Workload("paper2", H0, Hc, L, psi0, tgt, T, nt, u0, np.ones((2, nt)),
                    np.full(2, 2.0), M, seed, 3)


def run_oracle_forward(w, u=None, M=None, iteration=0, trajectories=None):
    sysd = oracle_system(w)
    u = w.u0 if u is None else u
    return okrotov.plain_forward(sysd, w.psi0, w.psi_tgt, u, w.T, w.M if M is None else M,
                                 w.seed, iteration)


@pytest.mark.parametrize("case", ["chain2_fock2", "chain2_fock2_ragged", "paper2"])
def test_forward_pass_matches_oracle(tk, case):
    if case == "chain2_fock2":
        w = small_workload()
    elif case == "chain2_fock2_ragged":
        w = small_workload(M=13, nt=137, seed=5)
        w = w.replace(u0=w.u0 * 3.0)  # stronger drive: more jumps
    else:
        w = paper_workload()
    say("forward", case, "d", w.dim, "M", w.M, "nt", w.nt)
    ref = run_oracle_forward(w)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        psiT, tau, rec, n = ctx.propagate_forward(w.M, w.seed, 0)
    say("  records gpu", n, "oracle", len(ref.records))
    assert n > 0
    dt = compare_records(gpu_records(rec), oracle_records(ref.records, 0), t_tol(w))
    assert max_abs(psiT, ref.psi_hat_T) <= STATE_TOL
    assert max_abs(tau, ref.tau) <= STATE_TOL
    say("  max |dt*|", dt, "max |dpsi|", max_abs(psiT, ref.psi_hat_T))


@pytest.mark.parametrize("case", ["chain2_fock2", "paper2"])
def test_backward_pass_matches_oracle(tk, case):
    w = small_workload(M=8, nt=300, seed=2) if case == "chain2_fock2" else paper_workload()
    say("backward", case, "d", w.dim, "M", w.M, "nt", w.nt)
    sysd = oracle_system(w)
    fw = run_oracle_forward(w)
    chi_ref, brec = okrotov.costates(sysd, w.psi_tgt, fw.tau, w.u0, w.T, w.M, w.seed, 1)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        _, tau, _, _ = ctx.propagate_forward(w.M, w.seed, 0)
        assert max_abs(tau, fw.tau) <= STATE_TOL
        rec, n = ctx.propagate_backward(w.M, w.seed, 1)
        worst = 0.0
        for j in sorted({0, 1, w.nt // 3, w.nt // 2, w.nt - 2, w.nt - 1}):
            chi = ctx.get_costate(j, w.M)
            worst = max(worst, max_abs(chi, chi_ref[j]))
    say("  records gpu", n, "oracle", len(brec), "max |dchi|", worst)
    compare_records(gpu_records(rec), oracle_records(brec, 1), t_tol(w))
    assert worst <= STATE_TOL


def _oracle_optimise(w, n_iter):
    return okrotov.optimise(oracle_system(w), w.psi0, w.psi_tgt, w.u0, w.S, w.lam, w.T, w.M,
                            w.seed, n_iter)


@pytest.mark.parametrize("case,n_iter", [("chain2_fock2", 10), ("paper2", 3)])
def test_krotov_iterations_match_oracle(tk, case, n_iter):
    """The full small workload: 2 nodes, cavity at 2 levels, M = 8, nt = 500."""
    w = small_workload() if case == "chain2_fock2" else paper_workload()
    say("krotov", case, "iterations", n_iter)
    ref = _oracle_optimise(w, n_iter)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        J, rec, n = ctx.krotov_iterate(w.M, w.seed, n_iter)
        u = ctx.get_pulses()
    say("  J gpu", J[:4], "... oracle", ref.J_T[:4])
    assert max_abs(J, ref.J_T) <= STATE_TOL
    assert max_abs(u, ref.u[-1]) <= STATE_TOL
    assert np.abs(ref.u[-1] - ref.u[0]).max() > 1e-6  # the pulses did move
    ref_rec = oracle_records(ref.passes[0].records, 0)
    for it in range(1, n_iter + 1):
        ref_rec += oracle_records(ref.backward_records[it - 1], it)
        ref_rec += oracle_records(ref.passes[it].records, it)
    compare_records(gpu_records(rec), sorted(ref_rec), t_tol(w))


def test_krotov_continuation_equals_single_call(tk):
    w = small_workload(M=6, nt=120, seed=4)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        J_all, _, _ = ctx.krotov_iterate(w.M, w.seed, 3)
        u_all = ctx.get_pulses()
        ctx.set_pulses(w.u0, w.T, w.S, w.lam)
        J0, _, _ = ctx.krotov_iterate(w.M, w.seed, 1)
        J1, _, _ = ctx.krotov_iterate(w.M, w.seed, 2, first_iteration=2)
        u_split = ctx.get_pulses()
    assert np.array_equal(np.concatenate([J0, J1]), J_all)
    assert np.array_equal(u_split, u_all)


def test_medium_krotov_matches_oracle(tk):
    """2 nodes, cavity at 3 levels (d = 81): two rows per lane."""
    w = config_workload("chain2_fock3", M=16, nt=200, seed=1)
    say("krotov d=81 M", w.M, "nt", w.nt)
    ref = _oracle_optimise(w, 2)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        J, rec, n = ctx.krotov_iterate(w.M, w.seed, 2)
        u = ctx.get_pulses()
    assert max_abs(J, ref.J_T) <= STATE_TOL
    assert max_abs(u, ref.u[-1]) <= STATE_TOL
    assert n == len(ref.passes[0].records) + sum(len(p.records) for p in ref.passes[1:]) + \
        sum(len(b) for b in ref.backward_records)


def test_fp32_form_against_oracle(tk):
    w = small_workload()
    say("fp32 krotov")
    ref = _oracle_optimise(w, 3)
    fw = ref.passes[0]
    with tk.Context(precision="fp32") as ctx:
        ctx.load(w)
        psiT, tau, rec, n = ctx.propagate_forward(w.M, w.seed, 0)
        J, krec, _ = ctx.krotov_iterate(w.M, w.seed, 3)
        u = ctx.get_pulses()
    # FP32 states carry ~1e-7 relative error; a jump time moves by that over the
    # norm's decay rate, so times are held to 1% of dt (discrete fields exact)
    worst_t = compare_records(gpu_records(rec), oracle_records(fw.records, 0), 1e-2 * w.dt)
    assert max_abs(psiT, fw.psi_hat_T) <= 1e-5
    assert max_abs(J, ref.J_T) <= 1e-4
    say("  fp32 |dJ|", max_abs(J, ref.J_T), "|du|", max_abs(u, ref.u[-1]), "max |dt*|", worst_t)


def test_no_dissipation_conserves_norm(tk):
    spec = CascadeSpec(2, 2)
    H0, Hc, _ = build_cascade(spec)
    w = small_workload(M=5, nt=80)
    w = w.replace(L_jump=[], H0=H0, H_ctrl=Hc)
    ref = run_oracle_forward(w)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        psiT, tau, rec, n = ctx.propagate_forward(w.M, w.seed, 0)
    assert n == 0 and not ref.records
    assert max_abs(psiT, ref.psi_hat_T) <= STATE_TOL


@pytest.mark.parametrize("M,nt", [(1, 1), (1, 7), (5, 1), (67, 3)])
def test_edge_shapes(tk, M, nt):
    w = small_workload(M=M, nt=nt, seed=9)
    w = w.replace(T=4.0 if nt > 1 else 0.2)  # nt = 3: steps of 4/3 need substeps
    ref = run_oracle_forward(w)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        psiT, tau, rec, n = ctx.propagate_forward(M, w.seed, 0)
        J, _ = ctx.functional(M, w.seed, 0)
    assert max_abs(psiT, ref.psi_hat_T) <= STATE_TOL
    assert abs(J - ref.J_T) <= STATE_TOL
    compare_records(gpu_records(rec), oracle_records(ref.records, 0), t_tol(w))


def test_single_node_system(tk):
    spec = CascadeSpec(1, 2)
    H0, Hc, L = build_cascade(spec)
    nt, T = 60, 6.0
    u0 = np.full((1, nt), 0.8)
    tgt = np.zeros(spec.dim, complex)
    tgt[2 * spec.n_fock] = 1.0
    w = Workload("node1", H0, Hc, L, initial_state(spec), tgt, T, nt, u0, np.ones((1, nt)),
                 np.ones(1), 40, 11, 1)
    ref = _oracle_optimise(w, 1)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        J, rec, n = ctx.krotov_iterate(w.M, w.seed, 1)
    assert max_abs(J, ref.J_T) <= STATE_TOL
    assert n > 5


def test_determinism(tk):
    w = config_workload("chain2_fock3", M=40, nt=100, seed=2)
    outs = []
    for _ in range(2):
        with tk.Context(precision="fp64") as ctx:
            ctx.load(w)
            J, rec, n = ctx.krotov_iterate(w.M, w.seed, 2)
            outs.append((J, ctx.get_pulses(), rec))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert np.array_equal(outs[0][2], outs[1][2])


def test_trajectory_record_independent_of_M(tk):
    """Counter-based streams: trajectory k's record does not depend on M."""
    w = small_workload(M=8, nt=200)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        psi_a, _, rec_a, _ = ctx.propagate_forward(8, w.seed, 0)
        psi_b, _, rec_b, _ = ctx.propagate_forward(67, w.seed, 0)
    assert np.array_equal(psi_a, psi_b[:8])
    sel = rec_b[rec_b["traj"] < 8]
    assert np.array_equal(rec_a, sel)


def test_error_paths(tk):
    w = small_workload(M=4, nt=50)
    with tk.Context(precision="fp64") as ctx:
        with pytest.raises(tk.TkError) as e:
            ctx.propagate_forward(4, 0, 0)
        assert e.value.code == tk.TK_ESTATE
        bad = w.H0.tolil()
        bad[0, 1] = 1.0  # not Hermitian
        with pytest.raises(tk.TkError) as e:
            ctx.set_system(bad.tocsr(), w.H_ctrl, w.L_jump)
        assert e.value.code == tk.TK_ENOTHERM
        ctx.set_system(w.H0, w.H_ctrl, w.L_jump)
        with pytest.raises(tk.TkError) as e:
            ctx.set_states(2 * w.psi0, w.psi_tgt)
        assert e.value.code == tk.TK_EINVAL
        ctx.set_states(w.psi0, w.psi_tgt)
        with pytest.raises(tk.TkError) as e:
            ctx.set_pulses(np.full_like(w.u0, np.nan), w.T)
        assert e.value.code == tk.TK_EINVAL
        ctx.set_pulses(w.u0 * 4, w.T, w.S, w.lam)
        with pytest.raises(tk.TkError) as e:
            ctx.propagate_forward(0, 0, 0)
        assert e.value.code == tk.TK_EINVAL
        _, _, _, n_all = ctx.propagate_forward(4, 0, 0)
        assert n_all > 1
        with pytest.raises(tk.TkError) as e:
            ctx.propagate_forward(4, 0, 0, rec_cap=1)
        assert e.value.code == tk.TK_ERECCAP
        with pytest.raises(tk.TkError) as e:
            ctx.krotov_iterate(4, 0, 1, first_iteration=5)
        assert e.value.code == tk.TK_ESTATE
        with pytest.raises(tk.TkError) as e:
            ctx.get_costate(0, 4)
        assert e.value.code == tk.TK_ESTATE


# ---------------------------------------------------------------------------
# full size: 2 nodes, cavity at 3 levels, M = 1024, nt = 2000 (sampled)
# ---------------------------------------------------------------------------

SAMPLED = [0, 511, 1023]


def _single_trajectory(w, k, u, iteration, direction, chi_start=None, tau_k=None):
    """Oracle for trajectory k alone: its stream depends only on (seed, k)."""
    from oracle.mcwf import Ensemble
    sysd = oracle_system(w)
    dt = w.T / w.nt
    start = w.psi0 if direction == 0 else w.psi_tgt / np.linalg.norm(w.psi_tgt)
    ens = Ensemble(sysd, start[None, :], 1, w.seed, iteration, direction)
    ens.streams[0] = type(ens.streams[0])(w.seed, k, iteration, direction)
    ens.r[0] = ens.streams[0].threshold(0)
    saved = {}
    steps = range(w.nt) if direction == 0 else range(w.nt - 1, -1, -1)
    for j in steps:
        ens.advance(j, u[:, j], dt, j * dt if direction == 0 else (j + 1) * dt)
        if direction == 1 and j in (0, w.nt // 2, w.nt - 1):
            saved[j] = tau_k * ens.normalised()[0]
    recs = [r.__class__(k, r.step, r.op, r.ordinal, r.direction, r.t) for r in ens.records]
    return ens.normalised()[0], recs, saved


def test_full_size_sampled_trajectories(tk):
    w = config_workload("chain2_fock3")
    assert (w.dim, w.M, w.nt) == (81, 1024, 2000)
    say("full size forward+backward, sampled", SAMPLED)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        psiT, tau, rec, n = ctx.propagate_forward(w.M, w.seed, 0)
        brec, bn = ctx.propagate_backward(w.M, w.seed, 1)
        chis = {j: ctx.get_costate(j, w.M) for j in (0, w.nt // 2, w.nt - 1)}
    say("  records", n, bn)
    for k in SAMPLED:
        psi_k, recs_k, _ = _single_trajectory(w, k, w.u0, 0, 0)
        tau_k = np.vdot(w.psi_tgt, psi_k)
        assert max_abs(psiT[k], psi_k) <= STATE_TOL
        assert abs(tau[k] - tau_k) <= STATE_TOL
        compare_records(gpu_records(rec[rec["traj"] == k]), oracle_records(recs_k, 0), t_tol(w))
        _, brecs_k, chi_k = _single_trajectory(w, k, w.u0, 1, 1, tau_k=tau_k)
        compare_records(gpu_records(brec[brec["traj"] == k]), oracle_records(brecs_k, 1), t_tol(w))
        for j, c in chi_k.items():
            assert max_abs(chis[j][k], c) <= STATE_TOL
    # properties over all trajectories
    assert np.allclose(np.linalg.norm(psiT, axis=1), 1.0, atol=1e-12)
    assert np.all(np.abs(tau) <= 1.0 + 1e-12)


def test_full_size_krotov_iteration_properties(tk):
    w = config_workload("chain2_fock3")
    say("full size one Krotov iteration")
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        J, rec, n = ctx.krotov_iterate(w.M, w.seed, 1)
        u = ctx.get_pulses()
        info = ctx.launch_info()
    say("  J", J, "launch", info)
    assert np.all((J >= 0) & (J <= 1))
    du = u - w.u0
    assert np.abs(du).max() > 0 and np.abs(du).max() < 0.1
    # update bound: |du_ij| <= S / lambda * max_k |<chi_k|H_i|psi_k>| <= ||H_i|| / lambda
    assert np.abs(du).max() <= 0.5 / w.lam[0] + 1e-12
