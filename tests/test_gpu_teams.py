"""GPU parity of multi-wave teams: one trajectory advanced by G wavefronts.

G = 2 is forced on the small workload (TK_VARIANT) and checked against the
oracle at the FP64 bars of the one-wave tests; the chain of 4 nodes
(d = 1296) selects the 8-wave FP32 shape and is checked at the FP32 bars.
"""

import numpy as np
import pytest

from oracle import krotov as okrotov
from oracle.gradient import gradient_adjoint, paths_from_records, replay_functional
from parity import (compare_records, gpu_records, max_abs, oracle_records, oracle_system,
                    say)
from workloads import config_workload

pytestmark = pytest.mark.gpu

TOL = 1e-10


def t_tol(w):
    """FP64 jump times: within 1e-10 of the step length."""
    return 1e-10 * w.T / w.nt


@pytest.fixture(scope="module")
def tk():
    from paper_1801_04382_amd import trajkrotov
    return trajkrotov


def to_tk_records(tk, recs):
    arr = np.zeros(len(recs), dtype=tk.JUMP_DTYPE)
    for q, r in enumerate(recs):
        arr[q] = (0, r.traj, r.step, r.op, r.ordinal, r.direction, 0, 0, r.t)
    return arr


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_two_wave_team_matches_oracle(tk, monkeypatch, precision):
    monkeypatch.setenv("TK_VARIANT", f"{precision} R=1 WS=4 NC=2 G=2")
    w = config_workload("chain2_fock2", M=8, nt=300, seed=2)
    say("G=2", precision, "d", w.dim, "M", w.M, "nt", w.nt)
    sysd = oracle_system(w)
    ref = okrotov.optimise(sysd, w.psi0, w.psi_tgt, w.u0, w.S, w.lam, w.T, w.M, w.seed, 3)
    fw = ref.passes[0]  # the guess pass (iteration 0)
    paths = paths_from_records(fw.records, w.M)
    g_ref = gradient_adjoint(sysd, w.psi0, w.psi_tgt, w.u0, w.T, paths)
    fp64 = precision == "fp64"
    with tk.Context(precision=precision) as ctx:
        ctx.load(w)
        assert "G=2" in ctx.launch_info()["variant"]
        psiT, tau, rec, n = ctx.propagate_forward(w.M, w.seed, 0)
        compare_records(gpu_records(rec), oracle_records(fw.records, 0),
                        t_tol(w) if fp64 else 1e-2 * w.T / w.nt)
        assert max_abs(psiT, fw.psi_hat_T) <= (TOL if fp64 else 1e-5)
        _, _, g = ctx.grad_pathwise(w.M, to_tk_records(tk, fw.records))
        ctx.load(w)
        J, _, _ = ctx.krotov_iterate(w.M, w.seed, 3)
        u = ctx.get_pulses()
    say("  J gpu", J.tolist(), "oracle", ref.J_T, "max|dg|", max_abs(g, g_ref))
    assert max_abs(J, ref.J_T) <= (TOL if fp64 else 1e-4)
    assert max_abs(u, ref.u[-1]) <= (TOL if fp64 else 1e-4)
    assert max_abs(g, g_ref) <= (1e-9 if fp64 else 1e-4) * np.max(np.abs(g_ref))


def test_chain_of_four_nodes_fp32(tk):
    """d = 1296 (8-wave teams): forward records and overlaps, one Krotov
    iteration and the pathwise gradient against the oracle (FP32 bars)."""
    w = config_workload("chain4_fock2", M=4, nt=30, seed=1)
    say("d=1296", "M", w.M, "nt", w.nt)
    sysd = oracle_system(w)
    ref = okrotov.optimise(sysd, w.psi0, w.psi_tgt, w.u0, w.S, w.lam, w.T, w.M, w.seed, 1)
    fw = ref.passes[0]  # the guess pass (iteration 0)
    paths = paths_from_records(fw.records, w.M)
    g_ref = gradient_adjoint(sysd, w.psi0, w.psi_tgt, w.u0, w.T, paths)
    J_ref, _ = replay_functional(sysd, w.psi0, w.psi_tgt, w.u0, w.T, paths)
    with tk.Context(precision="fp32") as ctx:
        ctx.load(w)
        info = ctx.launch_info()
        say("  variant", info["variant"])
        assert "G=8" in info["variant"]
        psiT, tau, rec, n = ctx.propagate_forward(w.M, w.seed, 0)
        say("  records gpu", n, "oracle", len(fw.records))
        compare_records(gpu_records(rec), oracle_records(fw.records, 0), 1e-2 * w.T / w.nt)
        assert max_abs(tau, fw.tau) <= 1e-5
        Jg, _, g = ctx.grad_pathwise(w.M, to_tk_records(tk, fw.records))
        ctx.load(w)
        J, _, _ = ctx.krotov_iterate(w.M, w.seed, 1)
    say("  J gpu", J.tolist(), "oracle", ref.J_T, "grad J", Jg, J_ref, "max|dg|",
        max_abs(g, g_ref), "scale", np.max(np.abs(g_ref)))
    assert max_abs(J, ref.J_T) <= 1e-4
    assert abs(Jg - J_ref) <= 1e-5
    assert max_abs(g, g_ref) <= 1e-4 * np.max(np.abs(g_ref))


def test_two_wave_shape_selected_for_d216_fp64(tk):
    """d = 216 in FP64 selects the 2-wave, 2-rows-per-lane shape (the 4-rows
    one spills registers): records, a Krotov iteration and the gradient against
    the oracle at the FP64 bars."""
    w = config_workload("chain3_fock2", M=2, nt=16, seed=2)
    say("d=216 fp64", "M", w.M, "nt", w.nt)
    sysd = oracle_system(w)
    ref = okrotov.optimise(sysd, w.psi0, w.psi_tgt, w.u0, w.S, w.lam, w.T, w.M, w.seed, 1)
    fw = ref.passes[0]
    paths = paths_from_records(fw.records, w.M)
    g_ref = gradient_adjoint(sysd, w.psi0, w.psi_tgt, w.u0, w.T, paths)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        assert ctx.launch_info()["variant"] == "fp64 R=2 WS=5/2 NC=3 G=2"
        psiT, tau, rec, n = ctx.propagate_forward(w.M, w.seed, 0)
        compare_records(gpu_records(rec), oracle_records(fw.records, 0), t_tol(w))
        assert max_abs(psiT, fw.psi_hat_T) <= TOL
        _, _, g = ctx.grad_pathwise(w.M, to_tk_records(tk, fw.records))
        ctx.load(w)
        J, _, _ = ctx.krotov_iterate(w.M, w.seed, 1)
        u = ctx.get_pulses()
    say("  J gpu", J.tolist(), "oracle", ref.J_T, "records", n)
    assert max_abs(J, ref.J_T) <= TOL
    assert max_abs(u, ref.u[-1]) <= TOL
    assert max_abs(g, g_ref) <= 1e-9 * max(np.max(np.abs(g_ref)), 1e-12)
