"""GPU parity of the batched form (many instances per launch) against the oracle.

Each instance of a batch is an independent optimisation whose random streams
carry its instance id; the oracle runs every instance on its own.  Bars as the
single-system tests: FP64 -- J_T and pulses within 1e-10 for every instance
and iteration; FP32 -- |dJ_T| <= 1e-4.  Instance isolation is bit-exact: an
instance gives identical pulses alone and inside a larger batch.
"""

import numpy as np
import pytest

from oracle import krotov as okrotov
from parity import max_abs, oracle_system, say
from workloads import batch_instances, build_paper_model, config_workload
from workloads.cascade import Workload, guess_pulses

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def tk():
    from paper_1801_04382_amd import trajkrotov
    return trajkrotov


def paper_instance(M=5, nt=100, T=5.0, seed=4, instance=1):
    H0, Hc, L, psi0, tgt = build_paper_model(2, delta=2.0)
    u0 = guess_pulses(2, nt, T, np.random.default_rng(seed), amplitude=3.0)
    return Workload("paper2", H0, Hc, L, psi0, tgt, T, nt, u0, np.ones((2, nt)),
                    np.full(2, 2.0), M, seed, 2, instance=instance)


def mixed_instances():
    a = config_workload("chain2_fock2", M=6, nt=120, seed=1).replace(instance=0)
    b = paper_instance(instance=5)
    c = config_workload("chain2_fock3", M=4, nt=90, seed=2).replace(instance=2)
    d = config_workload("chain3_fock2", M=3, nt=24, seed=3).replace(instance=9)
    return [a, b, c, d]


def oracle_run(w, n_iter):
    return okrotov.optimise(oracle_system(w), w.psi0, w.psi_tgt, w.u0, w.S, w.lam, w.T, w.M,
                            w.seed, n_iter, instance=w.instance)


def test_batch_matches_oracle_per_instance(tk):
    ws = mixed_instances()
    with tk.Batch(precision="fp64") as b:
        for w in ws:
            say("batch add", w.name, "d", w.dim, "M", w.M, "nt", w.nt, "id", w.instance)
            b.add(w)
        J1 = b.krotov_iterate(2)          # guess, iteration 1 (tuned), iteration 2 (graph)
        J2 = b.krotov_iterate(1, first_iteration=3)
        info = b.info()
        pulses = [b.get_pulses(i) for i in range(len(ws))]
    say("  launch", info)
    assert info["autotuned"] == 1
    for i, w in enumerate(ws):
        ref = oracle_run(w, 3)
        J = np.concatenate([J1[i], J2[i]])
        say("  instance", i, "J gpu", J.tolist(), "oracle", ref.J_T)
        assert max_abs(J, ref.J_T) <= TOL
        assert max_abs(pulses[i], ref.u[-1]) <= TOL


def test_batch_instance_isolation_is_bit_exact(tk):
    ws = mixed_instances()
    target = ws[2]
    with tk.Batch(precision="fp64") as b:
        b.add(target)
        J_alone = b.krotov_iterate(2)
        u_alone = b.get_pulses(0)
    with tk.Batch(precision="fp64") as b:
        for w in (ws[1], ws[0], target, ws[3]):
            b.add(w)
        J_all = b.krotov_iterate(2)
        u_all = b.get_pulses(2)
    assert np.array_equal(J_alone[0], J_all[2])
    assert np.array_equal(u_alone, u_all)


def test_batch_agrees_with_single_system_path(tk):
    w = config_workload("chain2_fock2", M=16, nt=200, seed=2)
    with tk.Batch(precision="fp64") as b:
        b.add(w)
        Jb = b.krotov_iterate(3)[0]
        ub = b.get_pulses(0)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        Js, _, _ = ctx.krotov_iterate(w.M, w.seed, 3, rec_cap=0)
        us = ctx.get_pulses()
    say("batch vs single: max|dJ|", max_abs(Jb, Js), "max|du|", max_abs(ub, us))
    assert max_abs(Jb, Js) <= 1e-12
    assert max_abs(ub, us) <= 1e-12


def test_batch_fp32_form_against_oracle(tk):
    """All four mixed instances in FP32, the d = 216 one (one-wave, four rows
    per lane) included."""
    ws = mixed_instances()
    with tk.Batch(precision="fp32") as b:
        for w in ws:
            b.add(w)
        J = b.krotov_iterate(2)
    for i, w in enumerate(ws):
        ref = oracle_run(w, 2)
        say("  fp32 instance", i, "max|dJ|", max_abs(J[i], ref.J_T))
        assert max_abs(J[i], ref.J_T) <= 1e-4


def test_batch_of_uneven_instances_at_scale(tk):
    """Eight instances of the batching workload (chains of 2, 3 or 4 nodes --
    this draw has four d = 1296 instances, run by the eight-wave kernels with
    costate segments --, M in [64, 2048], nt in [500, 4000]), FP32, two
    iterations: every J_T is a valid fidelity error, and the two d = 36
    instances of the draw (M = 675, nt = 643 and M = 96, nt = 1113) agree with
    the oracle's own runs of them (stored by tests/golden/make_golden.py)."""
    import os
    ws = batch_instances(8, seed=0, nodes=(2, 3, 4))
    with tk.Batch(precision="fp32") as b:
        for w in ws:
            b.add(w)
        J = b.krotov_iterate(2)
        info = b.info()
        u = {i: b.get_pulses(i) for i in (1, 2)}
    say("  uneven batch", [(w.dim, w.M, w.nt) for w in ws], info)
    assert info["multiwave_instances"] == sum(1 for w in ws if w.dim == 1296)
    assert np.all(np.isfinite(J)) and np.all(J >= 0.0) and np.all(J <= 1.0 + 1e-12)
    g = dict(np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                  "batch_seed0_inst1_2.npz")))
    for i in (1, 2):
        assert ws[i].dim == 36
        say("  instance", i, "J gpu", J[i].tolist(), "oracle", g[f"J{i}"].tolist())
        assert max_abs(J[i], g[f"J{i}"]) <= 1e-4
        assert max_abs(u[i], g[f"u{i}"][-1]) <= 1e-4


def test_batch_error_paths(tk):
    w = config_workload("chain2_fock2", M=4, nt=50, seed=1)
    with tk.Batch(precision="fp64") as b:
        with pytest.raises(tk.TkError) as e:
            b.krotov_iterate(1)
        assert e.value.code == tk.TK_ESTATE
        b.add(w, instance_id=3)
        with pytest.raises(tk.TkError) as e:
            b.add(w, instance_id=3)
        assert e.value.code == tk.TK_EINVAL
        b.krotov_iterate(1)
        with pytest.raises(tk.TkError) as e:
            b.krotov_iterate(1, first_iteration=5)
        assert e.value.code == tk.TK_ESTATE
        with pytest.raises(tk.TkError) as e:
            b.add(w, instance_id=4)
        assert e.value.code == tk.TK_ESTATE


def test_batch_multiwave_segments_match_oracle(tk):
    """d = 216 in FP64 runs the two-wave batched kernels, whose Krotov pass
    recomputes the costates segment by segment (64 steps) from the backward
    pass's checkpoints: nt = 150 spans two full segments and a ragged one.  J_T
    and pulses against the oracle at the FP64 bars, beside a one-wave instance."""
    big = config_workload("chain3_fock2", M=3, nt=150, seed=5).replace(instance=7)
    small = config_workload("chain2_fock2", M=4, nt=70, seed=1).replace(instance=2)
    with tk.Batch(precision="fp64") as b:
        b.add(big)
        b.add(small)
        J = b.krotov_iterate(2)
        u_big = b.get_pulses(0)
        u_small = b.get_pulses(1)
    for w, Jw, uw in ((big, J[0], u_big), (small, J[1], u_small)):
        ref = oracle_run(w, 2)
        say("  segments", w.name, "d", w.dim, "nt", w.nt, "J gpu", Jw.tolist(), "oracle", ref.J_T)
        assert max_abs(Jw, ref.J_T) <= TOL
        assert max_abs(uw, ref.u[-1]) <= TOL


def test_batch_chain_of_four_nodes_fp32(tk):
    """d = 1296 (eight-wave teams, costate segments) in an FP32 batch: J_T
    against the oracle at the FP32 bar, and pulses against the single-system
    path (same kernels for the step; only the summation order of the update
    differs)."""
    w = config_workload("chain4_fock2", M=4, nt=70, seed=1).replace(instance=0)
    ref = oracle_run(w, 1)
    with tk.Batch(precision="fp32") as b:
        b.add(w)
        J = b.krotov_iterate(1)[0]
        ub = b.get_pulses(0)
    with tk.Context(precision="fp32") as ctx:
        ctx.load(w)
        Js, _, _ = ctx.krotov_iterate(w.M, w.seed, 1, rec_cap=0)
        us = ctx.get_pulses()
    say("  d=1296 batch J", J.tolist(), "single", Js.tolist(), "oracle", ref.J_T,
        "max|du| batch-single", max_abs(ub, us))
    assert max_abs(J, ref.J_T) <= 1e-4
    assert max_abs(J, Js) <= 1e-10
    assert max_abs(ub, us) <= 1e-10
