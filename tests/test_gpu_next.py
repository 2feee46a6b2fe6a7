"""GPU parity of the parts of the method beyond the independent-trajectory
pass: the pulse-noise measure of Sec. 3.4 and the cross-trajectory update of
Sec. 2.3, each against the FP64 oracle."""

import numpy as np
import pytest

from oracle import krotov as okrotov
from oracle.noise import pulse_noise
from parity import compare_records, gpu_records, max_abs, oracle_records, oracle_system, say
from workloads import build_paper_model, config_workload
from workloads.cascade import Workload, guess_pulses

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tk():
    from paper_1801_04382_amd import trajkrotov
    return trajkrotov


# ---------------------------------------------------------------------------
# pulse noise (Sec. 3.4)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n_ctrl,nt", [(1, 5), (2, 6), (3, 257), (4, 4000)])
def test_pulse_noise_matches_oracle(tk, n_ctrl, nt):
    rng = np.random.default_rng(nt)
    T = 50.0
    u = guess_pulses(n_ctrl, nt, T, rng) + 0.003 * rng.standard_normal((n_ctrl, nt))
    w = config_workload("chain2_fock2", M=2, nt=10)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        nu = ctx.pulse_noise(u, T)
    ref = pulse_noise(u, T)
    say("noise", n_ctrl, nt, nu.tolist(), ref.tolist())
    assert np.all(np.abs(nu - ref) <= 1e-12 * np.abs(ref) + 1e-15)


def test_pulse_noise_of_optimised_pulses_and_errors(tk):
    w = config_workload("chain2_fock2", M=8, nt=300, seed=1)
    ref = okrotov.optimise(oracle_system(w), w.psi0, w.psi_tgt, w.u0, w.S, w.lam, w.T, w.M,
                           w.seed, 2)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        ctx.krotov_iterate(w.M, w.seed, 2)
        nu = ctx.pulse_noise()  # the context's current (optimised) pulses
        with pytest.raises(tk.TkError) as e:
            ctx.pulse_noise(np.zeros((2, 4)), w.T)
        assert e.value.code == tk.TK_EINVAL
    nu_ref = pulse_noise(ref.u[-1], w.T)
    say("noise of optimised pulses", nu.tolist(), nu_ref.tolist())
    assert np.all(np.abs(nu - nu_ref) <= 1e-9 * np.abs(nu_ref))


# ---------------------------------------------------------------------------
# cross-trajectory update (Sec. 2.3, eq. cross_traj_update)
# ---------------------------------------------------------------------------

def _cross_oracle(w, n_iter):
    return okrotov.optimise_cross(oracle_system(w), w.psi0, w.psi_tgt, w.u0, w.S, w.lam, w.T,
                                  w.M, w.seed, n_iter, instance=w.instance)


def _cross_records(ref, n_iter):
    out = oracle_records(ref.passes[0].records, 0)
    for it in range(1, n_iter + 1):
        out += oracle_records(ref.backward_records[it - 1], it)
        out += oracle_records(ref.passes[it].records, it)
    return sorted(out)


@pytest.mark.parametrize("case,M,nt,n_iter", [("chain2_fock2", 8, 200, 3),
                                              ("chain2_fock3", 24, 120, 2),
                                              ("chain2_fock2", 67, 50, 1)])
def test_cross_update_matches_oracle(tk, case, M, nt, n_iter):
    w = config_workload(case, M=M, nt=nt, seed=2)
    say("cross", case, "d", w.dim, "M", M, "nt", nt)
    ref = _cross_oracle(w, n_iter)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        J, rec, n = ctx.krotov_iterate_cross(w.M, w.seed, n_iter)
        u = ctx.get_pulses()
    say("  J gpu", J.tolist(), "oracle", ref.J_T, "max|du|", max_abs(u, ref.u[-1]))
    assert np.abs(ref.u[-1] - ref.u[0]).max() > 1e-6  # the pulses moved
    assert max_abs(J, ref.J_T) <= 1e-10
    assert max_abs(u, ref.u[-1]) <= 1e-10
    compare_records(gpu_records(rec), _cross_records(ref, n_iter), 1e-10 * w.T / w.nt)


def test_cross_update_fp32_form(tk):
    w = config_workload("chain2_fock2", M=8, nt=200, seed=2)
    ref = _cross_oracle(w, 2)
    with tk.Context(precision="fp32") as ctx:
        ctx.load(w)
        J, rec, n = ctx.krotov_iterate_cross(w.M, w.seed, 2)
        u = ctx.get_pulses()
    say("cross fp32 J", J.tolist(), "oracle", ref.J_T)
    assert max_abs(J, ref.J_T) <= 1e-4
    assert max_abs(u, ref.u[-1]) <= 1e-4
    compare_records(gpu_records(rec), _cross_records(ref, 2), 1e-2 * w.T / w.nt)


def test_cross_update_paper_model(tk):
    """The paper's own model (complex control operators, d = 5)."""
    H0, Hc, L, psi0, tgt = build_paper_model(2, delta=2.0)
    nt, T = 150, 5.0
    u0 = guess_pulses(2, nt, T, np.random.default_rng(3), amplitude=3.0)
    w = Workload("paper2", H0, Hc, L, psi0, tgt, T, nt, u0, np.ones((2, nt)),
                 np.full(2, 2.0), 10, 3, 2)
    ref = _cross_oracle(w, 2)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        J, rec, n = ctx.krotov_iterate_cross(w.M, w.seed, 2)
        u = ctx.get_pulses()
    assert max_abs(J, ref.J_T) <= 1e-10
    assert max_abs(u, ref.u[-1]) <= 1e-10


def test_cross_update_many_trajectories(tk):
    """M = 1100 (waves keep two trajectories each; the Gram matrices sum 1100
    backward states on the matrix cores), against stored oracle values."""
    import os
    g = dict(np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                  "cross_chain2_fock2_M1100_nt60.npz")))
    w = config_workload("chain2_fock2", M=1100, nt=60)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        J, rec, n = ctx.krotov_iterate_cross(w.M, w.seed, 2)
        u = ctx.get_pulses()
        info = ctx.launch_info()
    say("cross M=1100 launch", info, "J", J.tolist(), "oracle", g["J"].tolist())
    assert info["traj_per_wave"] >= 2
    assert max_abs(J, g["J"]) <= 1e-10
    assert max_abs(u, g["u"][-1]) <= 1e-10


def test_cross_update_unsupported_shape(tk):
    w = config_workload("chain3_fock2", M=2, nt=8)
    with tk.Context(precision="fp64") as ctx:  # d = 216 FP64 runs two-wave teams
        ctx.load(w)
        with pytest.raises(tk.TkError) as e:
            ctx.krotov_iterate_cross(w.M, w.seed, 1)
        assert e.value.code == tk.TK_EUNSUPPORTED


# ---------------------------------------------------------------------------
# one step on the matrix cores versus the sparse step (the K7 measurement)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case,precision", [("chain2_fock2", "fp64"), ("chain2_fock3", "fp64"),
                                            ("chain2_fock2", "fp32"), ("chain2_fock3", "fp32"),
                                            ("chain3_fock2", "fp32")])
def test_dense_and_sparse_step_agree_with_exact_propagator(tk, case, precision):
    """Both methods give the K-term Taylor step; against the oracle's exact
    exp(-i dt H_eff) within the truncation bound x^(K+1)/(K+1)! e^x (x =
    ||H_eff|| dt) plus rounding, and against each other."""
    import math
    from oracle.mcwf import propagator
    w = config_workload(case, M=70, nt=400, seed=5)
    sysd = oracle_system(w)
    H = sysd.effective_hamiltonian(w.u0[:, 0])
    dt = w.T / w.nt
    K = 12 if precision == "fp64" else 6
    rng = np.random.default_rng(1)
    x = rng.standard_normal((w.M, w.dim)) + 1j * rng.standard_normal((w.M, w.dim))
    x /= np.linalg.norm(x, axis=1)[:, None]
    y_exact = x @ propagator(H, dt, 0).T
    xn = np.linalg.norm(H, 2) * dt
    trunc = xn ** (K + 1) / math.factorial(K + 1) * math.exp(xn)
    rnd = 1e-13 if precision == "fp64" else 1e-5
    with tk.Context(precision=precision) as ctx:
        ctx.load(w)
        ys, ms_s = ctx.step_bench(tk.TK_STEP_SPARSE, x, K, reps=2)
        yd, ms_d = ctx.step_bench(tk.TK_STEP_DENSE_MFMA, x, K, reps=2)
    say("step", case, precision, "sparse", max_abs(ys, y_exact), "dense", max_abs(yd, y_exact),
        "bound", trunc, "ms", ms_s, ms_d)
    assert max_abs(ys, y_exact) <= trunc + rnd
    assert max_abs(yd, y_exact) <= trunc + rnd
    assert max_abs(yd, ys) <= 2 * rnd


# ---------------------------------------------------------------------------
# density-matrix functional and Krotov's method in Liouville space (Sec. 2.2)
# ---------------------------------------------------------------------------

def _paper_w(nt=120, T=5.0, M=1):
    H0, Hc, L, psi0, tgt = build_paper_model(2, delta=2.0)
    u0 = guess_pulses(2, nt, T, np.random.default_rng(3), amplitude=3.0)
    return Workload("paper2", H0, Hc, L, psi0, tgt, T, nt, u0, np.ones((2, nt)),
                    np.full(2, 2.0), M, 3, 2)


@pytest.mark.parametrize("case", ["chain2_fock2", "chain2_fock3", "paper2"])
def test_density_functional_matches_oracle(tk, case):
    from oracle import density
    w = _paper_w() if case == "paper2" else config_workload(case, M=1, nt=150, seed=1)
    sysd = oracle_system(w)
    ref = density.rho_functional(density.forward_rho(sysd, w.psi0, w.u0, w.T), w.psi_tgt)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        J = ctx.density_functional()
    say("density J", case, J, ref)
    assert abs(J - ref) <= 1e-10


@pytest.mark.parametrize("case", ["chain2_fock2", "paper2"])
def test_density_krotov_matches_oracle(tk, case):
    from oracle import density
    w = _paper_w(nt=80) if case == "paper2" else config_workload(case, M=1, nt=80, seed=2)
    sysd = oracle_system(w)
    ref = density.optimise_rho(sysd, w.psi0, w.psi_tgt, w.u0, w.S, w.lam, w.T, 2)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        J = ctx.density_krotov_iterate(2)
        u = ctx.get_pulses()
    say("density krotov", case, J.tolist(), ref.J_T)
    assert np.abs(ref.u[-1] - ref.u[0]).max() > 1e-5
    assert max_abs(J, ref.J_T) <= 1e-10
    assert max_abs(u, ref.u[-1]) <= 1e-10


# ---------------------------------------------------------------------------
# the paper's own network optimised three ways (Sec. 3.2-3.4)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("method", ["independent", "cross", "density"])
def test_paper_model_runs_match_oracle(tk, method):
    """A short optimisation of the paper's two-node network (Delta = 100 g,
    T = 5) by the experiment runner: the density-matrix error recorded after
    each iteration and the final pulses against the oracle's own optimisation,
    and the noise measure of those pulses."""
    from oracle import density
    from oracle.noise import pulse_noise
    from oracle.mcwf import System
    from paper_1801_04382_amd.experiments import paper_model_problem, run_optimisation
    problem = paper_model_problem(2, T=5.0)
    H0, Hc, L, psi0, tgt, u0, S, lam, T = problem
    sysd = System.from_sparse(H0, Hc, L)
    n_iter, M = 3, 4
    r = run_optimisation(problem, method, M, n_iter)
    if method == "density":
        ref = density.optimise_rho(sysd, psi0, tgt, u0, S, lam, T, n_iter)
        J_ref, u_ref = ref.J_T, ref.u
    else:
        opt = okrotov.optimise if method == "independent" else okrotov.optimise_cross
        ref = opt(sysd, psi0, tgt, u0, S, lam, T, M, 0, n_iter)
        J_ref = [density.rho_functional(density.forward_rho(sysd, psi0, u, T), tgt)
                 for u in ref.u]
        u_ref = ref.u
        assert max_abs(r["J_traj"], ref.J_T) <= 1e-10
    say("paper model", method, "J_rho gpu", r["J_rho"], "oracle", J_ref)
    assert max_abs(r["J_rho"], J_ref) <= 1e-10
    assert max_abs(r["u"], u_ref[-1]) <= 1e-8 * np.abs(u_ref[-1]).max()
    assert np.allclose(r["nu"], pulse_noise(u_ref[-1], T), rtol=1e-8, atol=1e-12)
    assert r["J_rho"][-1] < r["J_rho"][0]
