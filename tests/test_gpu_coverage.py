"""GPU parity at the launch shapes the larger workloads run, against the oracle.

* The sequential Krotov pass with its full grid exchange: d = 81, M = 1024
  trajectories (256 blocks of 4 one-wave teams), and passes whose waves keep
  several trajectories' states in LDS (M = 1100: more trajectories than one
  cooperative launch holds one to a wave), in FP64 (d = 36) and in the FP32
  four-rows-per-lane shape of d = 216.
* Several jumps inside one substep, forward and backward.
* The pathwise gradient on the eight-wave d = 1296 path over many 64-step
  checkpoint segments, against the oracle's adjoint and its central
  differences.

Expected values of the cases whose oracle runs take minutes are stored under
tests/golden/ by tests/golden/make_golden.py (oracle only).  Bars: FP64 --
discrete record fields identical, jump times within 1e-10 dt, J_T and pulses
within 1e-10; FP32 -- record fields identical, times within 1e-2 dt, states
within 1e-5, |dJ_T| <= 1e-4; gradients within 1e-4 of max |dJ_T/du| (FP32).
"""

import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import krotov as okrotov
from oracle.mcwf import Ensemble, System, forward_pass
from parity import (compare_records, gpu_records, max_abs, oracle_records, oracle_system, say,
                    slow_crossing_allowance)
from workloads import config_workload
from workloads.cascade import Workload

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def tk():
    from paper_1801_04382_amd import trajkrotov
    return trajkrotov


def golden(name):
    path = os.path.join(GOLDEN, name + ".npz")
    if not os.path.exists(path):
        pytest.fail(f"missing {path}: run tests/golden/make_golden.py {name}")
    return dict(np.load(path))


def golden_records(g, iteration=None, direction=None, with_rate=False):
    out = []
    rates = g["rec_rate"] if "rec_rate" in g else np.full(len(g["rec_t"]), np.nan)
    for row, t, q in zip(g["rec_int"], g["rec_t"], rates):
        it, dr = int(row[0]), int(row[1])
        if iteration is not None and it != iteration:
            continue
        if direction is not None and dr != direction:
            continue
        out.append((it, dr, int(row[2]), int(row[3]), int(row[4]), int(row[5]), float(t), float(q)))
    out.sort()
    if with_rate:
        return [r[:7] for r in out], [r[7] for r in out]
    return [r[:7] for r in out]


def compare_golden_records(gpu, g, nt, t_tol):
    """GPU records against the stored oracle records: t_tol plus the
    slow-crossing allowance of each record (FP64 step tolerance)."""
    ref, rates = golden_records(g, with_rate=True)
    return compare_records(gpu, ref, t_tol, slow_crossing_allowance(rates, ref, nt))


def to_tk_records(tk, g):
    arr = np.zeros(len(g["rec_t"]), dtype=tk.JUMP_DTYPE)
    for q, (row, t) in enumerate(zip(g["rec_int"], g["rec_t"])):
        it, dr, k, n, j, op = (int(x) for x in row)
        arr[q] = (0, k, j, op, n, dr, it, 0, t)
    return arr


# ---------------------------------------------------------------------------
# Krotov pass: full grid exchange and several states per wave
# ---------------------------------------------------------------------------

def test_krotov_full_grid_exchange_matches_oracle(tk):
    """d = 81, M = 1024 (the headline launch: 256 blocks x 4 waves, one
    trajectory each), nt = 200, two iterations."""
    g = golden("krotov_chain2_fock3_M1024_nt200")
    w = config_workload("chain2_fock3", M=1024, nt=200)
    say("krotov full exchange d", w.dim, "M", w.M, "nt", w.nt)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        J, rec, n = ctx.krotov_iterate(w.M, w.seed, 2)
        u = ctx.get_pulses()
        info = ctx.launch_info()
    say("  launch", info, "J gpu", J.tolist(), "oracle", g["J"].tolist(), "records", n)
    assert (info["blocks"], info["waves_per_block"], info["traj_per_wave"]) == (256, 4, 1)
    assert max_abs(J, g["J"]) <= 1e-10
    assert max_abs(u, g["u"][-1]) <= 1e-10
    worst = compare_golden_records(gpu_records(rec), g, w.nt, 1e-10 * w.dt)
    say("  max |dJ|", max_abs(J, g["J"]), "max |du|", max_abs(u, g["u"][-1]), "max |dt*|", worst)


def test_krotov_several_states_per_wave_fp64(tk):
    """d = 36, M = 1100: each wave keeps two trajectories' states in LDS."""
    g = golden("krotov_chain2_fock2_M1100_nt60")
    w = config_workload("chain2_fock2", M=1100, nt=60)
    say("krotov traj_per_wave > 1, fp64 d", w.dim, "M", w.M)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        J, rec, n = ctx.krotov_iterate(w.M, w.seed, 2)
        u = ctx.get_pulses()
        info = ctx.launch_info()
    say("  launch", info, "J gpu", J.tolist(), "oracle", g["J"].tolist())
    assert info["traj_per_wave"] >= 2
    assert max_abs(J, g["J"]) <= 1e-10
    assert max_abs(u, g["u"][-1]) <= 1e-10
    compare_golden_records(gpu_records(rec), g, w.nt, 1e-10 * w.dt)


def _single_costate(w, k, u, iteration, tau_k, js):
    """Oracle costate of trajectory k alone (its stream depends only on seed, k)."""
    sysd = oracle_system(w)
    dt = w.T / w.nt
    start = w.psi_tgt / np.linalg.norm(w.psi_tgt)
    ens = Ensemble(sysd, start[None, :], 1, w.seed, iteration, 1)
    ens.streams[0] = type(ens.streams[0])(w.seed, k, iteration, 1)
    ens.r[0] = ens.streams[0].threshold(0)
    out = {}
    for j in range(w.nt - 1, -1, -1):
        ens.advance(j, u[:, j], dt, (j + 1) * dt)
        if j in js:
            out[j] = tau_k * ens.normalised()[0]
    return out


def test_fp32_four_rows_per_lane_shape_d216(tk):
    """C3's FP32 kernel shape (d = 216, four rows per lane, one wave): guess
    pass, costate pass and two Krotov iterations with M = 1100 (two states per
    wave in the Krotov pass)."""
    g = golden("krotov_chain3_fock2_M1100_nt40")
    w = config_workload("chain3_fock2", M=1100, nt=40, T=2.0)
    dt = w.T / w.nt
    say("fp32 d=216 M", w.M, "nt", w.nt)
    with tk.Context(precision="fp32") as ctx:
        ctx.load(w)
        assert ctx.launch_info()["variant"] == "fp32 R=4 WS=5/3 NC=3"
        psiT, tau, rec, n = ctx.propagate_forward(w.M, w.seed, 0)
        worst = compare_records(gpu_records(rec), golden_records(g, 0, 0), 1e-2 * dt)
        assert max_abs(psiT[g["sample_k"]], g["sample_psi"]) <= 1e-5
        # tau_k = <tgt|psi_hat_k> with ||tgt|| = 1: |dtau| <= ||dpsi||_2, which the
        # elementwise state bar bounds by sqrt(d) 1e-5
        assert max_abs(tau, g["tau0"]) <= 1e-5 * np.sqrt(w.dim)
        brec, bn = ctx.propagate_backward(w.M, w.seed, 1)
        compare_records(gpu_records(brec), golden_records(g, 1, 1), 1e-2 * dt)
        chis = {j: ctx.get_costate(j, w.M) for j in (0, w.nt // 2)}
        for k in (0, 1099):
            for j, c in _single_costate(w, k, w.u0, 1, g["tau0"][k], (0, w.nt // 2)).items():
                assert max_abs(chis[j][k], c) <= 1e-5
        ctx.load(w)
        J, krec, _ = ctx.krotov_iterate(w.M, w.seed, 2)
        u = ctx.get_pulses()
        info = ctx.launch_info()
    say("  launch", info, "J gpu", J.tolist(), "oracle", g["J"].tolist(), "fw records", n,
        "max |dt*|", worst)
    assert info["traj_per_wave"] >= 2
    assert max_abs(J, g["J"]) <= 1e-4
    assert max_abs(u, g["u"][-1]) <= 1e-4
    compare_records(gpu_records(krec), golden_records(g), 1e-2 * dt)


# ---------------------------------------------------------------------------
# several jumps inside one substep
# ---------------------------------------------------------------------------

def cavity_workload(M=256, nt=40, T=18.0, seed=21):
    """A lone cavity truncated at 3 levels starting with two photons, no drive:
    H_eff = -(i/2) a^+a has norm 1, so a step of 0.45 is a single substep, in
    which a photon decays at rate 2 and then the second at rate 1 -- many
    trajectories lose both photons inside one (sub)step."""
    a = sp.csr_matrix(np.diag([1.0, math.sqrt(2.0)], 1).astype(complex))
    H0 = sp.csr_matrix((3, 3), dtype=complex)
    Hc = [sp.csr_matrix((a + a.T).astype(complex))]
    psi0 = np.array([0, 0, 1], complex)
    tgt = np.array([1, 0, 1], complex) / math.sqrt(2.0)
    u0 = np.zeros((1, nt))
    return Workload("cavity2", H0, Hc, [a], psi0, tgt, T, nt, u0, np.ones((1, nt)),
                    np.ones(1), M, seed, 1)


def _same_step_pairs(recs, direction):
    seen = {}
    for r in recs:
        if r[1] == direction:
            seen[(r[2], r[4])] = seen.get((r[2], r[4]), 0) + 1
    return sum(1 for v in seen.values() if v >= 2)


def test_two_jumps_in_one_substep_forward_and_backward(tk):
    w = cavity_workload()
    dt = w.T / w.nt
    sysd = oracle_system(w)
    fw = okrotov.plain_forward(sysd, w.psi0, w.psi_tgt, w.u0, w.T, w.M, w.seed, 0)
    chi_ref, brec = okrotov.costates(sysd, w.psi_tgt, fw.tau, w.u0, w.T, w.M, w.seed, 1)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        psiT, tau, rec, n = ctx.propagate_forward(w.M, w.seed, 0)
        brec_g, bn = ctx.propagate_backward(w.M, w.seed, 1)
        chi0 = ctx.get_costate(0, w.M)
    ref_f = oracle_records(fw.records, 0)
    ref_b = oracle_records(brec, 1)
    pairs_f, pairs_b = _same_step_pairs(ref_f, 0), _same_step_pairs(ref_b, 1)
    say("two jumps per step: forward", pairs_f, "backward", pairs_b, "records", n, bn)
    assert pairs_f >= 5 and pairs_b >= 5
    worst_f = compare_records(gpu_records(rec), ref_f, 1e-10 * dt)
    worst_b = compare_records(gpu_records(brec_g), ref_b, 1e-10 * dt)
    assert max_abs(psiT, fw.psi_hat_T) <= 1e-10
    assert max_abs(chi0, chi_ref[0]) <= 1e-10
    say("  max |dt*| forward", worst_f, "backward", worst_b)


# ---------------------------------------------------------------------------
# pathwise gradient on the eight-wave d = 1296 path
# ---------------------------------------------------------------------------

def test_gradient_d1296_full_nt_against_oracle_adjoint(tk):
    """One trajectory of the four-node chain over the full nt = 4000 (63
    checkpoint segments of the eight-wave gradient kernel)."""
    g = golden("grad_chain4_fock2_nt4000_M1")
    w = config_workload("chain4_fock2", M=1, nt=4000)
    with tk.Context(precision="fp32") as ctx:
        ctx.load(w)
        assert "G=8" in ctx.launch_info()["variant"]
        J, tau, grad = ctx.grad_pathwise(w.M, to_tk_records(tk, g))
    scale = float(np.max(np.abs(g["g"])))
    say("grad d=1296 nt=4000: records", len(g["rec_t"]), "J", J, float(g["J"]), "max|dg|",
        max_abs(grad, g["g"]), "scale", scale)
    assert abs(J - float(g["J"])) <= 1e-5
    assert max_abs(grad, g["g"]) <= 1e-4 * scale


def test_gradient_d1296_segments_against_central_differences(tk):
    """d = 1296, M = 4, nt = 200 (four segments): the gradient against the
    oracle's adjoint and its central differences (h = 1e-4) on 16 entries,
    five at segment boundaries, with the oracle's jump records fixed."""
    g = golden("grad_chain4_fock2_nt200_M4")
    w = config_workload("chain4_fock2", M=4, nt=200, T=25.0)
    with tk.Context(precision="fp32") as ctx:
        ctx.load(w)
        J, tau, grad = ctx.grad_pathwise(w.M, to_tk_records(tk, g))
    scale = float(np.max(np.abs(g["g"])))
    ent = g["fd_entries"]
    fd_gpu = grad[ent[:, 0], ent[:, 1]]
    say("grad d=1296 nt=200: records", len(g["rec_t"]), "max|dg| adjoint",
        max_abs(grad, g["g"]), "fd", max_abs(fd_gpu, g["fd"]), "scale", scale)
    assert len(g["rec_t"]) >= 1
    assert abs(J - float(g["J"])) <= 1e-5
    assert max_abs(grad, g["g"]) <= 1e-4 * scale
    assert max_abs(fd_gpu, g["fd"]) <= 1e-4 * scale


# ---------------------------------------------------------------------------
# Krotov pass with its states in global memory (more trajectories than LDS holds)
# ---------------------------------------------------------------------------

def _krotov_run(tk, w, precision, n_iter):
    with tk.Context(precision=precision) as ctx:
        ctx.load(w)
        J, rec, n = ctx.krotov_iterate(w.M, w.seed, n_iter)
        return J, ctx.get_pulses(), gpu_records(rec), ctx.launch_info()


def test_krotov_states_in_global_memory_fp64_against_oracle(tk, monkeypatch):
    """d = 36, M = 1100 with the states in global memory (forced): the stored
    oracle values to 1e-10, and the same bits as the LDS form."""
    g = golden("krotov_chain2_fock2_M1100_nt60")
    w = config_workload("chain2_fock2", M=1100, nt=60)
    J0, u0, r0, _ = _krotov_run(tk, w, "fp64", 2)
    monkeypatch.setenv("TK_KROTOV_STATES", "global")
    J1, u1, r1, info = _krotov_run(tk, w, "fp64", 2)
    say("krotov states in global memory d", w.dim, "M", w.M, "launch", info)
    assert max_abs(J1, g["J"]) <= 1e-10
    assert max_abs(u1, g["u"][-1]) <= 1e-10
    compare_golden_records(r1, g, w.nt, 1e-10 * w.dt)
    assert np.array_equal(J0, J1) and np.array_equal(u0, u1) and r0 == r1


def test_krotov_states_in_global_memory_eight_wave_same_bits(tk, monkeypatch):
    """d = 1296 (eight-wave teams), M = 16: the global-memory form gives the
    bits of the LDS form."""
    w = config_workload("chain4_fock2", M=16, nt=20, T=0.25)
    J0, u0, r0, _ = _krotov_run(tk, w, "fp32", 2)
    monkeypatch.setenv("TK_KROTOV_STATES", "global")
    J1, u1, r1, _ = _krotov_run(tk, w, "fp32", 2)
    say("eight-wave global states: J", J0.tolist(), J1.tolist(), "records", len(r0))
    assert np.array_equal(J0, J1) and np.array_equal(u0, u1) and r0 == r1



def test_krotov_d1296_more_trajectories_than_lds_holds(tk):
    """d = 1296, M = 1100 (the LDS form holds about a thousand): one Krotov
    iteration against the stored oracle values (FP32 bars; the pulse update is
    checked relative to its own size)."""
    g = golden("krotov_chain4_fock2_M1100_nt80")
    w = config_workload("chain4_fock2", M=1100, nt=80, T=10.0, lam=0.05)
    J, u, rec, info = _krotov_run(tk, w, "fp32", 1)
    du_ref = g["u"][-1] - g["u"][0]
    say("krotov d=1296 M=1100: launch", info, "J gpu", J.tolist(), "oracle", g["J"].tolist(),
        "records", len(rec), "max |du| oracle", float(np.max(np.abs(du_ref))),
        "max |u - u_ref|", max_abs(u, g["u"][-1]))
    assert "G=8" in info["variant"]
    assert info["traj_per_wave"] * info["blocks"] >= w.M and info["traj_per_wave"] >= 5
    assert np.max(np.abs(du_ref)) > 1e-4
    assert max_abs(J, g["J"]) <= 1e-4
    assert max_abs(u, g["u"][-1]) <= 1e-3 * float(np.max(np.abs(du_ref)))
    compare_records(rec, golden_records(g), 1e-2 * w.dt)


# ---------------------------------------------------------------------------
# fewer static slots past row slot 0 (basis ordered by non-zeros per row)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,precision,uniform,light", [
    ("chain2_fock3", "fp64", "fp64 R=2 WS=4 NC=2", "fp64 R=2 WS=3/1 NC=2"),
    ("chain3_fock2", "fp32", "fp32 R=4 WS=6 NC=3", "fp32 R=4 WS=5/3 NC=3"),
    ("chain4_fock2", "fp32", "fp32 R=3 WS=9 NC=4 G=8", "fp32 R=3 WS=8/4 NC=4 G=8"),
])
def test_reordered_basis_shape_matches_uniform_shape(tk, monkeypatch, name, precision, uniform,
                                                     light):
    """The shape that puts the rows with the most non-zeros in row slot 0 (and
    fewer static slots in the others) runs the same trajectories as the uniform
    shape: final states (returned in the basis order), overlaps, records, a
    Krotov iteration and costates, to the rounding of the reordered sums."""
    w = config_workload(name, M=32, nt=40, T=2.0)
    out = {}
    for label, variant in (("uniform", uniform), ("light", light)):
        monkeypatch.setenv("TK_VARIANT", variant)
        with tk.Context(precision=precision) as ctx:
            ctx.load(w)
            assert ctx.launch_info()["variant"] == variant
            psiT, tau, rec, n = ctx.propagate_forward(w.M, w.seed, 0)
            brec, _ = ctx.propagate_backward(w.M, w.seed, 1)
            chi = ctx.get_costate(w.nt // 2, w.M)
            ctx.load(w)
            J, krec, _ = ctx.krotov_iterate(w.M, w.seed, 1)
            out[label] = (psiT, tau, gpu_records(rec), gpu_records(brec), chi, J,
                          ctx.get_pulses(), gpu_records(krec))
    a, b = out["uniform"], out["light"]
    tol = 1e-12 if precision == "fp64" else 1e-5
    say(name, precision, "max |dpsi|", max_abs(a[0], b[0]), "max |dchi|", max_abs(a[4], b[4]),
        "max |dJ|", max_abs(a[5], b[5]), "records", len(a[2]), len(a[7]))
    assert max_abs(a[0], b[0]) <= tol
    assert max_abs(a[1], b[1]) <= tol
    assert max_abs(a[4], b[4]) <= tol
    assert max_abs(a[5], b[5]) <= tol
    assert max_abs(a[6], b[6]) <= tol
    t_tol = (1e-10 if precision == "fp64" else 1e-2) * w.T / w.nt
    for ra, rb in ((a[2], b[2]), (a[3], b[3]), (a[7], b[7])):
        compare_records(rb, ra, t_tol)


def test_complex_controls_take_a_uniform_shape(tk):
    """Control operators with complex elements (the cascade's H_i conjugated by
    random diagonal phases: Hermitian, complex off-diagonal elements) never get
    a shape for real control elements: d = 81 runs the uniform shape, and two
    Krotov iterations match the oracle at the FP64 bars (the first update of
    this small draw is zero, the second is not)."""
    w = config_workload("chain2_fock3", M=4, nt=40, T=10.0, lam=0.05)
    rng = np.random.default_rng(5)
    ph = sp.diags(np.exp(1j * rng.uniform(0.0, 2.0 * np.pi, w.dim)))
    Hc = [sp.csr_matrix(ph @ H @ ph.conj().T) for H in w.H_ctrl]
    assert max(float(np.abs(H.data.imag).max()) for H in Hc) > 0.1
    w = w.replace(H_ctrl=Hc)
    n_iter = 2
    ref = okrotov.optimise(oracle_system(w), w.psi0, w.psi_tgt, w.u0, w.S, w.lam, w.T, w.M,
                           w.seed, n_iter)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        variant = ctx.launch_info()["variant"]
        J, rec, n = ctx.krotov_iterate(w.M, w.seed, n_iter)
        u = ctx.get_pulses()
    # oracle records with the norm's decay rate at each crossing
    runs = [(0, ref.passes[0].records)]
    for it in range(1, n_iter + 1):
        runs += [(it, ref.backward_records[it - 1]), (it, ref.passes[it].records)]
    pairs = sorted((((it, r.direction, r.traj, r.ordinal, r.step, r.op, r.t), r.rate)
                    for it, recs in runs for r in recs), key=lambda q: q[0])
    ref_rec = [q[0] for q in pairs]
    say("complex controls: variant", variant, "J gpu", J.tolist(), "oracle", list(ref.J_T),
        "records", n, len(ref_rec), "max |du|", float(np.abs(ref.u[-1] - ref.u[0]).max()))
    assert variant == "fp64 R=2 WS=4 NC=2"
    assert max_abs(J, ref.J_T) <= 1e-10
    assert max_abs(u, ref.u[-1]) <= 1e-10
    assert np.abs(ref.u[-1] - ref.u[0]).max() > 1e-3
    compare_records(gpu_records(rec), ref_rec, 1e-10 * w.T / w.nt,
                    slow_crossing_allowance([q[1] for q in pairs], ref_rec, w.nt))


# ---------------------------------------------------------------------------
# FP64 at d = 1296 (eight-wave teams; substeps short enough for the LDS)
# ---------------------------------------------------------------------------

def test_fp64_d1296_shape_against_oracle(tk):
    """The FP64 d = 1296 shape: one Krotov iteration of M = 1100 (states in
    global memory) against the stored oracle values at the FP64 bars.  Its
    series hold at most five terms, so its steps take ~20 substeps, each kept
    to 1e-15: the slow-crossing allowance of the jump times uses 2e-14 per step."""
    g = golden("krotov_chain4_fock2_M1100_nt80")
    w = config_workload("chain4_fock2", M=1100, nt=80, T=10.0, lam=0.05)
    J, u, rec, info = _krotov_run(tk, w, "fp64", 1)
    say("fp64 d=1296: launch", info, "J gpu", J.tolist(), "oracle", g["J"].tolist(),
        "max |du|", max_abs(u, g["u"][-1]), "records", len(rec))
    assert info["variant"] == "fp64 R=3 WS=8/4 NC=4 G=8"
    assert max_abs(J, g["J"]) <= 1e-10
    assert max_abs(u, g["u"][-1]) <= 1e-10
    ref, rates = golden_records(g, with_rate=True)
    worst = compare_records(rec, ref, 1e-10 * w.dt,
                            slow_crossing_allowance(rates, ref, w.nt, step_tol=2e-14))
    say("  max |dt*|", worst)
