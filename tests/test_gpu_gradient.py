"""GPU parity of the pathwise gradient (jump record fixed) against the oracle.

The jump records fed to both sides come from the oracle's own forward pass.
Bars: FP64 -- J_T and overlaps within 1e-10, every gradient entry within
1e-9 of max |dJ_T/du|; FP32 bulk -- J_T within 1e-5, gradient within 1e-4 of
max |dJ_T/du|.  At the full workload size the gradient is checked against
central differences of the library's own replayed functional.
"""

import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import krotov as okrotov
from oracle.gradient import gradient_adjoint, paths_from_records, replay_functional
from parity import max_abs, oracle_system, say
from workloads import build_paper_model, config_workload
from workloads.cascade import (CascadeSpec, G_LEVEL, Workload, basis_index, build_cascade,
                               guess_pulses)

pytestmark = pytest.mark.gpu

J_TOL = 1e-10
G_RTOL = 1e-9


@pytest.fixture(scope="module")
def tk():
    from paper_1801_04382_amd import trajkrotov
    return trajkrotov


def to_tk_records(tk, recs):
    arr = np.zeros(len(recs), dtype=tk.JUMP_DTYPE)
    for q, r in enumerate(recs):
        arr[q] = (0, r.traj, r.step, r.op, r.ordinal, r.direction, 0, 0, r.t)
    return arr


def oracle_gradient(w, recs):
    sysd = oracle_system(w)
    paths = paths_from_records(recs, w.M)
    g = gradient_adjoint(sysd, w.psi0, w.psi_tgt, w.u0, w.T, paths)
    J, tau = replay_functional(sysd, w.psi0, w.psi_tgt, w.u0, w.T, paths)
    return J, tau, g


def oracle_forward_records(w):
    return okrotov.plain_forward(oracle_system(w), w.psi0, w.psi_tgt, w.u0, w.T, w.M,
                                 w.seed, 0).records


def paper_workload(M=5, nt=120, T=5.0, seed=3):
    H0, Hc, L, psi0, tgt = build_paper_model(2, delta=2.0)
    u0 = guess_pulses(2, nt, T, np.random.default_rng(seed), amplitude=3.0)
    return Workload("paper2", H0, Hc, L, psi0, tgt, T, nt, u0, np.ones((2, nt)),
                    np.full(2, 2.0), M, seed, 1)


def long_step_workload():
    """One driven node, two long steps: several jumps and many substeps per step."""
    spec = CascadeSpec(1, 3)
    H0, Hc, L = build_cascade(spec)
    psi0 = np.zeros(spec.dim, complex)
    psi0[basis_index(spec, [G_LEVEL], [2])] = 1.0
    tgt = np.ones(spec.dim, complex) / math.sqrt(spec.dim)
    u0 = np.array([[0.9, 0.4]])
    return Workload("long_steps", H0, Hc, L, psi0, tgt, 16.0, 2, u0, np.ones((1, 2)),
                    np.ones(1), 10, 7, 1)


def check_against_oracle(tk, w, precision="fp64", j_tol=J_TOL, g_rtol=G_RTOL):
    recs = oracle_forward_records(w)
    J_ref, tau_ref, g_ref = oracle_gradient(w, recs)
    with tk.Context(precision=precision) as ctx:
        ctx.load(w)
        J, tau, g = ctx.grad_pathwise(w.M, to_tk_records(tk, recs))
    scale = float(np.max(np.abs(g_ref)))
    err = max_abs(g, g_ref)
    say("  records", len(recs), "J gpu", J, "oracle", J_ref, "max|dg|", err, "scale", scale)
    assert scale > 0.0
    assert abs(J - J_ref) <= j_tol
    assert max_abs(tau, tau_ref) <= max(j_tol, 1e-10)
    assert err <= g_rtol * scale
    return len(recs)


@pytest.mark.parametrize("case", ["chain2_fock2", "chain2_fock2_strong", "paper2"])
def test_gradient_matches_oracle(tk, case):
    if case == "chain2_fock2":
        w = config_workload("chain2_fock2", M=6, nt=150, seed=1)
    elif case == "chain2_fock2_strong":
        w = config_workload("chain2_fock2", M=7, nt=97, seed=5)
        w = w.replace(u0=w.u0 * 1.5)  # stronger drive: one or two jumps per trajectory
    else:
        w = paper_workload(M=8, seed=4)
    say("grad", case, "d", w.dim, "M", w.M, "nt", w.nt)
    assert check_against_oracle(tk, w) > 0


def test_gradient_several_jumps_per_step_and_substeps(tk):
    w = long_step_workload()
    say("grad long steps", "d", w.dim, "M", w.M, "nt", w.nt)
    recs = oracle_forward_records(w)
    steps = [(r.traj, r.step) for r in recs]
    assert any(steps.count(s) > 1 for s in steps)
    check_against_oracle(tk, w)


def test_gradient_two_level_closed_form(tk):
    """H = u sigma_x / 2, |0> -> |1>, no dissipation: dJ/du_j = -sin(theta) dt / 2."""
    nt, T = 40, 3.0
    u = np.random.default_rng(4).uniform(0.1, 0.6, size=(1, nt))
    sx = sp.csr_matrix(np.array([[0, 0.5], [0.5, 0]], complex))
    with tk.Context(precision="fp64") as ctx:
        ctx.set_system(sp.csr_matrix((2, 2), dtype=complex), [sx], [])
        ctx.set_states(np.array([1, 0], complex), np.array([0, 1], complex))
        ctx.set_pulses(u, T)
        J, _, g = ctx.grad_pathwise(3, np.zeros(0, dtype=tk.JUMP_DTYPE))
    theta = float(np.sum(u) * T / nt)
    assert abs(J - (1 - math.sin(theta / 2) ** 2)) < 1e-13
    assert np.max(np.abs(g + math.sin(theta) * (T / nt) / 2)) < 1e-13


def test_gradient_fp32_form(tk):
    w = config_workload("chain2_fock2", M=6, nt=150, seed=1)
    say("grad fp32", "d", w.dim, "M", w.M, "nt", w.nt)
    check_against_oracle(tk, w, precision="fp32", j_tol=1e-5, g_rtol=1e-4)


def test_autograd_function_returns_library_gradient(tk):
    import torch
    from paper_1801_04382_amd.autograd import pathwise_functional
    w = config_workload("chain2_fock2", M=6, nt=150, seed=1)
    recs = to_tk_records(tk, oracle_forward_records(w))
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        J_ref, _, g_ref = ctx.grad_pathwise(w.M, recs)
        u = torch.tensor(w.u0, dtype=torch.float64, requires_grad=True)
        J = pathwise_functional(u, ctx, w.M, recs)
        (3.0 * J).backward()
    assert float(J.detach()) == J_ref
    assert np.array_equal(u.grad.numpy(), 3.0 * g_ref)


def test_gradient_full_size_against_finite_differences(tk):
    """chain2_fock3, M = 1024, nt = 2000: the replay reproduces the forward pass,
    and sampled gradient entries match central differences (h = 1e-4) of the
    library's replayed functional."""
    w = config_workload("chain2_fock3")
    say("grad full size", "d", w.dim, "M", w.M, "nt", w.nt)
    h = 1e-4
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        _, tau_fw, rec, n = ctx.propagate_forward(w.M, w.seed, 0, want_states=False,
                                                  rec_cap=8 * w.M)
        assert n == len(rec) and n > 0
        J, tau, g = ctx.grad_pathwise(w.M, rec)
        say("  records", n, "J", J, "max|dtau| vs forward", max_abs(tau, tau_fw))
        assert max_abs(tau, tau_fw) <= 1e-8
        scale = float(np.max(np.abs(g)))
        rng = np.random.default_rng(0)
        entries = [(int(rng.integers(0, 2)), int(rng.integers(0, w.nt))) for _ in range(5)]
        entries.append(tuple(int(x) for x in np.unravel_index(np.argmax(np.abs(g)), g.shape)))
        for i, j in entries:
            up, dn = w.u0.copy(), w.u0.copy()
            up[i, j] += h
            dn[i, j] -= h
            ctx.set_pulses(up, w.T, w.S, w.lam)
            Jp, _, _ = ctx.grad_pathwise(w.M, rec)
            ctx.set_pulses(dn, w.T, w.S, w.lam)
            Jm, _, _ = ctx.grad_pathwise(w.M, rec)
            fd = (Jp - Jm) / (2 * h)
            say("  entry", (i, j), "adjoint", g[i, j], "fd", fd)
            assert abs(fd - g[i, j]) <= 1e-6 * scale


def test_gradient_error_paths(tk):
    w = config_workload("chain2_fock2", M=4, nt=50, seed=1)
    rec = np.zeros(1, dtype=tk.JUMP_DTYPE)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        dt = w.T / w.nt
        rec[0] = (0, 4, 3, 0, 0, 0, 0, 0, 3.5 * dt)  # trajectory >= M
        with pytest.raises(tk.TkError) as e:
            ctx.grad_pathwise(w.M, rec)
        assert e.value.code == tk.TK_EINVAL
        rec[0] = (0, 1, 3, 0, 0, 0, 0, 0, 5.5 * dt)  # time outside its step
        with pytest.raises(tk.TkError) as e:
            ctx.grad_pathwise(w.M, rec)
        assert e.value.code == tk.TK_EINVAL
        rec[0] = (0, 9, 3, 0, 0, 1, 0, 0, 3.5 * dt)  # backward records are ignored
        J, _, g = ctx.grad_pathwise(w.M, rec)
        assert np.isfinite(J) and np.all(np.isfinite(g))


def test_autograd_on_device_tensors_uses_device_entry_points(tk):
    """Pulses on the GPU go through tk_set_pulses_dev / tk_grad_pathwise_dev on
    torch's current stream: J_T and the gradient equal the host path's bit for
    bit, and the gradient tensor stays on the device."""
    import torch
    from paper_1801_04382_amd.autograd import pathwise_functional
    w = config_workload("chain2_fock2", M=6, nt=150, seed=1)
    recs = to_tk_records(tk, oracle_forward_records(w))
    J_o, tau_o, g_o = oracle_gradient(w, oracle_forward_records(w))
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        J_ref, _, g_ref = ctx.grad_pathwise(w.M, recs)
        u = torch.tensor(w.u0, dtype=torch.float64, device="cuda:0", requires_grad=True)
        J = pathwise_functional(u, ctx, w.M, recs)
        (2.0 * J).backward()
        assert J.is_cuda and u.grad.is_cuda
        J_host, g_dev = float(J.detach().cpu()), u.grad.detach().cpu().numpy()
        # the device pulses became the context's pulses
        assert np.array_equal(ctx.get_pulses(), w.u0)
    assert J_host == J_ref
    assert np.array_equal(g_dev, 2.0 * g_ref)
    assert abs(J_host - J_o) <= J_TOL
    assert max_abs(g_ref, g_o) <= G_RTOL * float(np.max(np.abs(g_o)))


def test_device_pointer_entry_points_match_host_calls(tk):
    """tk_functional_dev, tk_krotov_iterate_dev and tk_get_pulses_dev with
    torch device tensors and a non-default stream give the host calls' values."""
    import torch
    w = config_workload("chain2_fock2", M=8, nt=120, seed=3)
    dev = torch.device("cuda:0")
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        J_h, tau_h = ctx.functional(w.M, w.seed, 0)
        Jk_h, _, _ = ctx.krotov_iterate(w.M, w.seed, 2, rec_cap=0)
        u_h = ctx.get_pulses()
        s = torch.cuda.Stream(device=dev)
        with torch.cuda.stream(s):
            u0 = torch.tensor(w.u0, dtype=torch.float64, device=dev)
            S = torch.tensor(w.S, dtype=torch.float64, device=dev)
            lam = torch.tensor(w.lam, dtype=torch.float64, device=dev)
            J = torch.full((1,), -1.0, dtype=torch.float64, device=dev)
            tau = torch.zeros(2 * w.M, dtype=torch.float64, device=dev)
            Jk = torch.zeros(3, dtype=torch.float64, device=dev)
            u_out = torch.zeros_like(u0)
            h = s.cuda_stream
            ctx.set_pulses_dev(w.nt, w.T, u0.data_ptr(), S.data_ptr(), lam.data_ptr(), h)
            ctx.functional_dev(w.M, w.seed, 0, J.data_ptr(), tau.data_ptr(), h)
            ctx.krotov_iterate_dev(w.M, w.seed, 2, Jk.data_ptr(), stream=h)
            ctx.get_pulses_dev(u_out.data_ptr(), h)
            got = (J.cpu().numpy(), tau.cpu().numpy(), Jk.cpu().numpy(), u_out.cpu().numpy())
    assert got[0][0] == J_h
    assert np.array_equal(got[1].view(np.complex128), tau_h)
    assert np.array_equal(got[2], Jk_h)
    assert np.array_equal(got[3], u_h)
