"""Pins of the FP64 oracle against facts fixed outside it.

Each test checks the oracle against something it does not compute itself:
a library routine (NumPy's Philox), a closed form, an invariant, a textbook
limit, or the Lindblad master equation (whose integrator is pinned by its own
closed form below).
"""

import math

import numpy as np
import pytest
import scipy.optimize

from oracle import krotov, lindblad, philox
from oracle.mcwf import Ensemble, System, choose_operator, forward_pass, norm2
from workloads import build_paper_model
from workloads.cascade import (CascadeSpec, E_LEVEL, G_LEVEL, R_LEVEL, basis_index,
                               build_cascade, initial_state)


# ---------------------------------------------------------------------------
# Philox4x64-10 versus NumPy's implementation
# ---------------------------------------------------------------------------

def _numpy_block(counter, key):
    """NumPy advances the counter before producing a block: start one below."""
    v = sum(int(c) << (64 * i) for i, c in enumerate(counter))
    v = (v - 1) % (1 << 256)
    c = np.array([(v >> (64 * i)) & philox.MASK64 for i in range(4)], dtype=np.uint64)
    g = np.random.Philox(counter=c, key=np.array(key, dtype=np.uint64))
    return tuple(int(x) for x in g.random_raw(4))


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((7, 3, 1, 0), (12345, (5 << 32) | 99)),
    ((0, 2 ** 64 - 1, 0, 0), (2 ** 64 - 1, 1)),
    ((2 ** 64 - 1, 2 ** 64 - 1, 2 ** 64 - 1, 0), (3, 4)),
])
def test_philox_matches_numpy(counter, key):
    assert philox.block(counter, key) == _numpy_block(counter, key)


def test_philox_stream_layout():
    s = philox.TrajectoryStream(seed=11, trajectory=6, iteration=2, direction=1, instance=3)
    w = philox.block((4, 2, 1, 0), (11, (3 << 32) | 6))
    assert s.threshold(4) == (w[0] >> 11) * 2.0 ** -53
    assert s.choice(4) == (w[1] >> 11) * 2.0 ** -53
    u = [philox.to_unit(x) for x in (0, 2 ** 64 - 1, 2 ** 11)]
    assert u[0] == 0.0 and u[1] == 1.0 - 2.0 ** -53 and u[2] == 2.0 ** -53


# ---------------------------------------------------------------------------
# MCWF closed forms
# ---------------------------------------------------------------------------

def _single_cavity(n_fock=2):
    spec = CascadeSpec(1, n_fock)
    H0, Hc, L = build_cascade(spec)
    return spec, System.from_sparse(H0, Hc, L)


def test_single_cavity_norm_decay_and_jump_time():
    """One photon, atom in g, no drive: ||psi||^2 = exp(-kappa t), t* = -ln(r)/kappa."""
    spec, sysd = _single_cavity()
    psi0 = np.zeros(spec.dim, complex)
    psi0[basis_index(spec, [G_LEVEL], [1])] = 1.0
    T, nt, M, seed = 5.0, 10, 24, 3
    dt = T / nt
    ens = Ensemble(sysd, psi0, M, seed, 0, 0)
    jumped_at = {}
    for j in range(nt):
        ens.advance(j, [0.0], dt, j * dt)
        for rec in ens.records:
            jumped_at.setdefault(rec.traj, rec)
        for k in range(M):
            if k not in jumped_at:
                assert abs(norm2(ens.psi[k]) - math.exp(-(j + 1) * dt)) < 1e-13
    n_jumps = 0
    for k in range(M):
        r0 = philox.TrajectoryStream(seed, k, 0, 0).threshold(0)
        if r0 > math.exp(-T):
            rec = jumped_at[k]
            assert abs(rec.t - (-math.log(r0))) < 1e-11
            assert rec.step == int(-math.log(r0) // dt) and rec.ordinal == 0 and rec.op == 0
            n_jumps += 1
            # after the jump the cavity is empty and the state is dark
            ground = basis_index(spec, [G_LEVEL], [0])
            assert abs(abs(ens.psi[k][ground]) - 1.0) < 1e-12
        else:
            assert k not in jumped_at
    assert n_jumps >= 10


def test_two_jumps_inside_one_step():
    """Two photons decay in one long step: t1 = -ln r0 / 2, t2 = t1 - ln r1."""
    spec, sysd = _single_cavity(n_fock=3)
    psi0 = np.zeros(spec.dim, complex)
    psi0[basis_index(spec, [G_LEVEL], [2])] = 1.0
    T, M, seed = 40.0, 12, 5
    ens, _ = forward_pass(sysd, psi0, np.zeros((1, 1)), T, M, seed, 0)
    checked = 0
    for k in range(M):
        st = philox.TrajectoryStream(seed, k, 0, 0)
        t1 = -math.log(st.threshold(0)) / 2.0
        t2 = t1 - math.log(st.threshold(1))
        recs = [r for r in ens.records if r.traj == k]
        if t2 < T:
            assert [(r.step, r.ordinal) for r in recs] == [(0, 0), (0, 1)]
            assert abs(recs[0].t - t1) < 1e-11 and abs(recs[1].t - t2) < 1e-10
            checked += 1
    assert checked >= 8


def test_cascade_two_nodes_closed_form():
    """Photon in cavity 1 feeds cavity 2: c1 = e^{-t/2}, c2 = -t e^{-t/2} (kappa = 1).

    ||psi||^2 = e^{-t}(1 + t^2); the first jump takes both photon amplitudes to
    the empty network.  This fixes the cascade's direction and sign.
    """
    spec = CascadeSpec(2, 2)
    H0, Hc, L = build_cascade(spec)
    sysd = System.from_sparse(H0, Hc, L)
    i10 = basis_index(spec, [G_LEVEL, G_LEVEL], [1, 0])
    i01 = basis_index(spec, [G_LEVEL, G_LEVEL], [0, 1])
    i00 = basis_index(spec, [G_LEVEL, G_LEVEL], [0, 0])
    psi0 = np.zeros(spec.dim, complex)
    psi0[i10] = 1.0
    T, nt, M, seed = 6.0, 30, 16, 1
    dt = T / nt
    u = np.zeros((2, nt))
    ens, states = forward_pass(sysd, psi0, u, T, M, seed, 0, keep_states=True)
    f = lambda t: math.exp(-t) * (1 + t * t)
    first = {}
    for rec in ens.records:
        first.setdefault(rec.traj, rec)
    for k in range(M):
        r0 = philox.TrajectoryStream(seed, k, 0, 0).threshold(0)
        t_jump = first[k].t if k in first else T + 1
        for j in range(nt + 1):
            t = j * dt
            if t < t_jump:
                ref = np.zeros(spec.dim, complex)
                ref[i10], ref[i01] = 1.0, -t
                ref /= np.linalg.norm(ref)
                assert np.abs(states[j, k] - ref).max() < 1e-12
        if r0 > f(T):
            rec = first[k]
            # residual of the closed-form norm at the recorded time
            assert abs(f(rec.t) - r0) < 1e-13
            t_ref = scipy.optimize.brentq(lambda t: f(t) - r0, 0.0, T, xtol=1e-15)
            slope = math.exp(-t_ref) * (1 - t_ref) ** 2
            if slope > 1e-3:
                assert abs(rec.t - t_ref) < 1e-10
            assert abs(abs(ens.psi[k][i00]) - 1.0) < 1e-12
        else:
            assert k not in first


def test_norm_conserved_without_dissipation():
    spec = CascadeSpec(2, 2)
    H0, Hc, _ = build_cascade(spec)
    sysd = System.from_sparse(H0, Hc, [])
    rng = np.random.default_rng(0)
    u = rng.normal(0, 0.5, (2, 40))
    ens, _ = forward_pass(sysd, initial_state(spec), u, 8.0, 4, 0, 0)
    assert not ens.records
    for k in range(4):
        assert abs(norm2(ens.psi[k]) - 1.0) < 1e-12


def test_choose_operator_rule():
    d = 4
    L1 = np.zeros((d, d), complex); L1[0, 1] = 1.0
    L2 = np.zeros((d, d), complex); L2[0, 2] = 2.0
    psi = np.array([0, 1, 1, 0], complex) / math.sqrt(2)  # weights 0.5 and 2.0
    assert choose_operator(psi, [L1, L2], 0.0) == 0
    assert choose_operator(psi, [L1, L2], 0.199) == 0
    assert choose_operator(psi, [L1, L2], 0.2) == 1
    assert choose_operator(psi, [L1, L2], 0.999) == 1
    psi2 = np.array([0, 0, 1, 0], complex)
    assert choose_operator(psi2, [L1, L2], 0.0) == 1
    with pytest.raises(FloatingPointError):
        choose_operator(np.array([1, 0, 0, 0], complex), [L1, L2], 0.5)


# ---------------------------------------------------------------------------
# Lindblad integrator (closed form) and the trajectory ensemble against it
# ---------------------------------------------------------------------------

def test_lindblad_single_cavity_closed_form():
    spec, sysd = _single_cavity()
    i1 = basis_index(spec, [G_LEVEL], [1])
    i0 = basis_index(spec, [G_LEVEL], [0])
    rho0 = np.zeros((spec.dim, spec.dim), complex)
    rho0[i1, i1] = 1.0
    rhos = lindblad.propagate_rho(sysd, rho0, np.zeros((1, 8)), 4.0, keep=True)
    for j, rho in enumerate(rhos):
        t = j * 0.5
        assert abs(rho[i1, i1] - math.exp(-t)) < 1e-12
        assert abs(rho[i0, i0] - (1 - math.exp(-t))) < 1e-12
        assert abs(np.trace(rho) - 1) < 1e-12


def _ensemble_vs_lindblad(sysd, psi0, u, T, M, seed, tol_sigma=5.0):
    ens, _ = forward_pass(sysd, psi0, u, T, M, seed, 0)
    psi_hat = ens.normalised()
    rho_traj = np.einsum("ki,kj->ij", psi_hat, psi_hat.conj()) / M
    rho = lindblad.propagate_rho(sysd, np.outer(psi0, psi0.conj()), u, T)
    # per-entry standard error of the trajectory mean
    vals = np.einsum("ki,kj->kij", psi_hat, psi_hat.conj())
    se_re = vals.real.std(axis=0) / math.sqrt(M) + 1e-12
    se_im = vals.imag.std(axis=0) / math.sqrt(M) + 1e-12
    z_re = np.abs(rho_traj.real - rho.real) / se_re
    z_im = np.abs(rho_traj.imag - rho.imag) / se_im
    assert z_re.max() < tol_sigma and z_im.max() < tol_sigma, (z_re.max(), z_im.max())
    return ens, rho


def test_ensemble_matches_lindblad_single_node():
    spec, sysd = _single_cavity()
    u = np.full((1, 30), 0.8)
    ens, rho = _ensemble_vs_lindblad(sysd, initial_state(spec), u, 6.0, 3000, 7)
    assert len(ens.records) > 300  # the check is informative: many jumps happened
    assert rho[basis_index(spec, [R_LEVEL], [0]), basis_index(spec, [R_LEVEL], [0])].real > 0.1


def test_ensemble_matches_lindblad_two_channels():
    """Two nodes with separate decay channels exercise the operator choice."""
    spec = CascadeSpec(2, 2)
    H0, Hc, L = build_cascade(spec)
    from workloads.cascade import _embed, _local_ops
    a = _local_ops(2)["a"]
    Ls = [_embed(a, i, 2, spec.local_dim) for i in range(2)]
    sysd = System.from_sparse(H0, Hc, Ls)
    u = np.vstack([np.full(20, 0.9), np.full(20, 0.5)])
    ens, _ = _ensemble_vs_lindblad(sysd, initial_state(spec), u, 4.0, 800, 2)
    ops = {r.op for r in ens.records}
    assert ops == {0, 1}


def test_ensemble_matches_lindblad_paper_model():
    H0, Hc, L, psi0, tgt = build_paper_model(2, delta=2.0)
    sysd = System.from_sparse(H0, Hc, L)
    u = np.vstack([np.full(20, 1.5), np.full(20, -1.0)])
    _ensemble_vs_lindblad(sysd, psi0, u, 3.0, 1500, 4)


# ---------------------------------------------------------------------------
# costates: adjoint propagation conserves the overlap with the forward state
# ---------------------------------------------------------------------------

def test_backward_forward_overlap_is_conserved():
    """For jump-free trajectories <chi~(t)|psi~(t)> is independent of t.

    <exp(i H^+ dt) chi | psi> = <chi | exp(-i H dt) psi>: the backward
    propagator is the adjoint of the forward one, also for non-Hermitian H_eff.
    """
    spec = CascadeSpec(2, 2)
    H0, Hc, L = build_cascade(spec)
    sysd = System.from_sparse(H0, Hc, L)
    rng = np.random.default_rng(3)
    nt, T, M = 24, 3.0, 24
    dt = T / nt
    u = rng.normal(0.4, 0.3, (2, nt))
    chiT = rng.normal(size=spec.dim) + 1j * rng.normal(size=spec.dim)
    chiT /= np.linalg.norm(chiT)
    fw = Ensemble(sysd, initial_state(spec), M, 9, 0, 0)
    psi = [fw.psi.copy()]
    for j in range(nt):
        fw.advance(j, u[:, j], dt, j * dt)
        psi.append(fw.psi.copy())
    bw = Ensemble(sysd, chiT, M, 9, 1, 1)
    chi = [None] * (nt + 1)
    chi[nt] = bw.psi.copy()
    for j in range(nt - 1, -1, -1):
        bw.advance(j, u[:, j], dt, (j + 1) * dt)
        chi[j] = bw.psi.copy()
    jumped = {r.traj for r in fw.records} | {r.traj for r in bw.records}
    clean = [k for k in range(M) if k not in jumped]
    assert len(clean) >= 5
    for k in clean:
        ov = np.array([np.vdot(chi[j][k], psi[j][k]) for j in range(nt + 1)])
        assert np.abs(ov - ov[-1]).max() < 1e-12 * max(1.0, abs(ov[-1]))
        assert abs(ov[-1]) > 1e-3


# ---------------------------------------------------------------------------
# Krotov update: kappa = 0 limit against the gradient and monotonicity
# ---------------------------------------------------------------------------

def _unitary_problem():
    spec = CascadeSpec(2, 2)
    H0, Hc, _ = build_cascade(spec)
    sysd = System.from_sparse(H0, Hc, [])
    tgt = np.zeros(spec.dim, complex)
    tgt[basis_index(spec, [E_LEVEL, G_LEVEL], [0, 0])] = 1.0
    tgt[basis_index(spec, [G_LEVEL, R_LEVEL], [0, 1])] = 1j
    tgt /= np.linalg.norm(tgt)
    return spec, sysd, tgt


def test_krotov_update_is_scaled_gradient():
    """Without dissipation, lambda Delta u_ij / S_ij -> -(1/(2 dt)) dJ_T/du_ij.

    For large lambda the forward states of the sequential pass equal the guess
    states to O(1/lambda); the left-point update then matches the central
    finite-difference gradient of J_T up to O(dt): the gap must halve when the
    time grid is refined twofold (a wrong factor or sign would not vanish).
    """
    spec, sysd, tgt = _unitary_problem()
    T, M, h = 4.0, 3, 1e-4
    times = [(0, 0.05), (1, 0.57 * T), (0, 0.5 * T), (1, 0.83 * T), (0, 0.99 * T)]
    gaps, preds = [], []
    for nt in (200, 400):
        dt = T / nt
        grid = np.linspace(0, 3, nt)
        u0 = 0.6 + 0.2 * np.sin(grid)[None, :] * np.array([[1.0], [-1.0]])
        lam = np.full(2, 1e6)
        res = krotov.optimise(sysd, initial_state(spec), tgt, u0, np.ones((2, nt)), lam,
                              T, M, 0, 1)
        du = res.u[1] - res.u[0]
        g, p = [], []
        for i, t in times:
            j = int(t / dt)
            up, um = u0.copy(), u0.copy()
            up[i, j] += h
            um[i, j] -= h
            Jp = krotov.plain_forward(sysd, initial_state(spec), tgt, up, T, 1, 0).J_T
            Jm = krotov.plain_forward(sysd, initial_state(spec), tgt, um, T, 1, 0).J_T
            pred = -(Jp - Jm) / (2 * h) / (2 * dt)
            g.append(lam[i] * du[i, j] - pred)
            p.append(pred)
        gaps.append(np.array(g))
        preds.append(np.array(p))
    scale = np.abs(preds[1]).max()
    assert np.abs(gaps[1]).max() < 0.05 * scale, (gaps[1], scale)
    ratio = np.abs(gaps[0]) / np.abs(gaps[1])
    assert np.all((ratio > 1.7) & (ratio < 2.3)), ratio


def test_krotov_monotone_without_dissipation():
    spec, sysd, tgt = _unitary_problem()
    T, nt = 4.0, 200
    rng = np.random.default_rng(2)
    u0 = 0.6 + 0.2 * rng.normal(size=(2, nt))
    res = krotov.optimise(sysd, initial_state(spec), tgt, u0, np.ones((2, nt)),
                          np.full(2, 0.5), T, 2, 0, 6)
    J = np.array(res.J_T)
    assert np.all(np.diff(J) < 0), J
    assert J[-1] < J[0] - 0.05


def test_functional_definition():
    tgt = np.array([1, 1j, 0], complex) / math.sqrt(2)
    psi = np.vstack([tgt, np.array([0, 0, 1], complex), np.array([1, 0, 0], complex)])
    tau = krotov.overlaps(psi, tgt)
    assert np.allclose(np.abs(tau) ** 2, [1, 0, 0.5])
    assert abs(krotov.functional(tau) - (1 - 1.5 / 3)) < 1e-15
    # the costate boundary is <tgt|psi> tgt (derivative of J_T wrt <psi|)
    assert abs(tau[0] - 1) < 1e-15 and abs(tau[2] - 1 / math.sqrt(2)) < 1e-15


# ---------------------------------------------------------------------------
# costate (backward) jumps: the reverse clock and the recorded times
# ---------------------------------------------------------------------------

def test_backward_single_cavity_closed_form():
    """Costate from one photon, atom in g, no drive, run backward from T.

    exp(+i H_eff^+ tau) with H_eff = H - (i/2) kappa a^+a damps the photon as
    exp(-kappa tau/2) in amplitude, so before its first jump the backward
    state has ||chi~(t)||^2 = exp(-kappa (T - t)); the jump happens when that
    reaches the threshold r0 of stream (seed, k, iteration, direction 1),
    i.e. at t = T + ln(r0)/kappa, recorded with direction 1 in the step
    that contains it; the jump leaves the empty (dark) cavity.
    """
    from oracle.mcwf import backward_pass
    spec, sysd = _single_cavity()
    i1 = basis_index(spec, [G_LEVEL], [1])
    i0 = basis_index(spec, [G_LEVEL], [0])
    chiT = np.zeros(spec.dim, complex)
    chiT[i1] = 1.0
    T, nt, M, seed, it = 5.0, 10, 24, 8, 3
    dt = T / nt
    ens, chi_hat = backward_pass(sysd, chiT[None, :].repeat(M, 0), np.zeros((1, nt)), T, M,
                                 seed, it)
    first = {}
    for rec in ens.records:
        assert rec.direction == 1
        first.setdefault(rec.traj, rec)
    n_jumps = 0
    for k in range(M):
        r0 = philox.TrajectoryStream(seed, k, it, 1).threshold(0)
        t_ref = T + math.log(r0)  # kappa = 1
        if t_ref > 0.0:
            rec = first[k]
            assert abs(rec.t - t_ref) < 1e-11, (rec.t, t_ref)
            assert rec.step == int(t_ref // dt) and rec.ordinal == 0 and rec.op == 0
            assert sum(r.traj == k for r in ens.records) == 1
            # normalised costates: |g,1> after t_ref, |g,0> before it
            for j in range(nt):
                ref = i1 if j * dt > t_ref else i0
                assert abs(abs(chi_hat[j, k, ref]) - 1.0) < 1e-12
            n_jumps += 1
        else:
            assert k not in first
            # no jump: the norm left at t = 0 is exp(-kappa T)
            assert abs(norm2(ens.psi[k]) - math.exp(-T)) < 1e-13
    assert n_jumps >= 10


def test_backward_two_jumps_inside_one_step():
    """Two photons, one step of length T run backward: the first jump is at
    elapsed time e1 = -ln(r0)/2 (decay rate 2 kappa), the second at
    e2 = e1 - ln(r1) (rate kappa), recorded as T - e1 and T - e2."""
    from oracle.mcwf import backward_pass
    spec, sysd = _single_cavity(n_fock=3)
    chiT = np.zeros(spec.dim, complex)
    chiT[basis_index(spec, [G_LEVEL], [2])] = 1.0
    T, M, seed, it = 40.0, 12, 6, 2
    ens, _ = backward_pass(sysd, chiT[None, :].repeat(M, 0), np.zeros((1, 1)), T, M, seed, it)
    checked = 0
    for k in range(M):
        st = philox.TrajectoryStream(seed, k, it, 1)
        e1 = -math.log(st.threshold(0)) / 2.0
        e2 = e1 - math.log(st.threshold(1))
        recs = sorted((r for r in ens.records if r.traj == k), key=lambda r: r.ordinal)
        if e2 < T:
            assert [(r.step, r.ordinal, r.direction) for r in recs] == [(0, 0, 1), (0, 1, 1)]
            assert abs(recs[0].t - (T - e1)) < 1e-11 and abs(recs[1].t - (T - e2)) < 1e-10
            # the norm falls at relative rate sum_l ||L psi||^2 / ||psi||^2 = kappa n:
            # 2 with two photons, 1 with one (kappa = 1)
            assert abs(recs[0].rate - 2.0) < 1e-12 and abs(recs[1].rate - 1.0) < 1e-12
            checked += 1
    assert checked >= 8


# ---------------------------------------------------------------------------
# the trajectory average converges to rho as 1/sqrt(M)
# ---------------------------------------------------------------------------

def test_ensemble_error_falls_as_inverse_sqrt_M():
    """RMS Frobenius error of (1/M) sum_k |psi_hat_k><psi_hat_k| against the
    master-equation rho(T), over disjoint groups of M trajectories of one run
    of 16384, for M = 256 .. 16384: the log-log slope is -1/2 (trajectory
    expansion of rho, Sec. 2.1; independent samples)."""
    spec, sysd = _single_cavity()
    u = np.full((1, 8), 0.8)
    T, total, seed = 3.0, 16384, 12
    psi0 = initial_state(spec)
    ens, _ = forward_pass(sysd, psi0, u, T, total, seed, 0)
    psi_hat = ens.normalised()
    rho = lindblad.propagate_rho(sysd, np.outer(psi0, psi0.conj()), u, T)
    Ms = [256, 1024, 4096, 16384]
    rms = []
    for M in Ms:
        errs = []
        for g in range(total // M):
            p = psi_hat[g * M:(g + 1) * M]
            rho_m = p.T @ p.conj() / M
            errs.append(np.linalg.norm(rho_m - rho) ** 2)
        rms.append(math.sqrt(np.mean(errs)))
    slope = np.polyfit(np.log(Ms), np.log(rms), 1)[0]
    assert len(ens.records) > 2000
    assert abs(slope + 0.5) < 0.1, (slope, rms)


# ---------------------------------------------------------------------------
# pulse-noise measure (Sec. 3.4): Savitzky-Golay five-point cubic
# ---------------------------------------------------------------------------

def test_noise_filter_matches_scipy_savgol():
    """The filter equals SciPy's Savitzky-Golay filter (window 5, order 3,
    polynomial fit at the ends) -- a library routine."""
    import scipy.signal
    from oracle.noise import smooth_cubic5
    rng = np.random.default_rng(4)
    for n in (5, 6, 17, 400):
        x = rng.normal(size=n) + np.linspace(0, 3, n) ** 2
        ref = scipy.signal.savgol_filter(x, 5, 3, mode="interp")
        assert np.abs(smooth_cubic5(x) - ref).max() < 1e-12


def test_noise_filter_closed_forms():
    """Cubic pulses pass unchanged (nu = 0); the centred weights are the
    classic (-3, 12, 17, 12, -3)/35; an alternating ripple of amplitude e on a
    smooth pulse leaves 48/35 e at every interior sample."""
    from oracle.noise import pulse_noise, smooth_cubic5
    t = np.linspace(-1.0, 2.0, 60)
    cubic = 0.3 - 0.7 * t + 0.2 * t ** 2 + 0.9 * t ** 3
    assert np.abs(smooth_cubic5(cubic) - cubic).max() < 1e-12
    assert pulse_noise(cubic[None, :], 5.0)[0] < 1e-11
    imp = np.zeros(11)
    imp[5] = 1.0
    w = smooth_cubic5(imp)[3:8]  # response of the samples around the impulse
    assert np.abs(w * 35 - np.array([-3, 12, 17, 12, -3])).max() < 1e-12
    e, n, T = 1e-3, 50, 10.0
    ripple = e * (-1.0) ** np.arange(n)
    resid = np.abs(ripple - smooth_cubic5(ripple))
    assert np.abs(resid[2:-2] - 48.0 / 35.0 * e).max() < 1e-15
    nu = pulse_noise(ripple[None, :], T)[0]
    assert abs(nu - T / n * resid.sum()) < 1e-15


# ---------------------------------------------------------------------------
# cross-trajectory update (Sec. 2.3): kappa = 0, one trajectory
# ---------------------------------------------------------------------------

def test_cross_update_equals_independent_update_at_first_step():
    """Without dissipation and with M = 1 the backward state xi and the costate
    chi = tau chi_hat are the same unitary trajectory, and at t = 0 the forward
    state is still psi0, so <psi0|xi(0)> = <psi(T)|tgt> = conj(tau): the two
    updates of the first interval coincide (to rounding)."""
    spec, sysd, tgt = _unitary_problem()
    T, nt = 4.0, 100
    rng = np.random.default_rng(7)
    u0 = 0.6 + 0.2 * rng.normal(size=(2, nt))
    S, lam = np.ones((2, nt)), np.full(2, 3.0)
    ind = krotov.optimise(sysd, initial_state(spec), tgt, u0, S, lam, T, 1, 0, 1)
    crs = krotov.optimise_cross(sysd, initial_state(spec), tgt, u0, S, lam, T, 1, 0, 1)
    d_ind = ind.u[1][:, 0] - u0[:, 0]
    d_crs = crs.u[1][:, 0] - u0[:, 0]
    assert np.abs(d_ind).max() > 1e-4
    assert np.abs(d_crs - d_ind).max() < 1e-13 * np.abs(d_ind).max() + 1e-16


def test_cross_update_approaches_independent_update_as_lambda_grows():
    """kappa = 0, M = 1: both updates are lambda^-1 times the same first-order
    gradient; they differ only through the updated forward state in the
    overlap <psi^(1)(t)|xi(t)>, i.e. at order lambda^-2: doubling lambda
    quarters the gap, while the updates themselves halve."""
    spec, sysd, tgt = _unitary_problem()
    T, nt = 4.0, 100
    rng = np.random.default_rng(8)
    u0 = 0.6 + 0.2 * rng.normal(size=(2, nt))
    S = np.ones((2, nt))
    gaps, sizes = [], []
    for lam in (20.0, 40.0):
        L = np.full(2, lam)
        ind = krotov.optimise(sysd, initial_state(spec), tgt, u0, S, L, T, 1, 0, 1)
        crs = krotov.optimise_cross(sysd, initial_state(spec), tgt, u0, S, L, T, 1, 0, 1)
        gaps.append(np.abs(crs.u[1] - ind.u[1]).max())
        sizes.append(np.abs(ind.u[1] - u0).max())
    assert 1.8 < sizes[0] / sizes[1] < 2.2
    assert 3.4 < gaps[0] / gaps[1] < 4.6, gaps
    assert gaps[0] < 0.2 * sizes[0]


def test_cross_update_with_jumps_is_real_and_finite():
    """With dissipation and several trajectories the cross update runs the
    reverse-time MCWF rules for xi; each term sum is real-valued input to a
    real pulse (the imaginary part of a complex sum), finite, and bounded by
    ||H_i|| (|<xi|H_i|psi><psi|xi>| <= ||H_i|| for unit vectors)."""
    spec = CascadeSpec(2, 2)
    H0, Hc, L = build_cascade(spec)
    sysd = System.from_sparse(H0, Hc, L)
    from workloads.cascade import w_target
    T, nt, M = 10.0, 60, 6
    u0 = np.full((2, nt), 0.7)
    res = krotov.optimise_cross(sysd, initial_state(spec), w_target(spec), u0,
                                np.ones((2, nt)), np.full(2, 2.0), T, M, 3, 1)
    du = res.u[1] - u0
    assert np.all(np.isfinite(du))
    assert np.abs(du).max() <= 0.5 / 2.0 + 1e-12
    assert len(res.backward_records[0]) > 0


# ---------------------------------------------------------------------------
# density-matrix (Liouville-space) optimisation, Sec. 2.2
# ---------------------------------------------------------------------------

def test_rho_functional_and_adjoint_propagation():
    """<<P(t)|rho(t)>> is the same at every t for the adjoint backward P and
    the forward rho (the adjoint map), so 1 - <<P(0)|rho(0)>> = J_T; and the
    functional equals 1 - the trajectory-free fidelity of the master equation."""
    from oracle import density
    spec = CascadeSpec(2, 2)
    H0, Hc, L = build_cascade(spec)
    sysd = System.from_sparse(H0, Hc, L)
    from workloads.cascade import w_target
    tgt = w_target(spec)
    rng = np.random.default_rng(5)
    nt, T = 30, 6.0
    u = rng.normal(0.5, 0.3, (2, nt))
    psi0 = initial_state(spec)
    rhos = density.forward_rho(sysd, psi0, u, T, keep=True)
    P = density.backward_P(sysd, tgt, u, T)
    J = density.rho_functional(rhos[-1], tgt)
    ovl = [np.trace(P[j].conj().T @ rhos[j]) for j in range(nt)]
    assert np.abs(np.array(ovl) - (1.0 - J)).max() < 1e-12
    rho_ref = lindblad.propagate_rho(sysd, np.outer(psi0, psi0.conj()), u, T)
    assert abs(J - (1.0 - np.real(tgt.conj() @ rho_ref @ tgt))) < 1e-12
    assert 0.0 < J < 1.0


def test_rho_update_is_twice_the_cross_update_for_pure_states():
    """kappa = 0 and a pure initial state: P(t) = |xi(t)><xi(t)| and
    rho(t) = |psi(t)><psi(t)| exactly, so Im <<P|[H_i, rho]>> =
    2 Im[<xi|H_i|psi><psi|xi>]: the density-matrix pass equals the
    cross-trajectory pass with one trajectory at twice the step (lambda / 2),
    interval by interval, although one propagates d x d matrices with the
    Liouvillian and the other wave functions."""
    from oracle import density
    spec, sysd, tgt = _unitary_problem()
    T, nt = 4.0, 80
    rng = np.random.default_rng(9)
    u0 = 0.6 + 0.2 * rng.normal(size=(2, nt))
    S, lam = np.ones((2, nt)), np.full(2, 4.0)
    rho = density.optimise_rho(sysd, initial_state(spec), tgt, u0, S, lam, T, 2)
    crs = krotov.optimise_cross(sysd, initial_state(spec), tgt, u0, S, lam / 2.0, T, 1, 0, 2)
    for n in (1, 2):
        assert np.abs(rho.u[n] - crs.u[n]).max() < 1e-10, n
        assert abs(rho.J_T[n] - crs.J_T[n]) < 1e-10
    assert np.abs(rho.u[2] - u0).max() > 1e-3
    assert rho.J_T[2] < rho.J_T[0]  # monotone without dissipation
