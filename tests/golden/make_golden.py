"""Write the stored expected values of the larger GPU parity cases.

Every value written here comes from the FP64 oracle (``oracle/``) on seeded
synthetic inputs from ``workloads/``; nothing reads the HIP library.  The
cases are those whose oracle run takes minutes (many trajectories or
d = 1296), so the GPU tests load the results instead of recomputing them:

* ``krotov_chain2_fock3_M1024_nt200``: two nodes, cavity at 3 levels (d = 81),
  M = 1024 trajectories, nt = 200 on T = 50, two Krotov iterations
  (the sequential independent-trajectory update of Sec. 2.3 on the MCWF
  trajectories of Sec. 2.1): J_T per iteration, the pulses after each
  iteration and every jump record of the five passes.
* ``krotov_chain2_fock2_M1100_nt60``: d = 36, M = 1100 (more trajectories
  than one cooperative launch holds one to a wave), nt = 60 on T = 50.
* ``krotov_chain3_fock2_M1100_nt40``: d = 216, M = 1100, nt = 40 on T = 2,
  with the guess pass's overlaps and final states of sampled trajectories.
* ``krotov_chain4_fock2_M1100_nt80``: four nodes (d = 1296), M = 1100 (more
  trajectories than the eight-wave Krotov pass holds in LDS), nt = 80 on
  T = 10, lambda = 0.05, one Krotov iteration.
* ``cross_chain2_fock2_M1100_nt60``: the same d = 36 case with the
  cross-trajectory update of Sec. 2.3 (eq. cross_traj_update): J_T and pulses.
* ``batch_seed0_inst1_2``: instances 1 and 2 (d = 36) of the eight-instance
  draw ``batch_instances(8, seed=0, nodes=(2, 3, 4))``, two iterations each.
* ``grad_chain4_fock2_nt4000_M1``: four nodes (d = 1296), one trajectory over
  the full nt = 4000 on T = 50: its forward jump record and the pathwise
  gradient dJ_T/du of the replay with that record fixed (reverse sweep with
  Van Loan's block exponential).
* ``grad_chain4_fock2_nt200_M4``: d = 1296, M = 4, nt = 200 on T = 25: records,
  the adjoint gradient and central differences (h = 1e-4) of the replayed
  functional on 16 entries, five of them at the 64-step boundaries.

Usage: ``python tests/golden/make_golden.py [case ...]`` (all cases by
default, each in a process of its own).
"""

from __future__ import annotations

import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

# the oracle's dense products are small: one BLAS thread per case process
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _one_thread():
    from threadpoolctl import threadpool_limits
    return threadpool_limits(limits=1)


def record_columns(recs, iteration, with_rate=False):
    """Jump records as sorted columns (iteration, direction, traj, ordinal, step, op) + t
    (and the relative norm decay rate at each crossing)."""
    rows = sorted((iteration, r.direction, r.traj, r.ordinal, r.step, r.op, r.t, r.rate)
                  for r in recs)
    ints = np.array([r[:6] for r in rows], dtype=np.int64).reshape(-1, 6)
    ts = np.array([r[6] for r in rows], dtype=np.float64)
    if with_rate:
        return ints, ts, np.array([r[7] for r in rows], dtype=np.float64)
    return ints, ts


def _optimise(w, n_iter, keep_guess_states=None):
    from oracle import krotov as ok
    from oracle.mcwf import System
    sysd = System.from_sparse(w.H0, w.H_ctrl, w.L_jump)
    res = ok.optimise(sysd, w.psi0, w.psi_tgt, w.u0, w.S, w.lam, w.T, w.M, w.seed, n_iter,
                      instance=w.instance)
    ints, ts, rates = [], [], []
    i, t, q = record_columns(res.passes[0].records, 0, True)
    ints.append(i)
    ts.append(t)
    rates.append(q)
    for it in range(1, n_iter + 1):
        for recs in (res.backward_records[it - 1], res.passes[it].records):
            i, t, q = record_columns(recs, it, True)
            ints.append(i)
            ts.append(t)
            rates.append(q)
    order = np.lexsort(tuple(np.concatenate(ints).T[::-1]))
    out = dict(J=np.array(res.J_T), u=np.array(res.u), rec_int=np.concatenate(ints)[order],
               rec_t=np.concatenate(ts)[order], rec_rate=np.concatenate(rates)[order],
               tau0=res.passes[0].tau)
    if keep_guess_states is not None:
        out["sample_k"] = np.array(keep_guess_states)
        out["sample_psi"] = res.passes[0].psi_hat_T[keep_guess_states]
    return out


def case_krotov_chain2_fock3_M1024_nt200():
    from workloads import config_workload
    return _optimise(config_workload("chain2_fock3", M=1024, nt=200), 2)


def case_krotov_chain2_fock2_M1100_nt60():
    from workloads import config_workload
    return _optimise(config_workload("chain2_fock2", M=1100, nt=60), 2)


def case_krotov_chain3_fock2_M1100_nt40():
    from workloads import config_workload
    return _optimise(config_workload("chain3_fock2", M=1100, nt=40, T=2.0), 2,
                     keep_guess_states=[0, 1, 517, 1098, 1099])


def case_krotov_chain4_fock2_M1100_nt80():
    from workloads import config_workload
    return _optimise(config_workload("chain4_fock2", M=1100, nt=80, T=10.0, lam=0.05), 1)


def case_cross_chain2_fock2_M1100_nt60():
    from oracle import krotov as ok
    from oracle.mcwf import System
    from workloads import config_workload
    w = config_workload("chain2_fock2", M=1100, nt=60)
    sysd = System.from_sparse(w.H0, w.H_ctrl, w.L_jump)
    res = ok.optimise_cross(sysd, w.psi0, w.psi_tgt, w.u0, w.S, w.lam, w.T, w.M, w.seed, 2)
    return dict(J=np.array(res.J_T), u=np.array(res.u))


def case_batch_seed0_inst1_2():
    from workloads import batch_instances
    ws = batch_instances(8, seed=0, nodes=(2, 3, 4))
    out = {}
    for i in (1, 2):
        r = _optimise(ws[i], 2)
        out[f"J{i}"] = r["J"]
        out[f"u{i}"] = r["u"]
    return out


def _grad_case(w, fd_entries=None):
    from oracle import krotov as ok
    from oracle.gradient import gradient_adjoint, gradient_fd, paths_from_records, replay_functional
    from oracle.mcwf import System
    sysd = System.from_sparse(w.H0, w.H_ctrl, w.L_jump)
    fw = ok.plain_forward(sysd, w.psi0, w.psi_tgt, w.u0, w.T, w.M, w.seed, 0)
    paths = paths_from_records(fw.records, w.M)
    g = gradient_adjoint(sysd, w.psi0, w.psi_tgt, w.u0, w.T, paths)
    J, tau = replay_functional(sysd, w.psi0, w.psi_tgt, w.u0, w.T, paths)
    ints, ts = record_columns(fw.records, 0)
    out = dict(g=g, J=np.array(J), tau=tau, rec_int=ints, rec_t=ts, J_mcwf=np.array(fw.J_T))
    if fd_entries is not None:
        ent = np.array(fd_entries, dtype=np.int64)
        out["fd_entries"] = ent
        out["fd"] = gradient_fd(sysd, w.psi0, w.psi_tgt, w.u0, w.T, paths,
                                [tuple(e) for e in ent], h=1e-4)
    return out


def case_grad_chain4_fock2_nt4000_M1():
    from workloads import config_workload
    return _grad_case(config_workload("chain4_fock2", M=1, nt=4000))


def fd_entries_nt200(n_ctrl=4, nt=200, seed=17):
    """16 (control, step) entries: five at the 64-step boundaries, the rest drawn."""
    rng = np.random.default_rng(seed)
    fixed = [(0, 63), (1, 64), (2, 127), (3, 128), (0, 192)]
    drawn = [(int(rng.integers(n_ctrl)), int(rng.integers(nt))) for _ in range(11)]
    return fixed + drawn


def case_grad_chain4_fock2_nt200_M4():
    from workloads import config_workload
    return _grad_case(config_workload("chain4_fock2", M=4, nt=200, T=25.0),
                      fd_entries=fd_entries_nt200())


CASES = {name[5:]: fn for name, fn in globals().items() if name.startswith("case_")}


def run(name):
    _one_thread()
    t0 = time.time()
    out = CASES[name]()
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, **out)
    return f"{name}: {time.time() - t0:.0f} s -> {os.path.relpath(path, ROOT)}"


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    from concurrent.futures import as_completed
    with ProcessPoolExecutor(max_workers=min(len(names), 6)) as ex:
        futs = [ex.submit(run, n) for n in names]
        for f in as_completed(futs):
            print(f.result(), flush=True)
