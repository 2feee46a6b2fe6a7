"""The entry point that allocates nothing (tk_functional_dev_noalloc) against
tk_functional, through the C ABI, on two calls in a row (the second with
fewer trajectories, so it must not depend on what the first left in the
shared scratch)."""

import numpy as np
import pytest

from parity import say
from workloads import config_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tk():
    from paper_1801_04382_amd import trajkrotov
    return trajkrotov


def test_no_alloc_functional_matches_functional(tk):
    import torch
    dev = torch.device("cuda:0")
    w = config_workload("chain2_fock3", M=300, nt=400, seed=4)
    with tk.Context(precision="fp64") as ctx:
        ctx.load(w)
        for M, it in ((300, 0), (37, 5)):
            J_ref, tau_ref = ctx.functional(M, w.seed, it)
            J = torch.full((1,), -1.0, dtype=torch.float64, device=dev)
            tau = torch.zeros(2 * M, dtype=torch.float64, device=dev)
            s = torch.cuda.current_stream(dev).cuda_stream
            tk.tk_functional_dev_noalloc(ctx.h, M, w.seed, it, J.data_ptr(), tau.data_ptr(), s)
            J_h = float(J.cpu()[0])
            tau_h = tau.cpu().numpy().view(np.complex128)
            say("no-alloc M", M, "J", J_h, "reference", J_ref)
            # same kernels, same order: bit-identical to the allocating call
            assert J_h == J_ref
            assert np.array_equal(tau_h, tau_ref)
            # J without the overlaps
            J2 = torch.full((1,), -1.0, dtype=torch.float64, device=dev)
            tk.tk_functional_dev_noalloc(ctx.h, M, w.seed, it, J2.data_ptr(), 0, s)
            assert float(J2.cpu()[0]) == J_ref
        with pytest.raises(tk.TkError) as e:
            tk.tk_functional_dev_noalloc(ctx.h, 65505, w.seed, 0, J.data_ptr(), 0, s)
        assert e.value.code == tk.TK_EINVAL
