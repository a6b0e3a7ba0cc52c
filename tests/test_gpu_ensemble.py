"""Ensembles of independent solves (FD directions, parameter sweeps) through
rsfde_march_ensemble: members run concurrently on their own streams and host
threads, and each must give exactly what the same plan gives when marched
alone (the computation of a member does not depend on the others)."""

import numpy as np
import pytest
import torch

from workloads.configs import make_config, fd_direction

pytestmark = pytest.mark.gpu

rsfde = pytest.importorskip("paper_2102_11576_amd")
from paper_2102_11576_amd import RsfdePlan, make_opts, march_ensemble  # noqa: E402

DEV = "cuda:0"


def _members(n, count):
    w = make_config("c4", n=n, m=4)
    plans, u0s = [], []
    for i in range(count):
        pl = RsfdePlan.from_workload(w, kx=1.0 + 0.1 * i, ky=1.0 - 0.05 * i)
        du, _, _ = fd_direction(w.u0.shape, i)
        u0 = torch.as_tensor(w.u0 + 1e-3 * du * w.mask, device=DEV).reshape(-1).contiguous()
        plans.append(pl)
        u0s.append(u0)
    return w, plans, u0s


@pytest.mark.parametrize("sstep", [0, 8])
def test_ensemble_equals_members_marched_alone(sstep):
    w, plans, u0s = _members(127, 4)
    opts = make_opts(w.restart, 100000, w.tol, sstep=sstep)
    try:
        streams = [torch.cuda.Stream() for _ in plans]
        outs, sts = march_ensemble(plans, u0s, w.m, w.f_kind, opts, streams)
        torch.cuda.synchronize()
        for pl, u0, out, st in zip(plans, u0s, outs, sts):
            ref, it, _ = pl.march(u0, w.m, w.f_kind, opts)
            assert torch.equal(out, ref)
            assert st.iters == sum(it) and st.status == 0
    finally:
        for pl in plans:
            pl.close()


def test_ensemble_zero_steps_and_argument_checks():
    w, plans, u0s = _members(63, 2)
    opts = make_opts(w.restart, 100000, w.tol)
    try:
        outs, _ = march_ensemble(plans, u0s, 0, w.f_kind, opts)
        for u0, out in zip(u0s, outs):
            assert torch.equal(out, u0)
        with pytest.raises(rsfde.RsfdeError) as ei:   # the same plan twice
            march_ensemble([plans[0], plans[0]], u0s, 1, w.f_kind, opts)
        assert ei.value.code == rsfde._lib.RSFDE_EINVAL
        with pytest.raises(rsfde.RsfdeError) as ei:   # output aliasing the input
            rsfde._lib.rsfde_march_ensemble([plans[0].handle], [u0s[0]], 1, w.f_kind, opts,
                                            [u0s[0]], [plans[0].empty(), plans[0].empty()])
        assert ei.value.code == rsfde._lib.RSFDE_EINVAL
    finally:
        for pl in plans:
            pl.close()
