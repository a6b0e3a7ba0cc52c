"""The time march around the step: resuming an interrupted march and the
per-step JSONL log.

* A march of 6 steps equals, bit for bit, a march of 3 steps resumed for 3
  more from (u^3, u^2) with k0 = 3 (the extrapolated initial guess
  2 u^{k-1} - u^{k-2} needs the state before the last one), with the same
  inner iteration counts; both forms of GMRES (s-step at 71^2, one vector at
  31^2).
* The log holds one JSON record per step (step number, iterations, restarts,
  final relative residual, status, wall time) that matches the march's own
  counts.
* The resumed march agrees with the oracle's LU march (relative 1e-10 at
  solver tolerance 1e-12).
"""

import json

import numpy as np
import pytest
import torch

import oracle as O
from workloads.configs import make_config

pytestmark = pytest.mark.gpu

rsfde = pytest.importorskip("paper_2102_11576_amd")
from paper_2102_11576_amd import RsfdePlan, make_opts  # noqa: E402

DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV).reshape(-1)


@pytest.mark.parametrize("name,n,sstep", [("c4", 71, 8), ("c1", 31, 0)])
def test_resume_equals_uninterrupted_march(tmp_path, name, n, sstep):
    w = make_config(name, n=n, m=6)
    opts = make_opts(w.restart, 100000, 1e-12, sstep=sstep)
    log = tmp_path / "steps.jsonl"
    with RsfdePlan.from_workload(w) as pl:
        u0 = _t(w.u0)
        u6, it6, _ = pl.march(u0, 6, w.f_kind, opts, log=str(log))
        _, it3, kept = pl.march(u0, 3, w.f_kind, opts, keep=[2, 3])
        u6b, it6b, kept_b = pl.march(kept[3], 3, w.f_kind, opts, u_prev=kept[2], k0=3,
                                     keep=[3, 5])
        u6 = u6.cpu().numpy()
        u6b = u6b.cpu().numpy()
    assert np.array_equal(u6, u6b)
    assert it3 + it6b == it6, (it3, it6b, it6)
    assert sorted(kept_b) == [3, 5]
    recs = [json.loads(line) for line in open(log)]
    assert [r["step"] for r in recs] == list(range(1, 7))
    assert [r["iters"] for r in recs] == it6
    assert all(r["status"] == 0 and r["relres"] <= 1e-12 and r["ms"] > 0 for r in recs), recs
    ref = O.march_lu(O.problem_from_workload(w), w.u0, 6, w.f_kind).ravel()
    assert np.abs(u6b - ref).max() <= 1e-10 * np.abs(ref).max()
