"""Host-side logic of the differentiable march (no GPU): the checkpoint schedule."""

import math

import pytest

pytest.importorskip("torch")


def _sched():
    # the schedule is pure Python; import without touching the GPU
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location(
        "rsfde_autograd_sched",
        os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_2102_11576_amd", "autograd.py"))
    src = open(spec.origin).read()
    ns = {}
    # evaluate only checkpoint_schedule (the rest imports the HIP binding)
    start = src.index("def checkpoint_schedule")
    end = src.index("class RsfdeMarch")
    exec("import math\nfrom typing import List, Tuple\n" + src[start:end], ns)
    return ns["checkpoint_schedule"]


@pytest.mark.parametrize("m", [1, 2, 3, 7, 16, 32, 33, 100])
def test_schedule_covers_every_step_once(m):
    sched = _sched()
    segs = sched(m)
    steps = [k for a, b in segs for k in range(a + 1, b + 1)]
    assert steps == list(range(1, m + 1))
    s = max(1, math.ceil(math.sqrt(m)))
    assert all(b - a <= s for a, b in segs)
    assert len(segs) == math.ceil(m / s)


def test_schedule_explicit_interval():
    sched = _sched()
    assert sched(10, 4) == [(0, 4), (4, 8), (8, 10)]
    assert sched(0) == []
