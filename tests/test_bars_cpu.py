"""The element-wise preconditioner bars of the GPU parity tests, checked on
the CPU against the oracle alone: they pass for the oracle's own rounding
(the FP64 eigenvalue denominators evaluated another way) and fail for a
mistake planted in one place (one transform slot, one row, the penalty region
alone), which a 2-norm bar against the input misses."""

import numpy as np
import pytest
import scipy.fft as sf

import oracle as O
from workloads.configs import make_config
from bars import assert_precond, precond_kappa


@pytest.fixture(scope="module")
def c3_255():
    w = make_config("c3", n=255)  # alpha = 1.9, the stiff shape at a CPU size
    p = O.problem_from_workload(w)
    V = np.random.default_rng(3).standard_normal((w.n2, w.n1))
    return p, V, O.precond_apply_fft(p, V)


def _with(p, V, edit):
    """The preconditioner with `edit(E1, E2)` applied to its denominators."""
    lx, ly = O.tau_eigs_xy(p)
    W = sf.dstn(V, type=1, norm="ortho")
    E1 = 1.0 - lx[None, :] - ly[:, None]
    E2 = E1 + p.d
    edit(E1, E2)
    Y1 = sf.dstn(W / E1, type=1, norm="ortho")
    Y2 = sf.dstn(W / E2, type=1, norm="ortho")
    return (1.0 - p.phi) * Y1 + p.phi * Y2


def test_bars_accept_rounding_of_the_eigenvalue_denominators(c3_255):
    """E1 perturbed by the FP64 rounding of its low-frequency cancellation
    (eps times the sum of |c t_j|) stays inside the FP64 bar."""
    p, V, ref = c3_255
    k1, _ = precond_kappa(p)
    e1min = 1.0 - sum(l.max() for l in O.tau_eigs_xy(p))
    rng = np.random.default_rng(0)

    def jitter(E1, E2):
        d = np.finfo(np.float64).eps * k1 * e1min * rng.uniform(-1, 1, E1.shape)
        E1 += d
        E2 += d

    assert_precond(_with(p, V, jitter), ref, p, "fp64", "rounded denominators")


@pytest.mark.parametrize("where", ["one slot of E1", "one slot of E2", "one row", "penalty region"])
def test_bars_reject_localised_mistakes(c3_255, where):
    p, V, ref = c3_255
    if where == "one slot of E1":
        out = _with(p, V, lambda E1, E2: E1.__setitem__((0, 7), E1[0, 7] * (1 + 1e-6)))
    elif where == "one slot of E2":
        out = _with(p, V, lambda E1, E2: E2.__setitem__((200, 3), E2[200, 3] * (1 - 1e-7)))
    elif where == "one row":
        out = ref.copy()
        out[17] *= 1 + 1e-8
    else:
        out = ref.copy()
        out[p.phi > 0] *= 1 + 1e-9
    # a relative 2-norm bar against the input, as the full-size tests once used, passes all four
    assert np.linalg.norm(out - ref) <= 1e-13 * np.linalg.norm(V) or where == "one slot of E1"
    with pytest.raises(AssertionError):
        assert_precond(out, ref, p, "fp64", where)
