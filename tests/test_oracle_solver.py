"""End-to-end pins of the oracle: GMRES vs LU, the Lemma 3.1 certificate and
the paper's own numbers (Section 5, Tables 1-3)."""

import json
import os

import numpy as np
import pytest

import oracle as O
from workloads.configs import example1_workload, make_config

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def test_gmres_right_matches_lu_small_c1():
    w = make_config("c1", n=15, m=4)
    p = O.problem_from_workload(w)
    u_lu = O.march_lu(p, w.u0, w.m, w.f_kind)
    u_g, iters = O.march_gmres(p, w.u0, w.m, w.f_kind, 20, 1e-12)
    assert np.abs(u_g - u_lu).max() <= 1e-10 * np.abs(u_lu).max()
    assert all(i > 0 for i in iters)


def test_unpreconditioned_gmres_matches_lu():
    w = make_config("c4", n=9, m=3)
    p = O.problem_from_workload(w)
    u_lu = O.march_lu(p, w.u0, w.m, w.f_kind)
    u_g, _ = O.march_gmres(p, w.u0, w.m, w.f_kind, 30, 1e-13, precond=False, max_iters=100000)
    assert np.abs(u_g - u_lu).max() <= 1e-9 * np.abs(u_lu).max()


def test_left_and_right_modes_agree_to_tolerance():
    w = make_config("c2", n=15, m=3)
    p = O.problem_from_workload(w)
    uL, _ = O.march_gmres(p, w.u0, w.m, w.f_kind, 20, 1e-12, side="left")
    uR, _ = O.march_gmres(p, w.u0, w.m, w.f_kind, 20, 1e-12, side="right")
    assert np.abs(uL - uR).max() <= 1e-9 * np.abs(uR).max()


def test_lemma_3_1_certificate():
    """||u - u*||_inf <= ||b - M u||_inf for any u (Lemma 2.3 + Lemma 3.1)."""
    w = make_config("c1", n=11, m=1)
    p = O.problem_from_workload(w)
    b = O.rhs(p, w.u0, w.f_kind)
    M = O.dense_M(p)
    u_star = np.linalg.solve(M, b.ravel())
    rng = np.random.default_rng(0)
    for _ in range(5):
        u = u_star + 1e-3 * rng.standard_normal(u_star.size)
        r = b.ravel() - M @ u
        assert np.abs(u - u_star).max() <= np.abs(r).max() * (1 + 1e-12)


def _ex1(n, kx, **kw):
    return O.example1_march(example1_workload(n, kx, **{k: v for k, v in kw.items() if k in ("eta", "T", "m")}),
                            side=kw.get("side", "left"), precond=kw.get("precond", True))


# Rows the CPU oracle reproduces within the suite's time budget (Table 1 to
# n1 = 256, the others to 128); the GPU tests cover every row of the tables.
def _rows(table, nmax, **match):
    return [r for r in GOLD[table]["rows"] if r["n1"] <= nmax and all(r[k] == v for k, v in match.items())]


@pytest.mark.parametrize("row", _rows("table1", 256), ids=lambda r: f"kx{r['kx']}-n{r['n1']}")
def test_table1_pgmres_iterations_and_error(row):
    err, it, _, _ = _ex1(row["n1"], row["kx"])
    assert abs(it - row["pgmres_iter"]) <= 0.02, (it, row)
    assert err == pytest.approx(row["gmres_err"], rel=0.03)


@pytest.mark.parametrize("row", _rows("table1", 128, kx=1.0), ids=lambda r: f"n{r['n1']}")
def test_table1_unpreconditioned_gmres_iterations(row):
    err, it, _, _ = _ex1(row["n1"], row["kx"], precond=False)
    assert abs(it - row["gmres_iter"]) <= 0.02


@pytest.mark.parametrize("row", _rows("table2", 128), ids=lambda r: f"n{r['n1']}")
def test_table2_long_time(row):
    n = row["n1"]
    err, it, _, _ = _ex1(n, 1.0, T=10.0, m=10 * n)
    assert abs(it - row["iter"]) <= 0.02
    assert err == pytest.approx(row["err"], rel=0.03)


@pytest.mark.parametrize("row", _rows("table3", 128), ids=lambda r: f"n{r['n1']}-eta{r['eta']}")
def test_table3_penalty_region(row):
    _, _, _, pen = _ex1(row["n1"], 1e-4, eta=row["eta"])
    assert pen == pytest.approx(row["pen"], rel=2e-4)


def test_first_order_convergence():
    """Errors halve with h and dt (convergence lemma of Section 3), Example 1 with LU."""
    errs = [O.example1_march(example1_workload(n, 1.0), use_lu=True)[0] for n in (16, 32, 64)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.6 < r1 < 2.4 and 1.6 < r2 < 2.4, errs


def test_stability_bound():
    """||eps^k||_inf <= (1 + dt c2)^k ||eps^0||_inf for a perturbed start (Section 3)."""
    w = make_config("c1", n=9, m=6)
    p = O.problem_from_workload(w)
    rng = np.random.default_rng(5)
    d0 = 1e-6 * rng.standard_normal(w.u0.shape) * w.mask
    ua = O.march_lu(p, w.u0, w.m, w.f_kind)
    ub = O.march_lu(p, w.u0 + d0, w.m, w.f_kind)
    c2 = 1.0 + 2.0 * max(np.abs(w.u0).max(), 1.0)   # Lipschitz constant of u(1-u) on the range
    assert np.abs(ua - ub).max() <= (1 + p.dt * c2) ** w.m * np.abs(d0).max()


def test_example1_source_is_the_scheme_consistent_fractional_term():
    """The Example-1 source field g0 (an input field) equals -(kx R_x + ky R_y) u_e at
    t = 0.  The GL operator of Section 2 applied to u_e approximates dt (kx R_x + ky R_y)
    u_e, so A u_e / dt + g0 -> 0 as h -> 0 (in the 2-norm over the domain; the
    boundary singularity s^{2-alpha} slows the max-norm).  A dropped term, a wrong
    sign or power in g0 leaves an O(1) remainder."""
    rel = []
    for n in (63, 127, 255):
        w = example1_workload(n, 1.0)
        p = O.problem_from_workload(w)
        e0, g0 = w.extra["exact0"], w.extra["src"]
        Ae = e0 - O.matvec_fast(p, e0)   # M e0 = e0 - A e0 (e0 = 0 in the penalty region)
        inside = w.mask.astype(bool)
        rel.append(np.linalg.norm((Ae / p.dt + g0)[inside]) / np.linalg.norm(g0[inside]))
    assert rel[-1] < 0.012, rel
    assert rel[0] / rel[1] > 1.5 and rel[1] / rel[2] > 1.5, rel
