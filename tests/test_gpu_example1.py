"""Grids whose n + 1 is not a power of two, the paper's stopping rule (left
preconditioning) and the paper's own workload, Example 1 of Section 5, on the
HIP path.

* preconditioner, chirp form: whole output against the oracle's dense DST
  (small grids) or library DST (larger), entry by entry on the whole grid and
  separately on the domain and on the penalty region, with the bars of the
  full-size preconditioner tests (1e-12 plus the eigenvalue conditioning for
  FP64 internals, each region against its own scale; 2e-5 for FP32);
* Example 1 in paper mode (GMRES(20), tol 1e-8, left preconditioning,
  x0 = 2u^{k-1} - u^{k-2}), every row of Tables 1-3 (n1 = 32 .. 512, Table 3
  to 1024): mean iterations per step within 0.02 of the values printed in
  Tables 1 and 2 for n1 <= 256 and within 0.1 at n1 = 512, errors within 3 %,
  penalty-region values of Table 3 to 2e-4 relative.  At n1 = 512 about a
  third of the steps stop on an estimate within 25 % of the threshold, and the
  extrapolated initial guess carries each step's stopping point into the
  next: runs that differ only in rounding (modified, classical or two-pass
  Gram-Schmidt on the CPU, or iterates perturbed by 1e-15 relative) have
  identical per-step counts for the first ~200 steps and then diverge, with
  mean Iter between 2.48 and 2.57 over eight such oracle runs (standard
  deviation 0.03; the paper prints 2.53).  The bar there is therefore 0.1
  (about three standard deviations), and the per-step counts are compared
  with the oracle's over the first 128 steps, where they are fixed;
* per-step iteration counts equal to the oracle's paper-mode GMRES at every
  step for n1 = 32, 128 and 256;
* first-order convergence in h and dt (Section 3) at n = 128, 256, 512.
"""

import json
import math
import os

import numpy as np
import pytest
import torch

import oracle as O
from workloads.configs import domain_mask, _ellipse, example1_workload, make_config
from bars import assert_precond

pytestmark = pytest.mark.gpu

rsfde = pytest.importorskip("paper_2102_11576_amd")
from paper_2102_11576_amd import RsfdePlan, make_opts  # noqa: E402

DEV = "cuda:0"
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV).reshape(-1)


def _problem(n1, n2):
    w = make_config("c2", n=max(n1, n2))
    box = (0.0, 1.0, 0.0, 1.2)
    mask = domain_mask(n1, n2, box, _ellipse(0.5, 0.6, 0.42, 0.5, 10.0))
    return O.Problem(n1, n2, box, w.alpha1, w.alpha2, 1.1, 0.7, w.eta, 1.0 / 64, mask)


def _plan(p, max_restart=30):
    return RsfdePlan(p.n1, p.n2, p.box, p.alpha1, p.alpha2, p.kx, p.ky, torch.as_tensor(p.mask),
                     p.eta, p.dt, max_restart)


CHIRP_SHAPES = [(1, 2), (2, 2), (4, 5), (31, 20), (32, 32), (33, 20), (64, 64), (100, 37),
                (20, 130), (300, 200)]


@pytest.mark.parametrize("n1,n2", CHIRP_SHAPES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_chirp_precond_parity(n1, n2, precision):
    p = _problem(n1, n2)
    V = np.random.default_rng(n1 * 7 + n2).standard_normal((n2, n1))
    ref = O.precond_apply(p, V) if n1 * n2 <= 4096 else O.precond_apply_fft(p, V)
    with _plan(p) as pl:
        out = pl.precond(_t(V), precision=precision).cpu().numpy().reshape(n2, n1)
    assert_precond(out, ref, p, precision, f"chirp {n1}x{n2} {precision}")


def test_chirp_precond_large_and_maximum_size():
    """n = 1000 x 999 (convolution length 2048) and the largest grid, 4096^2
    (length 8192), against the library DST of the oracle; at 4096^2 also the
    FP32 internals and the whole matrix-vector product against the oracle's
    FFT-Toeplitz form."""
    for n1, n2 in ((1000, 999), (4096, 4096)):
        p = _problem(n1, n2)
        V = np.random.default_rng(n1).standard_normal((n2, n1))
        ref = O.precond_apply_fft(p, V)
        with _plan(p, 8) as pl:
            out = pl.precond(_t(V), precision="fp64").cpu().numpy().reshape(n2, n1)
            assert_precond(out, ref, p, "fp64", f"chirp {n1}x{n2} fp64")
            if n1 == 4096:
                out = pl.precond(_t(V), precision="fp32").cpu().numpy().reshape(n2, n1)
                assert_precond(out, ref, p, "fp32", f"chirp {n1}x{n2} fp32")
                mv = pl.matvec(_t(V)).cpu().numpy().reshape(n2, n1)
                tx = np.abs(p.cx * O.toeplitz_first_column(p.alpha1, p.n1)).sum()
                ty = np.abs(p.cy * O.toeplitz_first_column(p.alpha2, p.n2)).sum()
                bound = 1e-13 * (1.0 + p.d + 2 * tx + 2 * ty) * np.abs(V).max()
                err = np.abs(mv - O.matvec_fast(p, V))
                assert err.max() <= bound, np.unravel_index(err.argmax(), err.shape)


def test_nonpow2_step_matches_lu_both_sides():
    """One FGMRES step and one paper-mode step at 20 x 20 (chirp preconditioner)
    against the dense LU solve of the same step."""
    w = make_config("c4", n=20, m=2)
    p = O.problem_from_workload(w)
    ref = O.march_lu(p, w.u0, w.m, w.f_kind)
    with RsfdePlan.from_workload(w) as pl:
        for side in ("right", "left"):
            u, _, _ = pl.march(_t(w.u0), w.m, w.f_kind, make_opts(30, 10000, 1e-13, side=side))
            u = u.cpu().numpy().reshape(w.n2, w.n1)
            assert np.abs(u - ref).max() / np.abs(ref).max() <= 1e-10, side


def _ex1_gpu(n, kx, precond="tau", side="left", reorth=0, **kw):
    w = example1_workload(n, kx, **kw)
    dt = w.T / w.m
    with RsfdePlan.from_workload(w) as pl:
        u, iters, _ = pl.march(_t(w.u0), w.m, w.f_kind,
                               make_opts(w.restart, 10000, w.tol, "fp64", precond, reorth, side),
                               src=_t(w.extra["src"]),
                               src_scale=lambda k: math.exp(-(k - 1) * dt))
        u = u.cpu().numpy().reshape(n, n)
    ue = math.exp(-w.T) * w.extra["exact0"]
    inside = w.mask.astype(bool)
    err = np.abs(ue - u)[inside].max() / np.abs(ue)[inside].max()
    pen = np.abs(u[~inside]).max()
    return float(err), float(np.mean(iters)), u, float(pen), iters


def iter_bar(n1):
    """Bar on the mean iterations per step against the paper's tables: 0.02 up
    to n1 = 256, 0.1 at n1 = 512 (rounding decides the stopping step of about
    a third of the steps there; see the module docstring)."""
    return 0.02 if n1 <= 256 else 0.1


@pytest.mark.parametrize("row", GOLD["table1"]["rows"], ids=lambda r: f"kx{r['kx']}-n{r['n1']}")
def test_table1_paper_mode(row):
    err, it, _, _, _ = _ex1_gpu(row["n1"], row["kx"])
    assert abs(it - row["pgmres_iter"]) <= iter_bar(row["n1"]), (it, row)
    assert err == pytest.approx(row["gmres_err"], rel=0.03)


@pytest.mark.parametrize("row", [r for r in GOLD["table1"]["rows"] if r["kx"] == 1.0],
                         ids=lambda r: f"n{r['n1']}")
def test_table1_unpreconditioned(row):
    _, it, _, _, _ = _ex1_gpu(row["n1"], row["kx"], precond="none", reorth=1)
    assert abs(it - row["gmres_iter"]) <= 0.02, (it, row)


@pytest.mark.parametrize("row", GOLD["table2"]["rows"], ids=lambda r: f"n{r['n1']}")
def test_table2_long_time(row):
    n = row["n1"]
    err, it, _, _, _ = _ex1_gpu(n, 1.0, T=10.0, m=10 * n)
    assert abs(it - row["iter"]) <= iter_bar(n), (it, row)
    assert err == pytest.approx(row["err"], rel=0.03)


@pytest.mark.parametrize("row", GOLD["table3"]["rows"], ids=lambda r: f"n{r['n1']}-eta{r['eta']}")
def test_table3_penalty_region(row):
    _, _, _, pen, _ = _ex1_gpu(row["n1"], 1e-4, eta=row["eta"])
    assert pen == pytest.approx(row["pen"], rel=2e-4)


@pytest.mark.parametrize("n", [32, 128, 256])
def test_paper_mode_matches_oracle_step_by_step(n):
    """Same algorithm on both sides (left GMRES(20), paper stopping rule): the
    iteration count of every step agrees and the solutions agree to the
    solver tolerance."""
    w = example1_workload(n, 1.0)
    p = O.problem_from_workload(w)
    g0 = w.extra["src"]
    u_o, it_o = O.march_gmres(p, w.u0, w.m, O.F_NONE, w.restart, w.tol, side="left",
                              f_values_fn=lambda km1, u: -u + math.exp(-km1 * p.dt) * g0)
    err_g, _, u_g, _, it_g = _ex1_gpu(n, 1.0)
    assert it_g == it_o
    assert np.abs(u_g - u_o).max() <= 1e-9 * np.abs(u_o).max()


def test_paper_mode_n512_first_steps_match_oracle():
    """n1 = 512: the per-step counts agree with the oracle's over the first 128
    steps, before rounding starts to decide stopping steps (the first
    difference between rounding-equivalent runs falls between steps 199 and
    272)."""
    n, K = 512, 128
    w = example1_workload(n, 1.0)
    p = O.problem_from_workload(w)
    g0 = w.extra["src"]
    _, it_o = O.march_gmres(p, w.u0, K, O.F_NONE, w.restart, w.tol, side="left",
                            f_values_fn=lambda km1, u: -u + math.exp(-km1 * p.dt) * g0)
    _, _, _, _, it_g = _ex1_gpu(n, 1.0)
    assert it_g[:K] == it_o


def test_first_order_convergence_at_larger_n():
    """Errors halve as h and dt halve (Section 3), n = 128 .. 1024 beyond the
    paper's tables (chirp-form preconditioner; right and left modes agree to
    the solver tolerance)."""
    errs = []
    for n in (128, 256, 512, 1024):
        err, it, _, _, _ = _ex1_gpu(n, 1.0)
        errs.append(err)
        assert it < 8, (n, it)
    ratios = [a / b for a, b in zip(errs, errs[1:])]
    assert all(1.6 < r < 2.4 for r in ratios), errs
    err_r, _, _, _, _ = _ex1_gpu(256, 1.0, side="right")
    assert err_r == pytest.approx(errs[1], rel=1e-3)


def test_paper_mode_fp32_preconditioner():
    """Paper mode with FP32 internals of the preconditioner (chirp form at
    n = 64): Table 1's error is kept and the mean Iter stays within 0.1."""
    row = [r for r in GOLD["table1"]["rows"] if r["kx"] == 1.0 and r["n1"] == 64][0]
    w = example1_workload(64, 1.0)
    dt = w.T / w.m
    with RsfdePlan.from_workload(w) as pl:
        u, iters, _ = pl.march(_t(w.u0), w.m, w.f_kind,
                               make_opts(w.restart, 10000, w.tol, "fp32", side="left"),
                               src=_t(w.extra["src"]), src_scale=lambda k: math.exp(-(k - 1) * dt))
        u = u.cpu().numpy().reshape(64, 64)
    ue = math.exp(-w.T) * w.extra["exact0"]
    inside = w.mask.astype(bool)
    err = np.abs(ue - u)[inside].max() / np.abs(ue)[inside].max()
    assert err == pytest.approx(row["gmres_err"], rel=0.03)
    assert abs(np.mean(iters) - row["pgmres_iter"]) <= 0.1
