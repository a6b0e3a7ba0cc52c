#!/usr/bin/env python
"""Throughput of the tau-preconditioned GMRES time march on one MI355X.

Workload (default): the 2047^2 rotated-ellipse configuration — alpha1 = alpha2
= 1.9, kx = ky = 1, eta = 1e-6, 32 implicit steps to T = 1, f(u) = sin u,
seeded 8-bump u0, flexible GMRES(30) to ||b - Mx|| <= 1e-8 ||b||.  A "step" is
one implicit time step: right-hand side, initial guess and the full Krylov
solve (preconditioner, matvec, Arnoldi, Givens, update, true residual).

Prints one JSON line: unknown*timesteps/s of the FP64 path (inputs resident in
HBM), GMRES iterations, the FP32-preconditioner variant and its error against
the FP64 result, the HBM roofline of the dominant kernel (HIP events on the
library's stream, algorithmic bytes) and the CPU oracle timed on this host.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TFS = 78.6   # 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz


def fft_flops(family, n1, n2):
    """Algorithmic FP64 flops of one launch of an FFT-based kernel family: the
    conventional 5 L log2(L) per complex FFT of length L (two real lines share
    one complex FFT), pointwise products not counted.  None for other families."""
    import math

    def f(L):
        return 5.0 * L * math.log2(L)
    def p2(v):
        L = 1
        while L < v:
            L *= 2
        return L
    Lcx, Lcy = max(2, p2(2 * n1)), max(2, p2(2 * n2))
    Ldx, Ldy = 2 * (n1 + 1), 2 * (n2 + 1)
    table = {
        "mv_rows": ((n2 + 1) // 2) * 2 * f(Lcx),        # forward + inverse per row pair
        "mv_cols": ((n1 + 1) // 2) * 2 * f(Lcy),
        "pc_rows_fwd": ((n2 + 1) // 2) * f(Ldx),         # forward per row pair
        "pc_cols": ((n1 + 1) // 2) * 3 * f(Ldy),         # forward + two inverses per column pair
        "pc_rows_inv": n2 * f(Ldx),                      # inverse per row
        # pass C (inverse per row) fused with the matvec row pass (conv per row pair)
        "pc_inv_mv_rows": n2 * f(Ldx) + ((n2 + 1) // 2) * 2 * f(Lcx),
    }
    return table.get(family)


def fft_flops3(family, n1, n2, n3):
    """As fft_flops for the three-dimensional plan: (flops of one operator
    application's launches of `family`, launches per application).  mv_cols is
    the y pass (per z slice) plus the z pass; dst_cols the stand-alone y
    transforms before and after the z pass of the preconditioner."""
    import math

    def f(L):
        return 5.0 * L * math.log2(L)

    def p2(v):
        L = 1
        while L < v:
            L *= 2
        return L
    Lc = [max(2, p2(2 * n)) for n in (n1, n2, n3)]
    Ld = [2 * (n + 1) for n in (n1, n2, n3)]
    rows, ld = n2 * n3, n1 + 1
    table = {
        "mv_rows": (((rows + 1) // 2) * 2 * f(Lc[0]), 1),
        "mv_cols": (((n1 + 1) // 2) * n3 * 2 * f(Lc[1]) + ((n1 * n2 + 1) // 2) * 2 * f(Lc[2]), 2),
        "pc_rows_fwd": (((rows + 1) // 2) * f(Ld[0]), 1),
        "dst_cols": ((ld // 2) * n3 * f(Ld[1]) + ld * n3 * f(Ld[1]), 2),
        "pc_cols": ((ld * n2 // 2) * 3 * f(Ld[2]), 1),
        "pc_rows_inv": (rows * f(Ld[0]), 1),
        "pc_inv_mv_rows": (rows * f(Ld[0]) + ((rows + 1) // 2) * 2 * f(Lc[0]), 1),
    }
    return table.get(family)


METRIC = "unknown·timesteps/s at 2047², mixed vs FP64 at 1e-8 rel err; adjoint grads/s"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed implicit steps (default: all 32)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--n", type=int, default=None, help="override the grid size (testing only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-three-d", action="store_true")
    ap.add_argument("--ex1-sizes", default="128,256,512,1024,2048,4096",
                    help="grid sizes of --mode example1")
    ap.add_argument("--mode", choices=["march", "kernels", "ablations", "three_d", "example1"],
                    default="march",
                    help="kernels: repeat each operator in isolation (for counter profiles)")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed marches of the headline (the median is reported)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the c1 / c2 / c5 legs")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--jsonl", default=None,
                    help="per-step metrics: after the timed runs, one more FP64 march of the "
                         "workload writes a JSON line per step (iterations, restarts, relative "
                         "residual, status, ms) to this file, after a header line")
    ap.add_argument("--no-one-vector", action="store_true",
                    help="skip the one-vector-per-step comparison march (profiling runs)")
    ap.add_argument("--sstep", type=int, default=10,
                    help="GMRES form of the timed march: s >= 2 the s-step block form, "
                         "0 one Arnoldi vector per step (both are reported)")
    return ap.parse_args()


def kernel_mode(args):
    """Each operator in isolation at the workload's shape, for rocprofv3 runs:
    a 256 MiB device copy (counter calibration: FETCH_SIZE and WRITE_SIZE of a
    copy of known size), then --reps applications of the matvec, of the FP64
    and FP32 preconditioner, and two implicit steps (Krylov kernels)."""
    import torch
    from paper_2102_11576_amd import RsfdePlan, make_opts
    from workloads.configs import make_config
    w = make_config(args.workload, n=args.n)
    dev = torch.device("cuda:0")
    a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log("copy calibration: 3 x 256 MiB device-to-device copies")
    plan = RsfdePlan.from_workload(w, device=dev)
    u0 = torch.as_tensor(w.u0, device=dev).reshape(-1).contiguous()
    y = plan.empty()
    for _ in range(args.reps):
        plan.matvec(u0, y)
    torch.cuda.synchronize()
    log(f"matvec x{args.reps}")
    for prec in ("fp64", "fp32"):
        for _ in range(args.reps):
            plan.precond(u0, y, prec)
        torch.cuda.synchronize()
        log(f"precond {prec} x{args.reps}")
    plan.march(u0, 2, w.f_kind, make_opts(w.restart, 100000, w.tol, sstep=args.sstep))
    torch.cuda.synchronize()
    log("2 implicit steps")
    plan.close()


def cpu_baseline(w, gpu_iters_per_step, log=lambda m: None):
    """The oracle as it stands, timed on this host's cores on a bounded sample
    of the same workload.

    Main figure (c3 at its full size): the right-hand side and one whole
    restart cycle (GMRES(30): inner iterations j = 0..29 with their growing
    modified Gram-Schmidt cost, the update and the true residual) of step 1,
    with the oracle's fast operators (scipy FFT Toeplitz products and the scipy
    DST-I preconditioner).  Every cycle of a step has this j-profile, so a step
    of K inner iterations costs (set-up) + (K / 30) cycles; K is the GPU run's
    mean (same algorithm and stopping rule).  Also reported: the dense-LU
    oracle (forming M, one LU factorisation, 16 solves) on the 63^2 shape of
    c1, timed whole."""
    import numpy as np
    import oracle as O
    from workloads.configs import make_config

    p = O.problem_from_workload(w)
    lam = O.tau_eigs_xy(p)
    A = lambda V: O.matvec_fast(p, V)  # noqa: E731
    Pi = lambda V: O.precond_apply_fft(p, V, lam)  # noqa: E731
    t0 = time.perf_counter()
    b = O.rhs(p, w.u0, w.f_kind)
    t_rhs = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, its, _ = O.gmres(A, b, w.u0, w.restart, 1e-300, w.restart, Pi, "right")
    t_cycle = time.perf_counter() - t0
    log(f"CPU oracle: one GMRES({w.restart}) cycle at {w.n1}^2 in {t_cycle:.1f} s")
    t_step = t_rhs + (gpu_iters_per_step / w.restart) * t_cycle
    # dense LU on the 63^2 shape (the oracle's dense tier), whole
    w1 = make_config("c1")
    p1 = O.problem_from_workload(w1)
    t0 = time.perf_counter()
    O.march_lu(p1, w1.u0, w1.m, w1.f_kind)
    t_lu = time.perf_counter() - t0
    blas = None
    try:
        from threadpoolctl import threadpool_info
        blas = max((int(i.get("num_threads", 1)) for i in threadpool_info()), default=None)
    except Exception:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except Exception:
        affinity = os.cpu_count()
    return {
        "value": w.N / t_step,
        "unit": "unknown·timesteps/s",
        "cores": affinity,
        "kind": "oracle",
        "sample": (f"{w.n1}x{w.n2} workload, step 1: right-hand side ({t_rhs:.2f} s) and one whole "
                   f"GMRES({w.restart}) restart cycle ({its} inner iterations, MGS, scipy FFT "
                   f"Toeplitz matvec, scipy DST-I preconditioner: {t_cycle:.1f} s); a step = "
                   f"set-up + {gpu_iters_per_step:.1f}/{w.restart} cycles (the GPU's mean "
                   f"iterations per step)"),
        "threads": {"scipy_fft_workers": os.cpu_count(), "blas": blas, "affinity_cpus": affinity},
        "dense_lu_c1": {"value": w1.N * w1.m / t_lu, "seconds": t_lu,
                        "sample": f"c1 63x63, 16 steps: dense M, one LU factorisation, 16 solves"},
    }


def adjoint_rate(log, sstep=0):
    """Adjoint gradients per second on the differentiation workload: 511^2 disk
    r=0.4, alpha=(1.3,1.6), 32 FP64 steps, L = ||u(T) - u_tgt||^2 with u_tgt
    marched at (kx, ky) = (1.2, 0.8); one gradient = forward march with
    ceil(sqrt(32)) = 6-step checkpoints + the reverse sweep (segment
    recomputation and one adjoint GMRES solve per step).  Two central
    differences (h = 1e-6, tol 1e-12) check the gradient on the spot."""
    import numpy as np
    import torch
    from paper_2102_11576_amd import RsfdePlan, make_opts
    from paper_2102_11576_amd.autograd import RsfdeMarch
    from workloads.configs import make_config, fd_direction
    w = make_config("c4")
    dev = torch.device("cuda:0")
    res = {"workload": "c4: 511x511 disk r=0.4, alpha=(1.3,1.6), 32 steps, GMRES(30) tol 1e-8 "
                       "(FD check at tol 1e-12), loss ||u(T)-u_tgt||^2, grads w.r.t. u0, kx, ky",
           "gmres_form": f"s-step (s={sstep})" if sstep >= 2 else "one vector per step"}
    with RsfdePlan.from_workload(w, device=dev) as pl:
        u0 = torch.as_tensor(w.u0, device=dev).reshape(-1).contiguous()
        opts = make_opts(w.restart, 100000, w.tol, sstep=sstep)
        pl.set_coeffs(*w.extra["target_k"])
        u_tgt = pl.march(u0, w.m, w.f_kind, make_opts(w.restart, 100000, 1e-12))[0].clone()

        def grad(op):
            x0 = u0.clone().requires_grad_(True)
            kx = torch.tensor(w.kx, dtype=torch.float64, device=dev, requires_grad=True)
            ky = torch.tensor(w.ky, dtype=torch.float64, device=dev, requires_grad=True)
            uT = RsfdeMarch.apply(x0, kx, ky, pl, w.m, w.f_kind, op)
            ((uT - u_tgt) ** 2).sum().backward()
            return x0.grad, float(kx.grad), float(ky.grad)

        grad(opts)  # warm-up
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            grad(opts)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        res.update({"grads_per_s": 1.0 / dt, "s_per_grad": dt})
        log(f"adjoint: {dt:.3f} s per gradient (forward + reverse sweep)")
        tight = make_opts(w.restart, 100000, 1e-12, sstep=sstep)
        g0, gkx, gky = grad(tight)

        def loss(uu0, kx, ky):
            pl.set_coeffs(kx, ky)
            uT = pl.march(uu0, w.m, w.f_kind, tight)[0]
            return float(((uT - u_tgt) ** 2).sum())
        errs = []
        for i in range(2):
            du, dkx, dky = fd_direction(w.u0.shape, i)
            dut = torch.as_tensor(du, device=dev).reshape(-1)
            h = w.extra["fd_h"]
            fd = (loss(u0 + h * dut, w.kx + h * dkx, w.ky + h * dky)
                  - loss(u0 - h * dut, w.kx - h * dkx, w.ky - h * dky)) / (2 * h)
            an = float(torch.dot(g0, dut)) + gkx * dkx + gky * dky
            errs.append(abs(fd - an) / abs(an))
        res["fd_rel_err_2_dirs"] = errs
    return res


def configs_rates(log, sstep=10):
    """The other configurations of the benchmark family, each marched whole.

    c1 (63^2 disk, 16 steps, GMRES(20) tol 1e-10, one Arnoldi vector per step:
    the grid is below the s-step floor of 4096 unknowns): latency-bound, so
    microseconds per inner iteration are reported.  c2 (1023^2 ellipse, 64
    steps, GMRES(30) tol 1e-8, s-step): throughput.  c5 (4095^2 hexagon, 16
    steps, FP32 preconditioner inside FGMRES(20) tol 1e-8, s-step): forward
    march, then one backward pass (checkpointed forward + adjoint sweep, FP32
    preconditioner in both) for the gradient of L = ||u(T)||^2 with respect to
    u0, kx and ky, checked by central differences (h = 1e-4, tol 1e-10: the
    residual's rounding floor at this stiffness is near 5e-11) on two seeded
    directions."""
    import numpy as np
    import torch
    from paper_2102_11576_amd import RsfdePlan, make_opts
    from paper_2102_11576_amd.autograd import RsfdeMarch
    from workloads.configs import make_config, fd_direction
    dev = torch.device("cuda:0")
    res = {}

    def march(pl, w, opts, reps):
        u0 = torch.as_tensor(w.u0, device=dev).reshape(-1).contiguous()
        pl.march(u0, min(2, w.m), w.f_kind, opts)
        torch.cuda.synchronize()
        ts, its = [], None
        for _ in range(reps):
            t0 = time.perf_counter()
            _, its, _ = pl.march(u0, w.m, w.f_kind, opts)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), its

    w = make_config("c1")
    with RsfdePlan.from_workload(w, device=dev) as pl:
        t, its = march(pl, w, make_opts(w.restart, 100000, w.tol), 5)
    res["c1"] = {"workload": "c1: 63x63 disk r=0.45, alpha=(1.5,1.7), 16 steps, GMRES(20) tol 1e-10, "
                             "one vector per step", "unknown_timesteps_per_s": w.N * w.m / t,
                 "us_per_iteration": 1e6 * t / sum(its), "gmres_iters_per_step": float(np.mean(its)),
                 "ms_per_step": 1e3 * t / w.m, "timing": "median of 5 whole marches"}
    log(f"c1: {res['c1']['us_per_iteration']:.1f} us/iteration, {np.mean(its):.1f} iterations/step")

    w = make_config("c2")
    with RsfdePlan.from_workload(w, device=dev) as pl:
        t, its = march(pl, w, make_opts(w.restart, 100000, w.tol, sstep=sstep), 5)
    res["c2"] = {"workload": "c2: 1023x1023 ellipse .45/.30, alpha=(1.2,1.8), k=(1,0.5), 64 steps, "
                             f"GMRES(30) tol 1e-8, s-step (s={sstep})",
                 "unknown_timesteps_per_s": w.N * w.m / t, "ms_per_step": 1e3 * t / w.m,
                 "gmres_iters_per_step": float(np.mean(its)), "timing": "median of 5 whole marches"}
    log(f"c2: {res['c2']['unknown_timesteps_per_s']:.3e} unknown*timesteps/s, {np.mean(its):.1f} it/step")

    w = make_config("c5")
    opts = make_opts(w.restart, 100000, w.tol, "fp32", sstep=sstep)
    with RsfdePlan.from_workload(w, device=dev) as pl:
        t, its = march(pl, w, opts, 1)
        r5 = {"workload": "c5: 4095x4095 hexagon R=0.45, alpha=(1.4,1.75), 16 steps, f=u-u^3, "
                          f"FP32 preconditioner in FGMRES(20) tol 1e-8, s-step (s={sstep})",
              "unknown_timesteps_per_s": w.N * w.m / t, "ms_per_step": 1e3 * t / w.m,
              "gmres_iters_per_step": float(np.mean(its))}
        log(f"c5 forward: {r5['unknown_timesteps_per_s']:.3e} unknown*timesteps/s")
        u0 = torch.as_tensor(w.u0, device=dev).reshape(-1).contiguous()

        def grad(op):
            x0 = u0.clone().requires_grad_(True)
            kx = torch.tensor(w.kx, dtype=torch.float64, device=dev, requires_grad=True)
            ky = torch.tensor(w.ky, dtype=torch.float64, device=dev, requires_grad=True)
            uT = RsfdeMarch.apply(x0, kx, ky, pl, w.m, w.f_kind, op)
            (uT * uT).sum().backward()
            return x0.grad, float(kx.grad), float(ky.grad)

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        grad(opts)
        torch.cuda.synchronize()
        r5["backward_pass_s"] = time.perf_counter() - t0
        log(f"c5 gradient (checkpointed forward + adjoint sweep): {r5['backward_pass_s']:.2f} s")
        # FD at tol 1e-10 (the residual's rounding floor at 4095^2 is near
        # 5e-11) with h = 1e-4: noise ~ tol / h = 1e-6, truncation ~ h^2
        tight = make_opts(w.restart, 100000, 1e-10, "fp32", sstep=0)
        g0, gkx, gky = grad(tight)

        def loss(uu0, kx, ky):
            pl.set_coeffs(kx, ky)
            uT = pl.march(uu0, w.m, w.f_kind, tight)[0]
            return float((uT * uT).sum())
        errs = []
        for i in range(2):
            du, dkx, dky = fd_direction(w.u0.shape, i)
            dut = torch.as_tensor(du, device=dev).reshape(-1)
            h = 1e-4
            fd = (loss(u0 + h * dut, w.kx + h * dkx, w.ky + h * dky)
                  - loss(u0 - h * dut, w.kx - h * dkx, w.ky - h * dky)) / (2 * h)
            an = float(torch.dot(g0, dut)) + gkx * dkx + gky * dky
            errs.append(abs(fd - an) / abs(an))
        pl.set_coeffs(w.kx, w.ky)
        r5["fd_rel_err_2_dirs"] = errs
        r5["loss"] = "||u(T)||^2; gradient w.r.t. u0 (full field), kx, ky"
        log(f"c5 FD check: {errs}")
    res["c5"] = r5
    return res


def ensemble_rate(log, sstep=0, steps=8):
    """Independent marches of one grid (FD directions, parameter sweeps): B
    members with their own kx and perturbed u0, advanced `steps` steps each,
    three ways: one batched solve (rsfde_batch_step: every kernel launched once
    for all members, one host decision per inner step for the batch), the
    members as separate plans on their own streams (rsfde_march_ensemble), and
    one member alone (the single-march rate).  The 511^2 differentiation grid
    and the 63^2 grid of the small configuration, B = 8 and 16."""
    import numpy as np
    import torch
    from paper_2102_11576_amd import RsfdeBatch, RsfdePlan, make_opts, march_ensemble
    from workloads.configs import make_config, fd_direction
    dev = torch.device("cuda:0")
    out = {"note": "unknown*timesteps/s over all members; batched: one-vector FGMRES with two "
                   "Gram-Schmidt passes; streams and single: the same form"}
    for name in ("c4", "c1"):
        w = make_config(name)
        opts = make_opts(w.restart, 100000, w.tol, sstep=0)
        single = None
        for B in (8, 16):
            kxs = [1.0 + 0.02 * i for i in range(B)]
            kys = [w.ky] * B
            u0s = []
            for i in range(B):
                du, _, _ = fd_direction(w.u0.shape, i)
                u0s.append(w.u0 + 1e-3 * du * w.mask)
            u0b = torch.as_tensor(np.stack(u0s), device=dev).reshape(-1).contiguous()
            unk = float(w.N) * steps * B
            with RsfdeBatch.from_workload(w, kxs, kys, device=dev) as bt:
                bt.march(u0b, 1, w.f_kind, opts)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, itb = bt.march(u0b, steps, w.f_kind, opts)
                torch.cuda.synchronize()
                t_b = time.perf_counter() - t0
            plans = [RsfdePlan.from_workload(w, kx=kxs[i], device=dev) for i in range(B)]
            u0t = [torch.as_tensor(u, device=dev).reshape(-1).contiguous() for u in u0s]
            streams = [torch.cuda.Stream() for _ in plans]
            march_ensemble(plans, u0t, 1, w.f_kind, opts, streams)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            march_ensemble(plans, u0t, steps, w.f_kind, opts, streams)
            torch.cuda.synchronize()
            t_s = time.perf_counter() - t0
            if single is None:
                plans[0].march(u0t[0], 1, w.f_kind, opts)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                plans[0].march(u0t[0], steps, w.f_kind, opts)
                torch.cuda.synchronize()
                single = float(w.N) * steps / (time.perf_counter() - t0)
            for pl in plans:
                pl.close()
            row = {"members": B, "steps": steps,
                   "batched_unknown_timesteps_per_s": unk / t_b,
                   "streams_unknown_timesteps_per_s": unk / t_s,
                   "single_march_unknown_timesteps_per_s": single,
                   "batched_over_streams": t_s / t_b,
                   "batched_iters_per_member_step": float(np.mean(itb))}
            out[f"{name}_{w.n1}_B{B}"] = row
            log(f"ensemble {name} {w.n1}^2 B={B}: batched {row['batched_unknown_timesteps_per_s']:.3e}, "
                f"streams {row['streams_unknown_timesteps_per_s']:.3e}, single {single:.3e}")
    return out


def three_d_rate(log, sstep=10, steps=4, profile=True, one_vector=True, fp32=True):
    """The three-dimensional plan on its 255^3 workload (ellipsoid, alpha =
    (1.6, 1.7, 1.8), 16 steps to T = 1, f = u(1-u), GMRES(30) tol 1e-8): the
    first `steps` implicit steps after one warm-up step, s-step and one-vector
    GMRES with the FP64 preconditioner and s-step with FP32 internals, plus the
    per-family kernel times of the s-step run (HIP events)."""
    import numpy as np
    import torch
    from paper_2102_11576_amd import RsfdePlan, make_opts
    from paper_2102_11576_amd import _lib as L
    from workloads.three_d import make_config3d
    w = make_config3d()
    dev = torch.device("cuda:0")
    res = {"workload": (f"e3: {w.n1}x{w.n2}x{w.n3} grid, ellipsoid 0.45/0.35/0.30 in [0,1]^3, "
                        f"alpha=({w.alpha1},{w.alpha2},{w.alpha3}), k=(1,1,1), eta={w.eta}, "
                        f"{w.m} steps to T={w.T}, f=u(1-u), 6 seeded Gaussian bumps, "
                        f"FGMRES({w.restart}) tol {w.tol}; first {steps} steps timed"),
           "unit": "unknown·timesteps/s", "N": w.N}
    with RsfdePlan.from_workload3(w, device=dev) as pl:
        u0 = torch.as_tensor(w.u0, device=dev).reshape(-1).contiguous()

        def run(precision, ss, prof=False):
            opts = make_opts(w.restart, 100000, w.tol, precision, sstep=ss)
            pl.march(u0, 1, w.f_kind, opts)
            torch.cuda.synchronize()
            if prof:
                L.rsfde_profile(pl.handle, True)
                L.rsfde_profile_read(pl.handle)
            t0 = time.perf_counter()
            u, it, _ = pl.march(u0, steps, w.f_kind, opts)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            pr = None
            if prof:
                pr = L.rsfde_profile_read(pl.handle)
                L.rsfde_profile(pl.handle, False)
            form = f"s-step (s={ss})" if ss >= 2 else "one vector per step"
            log(f"3-D {precision}, {form}: {1e3 * dt / steps:.2f} ms/step, "
                f"{np.mean(it):.1f} iterations/step")
            return u, {"value": w.N * steps / dt, "ms_per_step": 1e3 * dt / steps,
                       "gmres_iters_per_step": float(np.mean(it)), "gmres_form": form,
                       "preconditioner": precision}, pr

        u8, main, _ = run("fp64", sstep)
        res.update(main)
        if one_vector:
            u1, one, _ = run("fp64", 0)
            one["rel_err_inf_vs_sstep"] = float((u1 - u8).abs().max() / u8.abs().max())
            res["one_vector_per_step"] = one
        if fp32:
            u32, r32, _ = run("fp32", sstep)
            r32["rel_err_inf_vs_fp64"] = float((u32 - u8).abs().max() / u8.abs().max())
            res["fp32"] = r32
        if profile:
            _, _, pr = run("fp64", sstep, prof=True)
            kernels = {}
            for name, (n, ms, by) in sorted(pr.items(), key=lambda kv: -kv[1][1]):
                kv = {"launches": n, "total_ms": ms, "avg_us": 1e3 * ms / n,
                      "alg_GBs": by / (ms * 1e-3) / 1e9 if ms > 0 else None}
                fl = fft_flops3(name, w.n1, w.n2, w.n3)
                if fl is not None and ms > 0:
                    kv["fp64_TFs"] = fl[0] * (n / fl[1]) / (ms * 1e-3) / 1e12
                    kv["frac_of_fp64_valu_peak"] = kv["fp64_TFs"] / FP64_VALU_PEAK_TFS
                kernels[name] = kv
            res["kernels"] = kernels
    return res


def example1_large(args):
    """The paper's Example 1 (Section 5: ellipse a = 2, b = 1 in (0,4) x (0,2),
    alpha = (1.4, 1.7), kx = ky = 1, eta = 1e-5, T = 1 with m = n1 steps,
    manufactured source, paper mode: left preconditioning, GMRES(20), tol 1e-8)
    on the GPU from the table sizes up to n1 = 4096 (n1 + 1 is not a power of
    two, so the chirp-form sine transforms run).  Per size: mean iterations per
    step, the error against the exact solution inside the domain (max norm,
    relative) and its ratio to the previous size (first order: about 2), time
    and unknown*timesteps/s.  One JSON line."""
    import math
    import numpy as np
    import torch
    from paper_2102_11576_amd import RsfdePlan, make_opts
    from workloads.configs import example1_workload
    sizes = [int(v) for v in args.ex1_sizes.split(",")]
    dev = torch.device("cuda:0")
    rows, prev = [], None
    for n in sizes:
        w = example1_workload(n, 1.0)
        dt = w.T / w.m
        opts = make_opts(w.restart, 10000, w.tol, "fp64", side="left")
        with RsfdePlan.from_workload(w, device=dev) as pl:
            u0 = torch.as_tensor(w.u0, device=dev).reshape(-1).contiguous()
            src = torch.as_tensor(w.extra["src"], device=dev).reshape(-1).contiguous()
            pl.march(u0, 2, w.f_kind, opts, src=src, src_scale=lambda k: math.exp(-(k - 1) * dt))
            torch.cuda.synchronize()
            # the march of solver.RsfdePlan.march, stepped here to report progress
            bufs = [u0.clone(), pl.empty(), pl.empty()]
            cur, prv, iters = 0, None, []
            t0 = time.perf_counter()
            for k in range(1, w.m + 1):
                nxt = [i for i in range(3) if i != cur and i != prv][0]
                _, st = pl.step(bufs[cur], None if prv is None else bufs[prv], w.f_kind, opts,
                                bufs[nxt], src=src, src_scale=math.exp(-(k - 1) * dt))
                iters.append(st.iters)
                prv, cur = cur, nxt
                if k % 512 == 0 and k < w.m:
                    log(f"example 1, n1 = {n}: step {k} of {w.m}")
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            u = bufs[cur].cpu().numpy().reshape(n, n)
        ue = math.exp(-w.T) * w.extra["exact0"]
        inside = w.mask.astype(bool)
        err = float(np.abs(ue - u)[inside].max() / np.abs(ue)[inside].max())
        row = {"n1": n, "steps": w.m, "iter_mean": float(np.mean(iters)), "rel_err_max": err,
               "err_ratio_to_previous": (prev / err) if prev else None, "seconds": el,
               "unknown_timesteps_per_s": n * n * w.m / el}
        prev = err
        rows.append(row)
        log(f"example 1, n1 = {n}: {w.m} steps in {el:.1f} s, Iter {row['iter_mean']:.2f}, "
            f"error {err:.3e}" + (f" (ratio {row['err_ratio_to_previous']:.2f})" if row['err_ratio_to_previous'] else ""))
    print(json.dumps({"example1": rows, "note": "paper mode (left preconditioning, GMRES(20), "
                      "tol 1e-8 on the preconditioned residual), kx = ky = 1, T = 1, m = n1"}))


def traffic_for(kernel, bytes_per_launch):
    """Measured HBM bytes per launch of `kernel` from the committed counter
    summary, if it was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "counters_c3_2047.txt")
    try:
        from paper_2102_11576_amd.profiling import source_hash
        d = json.load(open(path))
        if d.get("source_hash") != source_hash():
            return None
        f = d["families"].get(kernel) or d["families"].get(kernel + "<double>")
        return None if f is None else f["traffic_over_alg"] * bytes_per_launch
    except Exception:
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def ablations(args):
    """Arnoldi-traffic ablations on the benchmark march (FP64 preconditioner,
    tol 1e-8): GMRES form (one-vector CGS, CGS2, s-step s = 2..16, which is also the
    sweep of s) and restart
    length, each timed over the same steps.  One JSON line."""
    import numpy as np
    import torch
    from paper_2102_11576_amd import RsfdePlan, make_opts
    from workloads.configs import make_config
    w = make_config(args.workload, n=args.n)
    K = min(w.m, args.steps or 8)
    dev = torch.device("cuda:0")
    plan = RsfdePlan.from_workload(w, max_restart=64, device=dev)
    u0 = torch.as_tensor(w.u0, device=dev).reshape(-1).contiguous()

    def run(restart, sstep, reorth=0):
        opts = make_opts(restart, 100000, w.tol, "fp64", reorth=reorth, sstep=sstep)
        plan.march(u0, 1, w.f_kind, opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, it, _ = plan.march(u0, K, w.f_kind, opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        row = {"restart": restart, "sstep": sstep, "reorth": reorth, "ms_per_step": 1e3 * dt / K,
               "gmres_iters_per_step": float(np.mean(it))}
        log(f"ablation restart {restart} sstep {sstep} reorth {reorth}: "
            f"{row['ms_per_step']:.2f} ms/step, {row['gmres_iters_per_step']:.1f} it/step")
        return row
    rows = [run(w.restart, 0, -1), run(w.restart, 0, 1)]
    rows += [run(w.restart, s) for s in (2, 4, 6, 8, 10, 12, 16)]
    rows += [run(r, 8) for r in (10, 20, 40, 60)]
    rows += [run(r, 0, -1) for r in (10, 20, 40, 60)]
    plan.close()
    print(json.dumps({"ablations": rows, "workload": w.name, "n": w.n1, "steps": K,
                      "note": "sstep 0 = one Arnoldi vector per step (reorth -1: one CGS pass, "
                              "1: two); sstep s >= 2 = s-step blocks"}))


def main():
    args = parse()
    if args.mode == "kernels":
        kernel_mode(args)
        return
    if args.mode == "ablations":
        ablations(args)
        return
    if args.mode == "example1":
        example1_large(args)
        return
    if args.mode == "three_d":  # the 3-D leg alone (for kernel traces)
        print(json.dumps({"three_d": three_d_rate(log, args.sstep, args.steps or 4,
                                                  profile=not args.no_profile,
                                                  one_vector=not args.no_one_vector,
                                                  fp32=not args.no_mixed)}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; sharding the grid "
                                   "over several GPUs is not implemented. Use --gpus 1."}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2102_11576_amd import RsfdePlan, make_opts
    from paper_2102_11576_amd import _lib as L
    from workloads.configs import make_config

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = make_config(args.workload, n=args.n)
    K = w.m if args.steps is None else args.steps
    W = args.warmup
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    plan = RsfdePlan.from_workload(w, device=dev)
    u0 = torch.as_tensor(w.u0, device=dev).reshape(-1).contiguous()

    def timed_march(precision, steps, profile=False, sstep=args.sstep, zstore="fp64"):
        opts = make_opts(w.restart, 100000, w.tol, precision, sstep=sstep, zstore=zstore)
        if W > 0:
            plan.march(u0, min(W, w.m), w.f_kind, opts)
        torch.cuda.synchronize()
        if profile:
            L.rsfde_profile(plan.handle, True)
            L.rsfde_profile_read(plan.handle)
        t0 = time.perf_counter()
        u, iters, _ = plan.march(u0, steps, w.f_kind, opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = None
        if profile:
            prof = L.rsfde_profile_read(plan.handle)
            L.rsfde_profile(plan.handle, False)
        return u, iters, dt, prof

    log(f"workload {w.name} {w.n1}x{w.n2}, timing {K} steps after {W} warm-up steps, "
        f"{args.repeats} runs")
    runs = []
    for r in range(max(1, args.repeats)):
        u64, it64, t, _ = timed_march("fp64", K)
        runs.append(t)
        log(f"run {r + 1}: {1e3 * t / K:.2f} ms/step")
    t64 = float(np.median(runs))
    value = w.N * K / t64
    if args.jsonl:  # outside the timed region
        with open(args.jsonl, "a") as fh:
            fh.write(json.dumps({"workload": w.name, "n1": w.n1, "n2": w.n2, "steps": K,
                                 "precision": "fp64", "sstep": args.sstep, "restart": w.restart,
                                 "tol": w.tol, "ms_per_step_median": 1e3 * t64 / K}) + "\n")
            plan.march(u0, K, w.f_kind, make_opts(w.restart, 100000, w.tol, "fp64",
                                                  sstep=args.sstep), log=fh)
        log(f"per-step metrics written to {args.jsonl}")
    form = f"s-step (s={args.sstep})" if args.sstep >= 2 else "one vector per step"
    log(f"fp64, {form}: {1e3 * t64 / K:.2f} ms/step (median), {np.mean(it64):.1f} iterations/step")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "unknown·timesteps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * t64 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{w.name}: {w.n1}x{w.n2} grid, rotated ellipse 0.45/0.25 at 30 deg in [0,1]^2, "
                         f"alpha=({w.alpha1},{w.alpha2}), k=({w.kx},{w.ky}), eta={w.eta}, {w.m} steps "
                         f"to T={w.T}, f=sin(u), 8 seeded Gaussian bumps, FGMRES({w.restart}) tol {w.tol}"),
            "n1": w.n1, "n2": w.n2, "time_steps_total": w.m, "restart": w.restart, "tol": w.tol,
            "preconditioner": "fp64",
            "gmres_form": form,
        },
        "timing": {"statistic": f"median of {len(runs)} timed marches of {K} steps",
                   "ms_per_step_runs": [1e3 * t / K for t in runs]},
        "gmres_iters_per_step": float(np.mean(it64)),
        "gmres_iters": it64,
    }
    if args.sstep >= 2 and not args.no_one_vector:
        u1, it1, t1, _ = timed_march("fp64", K, sstep=0)
        log(f"fp64, one vector per step: {1e3 * t1 / K:.2f} ms/step, {np.mean(it1):.1f} iterations/step")
        out["one_vector_per_step"] = {
            "value": w.N * K / t1, "ms_per_step": 1e3 * t1 / K,
            "gmres_iters_per_step": float(np.mean(it1)),
            "rel_err_inf_vs_sstep": float((u1 - u64).abs().max() / u64.abs().max())}

    if not args.no_mixed:
        u32, it32, t32, _ = timed_march("fp32", K)
        log(f"fp32 preconditioner: {1e3 * t32 / K:.2f} ms/step, {np.mean(it32):.1f} iterations/step")
        d = float((u32 - u64).abs().max() / u64.abs().max())
        # the preconditioned basis Z kept in FP32 (with either preconditioner)
        zres = {}
        for prec in ("fp64", "fp32"):
            uz, itz, tz, _ = timed_march(prec, K, zstore="fp32")
            zres[prec] = {"value": w.N * K / tz, "ms_per_step": 1e3 * tz / K,
                          "gmres_iters_per_step": float(np.mean(itz)),
                          "rel_err_inf_vs_fp64": float((uz - u64).abs().max() / u64.abs().max())}
            log(f"{prec} preconditioner, Z in FP32: {1e3 * tz / K:.2f} ms/step, "
                f"{np.mean(itz):.1f} iterations/step")
        # Tight FP64 reference (one Arnoldi vector per step, two Gram-Schmidt
        # passes) at tol 1e-10: at this stiffness the true residual b - Mx
        # computed in FP64 carries a rounding floor of about eps sum_j |M_ij| |x_j|
        # (sum_j |M_ij| ~ 3.5e5), i.e. about 4e-11 of ||b||, so 1e-12 and 1e-11
        # are out of reach; the achieved relative residuals are reported.
        TIGHT = 1e-10
        opts_t = make_opts(w.restart, 3000, TIGHT, "fp64", sstep=0)
        bufs = [u0.clone(), plan.empty(), plan.empty()]
        cur, prv, it_t, rel_t = 0, None, [], []
        for _ in range(K):
            nxt = [i for i in range(3) if i != cur and i != prv][0]
            _, st_t = plan.step(bufs[cur], None if prv is None else bufs[prv], w.f_kind, opts_t,
                                bufs[nxt], check=False)
            it_t.append(st_t.iters)
            rel_t.append(st_t.relres)
            prv, cur = cur, nxt
            if len(it_t) % 8 == 0:
                log(f"tight reference: step {len(it_t)}, {st_t.iters} iterations, relres {st_t.relres:.2e}")
        torch.cuda.synchronize()
        u_t = bufs[cur]
        d64_t = float((u64 - u_t).abs().max() / u_t.abs().max())
        d32_t = float((u32 - u_t).abs().max() / u_t.abs().max())
        log(f"vs FP64 at tol {TIGHT:g} (largest relative residual {max(rel_t):.2e}): "
            f"fp64 {d64_t:.2e}, fp32 {d32_t:.2e}")
        # BF16 preconditioner: not supported at this stiffness.  Flexible GMRES
        # stalls from step 3 on (the BF16 rounding of each preconditioned
        # vector, about 6e-3 relative, is amplified by ||M|| ~ 1e5 in the next
        # product); the first KB steps converge and are reported as such.
        KB = min(2, K)
        u64b, _, _, _ = timed_march("fp64", KB, sstep=0)
        ub, itb, tb, profb = timed_march("bf16", KB, profile=not args.no_profile, sstep=0)
        log(f"bf16 preconditioner ({KB} steps): {1e3 * tb / KB:.2f} ms/step, "
            f"{np.mean(itb):.1f} iterations/step")
        db = float((ub - u64b).abs().max() / u64b.abs().max())
        out["mixed"] = {
            "fp32": {"value": w.N * K / t32, "ms_per_step": 1e3 * t32 / K, "steps": K,
                     "gmres_iters_per_step": float(np.mean(it32)), "rel_err_inf_vs_fp64": d,
                     "rel_err_inf_vs_fp64_tight": d32_t},
            "zstore_fp32": {"note": "preconditioned basis Z stored in FP32 (rounded when "
                                    "stored; M z formed from the stored vector)",
                            "fp64_preconditioner": zres["fp64"], "fp32_preconditioner": zres["fp32"]},
            "fp64_rel_err_inf_vs_fp64_tight": d64_t,
            "fp64_tight": {"tol": TIGHT, "iters_per_step": float(np.mean(it_t)),
                           "max_relres": float(max(rel_t)),
                           "note": "tol 1e-12 (and 1e-11) is below the FP64 rounding floor of "
                                   "the true residual at this stiffness (about eps "
                                   "max_i sum_j |M_ij| ~ 4e-11)"},
            "bf16": {"supported": False,
                     "reason": "flexible GMRES stalls from step 3 on at this stiffness: the BF16 "
                               "rounding of each preconditioned vector (about 6e-3 relative) is "
                               "amplified by ||M|| ~ 1e5 in the next matrix-vector product",
                     "first_steps": {"value": w.N * KB / tb, "ms_per_step": 1e3 * tb / KB,
                                     "steps": KB, "gmres_iters_per_step": float(np.mean(itb)),
                                     "rel_err_inf_vs_fp64": db}},
        }
        if profb and "pc_gemm_bf16" in profb:
            n_l, ms_l, _ = profb["pc_gemm_bf16"]
            n1p, n2p = (w.n1 + 127) // 128 * 128, (w.n2 + 127) // 128 * 128
            # forward products with split (3 MFMA) operands: 2*3*n1p*n2p*(n1p + n2p); inverse
            # products: 2*2*n1p*n2p*(n1p + n2p)  (20 n^3 per apply for n1 = n2)
            flops = 10.0 * n1p * n2p * (n1p + n2p)
            tfs = flops / (ms_l / n_l * 1e-3) / 1e12
            out["mixed"]["bf16"]["first_steps"]["mfma_roofline"] = {
                "kernel": "pc_gemm_bf16", "bound": "mfma", "achieved": tfs, "peak": 2500.0,
                "unit": "TFLOP/s", "frac": tfs / 2500.0, "avg_apply_us": 1e3 * ms_l / n_l,
                "flops_per_apply": flops}

    if not args.no_profile:
        _, _, tprof, prof = timed_march("fp64", K, profile=True)
        log(f"profiled run: {1e3 * tprof / K:.2f} ms/step")
        kernels = {}
        for name, (n, ms, by) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
            kernels[name] = {"launches": n, "total_ms": ms, "avg_us": 1e3 * ms / n,
                             "achieved_GBs": by / (ms * 1e-3) / 1e9 if ms > 0 else None,
                             "hbm_frac": (by / (ms * 1e-3) / 1e9) / HBM_PEAK_GBS if ms > 0 else None}
        dom = max(prof.items(), key=lambda kv: kv[1][1])
        name, (n, ms, by) = dom
        ach = by / (ms * 1e-3) / 1e9
        fl = fft_flops(name, w.n1, w.n2)
        if fl is not None:
            # FFT passes: bound by FP64 vector issue and LDS exchanges, not by HBM
            tfs = fl / (ms / n * 1e-3) / 1e12
            traf = traffic_for(name, by / n)
            out["roofline"] = {"bound": "alu", "kernel": name, "achieved": tfs,
                               "peak": FP64_VALU_PEAK_TFS, "unit": "TFLOP/s",
                               "frac": tfs / FP64_VALU_PEAK_TFS,
                               "traffic": traf,
                               "flops_per_launch": fl, "alg_bytes_per_launch": by / n,
                               "hbm_GBs_algorithmic": ach, "hbm_frac_algorithmic": ach / HBM_PEAK_GBS,
                               "hbm_frac_counters": (traf / (ms / n * 1e-3) / 1e9 / HBM_PEAK_GBS
                                                     if traf else None),
                               "avg_launch_us": 1e3 * ms / n}
        else:
            out["roofline"] = {"bound": "hbm", "kernel": name, "achieved": ach,
                               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                               "traffic": traffic_for(name, by / n),
                               "bytes_per_launch_avg": by / n, "avg_launch_us": 1e3 * ms / n}
        for nm, kv in kernels.items():
            flk = fft_flops(nm, w.n1, w.n2)
            if flk is not None and kv["total_ms"] > 0:
                kv["fp64_TFs"] = flk * kv["launches"] / (kv["total_ms"] * 1e-3) / 1e12
                kv["frac_of_fp64_valu_peak"] = kv["fp64_TFs"] / FP64_VALU_PEAK_TFS
                trk = traffic_for(nm, prof[nm][2] / kv["launches"])
                if trk:
                    kv["hbm_frac_counters"] = trk / (kv["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS
        out["kernels"] = kernels
        out["profiled_ms_per_step"] = 1e3 * tprof / K

    if not args.no_adjoint:
        out["adjoint"] = adjoint_rate(log, args.sstep)

    if not args.no_ensemble:
        out["ensemble"] = ensemble_rate(log)

    if not args.no_configs:
        out["configs"] = configs_rates(log, args.sstep)

    if not args.no_three_d:
        out["three_d"] = three_d_rate(log, args.sstep)

    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(w, float(np.mean(it64)), log)

    plan.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
