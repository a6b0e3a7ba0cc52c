"""Thin Python wrapper over the C ABI: a plan object and the time march.

Only device memory, streams and the loop over time steps live here; every
arithmetic step runs in librsfde's HIP kernels.
"""

from __future__ import annotations

import json
import time
from dataclasses import dataclass
from typing import List, Optional

import torch

from . import _lib as L


@dataclass
class StepStats:
    iters: int
    restarts: int
    relres: float
    status: int


class RsfdePlan:
    """Owns one rsfde_plan (device workspaces, tables) for a grid and parameters."""

    def __init__(self, n1, n2, box, alpha1, alpha2, kx, ky, mask, eta, dt, max_restart=30,
                 device=None):
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        if not isinstance(mask, torch.Tensor):
            mask = torch.as_tensor(mask)
        self.mask = mask.to(device=dev, dtype=torch.uint8).contiguous().reshape(-1)
        self.n1, self.n2 = int(n1), int(n2)
        self.box = tuple(float(v) for v in box)
        self.alpha1, self.alpha2 = float(alpha1), float(alpha2)
        self.kx, self.ky = float(kx), float(ky)
        self.eta, self.dt = float(eta), float(dt)
        self.device = dev
        with torch.cuda.device(dev):
            self.handle = L.rsfde_setup(self.n1, self.n2, self.box, alpha1, alpha2, kx, ky,
                                        self.mask, eta, dt, max_restart)

    @classmethod
    def from_workload(cls, w, kx=None, ky=None, max_restart=None, device=None):
        mask = torch.as_tensor(w.mask)
        return cls(w.n1, w.n2, w.box, w.alpha1, w.alpha2, w.kx if kx is None else kx,
                   w.ky if ky is None else ky, mask, w.eta, w.T / w.m,
                   w.restart if max_restart is None else max_restart, device)

    @classmethod
    def setup3(cls, n, box, alphas, ks, mask, eta, dt, max_restart=30, device=None):
        """A three-dimensional plan (rsfde_setup3): n = (n1, n2, n3), box of six
        bounds, per-axis alphas and ks, mask [n3][n2][n1]."""
        self = cls.__new__(cls)
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        if not isinstance(mask, torch.Tensor):
            mask = torch.as_tensor(mask)
        self.mask = mask.to(device=dev, dtype=torch.uint8).contiguous().reshape(-1)
        self.n1, self.n2, self.n3 = (int(v) for v in n)
        self.box = tuple(float(v) for v in box)
        self.alpha1, self.alpha2, self.alpha3 = (float(a) for a in alphas)
        self.kx, self.ky, self.kz = (float(k) for k in ks)
        self.is3d = True
        self.eta, self.dt = float(eta), float(dt)
        self.device = dev
        with torch.cuda.device(dev):
            self.handle = L.rsfde_setup3(n, box, alphas, ks, self.mask, eta, dt, max_restart)
        return self

    @classmethod
    def from_workload3(cls, w, max_restart=None, device=None):
        return cls.setup3((w.n1, w.n2, w.n3), w.box, (w.alpha1, w.alpha2, w.alpha3),
                          (w.kx, w.ky, w.kz), torch.as_tensor(w.mask), w.eta, w.T / w.m,
                          w.restart if max_restart is None else max_restart, device)

    n3 = 1  # two-dimensional unless set by setup3
    is3d = False

    @property
    def N(self):
        return self.n1 * self.n2 * self.n3

    def close(self):
        if getattr(self, "handle", None) is not None:
            L.rsfde_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_coeffs(self, kx, ky, kz=None):
        """New diffusion coefficients; kz (3-D plans) keeps its value when None."""
        if kz is None:
            L.rsfde_set_coeffs(self.handle, kx, ky)
        else:
            L.rsfde_set_coeffs3(self.handle, kx, ky, kz)
            if self.is3d:
                self.kz = float(kz)
        self.kx, self.ky = float(kx), float(ky)

    def empty(self):
        return torch.empty(self.N, dtype=torch.float64, device=self.device)

    def matvec(self, x, y=None):
        y = self.empty() if y is None else y
        L._check_vec(x, self.N, "x")
        L._check_vec(y, self.N, "y")
        L.rsfde_matvec(self.handle, x, y)
        return y

    def precond(self, r, z=None, precision="fp64"):
        z = self.empty() if z is None else z
        L._check_vec(r, self.N, "r")
        L._check_vec(z, self.N, "z")
        L.rsfde_precond_apply(self.handle, r, z, precision)
        return z

    def step(self, u_prev, u_prev2, f_kind, opts, u_next=None, check=True, src=None,
             src_scale=1.0):
        """One implicit step; with `src` (a field [n2][n1]) the right-hand side
        gains dt * mask * src_scale * src (rsfde_step_src)."""
        u_next = self.empty() if u_next is None else u_next
        L._check_vec(u_prev, self.N, "u_prev")
        if u_prev2 is not None:
            L._check_vec(u_prev2, self.N, "u_prev2")
        L._check_vec(u_next, self.N, "u_next")
        if src is None:
            st = L.rsfde_step(self.handle, u_prev, u_prev2, f_kind, opts, u_next, check=check)
        else:
            L._check_vec(src, self.N, "src")
            st = L.rsfde_step_src(self.handle, u_prev, u_prev2, f_kind, src, src_scale, opts,
                                  u_next, check=check)
        return u_next, StepStats(st.iters, st.restarts, st.relres, st.status)

    def solve(self, b, x, opts, check=True):
        L._check_vec(b, self.N, "b")
        L._check_vec(x, self.N, "x")
        st = L.rsfde_solve(self.handle, b, x, opts, check=check)
        return x, StepStats(st.iters, st.restarts, st.relres, st.status)

    def adjoint_step(self, u_prev, u_cur, lam_cur, f_kind, opts, lam_prev, dk, mu=None):
        for t, nm in ((u_prev, "u_prev"), (u_cur, "u_cur"), (lam_cur, "lam_cur"),
                      (lam_prev, "lam_prev")):
            L._check_vec(t, self.N, nm)
        L._check_vec(dk, 3 if self.is3d else 2, "dk")
        if mu is not None:
            L._check_vec(mu, self.N, "mu")
        st = L.rsfde_adjoint_step(self.handle, u_prev, u_cur, lam_cur, f_kind, opts, lam_prev,
                                  mu, dk)
        return StepStats(st.iters, st.restarts, st.relres, st.status)

    def march(self, u0, m, f_kind, opts, keep: Optional[List[int]] = None, src=None,
              src_scale=None, u_prev=None, k0: int = 0, log=None):
        """Run m implicit steps from u0 (flat FP64 tensor).  Returns (u^m, iters per
        step, {k: u^k for k in keep}).  src / src_scale(k): optional source field
        and its factor at step k (evaluated at t_{k-1}).

        Resume: a march interrupted after step k0 continues from u0 = u^{k0} and
        u_prev = u^{k0-1} (the state the extrapolated initial guess 2 u^{k0} -
        u^{k0-1} needs); step numbers (keep, src_scale, log) are then k0 + 1 ..
        k0 + m, and the result equals that of the uninterrupted march.
        log: a path or a text file; one JSON line per step with the step number,
        inner iterations, restarts, the solver's final relative residual, status
        and the host wall time of the step call in ms."""
        L._check_vec(u0, self.N, "u0")
        if u_prev is not None:
            L._check_vec(u_prev, self.N, "u_prev")
        bufs = [u0.clone(), self.empty() if u_prev is None else u_prev.clone(), self.empty()]
        cur, prev = 0, (None if u_prev is None else 1)
        iters = []
        saved = {}
        if keep and k0 in keep:
            saved[k0] = u0.clone()
        own = isinstance(log, (str, bytes)) or hasattr(log, "__fspath__")
        fh = open(log, "a") if own else log
        try:
            for k in range(k0 + 1, k0 + m + 1):
                nxt = [i for i in range(3) if i != cur and i != prev][0]
                t0 = time.perf_counter()
                _, st = self.step(bufs[cur], None if prev is None else bufs[prev], f_kind, opts,
                                  bufs[nxt], src=src,
                                  src_scale=1.0 if src_scale is None else src_scale(k))
                if fh is not None:
                    fh.write(json.dumps({"step": k, "iters": st.iters, "restarts": st.restarts,
                                         "relres": st.relres, "status": st.status,
                                         "ms": 1e3 * (time.perf_counter() - t0)}) + "\n")
                iters.append(st.iters)
                prev, cur = cur, nxt
                if keep and k in keep:
                    saved[k] = bufs[cur].clone()
        finally:
            if own:
                fh.close()
        return bufs[cur], iters, saved


def march_ensemble(plans, u0s, m, f_kind, opts, streams=None):
    """Advance independent plans (an ensemble: FD directions, parameter sweeps)
    by m steps each, concurrently (rsfde_march_ensemble: one host thread and,
    with `streams`, one stream per member).  Returns (list of u^m, list of
    StepStats with the iterations summed over the member's steps)."""
    if len(plans) != len(u0s):
        raise ValueError("one initial field per plan")
    outs, works = [], []
    for pl, u in zip(plans, u0s):
        L._check_vec(u, pl.N, "u0")
        outs.append(pl.empty())
        works += [pl.empty(), pl.empty()]
    sts = L.rsfde_march_ensemble([pl.handle for pl in plans], u0s, m, f_kind, opts, outs, works,
                                 streams)
    return outs, [StepStats(s.iters, s.restarts, s.relres, s.status) for s in sts]


class RsfdeBatch:
    """Owns one rsfde_batch: `count` independent members of one grid (shared
    orders, mask, eta, dt; own kx, ky, fields and Krylov state), stepped
    together (rsfde_batch_step).  Vectors are [count * N] FP64 tensors, member
    after member."""

    def __init__(self, n1, n2, box, alpha1, alpha2, kxs, kys, mask, eta, dt, max_restart=30,
                 device=None):
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        if not isinstance(mask, torch.Tensor):
            mask = torch.as_tensor(mask)
        self.mask = mask.to(device=dev, dtype=torch.uint8).contiguous().reshape(-1)
        self.n1, self.n2 = int(n1), int(n2)
        self.count = len(kxs)
        self.kxs, self.kys = [float(k) for k in kxs], [float(k) for k in kys]
        self.device = dev
        self.max_restart = int(max_restart)
        with torch.cuda.device(dev):
            self.handle = L.rsfde_batch_setup(self.n1, self.n2, box, alpha1, alpha2, kxs, kys,
                                              self.mask, eta, dt, max_restart)

    @classmethod
    def from_workload(cls, w, kxs, kys, max_restart=None, device=None):
        return cls(w.n1, w.n2, w.box, w.alpha1, w.alpha2, kxs, kys, torch.as_tensor(w.mask),
                   w.eta, w.T / w.m, w.restart if max_restart is None else max_restart, device)

    @property
    def N(self):
        return self.n1 * self.n2

    def close(self):
        if getattr(self, "handle", None) is not None:
            L.rsfde_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def empty(self):
        return torch.empty(self.count * self.N, dtype=torch.float64, device=self.device)

    def set_coeffs(self, kxs, kys):
        L.rsfde_batch_set_coeffs(self.handle, kxs, kys)
        self.kxs, self.kys = [float(k) for k in kxs], [float(k) for k in kys]

    def matvec(self, x, y=None):
        y = self.empty() if y is None else y
        L._check_vec(x, self.count * self.N, "x")
        L._check_vec(y, self.count * self.N, "y")
        L.rsfde_batch_matvec(self.handle, x, y)
        return y

    def precond(self, r, z=None, precision="fp64"):
        z = self.empty() if z is None else z
        L._check_vec(r, self.count * self.N, "r")
        L._check_vec(z, self.count * self.N, "z")
        L.rsfde_batch_precond_apply(self.handle, r, z, precision)
        return z

    def step(self, u_prev, u_prev2, f_kind, opts, u_next=None, check=True):
        if opts.sstep > 1:
            raise ValueError("batched solves run the one-vector form: build opts with sstep=0")
        u_next = self.empty() if u_next is None else u_next
        for t, nm in ((u_prev, "u_prev"), (u_next, "u_next")):
            L._check_vec(t, self.count * self.N, nm)
        if u_prev2 is not None:
            L._check_vec(u_prev2, self.count * self.N, "u_prev2")
        sts = L.rsfde_batch_step(self.handle, self.count, u_prev, u_prev2, f_kind, opts, u_next,
                                 check=check)
        return u_next, [StepStats(s.iters, s.restarts, s.relres, s.status) for s in sts]

    def march(self, u0, m, f_kind, opts):
        """m steps of every member from u0 ([count * N]).  Returns (u^m, per-step
        lists of the members' iteration counts)."""
        L._check_vec(u0, self.count * self.N, "u0")
        bufs = [u0.clone(), self.empty(), self.empty()]
        cur, prev = 0, None
        iters = []
        for _ in range(m):
            nxt = [i for i in range(3) if i != cur and i != prev][0]
            _, sts = self.step(bufs[cur], None if prev is None else bufs[prev], f_kind, opts,
                               bufs[nxt])
            iters.append([s.iters for s in sts])
            prev, cur = cur, nxt
        return bufs[cur], iters
