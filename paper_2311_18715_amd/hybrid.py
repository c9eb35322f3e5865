"""Hybrid full-order / online-DMD time stepping (the workflow of Sec. 2.1).

Each time step either accepts the DMD's prediction of the next state or
calls the full-order model (FOM) and appends the FOM's pair to the DMD:

    k = 0:  FOM step; the pair (u_0, u_1) initialises the DMD.
    k > 0:  the DMD predicts u_{k+1}; its residual in the FOM's own
            equations, r = b(u_k) - A u_{k+1} (Sec. 2.2: no solve needed),
            decides: ||r|| <= eps_dmd ||b||  accept the prediction as the
            next state; otherwise run the FOM and update the DMD with the
            pair (u_k, u_{k+1}).
    exit:   when the DMD has converged, predict the final state directly.

An accepted prediction replaces a FOM step, so the pair after it does not
chain with the one before (u_k was not the last FOM output): the DMD is a
general-pair handle (odmd_create_general).

Readings where the paper leaves details open:
  * predictions are anchored at the last FOM snapshot the DMD has seen;
    after j accepted steps the next prediction is state a + j + 1 of the
    rollout from that anchor (one rollout of `horizon` states is computed
    after each update and consumed step by step);
  * accepted predictions do not update the DMD (only FOM snapshots do);
  * convergence: the eigenvalues of A~ (|lambda| >= 1e-2 max|lambda|,
    greedily matched) move by less than conv_eps (relative) over
    conv_window consecutive updates.

The FOM here is a stand-in with the properties the workflow needs (an
implicit linear solve per step and a residual that costs one operator
application): implicit Euler for u_t = nu lap(u) - gamma u +
f(x, y) cos(omega t) on a periodic nx x ny grid, solved by conjugate
gradients.  The forced response settles onto a periodic orbit (a rank-2
linear evolution), as the cylinder wake settles into vortex shedding.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np


class HeatFOM:
    """Implicit Euler, periodic 5-point Laplacian L on the unit square:
    ((1 + dt gamma) I - dt nu L) u_{k+1} = u_k + dt f cos(omega t_{k+1}).
    nu = fourier / (dt nx^2) fixes the mesh Fourier number (and with it the
    conditioning of the solve) independent of the grid.  Vectors are flat
    torch tensors (row-major nx x ny)."""

    def __init__(self, torch, nx: int, ny: int, fourier: float = 0.5, gamma: float = 10.0,
                 dt: float = 0.05, omega: float = 2 * math.pi * 0.25, cg_tol: float = 1e-12,
                 cg_maxit: int = 500, seed: int = 231118715, device: str = "cuda", dtype=None):
        self.t = torch
        self.nx, self.ny, self.dt, self.omega = nx, ny, dt, omega
        self.nu = fourier / (dt * nx * nx)
        self.gamma = gamma
        self.cg_tol, self.cg_maxit = cg_tol, cg_maxit
        self.dtype = dtype or torch.float64
        self.device = device
        g = np.random.Generator(np.random.PCG64(seed))
        x = np.arange(nx)[:, None] / nx
        y = np.arange(ny)[None, :] / ny
        # a few smooth forcing blobs with random centres and widths
        f = np.zeros((nx, ny))
        for _ in range(3):
            cx, cy, w, a = g.uniform(0, 1), g.uniform(0, 1), g.uniform(0.05, 0.15), g.uniform(0.5, 1.5)
            dx = np.minimum(np.abs(x - cx), 1 - np.abs(x - cx))
            dy = np.minimum(np.abs(y - cy), 1 - np.abs(y - cy))
            f += a * np.exp(-(dx ** 2 + dy ** 2) / (2 * w ** 2))
        self.f = torch.from_numpy(f.reshape(-1)).to(device, self.dtype)
        self.solves = 0
        self.cg_iters = 0

    @property
    def n(self) -> int:
        return self.nx * self.ny

    def initial_state(self, transient: float = 0.1):
        """A start on the forced periodic orbit plus `transient` times one
        decaying Fourier mode (cos 2 pi x), so that the exact trajectory is
        a rank-3 linear evolution.  The orbit u_k = Re(z e^{i theta k}),
        theta = omega dt, solves the step exactly when
        ((1 + dt gamma) - dt nu L - e^{-i theta}) z = dt f, which the FFT
        diagonalises on the periodic grid."""
        t = self.t
        kx = t.arange(self.nx, dtype=self.dtype, device=self.device)[:, None]
        ky = t.arange(self.ny, dtype=self.dtype, device=self.device)[None, :]
        lam = -(4 * self.nx ** 2 * t.sin(math.pi * kx / self.nx) ** 2 +
                4 * self.ny ** 2 * t.sin(math.pi * ky / self.ny) ** 2)
        theta = self.omega * self.dt
        den = (1.0 + self.dt * self.gamma) - self.dt * self.nu * lam - complex(math.cos(theta), -math.sin(theta))
        F = t.fft.fft2(self.f.view(self.nx, self.ny).to(t.complex128))
        z = t.fft.ifft2(self.dt * F / den)
        x = t.arange(self.nx, dtype=self.dtype, device=self.device)[:, None] / self.nx
        mode = t.cos(2 * math.pi * x).expand(self.nx, self.ny)
        u0 = z.real + transient * mode * float(t.linalg.norm(z.real)) / math.sqrt(self.n) * 4
        return u0.reshape(-1).contiguous()

    def lap(self, u):
        t = self.t
        U = u.view(self.nx, self.ny)
        L = (t.roll(U, 1, 0) + t.roll(U, -1, 0) - 2 * U) * (self.nx ** 2) + \
            (t.roll(U, 1, 1) + t.roll(U, -1, 1) - 2 * U) * (self.ny ** 2)
        return L.reshape(-1)

    def apply_A(self, u):
        return (1.0 + self.dt * self.gamma) * u - self.dt * self.nu * self.lap(u)

    def rhs(self, u, k: int):
        """b(u_k) of the step k -> k+1."""
        return u + self.dt * self.f * math.cos(self.omega * self.dt * (k + 1))

    def residual(self, u_prev, u_next, k: int) -> float:
        """||b(u_k) - A u_{k+1}|| / ||b(u_k)||."""
        b = self.rhs(u_prev, k)
        return float(self.t.linalg.norm(b - self.apply_A(u_next)) / self.t.linalg.norm(b))

    def step(self, u, k: int):
        """u_{k+1} by conjugate gradients from the guess u_k."""
        t = self.t
        b = self.rhs(u, k)
        x = u.clone()
        r = b - self.apply_A(x)
        p = r.clone()
        rr = t.dot(r, r)
        bn = t.dot(b, b)
        it = 0
        while it < self.cg_maxit and float(rr) > (self.cg_tol ** 2) * float(bn):
            Ap = self.apply_A(p)
            alpha = rr / t.dot(p, Ap)
            x += alpha * p
            r -= alpha * Ap
            rr_new = t.dot(r, r)
            p = r + (rr_new / rr) * p
            rr = rr_new
            it += 1
        self.solves += 1
        self.cg_iters += it
        return x


@dataclasses.dataclass
class HybridResult:
    steps: int                       # time steps taken (k = 0 .. steps-1)
    kinds: List[str]                 # 'fom' or 'dmd' per step taken
    checks: List[tuple]              # (step, residual, accepted) of each prediction checked
    fom_calls: int
    converged_at: Optional[int]      # step at which the DMD was declared converged
    final: object                    # state at the final step
    final_step: int

    @property
    def fom_fraction_avoided(self) -> float:
        return 1.0 - self.fom_calls / max(1, self.final_step)


def _eig_shift(prev, cur) -> float:
    if prev is None or len(prev) != len(cur) or len(cur) == 0:
        return math.inf
    big = np.abs(cur) >= 1e-2 * np.abs(cur).max()
    ref = list(prev)
    worst = 0.0
    for z in cur[big]:
        j = int(np.argmin([abs(z - w) for w in ref]))
        worst = max(worst, abs(z - ref.pop(j)) / abs(z))
    return worst


def run_hybrid(fom, u0, final_step: int, make_dmd: Callable, eps_dmd: float = 1e-6,
               horizon: int = 16, conv_eps: float = 1e-9, conv_window: int = 5,
               check_convergence: bool = True) -> HybridResult:
    """Advance u0 to step final_step with the hybrid FOM/DMD workflow.

    make_dmd(n) returns a general-pair DMD object with update(x, y),
    predict(steps) -> (steps, n) states after the last y, eigs(vectors=False)
    and info().r (the library's ODMD with pairs='general')."""
    dmd = make_dmd(fom.n)
    u = u0
    kinds, checks = [], []
    fom_calls = 0
    preds, used = None, 0            # rollout from the last FOM snapshot, states consumed
    lam_prev, calm, converged_at = None, 0, None
    k = 0
    while k < final_step:
        nxt = None
        if preds is not None and used < preds.shape[0]:
            cand = preds[used]
            res = fom.residual(u, cand, k)
            checks.append((k, res, res <= eps_dmd))
            if res <= eps_dmd:
                nxt = cand
                used += 1
                kinds.append("dmd")
        if nxt is None:
            nxt = fom.step(u, k)
            fom_calls += 1
            kinds.append("fom")
            dmd.update(u, nxt)
            preds, used = None, 0
            if check_convergence and dmd.info().r > 0:
                lam, _ = dmd.eigs(vectors=False)
                calm = calm + 1 if _eig_shift(lam_prev, lam) < conv_eps else 0
                lam_prev = lam
                if calm >= conv_window:
                    converged_at = k + 1
            if dmd.info().r > 0:
                preds, used = dmd.predict(horizon), 0
        u = nxt
        k += 1
        if converged_at is not None:
            # straight to the final step from the last FOM snapshot (u)
            remaining = final_step - k
            if remaining > 0:
                u = dmd.predict(remaining)[remaining - 1]
                kinds.extend(["skip"] * remaining)
                k = final_step
            break
    return HybridResult(steps=len(kinds), kinds=kinds, checks=checks, fom_calls=fom_calls,
                        converged_at=converged_at, final=u, final_step=final_step)
