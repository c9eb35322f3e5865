"""Seeded synthetic snapshot streams (test and benchmark inputs only).

The paper's full-order model (an MFEM Navier-Stokes solver on a cylinder
mesh, Sec. 3) is not available, so every input here is a planted linear
stream of the form the DMD model assumes (Sec. 2.3):

    x_k = Re( sum_j phi_j * lam_j**k * b_j ) + noise_k

This module holds no DMD arithmetic: it only draws modes, eigenvalues,
amplitudes and noise, and evaluates the sum above.  Both the CPU oracle
(through the tests) and the GPU path (through the tests and the benchmark)
receive the arrays it produces; neither side imports the other.

Workloads (sizes from the study's workload list):
  * ``planted_small``   n=4096, three complex mode pairs (rank 6), no noise.
  * ``wake``            cylinder-wake-shaped stream on a (u, v) grid: mean
                        flow, a shedding fundamental and harmonics on the
                        unit circle, decaying transients, relative noise.
                        n=160,000 (400 x 200 grid) or n=6,000,000 (3000 x 1000).
  * ``random_planted``  Gaussian i.i.d. modes with random planted rank, for
                        the many-stream batched form.
Noise of relative level s is i.i.d. N(0, (s*||x_clean||/sqrt(n))^2) per
element, drawn from PCG64 seeded by (seed, k) so any snapshot can be
regenerated on its own.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 231118715


@dataclasses.dataclass
class PlantedStream:
    """A linear snapshot stream with known modes, eigenvalues and amplitudes.

    modes:  (n, p) complex128; a real mode (lam real) has a real column.
    lam:    (p,) complex128 eigenvalues.
    amp:    (p,) complex128 amplitudes b_j.
    real:   (p,) bool, True where the mode contributes one real direction.
    noise:  relative noise level (0 for exact data).
    seed:   seed for the per-snapshot noise.
    """

    modes: np.ndarray
    lam: np.ndarray
    amp: np.ndarray
    real: np.ndarray
    noise: float
    seed: int

    @property
    def n(self) -> int:
        return self.modes.shape[0]

    @property
    def planted_rank(self) -> int:
        return int(np.sum(np.where(self.real, 1, 2)))

    def planted_eigs(self) -> np.ndarray:
        """All eigenvalues of the planted operator on its invariant subspace
        (each complex mode brings lam and its conjugate)."""
        out = []
        for lam, re in zip(self.lam, self.real):
            out.append(lam)
            if not re:
                out.append(np.conj(lam))
        return np.asarray(out, dtype=np.complex128)

    def coeffs(self, k0: int, k1: int) -> np.ndarray:
        """(p, k1-k0) complex matrix of lam_j**k * b_j for k in [k0, k1)."""
        k = np.arange(k0, k1, dtype=np.float64)
        # lam**k through polar form keeps |error| ~ k*eps independent of order
        mag = np.abs(self.lam)[:, None] ** k[None, :]
        ph = np.angle(self.lam)[:, None] * k[None, :]
        return self.amp[:, None] * mag * np.exp(1j * ph)

    def clean(self, k0: int, k1: int) -> np.ndarray:
        """(n, k1-k0) float64 noise-free snapshots x_k0 .. x_{k1-1}."""
        t = self.coeffs(k0, k1)
        return self.modes.real @ t.real - self.modes.imag @ t.imag

    def snapshots(self, k0: int, k1: int) -> np.ndarray:
        """(n, k1-k0) float64 snapshots with noise."""
        x = self.clean(k0, k1)
        if self.noise > 0.0:
            n = self.n
            for c, k in enumerate(range(k0, k1)):
                g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([self.seed, k])))
                s = self.noise * np.linalg.norm(x[:, c]) / math.sqrt(n)
                x[:, c] += s * g.standard_normal(n)
        return x


def planted_small(n: int = 4096, seed: int = BASE_SEED) -> PlantedStream:
    """Three orthonormal complex mode pairs (real rank 6), exact data.

    phi_j = (q_{2j-1} + i q_{2j}) / sqrt(2) from a QR of an n x 6 Gaussian;
    lam = {e^{i 2pi 0.02}, 0.995 e^{i 2pi 0.04}, 0.98 e^{i 2pi 0.06}};
    b_j ~ CN(0, 1).
    """
    g = np.random.Generator(np.random.PCG64(seed))
    q, _ = np.linalg.qr(g.standard_normal((n, 6)))
    modes = (q[:, 0::2] + 1j * q[:, 1::2]) / math.sqrt(2.0)
    lam = np.array([
        np.exp(2j * np.pi * 0.02),
        0.995 * np.exp(2j * np.pi * 0.04),
        0.98 * np.exp(2j * np.pi * 0.06),
    ])
    amp = (g.standard_normal(3) + 1j * g.standard_normal(3)) / math.sqrt(2.0)
    return PlantedStream(modes, lam, amp, np.zeros(3, bool), 0.0, seed + 1)


def wake(nx: int = 400, ny: int = 200, harmonics: int = 5, transients: int = 5,
         noise: float = 1e-6, seed: int = BASE_SEED) -> PlantedStream:
    """Cylinder-wake-shaped stream on an (nx, ny) grid, n = 2*nx*ny (u then v).

    Grid: x in [0, 20) diameters, y in [-4, 4].  Mean flow (lam = 1): a
    Gaussian velocity deficit that widens downstream.  Harmonic h of the
    shedding frequency f0 = 0.01 cycles/step: lam_h = e^{i 2pi 0.01 h},
    |b_h| = 1/h^2, shape A(x) e^{i h kappa x} G(y) with G a Gaussian or its
    y-derivative, parity alternating between u and v.  Transients: |lam| in
    U[0.9, 0.99], arg in U[0, 2pi 0.05], |b| in U[0.1, 0.5], shapes with
    random wavenumbers and widths.  All real mode directions are
    orthonormalised together (QR) and scaled to unit RMS.
    """
    g = np.random.Generator(np.random.PCG64(seed))
    x = np.linspace(0.0, 20.0, nx, endpoint=False)
    y = np.linspace(-4.0, 4.0, ny)
    X, Y = np.meshgrid(x, y, indexing="ij")
    s = 0.5 + 0.05 * X
    amp_x = (X / 4.0) * np.exp(1.0 - X / 4.0)
    gauss = np.exp(-Y ** 2 / (2.0 * s ** 2))
    dgauss = -Y / s ** 2 * gauss
    kappa = 2.0 * np.pi / 5.0

    cols = []                                   # real directions before QR
    mean_u = 1.0 - 0.5 * np.exp(-X / 8.0) * gauss
    cols.append(np.concatenate([mean_u.ravel(), np.zeros(nx * ny)]))
    lam, amp, real = [1.0 + 0j], [1.0 + 0j], [True]
    for h in range(1, harmonics + 1):
        gu, gv = (gauss, dgauss) if h % 2 else (dgauss, gauss)
        ph = np.exp(1j * h * kappa * X) * amp_x
        mode = np.concatenate([(ph * gu).ravel(), (ph * gv).ravel()])
        cols += [mode.real, mode.imag]
        lam.append(np.exp(2j * np.pi * 0.01 * h))
        amp.append(np.exp(1j * g.uniform(0, 2 * np.pi)) / h ** 2)
        real.append(False)
    for _ in range(transients):
        kt = g.uniform(0.5, 3.0)
        st = g.uniform(0.3, 1.5)
        x0 = g.uniform(2.0, 12.0)
        env = np.exp(-(X - x0) ** 2 / 8.0) * np.exp(-Y ** 2 / (2 * st ** 2))
        ph = np.exp(1j * kt * X) * env
        mode = np.concatenate([(ph * (1.0 + 0.3 * Y)).ravel(), (ph * Y / st).ravel()])
        cols += [mode.real, mode.imag]
        lam.append(g.uniform(0.9, 0.99) * np.exp(1j * g.uniform(0.0, 2 * np.pi * 0.05)))
        amp.append(g.uniform(0.1, 0.5) * np.exp(1j * g.uniform(0, 2 * np.pi)))
        real.append(False)

    q, _ = np.linalg.qr(np.stack(cols, axis=1))
    q *= math.sqrt(q.shape[0])                  # unit RMS per direction
    modes = np.empty((q.shape[0], len(lam)), np.complex128)
    modes[:, 0] = q[:, 0]
    for j in range(1, len(lam)):
        modes[:, j] = q[:, 2 * j - 1] + 1j * q[:, 2 * j]
    return PlantedStream(modes, np.asarray(lam), np.asarray(amp), np.asarray(real),
                         noise, seed + 1)


def random_planted(n: int, rank: int, seed: int, noise: float = 0.0) -> PlantedStream:
    """Gaussian i.i.d. modes (not orthonormalised) of real rank ``rank``.

    An odd rank uses one real mode (lam real in [0.97, 1]).  Complex modes:
    |lam| in U[0.97, 1], arg in U[2pi 0.005, 2pi 0.1], b ~ CN(0, 1).
    """
    g = np.random.Generator(np.random.PCG64(seed))
    npair, nreal = rank // 2, rank % 2
    p = npair + nreal
    modes = np.empty((n, p), np.complex128)
    lam = np.empty(p, np.complex128)
    real = np.zeros(p, bool)
    for j in range(npair):
        modes[:, j] = (g.standard_normal(n) + 1j * g.standard_normal(n)) / math.sqrt(2 * n)
        lam[j] = g.uniform(0.97, 1.0) * np.exp(1j * g.uniform(2 * np.pi * 0.005, 2 * np.pi * 0.1))
    if nreal:
        modes[:, p - 1] = g.standard_normal(n) / math.sqrt(n)
        lam[p - 1] = g.uniform(0.97, 1.0)
        real[p - 1] = True
    amp = (g.standard_normal(p) + 1j * g.standard_normal(p)) / math.sqrt(2.0)
    amp[real] = amp[real].real
    return PlantedStream(modes, lam, amp, real, noise, seed + 7919)


def batched_streams(count: int = 256, n_lo: float = 1e4, n_hi: float = 1e6,
                    seed: int = BASE_SEED):
    """Stream descriptors of the many-stream form: n log-uniform in
    [n_lo, n_hi], planted rank uniform in {6..30}, r_max uniform in {16..64}.
    Returns a list of (n, rank, r_max, stream_seed)."""
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        out.append((n, int(g.integers(6, 31)), int(g.integers(16, 65)), seed + i))
    return out


def restarted_pairs(s: PlantedStream, segments: int, length: int, seed: int):
    """Unchained snapshot pairs of one planted operator.

    ``segments`` trajectories of ``length`` pairs each, every one started
    from fresh amplitudes b_j ~ CN(0, 1) (drawn from PCG64(seed)) at a random
    start time in [0, 200), with the stream's own relative noise (per-segment
    noise seeds).  Returns (X, Y), each (n, segments * length): Y[:, j] is
    the successor of X[:, j] inside its trajectory, and X[:, j + 1] differs
    from Y[:, j] wherever a new segment starts.
    """
    g = np.random.Generator(np.random.PCG64(seed))
    p = s.lam.shape[0]
    xs, ys = [], []
    for sgm in range(segments):
        amp = (g.standard_normal(p) + 1j * g.standard_normal(p)) / math.sqrt(2.0)
        k0 = int(g.integers(0, 200))
        t = dataclasses.replace(s, amp=amp, seed=s.seed + 7919 * (sgm + 1))
        z = t.snapshots(k0, k0 + length + 1)
        xs.append(z[:, :-1])
        ys.append(z[:, 1:])
    return np.hstack(xs), np.hstack(ys)


class DeviceSnapshots:
    """Snapshots of a PlantedStream formed on the device, for sizes where the
    host cannot hold them (n in the millions): the modes go to the device
    once, snapshot k is Re(sum_j phi_j lam_j^k b_j) plus relative noise from
    a device generator seeded by (seed, k), so any snapshot can again be
    regenerated on its own.  The noise values differ from ``snapshots``'s
    host PCG64 draws (same distribution and level)."""

    def __init__(self, torch, s: PlantedStream, device: str = "cuda"):
        self.t, self.s, self.device = torch, s, device
        self.re = torch.from_numpy(np.ascontiguousarray(s.modes.real.T)).to(device)
        self.im = torch.from_numpy(np.ascontiguousarray(s.modes.imag.T)).to(device)
        self.gen = torch.Generator(device=device)

    @property
    def n(self) -> int:
        return self.re.shape[1]

    def chunk(self, k0: int, count: int):
        """Snapshots k0 .. k0+count-1 as rows of a (count, n) FP64 tensor."""
        t = self.s.coeffs(k0, k0 + count).T
        cre = self.t.from_numpy(np.ascontiguousarray(t.real)).to(self.device)
        cim = self.t.from_numpy(np.ascontiguousarray(t.imag)).to(self.device)
        X = cre @ self.re - cim @ self.im
        if self.s.noise > 0.0:
            for c in range(count):
                self.gen.manual_seed(int(self.s.seed) * 1000003 + k0 + c)
                sc = self.s.noise * float(self.t.linalg.norm(X[c])) / math.sqrt(self.n)
                X[c] += sc * self.t.randn(self.n, generator=self.gen, device=self.device,
                                          dtype=X.dtype)
        return X


class DevicePlanted:
    """The many-stream planted recipe (as ``random_planted``: |lam| in
    U[0.97, 1], arg in U[2pi 0.005, 2pi 0.1], b ~ CN(0, 1), an odd rank with
    one real mode) with the Gaussian mode vectors drawn on the device from a
    torch generator seeded by ``seed``, for streams too large or too many to
    build on the host.  Eigenvalues and amplitudes come from the host
    PCG64(seed) draws; ``planted`` lists the rank's eigenvalues.  No noise."""

    def __init__(self, torch, n: int, rank: int, seed: int, device: str = "cuda",
                 dtype=None):
        g = np.random.Generator(np.random.PCG64(seed))
        npair, nreal = rank // 2, rank % 2
        p = npair + nreal
        lam = np.empty(p, np.complex128)
        for j in range(npair):
            lam[j] = g.uniform(0.97, 1.0) * np.exp(1j * g.uniform(2 * np.pi * 0.005, 2 * np.pi * 0.1))
        if nreal:
            lam[p - 1] = g.uniform(0.97, 1.0)
        amp = (g.standard_normal(p) + 1j * g.standard_normal(p)) / math.sqrt(2.0)
        if nreal:
            amp[p - 1] = amp[p - 1].real
        dtype = dtype or torch.float64
        tg = torch.Generator(device=device)
        tg.manual_seed(int(seed))
        self.re = torch.randn((p, n), generator=tg, device=device, dtype=dtype) / math.sqrt(2 * n)
        self.im = torch.randn((p, n), generator=tg, device=device, dtype=dtype) / math.sqrt(2 * n)
        if nreal:
            self.re[p - 1] *= math.sqrt(2.0)
            self.im[p - 1] = 0.0
        self.lam, self.amp, self.n, self.device = lam, amp, n, device
        self.planted = np.concatenate([lam[:npair], np.conj(lam[:npair]), lam[npair:]])
        self.torch = torch

    def chunk(self, k0: int, count: int):
        """Snapshots k0 .. k0+count-1 as rows of a (count, n) tensor."""
        k = np.arange(k0, k0 + count)[:, None]
        C = self.amp[None, :] * self.lam[None, :] ** k
        t = self.torch
        cre = t.from_numpy(np.ascontiguousarray(C.real)).to(self.device, self.re.dtype)
        cim = t.from_numpy(np.ascontiguousarray(C.imag)).to(self.device, self.re.dtype)
        return cre @ self.re - cim @ self.im
