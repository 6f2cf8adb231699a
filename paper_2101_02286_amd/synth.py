"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the solver: it only draws random numbers
and evaluates input fields.  Both the HIP path and the oracle receive the
arrays it returns.

Fields live on the periodic grid x_j = j * 2*pi / n along each axis, stored
C-order as (nz, ny, nx) with x the unit-stride index.

random_modes: f = sum_m A_m cos(kx_m x + ky_m y + kz_m z + phi_m) with
A_m ~ U(-1, 1), integer wavenumbers k ~ U{1..kmax} per axis and phase
phi_m ~ U(0, 2 pi), drawn from numpy.random.default_rng(seed).
"""
import math

import numpy as np
import torch


def draw_modes(seed, n_modes=8, kmax=8):
    rng = np.random.default_rng(seed)
    amp = rng.uniform(-1.0, 1.0, size=n_modes)
    k = rng.integers(1, kmax + 1, size=(n_modes, 3))  # columns: kx, ky, kz
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    return amp, k, phi


def random_modes(shape, seed=0, n_modes=8, kmax=8, device="cpu", dtype=torch.float64):
    """Evaluate the seeded Fourier-mode field on a (nz, ny, nx) grid.

    Returns (field, (amp, k, phi))."""
    nz, ny, nx = shape
    amp, k, phi = draw_modes(seed, n_modes, kmax)
    xs = [torch.arange(m, device=device, dtype=torch.float64) * (2.0 * math.pi / m) for m in (nx, ny, nz)]
    f = torch.zeros((nz, ny, nx), device=device, dtype=torch.float64)
    for m in range(n_modes):
        # cos(a+b+c+phi) evaluated separably: Re(e^{i phi} e^{ia} e^{ib} e^{ic})
        ex = torch.polar(torch.ones_like(xs[0]), float(k[m, 0]) * xs[0] + float(phi[m]))
        ey = torch.polar(torch.ones_like(xs[1]), float(k[m, 1]) * xs[1])
        ez = torch.polar(torch.ones_like(xs[2]), float(k[m, 2]) * xs[2])
        f.add_((ez[:, None, None] * ey[None, :, None] * ex[None, None, :]).real, alpha=float(amp[m]))
    return f.to(dtype), (amp, k, phi)


def random_uniform(shape, seed=0, device="cpu", dtype=torch.float64):
    """U(-1, 1) noise (adversarial, non-smooth right-hand sides)."""
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed))
    return (torch.rand(shape, generator=g, dtype=torch.float64) * 2.0 - 1.0).to(device=device, dtype=dtype)


def random_bands(n, r, seed=0, dominance=2.5):
    """Per-row bands (n, 2r+1), strictly diagonally dominant: diagonal in
    [dominance, dominance+1) times the off-diagonal sum bound."""
    rng = np.random.default_rng(seed)
    b = rng.uniform(-1.0, 1.0, size=(n, 2 * r + 1))
    off = np.abs(b).sum(axis=1) - np.abs(b[:, r])
    b[:, r] = (dominance + rng.uniform(0, 1, size=n)) * np.maximum(off, 1e-3)
    return b


def grid_batch_shapes(seed=0, count=12):
    """The uneven-grid batch: `count` shapes (nx, ny, nz) drawn from six sizes."""
    menu = [(64, 64, 64), (128, 128, 128), (192, 192, 192), (384, 384, 384),
            (1024, 128, 64), (96, 512, 32)]
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(menu), size=count)
    return [menu[i] for i in idx]
