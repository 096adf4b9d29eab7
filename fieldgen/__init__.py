"""Seeded synthetic input fields for the compression workloads.

This module only draws inputs: random numbers, coordinates and the test fields
built from them.  It holds none of the compression method's arithmetic, so the
CPU oracle, the tests and the benchmark can all take their inputs from here.

Recipes (each field is built in float64 and cast by the caller):

* ``bumps2d``      -- 129x129 uniform grid on [0,1]^2: eight Gaussian bumps
  (centre U[0,1]^2, amplitude U[0.5,2], width U[0.05,0.2]) plus
  sin(4 pi x) cos(6 pi y) plus N(0, 1e-3) noise.  Draw order: centres,
  amplitudes, widths, noise.
* ``spectral``     -- turbulence-like field with energy spectrum E(k) ~ k^beta:
  white normal noise on a periodic grid, Fourier transform, unit-modulus
  phases, amplitude |k|^((beta-(D-1))/2) with the k=0 mode removed, inverse
  transform, normalised to zero mean and unit standard deviation.  A side
  n that is odd is synthesised on the periodic n-1 grid and the wrap plane is
  appended, so 2^k+1 grids hold a whole number of periods.
* ``geometric_coords`` -- nonuniform coordinates with spacings growing by a
  fixed ratio, normalised to [0, 1].
* ``front3d``      -- spectral k^-3 field plus a tanh front of width 0.02
  through the domain centre, on geometric coordinates.
* ``batch_specs``  -- the uneven-shape batch: per field D in {2,3} with
  probability 1/2, each side integer log-uniform in [65, 2049] (2D) or
  [33, 257] (3D), slope beta ~ U[-4, -5/3].

The paper's own workloads (cosmology, plasma, climate data) are not available;
these fields stand in for them with the same dimensionality, precision and
spectral character.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "bumps2d",
    "spectral",
    "geometric_coords",
    "front3d",
    "batch_specs",
    "BatchSpec",
    "random_coords",
    "random_field",
]


def bumps2d(n: int = 129, seed: int = 1) -> np.ndarray:
    """2D field: 8 Gaussians + sin(4 pi x) cos(6 pi y) + N(0, 1e-3) noise, float64."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(8, 2))
    amps = rng.uniform(0.5, 2.0, size=8)
    widths = rng.uniform(0.05, 0.2, size=8)
    noise = rng.normal(0.0, 1e-3, size=(n, n))
    x = np.linspace(0.0, 1.0, n)
    X, Y = np.meshgrid(x, x, indexing="ij")
    u = np.sin(4 * np.pi * X) * np.cos(6 * np.pi * Y)
    for k in range(8):
        r2 = (X - centres[k, 0]) ** 2 + (Y - centres[k, 1]) ** 2
        u = u + amps[k] * np.exp(-r2 / (2.0 * widths[k] ** 2))
    return u + noise


def _periodic_side(n: int) -> int:
    return n - 1 if (n % 2 == 1 and n > 1) else n


def spectral(shape, beta: float, seed: int, device: str = "cpu", noise: str = "numpy"):
    """Spectral synthesis with E(k) ~ k^beta; returns float64 (numpy on cpu, torch on cuda).

    noise="numpy" draws the white noise with numpy's PCG64 (default_rng(seed));
    noise="torch" draws it on `device` with torch's generator seeded by `seed`
    (used for the large training and evaluation sets, where host generation
    would dominate).
    """
    import torch

    shape = tuple(int(s) for s in shape)
    D = len(shape)
    m = tuple(_periodic_side(s) for s in shape)
    if noise == "torch":
        g = torch.Generator(device=device).manual_seed(int(seed))
        w = torch.randn(m, generator=g, device=device, dtype=torch.float64)
    else:
        rng = np.random.default_rng(seed)
        w = torch.from_numpy(rng.standard_normal(size=m))
        if device != "cpu":
            w = w.to(device)
    W = torch.fft.rfftn(w)
    del w
    mag = W.abs()
    W = torch.where(mag > 0, W / torch.where(mag > 0, mag, torch.ones_like(mag)), torch.zeros_like(W))
    del mag
    # |k|^2 on the rfft grid
    k2 = None
    for d in range(D):
        if d == D - 1:
            k = torch.fft.rfftfreq(m[d], d=1.0 / m[d], dtype=torch.float64, device=W.device)
        else:
            k = torch.fft.fftfreq(m[d], d=1.0 / m[d], dtype=torch.float64, device=W.device)
        view = [1] * D
        view[d] = -1
        kk = (k * k).view(view)
        k2 = kk if k2 is None else k2 + kk
    expo = (beta - (D - 1)) / 2.0
    amp = torch.where(k2 > 0, torch.pow(torch.where(k2 > 0, k2, torch.ones_like(k2)), expo / 2.0), torch.zeros_like(k2))
    del k2
    W = W * amp
    del amp
    f = torch.fft.irfftn(W, s=m)
    del W
    f = (f - f.mean()) / f.std()
    for d in range(D):
        if shape[d] == m[d] + 1:
            f = torch.cat([f, f.narrow(d, 0, 1)], dim=d)
    f = f.contiguous()
    if device == "cpu":
        return f.numpy()
    return f


def geometric_coords(n: int, ratio: float = 1.01) -> np.ndarray:
    """Coordinates with spacing h_i = ratio^i, normalised to [0, 1]."""
    h = ratio ** np.arange(n - 1, dtype=np.float64)
    x = np.concatenate([[0.0], np.cumsum(h)])
    return x / x[-1]


def front3d(n: int = 500, seed: int = 3, ratio: float = 1.01, device: str = "cpu"):
    """Spectral k^-3 field on the index grid + tanh front on geometric coordinates."""
    import torch

    base = spectral((n, n, n), -3.0, seed, device=device)
    x = geometric_coords(n, ratio)
    if device == "cpu":
        s = (x[:, None, None] + x[None, :, None] + x[None, None, :]) / math.sqrt(3.0)
        return base + np.tanh((s - math.sqrt(3.0) / 2.0) / 0.02), [x, x, x]
    xt = torch.from_numpy(x).to(device)
    s = (xt[:, None, None] + xt[None, :, None] + xt[None, None, :]) / math.sqrt(3.0)
    return base + torch.tanh((s - math.sqrt(3.0) / 2.0) / 0.02), [x, x, x]


@dataclass
class BatchSpec:
    shape: tuple
    beta: float
    seed: int


def _log_uniform_int(rng, lo: int, hi: int) -> int:
    v = int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi + 1)))))
    return min(max(v, lo), hi)


def batch_specs(count: int = 256, shape_seed: int = 4, first_field_seed: int = 1000):
    """Shapes, slopes and seeds of the uneven-shape batch."""
    rng = np.random.default_rng(shape_seed)
    out = []
    for i in range(count):
        D = 2 if rng.random() < 0.5 else 3
        lo, hi = (65, 2049) if D == 2 else (33, 257)
        shape = tuple(_log_uniform_int(rng, lo, hi) for _ in range(D))
        beta = float(rng.uniform(-4.0, -5.0 / 3.0))
        out.append(BatchSpec(shape=shape, beta=beta, seed=first_field_seed + i))
    return out


def random_coords(n: int, rng: np.random.Generator, jitter: float = 0.4) -> np.ndarray:
    """Strictly increasing random coordinates: unit steps scaled by U[1-jitter, 1+jitter]."""
    h = rng.uniform(1.0 - jitter, 1.0 + jitter, size=max(n - 1, 0))
    return np.concatenate([[0.0], np.cumsum(h)])


def random_field(shape, rng: np.random.Generator) -> np.ndarray:
    """Smooth-plus-rough random field for small tests (float64)."""
    u = rng.standard_normal(size=shape)
    # a smooth large-scale part so coefficients span several magnitudes
    grids = np.meshgrid(*[np.linspace(0, 1, s) for s in shape], indexing="ij")
    smooth = np.ones(shape)
    for g in grids:
        smooth = smooth * np.cos(3.0 * g + 0.5)
    return 4.0 * smooth + 0.1 * u
