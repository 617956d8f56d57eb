"""Seeded synthetic scientific fields.

These generators stand in for the paper's datasets (Table III: CESM, Miranda,
SCALE, S3D, JHTDB), none of which is available here.  They are shared by the
CPU oracle's tests, the GPU parity tests and the benchmark, and they hold none
of the compression method's arithmetic: they only draw numbers.

Recipes (all values computed in float64, cast once at the end):

* ``gaussian_bumps``: sum of 8 Gaussian bumps (centres U[0,n) per axis,
  sigma U[4,12] cells, amplitude U[-1,1]) plus
  0.3*sin(2*pi*x/32)*sin(2*pi*y/24)*cos(2*pi*z/40) plus N(0, 1e-3) noise,
  with x, y, z the indices of axes 2, 1, 0.  Draw order: centres, sigmas,
  amplitudes, noise.
* ``power_law_field``: Gaussian random field with isotropic power spectrum
  E(k) ~ k^-alpha: white N(0,1) noise, FFT, amplitude k^(-(alpha+d-1)/2) with
  k in cycles per cell, k = 0 removed, inverse FFT, normalised to zero mean and
  unit standard deviation.  alpha = 5/3 is turbulence-like.
* ``zonal_bands``: 2D climate-like field: sum over m in {2, 5, 9} of
  a_m*cos(2*pi*m*i/n0 + phi_m) (a ~ U[0.5,1], phi ~ U[0,2*pi)) plus 0.3 times
  a unit-std k^-3 random field.
* ``sharp_fronts``: k^-5/3 field plus spherical tanh fronts of width 2 cells.
"""
from __future__ import annotations

import os

import numpy as np


def _fft_workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def gaussian_bumps(shape=(64, 64, 64), seed: int = 0, nbumps: int = 8,
                   dtype=np.float32) -> np.ndarray:
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    assert len(shape) == 3
    centres = rng.uniform(0.0, 1.0, size=(nbumps, 3)) * np.asarray(shape, dtype=np.float64)
    sig = rng.uniform(4.0, 12.0, size=nbumps)
    amp = rng.uniform(-1.0, 1.0, size=nbumps)
    noise = rng.normal(0.0, 1e-3, size=shape)
    z = np.arange(shape[0], dtype=np.float64)[:, None, None]
    y = np.arange(shape[1], dtype=np.float64)[None, :, None]
    x = np.arange(shape[2], dtype=np.float64)[None, None, :]
    v = np.zeros(shape, dtype=np.float64)
    for i in range(nbumps):
        r2 = (z - centres[i, 0]) ** 2 + (y - centres[i, 1]) ** 2 + (x - centres[i, 2]) ** 2
        v += amp[i] * np.exp(-r2 / (2.0 * sig[i] ** 2))
    v += 0.3 * np.sin(2 * np.pi * x / 32) * np.sin(2 * np.pi * y / 24) * np.cos(2 * np.pi * z / 40)
    v += noise
    return v.astype(dtype)


def power_law_field(shape, alpha: float = 5.0 / 3.0, seed: int = 1,
                    dtype=np.float32) -> np.ndarray:
    """Isotropic Gaussian random field with E(k) ~ k^-alpha (float64 math)."""
    import scipy.fft as sfft

    shape = tuple(int(s) for s in shape)
    d = len(shape)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    F = sfft.rfftn(w, workers=_fft_workers())
    del w
    expo = -(alpha + d - 1) / 2.0
    # k^2 accumulated slab by slab along axis 0 to bound memory.
    freqs = []
    for ax, n in enumerate(shape):
        f = np.fft.rfftfreq(n) if ax == d - 1 else np.fft.fftfreq(n)
        freqs.append(f)
    tail = 0.0
    for ax in range(1, d):
        shp = [1] * (d - 1)
        shp[ax - 1] = freqs[ax].size
        tail = tail + (freqs[ax] ** 2).reshape(shp)
    tail = np.asarray(tail, dtype=np.float64)
    for i0 in range(F.shape[0]):
        k2 = freqs[0][i0] ** 2 + tail
        with np.errstate(divide="ignore"):
            amp = np.where(k2 > 0, k2 ** (expo / 2.0), 0.0)
        F[i0] *= amp
    v = sfft.irfftn(F, s=shape, workers=_fft_workers())
    del F
    v -= v.mean()
    v /= v.std()
    return v.astype(dtype)


def zonal_bands(shape=(1800, 3600), seed: int = 2, dtype=np.float32) -> np.ndarray:
    rng = np.random.default_rng(seed)
    n0, n1 = shape
    i = np.arange(n0, dtype=np.float64)[:, None]
    v = np.zeros(shape, dtype=np.float64)
    for m in (2, 5, 9):
        a = rng.uniform(0.5, 1.0)
        phi = rng.uniform(0.0, 2 * np.pi)
        v += a * np.cos(2 * np.pi * m * i / n0 + phi)
    sub_seed = int(rng.integers(0, 2**31 - 1))
    v += 0.3 * power_law_field(shape, alpha=3.0, seed=sub_seed, dtype=np.float64)
    return v.astype(dtype)


def sharp_fronts(shape, seed: int = 4, frac: float = 0.01, radius: float = 32.0,
                 dtype=np.float32) -> np.ndarray:
    """k^-5/3 field plus spherical tanh fronts covering about ``frac`` of the volume."""
    base = power_law_field(shape, seed=seed, dtype=np.float64)
    rng = np.random.default_rng(seed + 1000)
    vol = float(np.prod(shape))
    nsph = max(1, int(round(frac * vol / (4.0 / 3.0 * np.pi * radius ** 3))))
    sd = base.std()
    idx = [np.arange(s, dtype=np.float64) for s in shape]
    for _ in range(nsph):
        c = rng.uniform(0.0, 1.0, size=3) * np.asarray(shape, dtype=np.float64)
        nrm = rng.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        lo = [max(0, int(c[a] - radius - 8)) for a in range(3)]
        hi = [min(shape[a], int(c[a] + radius + 8) + 1) for a in range(3)]
        z = idx[0][lo[0]:hi[0], None, None]
        y = idx[1][None, lo[1]:hi[1], None]
        x = idx[2][None, None, lo[2]:hi[2]]
        rc = np.sqrt((z - c[0]) ** 2 + (y - c[1]) ** 2 + (x - c[2]) ** 2)
        dp = (z - c[0]) * nrm[0] + (y - c[1]) * nrm[1] + (x - c[2]) * nrm[2]
        bump = 2.0 * sd * np.tanh(dp / 2.0) * 0.5 * (1.0 - np.tanh((rc - radius) / 2.0))
        base[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] += bump
    return base.astype(dtype)


def polynomial_field(shape, coeffs, dtype=np.float64) -> np.ndarray:
    """Separable-sum polynomial: sum over axes a and powers p of coeffs[a][p]*i_a**p.

    Integer coefficients give integer values, exactly representable in float64.
    """
    d = len(shape)
    v = np.zeros(shape, dtype=np.float64)
    for a in range(d):
        shp = [1] * d
        shp[a] = shape[a]
        i = np.arange(shape[a], dtype=np.float64).reshape(shp)
        for p, c in enumerate(coeffs[a]):
            if c:
                v = v + c * i ** p
    return v.astype(dtype)


def config1_field() -> np.ndarray:
    """64^3 float32 Gaussian bumps + waves + noise, seed 0."""
    return gaussian_bumps((64, 64, 64), seed=0)


def config2_field(n: int = 512, dtype=np.float32) -> np.ndarray:
    """n^3 k^-5/3 Gaussian random field, seed 1."""
    return power_law_field((n, n, n), alpha=5.0 / 3.0, seed=1, dtype=dtype)


# --------------------------------------------------------------------------
# Device-side variants of the same recipes (torch on the current GPU), for
# benchmark workloads too large to draw on the host in reasonable time.  They
# follow the recipes above step by step but draw from torch's generator and
# use torch's FFT, so their values differ from the NumPy versions; nothing
# compares them with the oracle.
# --------------------------------------------------------------------------

def power_law_field_torch(shape, alpha: float = 5.0 / 3.0, seed: int = 1, dtype=None, device="cuda"):
    """``power_law_field`` drawn on the device (float64 math, cast once)."""
    import torch

    dtype = dtype or torch.float32
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    w = torch.randn(shape, generator=g, dtype=torch.float64, device=device)
    F = torch.fft.rfftn(w)
    del w
    expo = -(alpha + d - 1) / 2.0
    k2 = None
    for ax, n in enumerate(shape):
        f = torch.fft.rfftfreq(n, dtype=torch.float64, device=device) if ax == d - 1 else \
            torch.fft.fftfreq(n, dtype=torch.float64, device=device)
        shp = [1] * d
        shp[ax] = f.numel()
        t = (f ** 2).reshape(shp)
        k2 = t if k2 is None else k2 + t
    for i0 in range(F.shape[0]):  # slab by slab along axis 0 (bounded memory)
        kk = k2[i0] if d > 1 else k2[i0:i0 + 1]
        amp = torch.where(kk > 0, kk.clamp_min(1e-300) ** (expo / 2.0), torch.zeros_like(kk))
        F[i0] *= amp
    v = torch.fft.irfftn(F, s=shape)
    del F
    v -= v.mean()
    v /= v.std(unbiased=False)
    return v.to(dtype)


def zonal_bands_torch(shape=(1800, 3600), seed: int = 2, dtype=None, device="cuda"):
    """``zonal_bands`` drawn on the device."""
    import torch

    dtype = dtype or torch.float32
    rng = np.random.default_rng(seed)
    n0, n1 = shape
    i = torch.arange(n0, dtype=torch.float64, device=device)[:, None]
    v = torch.zeros(shape, dtype=torch.float64, device=device)
    for m in (2, 5, 9):
        a = rng.uniform(0.5, 1.0)
        phi = rng.uniform(0.0, 2 * np.pi)
        v += a * torch.cos(2 * np.pi * m * i / n0 + phi)
    sub_seed = int(rng.integers(0, 2**31 - 1))
    v += 0.3 * power_law_field_torch(shape, alpha=3.0, seed=sub_seed, dtype=torch.float64, device=device)
    return v.to(dtype)


def sharp_fronts_torch(shape, seed: int = 4, frac: float = 0.01, radius: float = 32.0, dtype=None, device="cuda"):
    """``sharp_fronts`` drawn on the device (sphere centres and normals from
    the same NumPy draws as the host version)."""
    import torch

    dtype = dtype or torch.float32
    base = power_law_field_torch(shape, seed=seed, dtype=torch.float64, device=device)
    rng = np.random.default_rng(seed + 1000)
    vol = float(np.prod(shape))
    nsph = max(1, int(round(frac * vol / (4.0 / 3.0 * np.pi * radius ** 3))))
    sd = float(base.std(unbiased=False))
    for _ in range(nsph):
        c = rng.uniform(0.0, 1.0, size=3) * np.asarray(shape, dtype=np.float64)
        nrm = rng.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        lo = [max(0, int(c[a] - radius - 8)) for a in range(3)]
        hi = [min(shape[a], int(c[a] + radius + 8) + 1) for a in range(3)]
        z = torch.arange(lo[0], hi[0], dtype=torch.float64, device=device)[:, None, None]
        y = torch.arange(lo[1], hi[1], dtype=torch.float64, device=device)[None, :, None]
        x = torch.arange(lo[2], hi[2], dtype=torch.float64, device=device)[None, None, :]
        rc = torch.sqrt((z - c[0]) ** 2 + (y - c[1]) ** 2 + (x - c[2]) ** 2)
        dp = (z - c[0]) * nrm[0] + (y - c[1]) * nrm[1] + (x - c[2]) * nrm[2]
        bump = 2.0 * sd * torch.tanh(dp / 2.0) * 0.5 * (1.0 - torch.tanh((rc - radius) / 2.0))
        base[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] += bump
    return base.to(dtype)
