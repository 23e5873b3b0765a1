"""Seeded synthetic inputs: random-ellipse phantoms, their exact (analytic) parallel-beam
projections, and measurement noise.

This module holds none of the reconstruction method's arithmetic: it never applies the
discrete projector, its adjoint, the TV prox or the solver.  Sinograms are the continuous
line integrals of the ellipses (the closed form for the Radon transform of an ellipse,
Kak & Slaney, ch. 3), the way the paper's simulated experiment computes analytical projection
data (Sec. 2.2), so the same data serve the HIP path and the FP64 oracle unchanged.

Coordinates (pixel units): pixel (i, j) has centre (j - (nx-1)/2, i - (ny-1)/2); the ray of
angle t and detector coordinate s is {x cos t + y sin t = s}; bin u sits at
s_u = (u - (B-1)/2) * du + off.  Phantom parameters live in normalised coordinates [-1, 1]
scaled by R = min(nx, ny)/2 pixels (and nz/2 along z for ellipsoids).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Ellipse:
    cx: float      # centre, normalised
    cy: float
    a: float       # semi-axis along the rotated x axis, normalised
    b: float       # semi-axis along the rotated y axis, normalised
    phi: float     # rotation, radians
    rho: float     # additive intensity
    cz: float = 0.0  # ellipsoids only: centre and semi-axis along z, normalised
    c: float = 1.0


def random_ellipses(seed: int, count: int = 10, dims: int = 2) -> list[Ellipse]:
    """``count`` seeded random ellipses (dims=2) or z-aligned ellipsoids (dims=3).

    Centre uniform in the disc (ball) of radius 0.6, semi-axes U[0.05, 0.35], rotation
    U[0, pi), intensity U[0.1, 1]; the extent stays inside radius 0.95.
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        while True:
            cen = rng.uniform(-0.6, 0.6, size=dims)
            if np.dot(cen, cen) <= 0.36:
                break
        ax = rng.uniform(0.05, 0.35, size=3)
        phi = rng.uniform(0.0, math.pi)
        rho = rng.uniform(0.1, 1.0)
        e = Ellipse(float(cen[0]), float(cen[1]), float(ax[0]), float(ax[1]), float(phi),
                    float(rho))
        if dims == 3:
            e.cz, e.c = float(cen[2]), float(ax[2])
        out.append(e)
    return out


def _slice_ellipse(e: Ellipse, nz: int, z: int) -> tuple[float, float] | None:
    """Cross-section scale of a z-aligned ellipsoid at slice z (None if the slice misses it)."""
    if nz == 1:
        return 1.0, 1.0
    Z = (z - (nz - 1) / 2.0) / (nz / 2.0)
    t = (Z - e.cz) / e.c
    if abs(t) >= 1.0:
        return None
    f = math.sqrt(1.0 - t * t)
    return f, f


def rasterize(ellipses: list[Ellipse], nx: int, ny: int, nz: int = 1,
              supersample: int = 1) -> np.ndarray:
    """Phantom image [nz][ny][nx] (float64): mean of ss x ss point samples per pixel."""
    R = min(nx, ny) / 2.0
    ss = supersample
    offs = (np.arange(ss) + 0.5) / ss - 0.5
    xs = (np.arange(nx)[None, :] - (nx - 1) / 2.0 + offs[:, None]) / R  # [ss][nx]
    ys = (np.arange(ny)[None, :] - (ny - 1) / 2.0 + offs[:, None]) / R  # [ss][ny]
    img = np.zeros((nz, ny, nx))
    Xg = np.broadcast_to(xs[None, :, None, :], (ss, ss, ny, nx))  # [sub-y][sub-x][ny][nx]
    Yg = np.broadcast_to(ys[:, None, :, None], (ss, ss, ny, nx))
    for z in range(nz):
        acc = np.zeros((ss, ss, ny, nx))
        for e in ellipses:
            sc = _slice_ellipse(e, nz, z)
            if sc is None:
                continue
            a, b = e.a * sc[0], e.b * sc[1]
            dx, dy = Xg - e.cx, Yg - e.cy
            cp, sp = math.cos(e.phi), math.sin(e.phi)
            xr = dx * cp + dy * sp
            yr = -dx * sp + dy * cp
            acc += e.rho * ((xr / a) ** 2 + (yr / b) ** 2 <= 1.0)
        img[z] = acc.mean(axis=(0, 1))
    return img


def analytic_sinogram(ellipses: list[Ellipse], nx: int, ny: int, n_angles: int, n_bins: int,
                      nz: int = 1, du: float = 1.0, off: float = 0.0,
                      angles: np.ndarray | None = None) -> np.ndarray:
    """Exact line integrals [nz][A][B] (float64) of the ellipse phantom, in pixel units."""
    R = min(nx, ny) / 2.0
    th = (np.arange(n_angles) * math.pi / n_angles) if angles is None else np.asarray(angles)
    s = (np.arange(n_bins) - (n_bins - 1) / 2.0) * du + off
    ct, st = np.cos(th)[:, None], np.sin(th)[:, None]
    out = np.zeros((nz, n_angles, n_bins))
    for z in range(nz):
        for e in ellipses:
            sc = _slice_ellipse(e, nz, z)
            if sc is None:
                continue
            A, Bq = e.a * sc[0] * R, e.b * sc[1] * R
            s0 = e.cx * R * ct + e.cy * R * st           # centre's detector coordinate
            a2 = (A * np.cos(th - e.phi)) ** 2 + (Bq * np.sin(th - e.phi)) ** 2
            a2 = a2[:, None]
            t = s[None, :] - s0
            inside = t * t < a2
            chord = np.where(inside, 2.0 * A * Bq * np.sqrt(np.maximum(a2 - t * t, 0.0)) / a2, 0.0)
            out[z] += e.rho * chord
    return out


def add_gaussian_noise(sino: np.ndarray, seed: int, level: float = 0.01) -> np.ndarray:
    """b = sino + sigma N(0, 1), sigma = level * max(sino)."""
    rng = np.random.default_rng(seed)
    sigma = level * float(np.max(sino))
    return sino + sigma * rng.standard_normal(sino.shape)


def add_poisson_log_noise(sino: np.ndarray, seed: int, photons: float = 1e4,
                          max_attenuation: float = 2.0) -> np.ndarray:
    """Transmission noise: counts ~ Poisson(I0 exp(-mu sino)), b = -ln(max(counts,1)/I0)/mu,
    with mu chosen so that max(mu * sino) = max_attenuation."""
    rng = np.random.default_rng(seed)
    mu = max_attenuation / max(float(np.max(sino)), 1e-30)
    counts = rng.poisson(photons * np.exp(-mu * sino))
    return -np.log(np.maximum(counts, 1) / photons) / mu


@dataclasses.dataclass
class Problem:
    """One synthetic reconstruction problem (all arrays float64)."""
    phantom: np.ndarray   # [nz][ny][nx]
    b: np.ndarray         # [nz][A][B] noisy sinogram
    clean: np.ndarray     # [nz][A][B] exact line integrals


def make_problem(nx: int, ny: int, n_angles: int, n_bins: int, seed: int, nz: int = 1,
                 n_ellipses: int = 10, noise: str = "gaussian", du: float = 1.0,
                 off: float = 0.0, with_phantom: bool = True) -> Problem:
    """Phantom from ``seed``, noise from ``seed + 1`` (gaussian: 1% of max; poisson-log)."""
    ells = random_ellipses(seed, n_ellipses, dims=3 if nz > 1 else 2)
    clean = analytic_sinogram(ells, nx, ny, n_angles, n_bins, nz=nz, du=du, off=off)
    if noise == "gaussian":
        b = add_gaussian_noise(clean, seed + 1)
    elif noise == "poisson-log":
        b = add_poisson_log_noise(clean, seed + 1)
    elif noise == "none":
        b = clean.copy()
    else:
        raise ValueError(noise)
    ph = rasterize(ells, nx, ny, nz) if with_phantom else np.zeros((0,))
    return Problem(ph, b, clean)


def perturbed_batch(batch: int, nx: int, ny: int, seed: int) -> np.ndarray:
    """[batch][ny][nx] random-ellipse images plus N(0, 1) perturbations (differentiation check)."""
    rng = np.random.default_rng(seed + 1)
    out = np.empty((batch, ny, nx))
    for k in range(batch):
        out[k] = rasterize(random_ellipses(seed + 1000 * k, 10), nx, ny)[0]
    return out + rng.standard_normal(out.shape)


def analytic_sinogram_torch(ellipses: list[Ellipse], nx: int, ny: int, n_angles: int,
                            n_bins: int, nz: int = 1, du: float = 1.0, off: float = 0.0,
                            device="cuda", dtype=None):
    """Same line integrals as analytic_sinogram, evaluated with torch on ``device`` (float64 by
    default) -- for volumes too large to generate on the host in reasonable time."""
    import torch
    dtype = dtype or torch.float64
    R = min(nx, ny) / 2.0
    th = torch.arange(n_angles, device=device, dtype=torch.float64) * (math.pi / n_angles)
    s = (torch.arange(n_bins, device=device, dtype=torch.float64) - (n_bins - 1) / 2.0) * du + off
    ct, st = torch.cos(th)[:, None], torch.sin(th)[:, None]
    out = torch.zeros((nz, n_angles, n_bins), device=device, dtype=dtype)
    for z in range(nz):
        acc = torch.zeros((n_angles, n_bins), device=device, dtype=torch.float64)
        for e in ellipses:
            sc = _slice_ellipse(e, nz, z)
            if sc is None:
                continue
            A, Bq = e.a * sc[0] * R, e.b * sc[1] * R
            s0 = e.cx * R * ct + e.cy * R * st
            a2 = ((A * torch.cos(th - e.phi)) ** 2 + (Bq * torch.sin(th - e.phi)) ** 2)[:, None]
            t = s[None, :] - s0
            chord = 2.0 * A * Bq * torch.sqrt(torch.clamp(a2 - t * t, min=0.0)) / a2
            acc += e.rho * chord
        out[z] = acc.to(dtype)
    return out


def gaussian_noise_torch(sino, seed: int, level: float = 0.01):
    """sino + N(0, (level * max|sino|)^2) from a seeded torch generator on sino's device."""
    import torch
    gen = torch.Generator(device=sino.device).manual_seed(int(seed))
    sigma = level * float(sino.abs().max())
    return sino + sigma * torch.randn(sino.shape, generator=gen, device=sino.device, dtype=sino.dtype)


def poisson_log_noise_torch(sino, seed: int, photons: float = 1e4, max_attenuation: float = 2.0):
    """Transmission noise of add_poisson_log_noise, drawn with a seeded torch generator on the
    sinogram's device (in place on a float copy)."""
    import torch
    gen = torch.Generator(device=sino.device).manual_seed(seed)
    mu = max_attenuation / max(float(sino.max()), 1e-30)
    out = torch.empty_like(sino)
    for z in range(sino.shape[0]):  # slice by slice: bounded temporaries
        lam = photons * torch.exp(-mu * sino[z].double())
        counts = torch.poisson(lam, generator=gen)
        out[z] = (-torch.log(torch.clamp(counts, min=1.0) / photons) / mu).to(sino.dtype)
    return out
