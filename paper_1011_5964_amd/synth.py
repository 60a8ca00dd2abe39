"""Seeded synthetic inputs shaped like the paper's test problems.

The paper's own signal and image are shown only as figures, so every input
here is a seeded piecewise-constant phantom with the paper's kind of blur
(Gaussian, Section 5.2; out-of-focus uniform disk, Section 5.1, eq. (of))
and additive white Gaussian noise at a stated level.

This module produces DATA ONLY.  It contains none of the deblurring method's
arithmetic (no boundary conditions, no operators, no solver): the observed
image is the valid convolution of a larger scene with the PSF, i.e. the
physical model v = h * u + eta of Section 1, eq. (nbf), with a field of view
cropped from the scene as in Section 5.1.  Both the GPU library tests and the
oracle tests receive the same arrays from here.

Recipe (per image, numpy PCG64 generator seeded with `seed`):
  * field of (n+2m) x (n+2m) zeros; S shapes painted in order (later ones
    overwrite): rectangle or disk with probability 1/2 each; rectangle corner
    uniform on the field, sides uniform integers in [n/32, n/4]; disk centre
    uniform, radius uniform in [n/64, n/8]; intensity U[0, 1];
  * optional ramp rectangle covering about a quarter of the field with
    intensity 0.2 + 0.6 (i + j) / (2n);
  * v = valid convolution of the field with h, plus N(0, sigma^2) noise with
    sigma = level * ||h * u||_2 / sqrt(N);  u_true = central n x n crop.
"""

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.signal


def gaussian_psf(size, sigma):
    """size x size Gaussian exp(-(a^2+b^2)/(2 sigma^2)), normalised to sum 1."""
    if size % 2 != 1:
        raise ValueError("PSF size must be odd")
    m = size // 2
    a = np.arange(-m, m + 1, dtype=np.float64)
    g = np.exp(-(a[:, None] ** 2 + a[None, :] ** 2) / (2.0 * sigma * sigma))
    return g / g.sum()


def disk_psf(radius):
    """Out-of-focus uniform disk of the given radius on a (2r+1)^2 grid,
    normalised to sum 1."""
    r = int(radius)
    a = np.arange(-r, r + 1, dtype=np.float64)
    d = ((a[:, None] ** 2 + a[None, :] ** 2) <= r * r).astype(np.float64)
    return d / d.sum()


def phantom_field(n, m, shapes, rng, ramp=False):
    """(n+2m)^2 piecewise-constant scene (see module docstring)."""
    F = n + 2 * m
    img = np.zeros((F, F))
    ii, jj = np.mgrid[0:F, 0:F]
    lo_side = max(1, n // 32)
    hi_side = max(lo_side, n // 4)
    for _ in range(shapes):
        if rng.random() < 0.5:
            r0 = int(rng.integers(0, F))
            c0 = int(rng.integers(0, F))
            hgt = int(rng.integers(lo_side, hi_side + 1))
            wid = int(rng.integers(lo_side, hi_side + 1))
            img[r0:r0 + hgt, c0:c0 + wid] = rng.random()
        else:
            cy = rng.random() * F
            cx = rng.random() * F
            rad = n / 64.0 + rng.random() * (n / 8.0 - n / 64.0)
            img[(ii - cy) ** 2 + (jj - cx) ** 2 <= rad * rad] = rng.random()
    if ramp:
        r0 = int(rng.integers(0, F // 2))
        c0 = int(rng.integers(0, F // 2))
        side = F // 2
        sl = (slice(r0, r0 + side), slice(c0, c0 + side))
        img[sl] = 0.2 + 0.6 * (ii[sl] + jj[sl] - 2 * m) / (2.0 * n)
    return img


@dataclass
class Problem:
    name: str
    v: np.ndarray          # observed n x n
    u_true: np.ndarray     # central crop of the scene
    psf: np.ndarray
    bc: str
    alpha: float
    beta: float
    n_outer: int
    inner_tol: float
    max_inner: int
    noise: float
    seed: int
    fp_tol: float = 0.0


def make_problem(name, n, shapes, psf, bc, alpha, beta, n_outer, noise, seed,
                 inner_tol=1e-6, max_inner=100, ramp=False):
    rng = np.random.default_rng(seed)
    m = psf.shape[0] // 2
    scene = phantom_field(n, m, shapes, rng, ramp=ramp)
    blurred = scipy.signal.fftconvolve(scene, psf, mode="valid")
    sigma = noise * np.linalg.norm(blurred) / np.sqrt(blurred.size)
    v = blurred + sigma * rng.standard_normal(blurred.shape)
    u_true = scene[m:m + n, m:m + n].copy()
    return Problem(name, v, u_true, psf, bc, alpha, beta, n_outer, inner_tol,
                   max_inner, noise, seed)


# Named workloads (sizes and parameters of the test problems).
def config(name):
    """Return a Problem (or list of Problems for the batch) by name.

    c1      64^2,  8 shapes,  9x9 Gaussian s=1.5, AR,  a=1e-3, b=0.1, K=10
    c2_ar   256^2, 32 shapes, 15x15 Gaussian s=2.5, AR, a=5e-4, b=0.05, K=20
    c2_r    same image, reflective BCs
    c3_gauss 1024^2, 256 shapes + ramp, 31x31 Gaussian s=5, AR, noise 0.5%,
            a=1e-4, b=0.01, K=20
    c3_disk same scene family, out-of-focus disk r=5
    c5 / m512  512^2, 64 shapes, 21x21 Gaussian s=3, AR, a=5e-4, b=0.05, K=15
    """
    if name == "c1":
        return make_problem("c1", 64, 8, gaussian_psf(9, 1.5), "antireflective",
                            1e-3, 0.1, 10, 0.01, 1)
    if name in ("c2_ar", "c2_r"):
        bc = "antireflective" if name == "c2_ar" else "reflective"
        return make_problem(name, 256, 32, gaussian_psf(15, 2.5), bc,
                            5e-4, 0.05, 20, 0.01, 2)
    if name == "c3_gauss":
        return make_problem(name, 1024, 256, gaussian_psf(31, 5.0), "antireflective",
                            1e-4, 0.01, 20, 0.005, 3, ramp=True)
    if name == "c3_disk":
        return make_problem(name, 1024, 256, disk_psf(5), "antireflective",
                            1e-4, 0.01, 20, 0.005, 3, ramp=True)
    if name == "c5":
        return make_problem(name, 512, 64, gaussian_psf(21, 3.0), "antireflective",
                            5e-4, 0.05, 15, 0.01, 5)
    if name == "m512":
        return make_problem(name, 512, 64, gaussian_psf(21, 3.0), "antireflective",
                            5e-4, 0.05, 15, 0.01, 512)
    if name == "c4":
        return batch_problems(64)
    raise KeyError(name)


def batch_problems(count, base_seed=4000, sides=(128, 192, 256, 384, 512),
                   n_outer=10):
    """Uneven batch: side lengths uniform over `sides`, Gaussian PSF of odd
    size in [9, 21] with sigma U[1, 4], alpha log-uniform in [1e-4, 1e-2],
    beta = 0.05, anti-reflective, 1% noise, n/8 shapes."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        n = int(rng.choice(np.asarray(sides)))
        size = int(rng.choice(np.arange(9, 22, 2)))
        sigma = float(rng.uniform(1.0, 4.0))
        alpha = float(10.0 ** rng.uniform(-4.0, -2.0))
        out.append(make_problem(f"c4_{i}", n, max(1, n // 8), gaussian_psf(size, sigma),
                                "antireflective", alpha, 0.05, n_outer, 0.01,
                                base_seed + 10_000 + i))
    return out


def out_of_focus_1d(m):
    """Out-of-focus PSF of Section 5.1, eq. (of): h_i = c for |i| < m, else 0,
    with c normalising the sum to 1; returned as a 1 x (2m-1) PSF."""
    if m < 1:
        raise ValueError("m >= 1")
    return np.full((1, 2 * m - 1), 1.0 / (2 * m - 1))


def signal_half_width(n):
    """m(n) of eq. (of): the PSF reaches m-1 samples past each end of the
    field of view, which covers [0.1, 0.9] of the scene (Section 5.1), so the
    margin of 0.1 of the scene on each side is about n/8 samples."""
    return max(2, int(round(n / 8.0)))


def signal_problem(n=203, bc="antireflective", alpha=1e-3, beta=0.1, n_outer=100, fp_tol=1e-3,
                   noise=0.01, seed=203, inner_tol=1e-6, max_inner=1000, pieces=8):
    """1D signal deblurring of Section 5.1 as a 1 x n image: a seeded scene of
    n + 2(m-1) samples on [0, 1] made of `pieces` segments (constant or
    linear with probability 1/2 each, levels U[0, 1], breakpoints uniform),
    blurred by the out-of-focus PSF of half-width m = m(n), the field of view
    the central n samples, plus white Gaussian noise at the given level
    relative to ||h * u|| (1% as in Section 5.1).  The paper's own signal is
    shown only as a figure; only the shape of the set-up is reproduced."""
    rng = np.random.default_rng(seed)
    m = signal_half_width(n)
    F = n + 2 * (m - 1)
    x = np.arange(F, dtype=np.float64)
    cuts = np.sort(rng.choice(np.arange(1, F), size=pieces - 1, replace=False))
    edges = np.concatenate([[0], cuts, [F]])
    scene = np.zeros(F)
    for a, b in zip(edges[:-1], edges[1:]):
        lo, hi = rng.random(), rng.random()
        if rng.random() < 0.5:
            scene[a:b] = lo
        else:
            scene[a:b] = lo + (hi - lo) * (x[a:b] - a) / max(1, b - a)
    psf = out_of_focus_1d(m)
    blurred = np.convolve(scene, psf[0], mode="valid")
    sigma = noise * np.linalg.norm(blurred) / np.sqrt(blurred.size)
    v = blurred + sigma * rng.standard_normal(blurred.shape)
    p = Problem(f"signal_{n}", v[None, :].copy(), scene[m - 1:m - 1 + n][None, :].copy(), psf, bc, alpha,
                beta, n_outer, inner_tol, max_inner, noise, seed)
    p.fp_tol = fp_tol
    return p


def small_problem(n=32, psf_size=7, sigma=1.2, bc="antireflective", alpha=1e-3,
                  beta=0.1, n_outer=3, seed=7, shapes=6, ny=None):
    """Small case for tests (the oracle finishes it in well under a second).
    ny, if given, makes the image rectangular (ny x n) by cropping."""
    p = make_problem("small", max(n, ny or n), shapes, gaussian_psf(psf_size, sigma), bc,
                     alpha, beta, n_outer, 0.01, seed)
    if ny is not None and ny != n:
        p.v = np.ascontiguousarray(p.v[:ny, :n])
        p.u_true = np.ascontiguousarray(p.u_true[:ny, :n])
    return p
