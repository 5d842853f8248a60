"""Seeded synthetic inputs shaped like the paper's workloads.

This module only makes data: Gaussian-mixture point sets and per-sample
(s, k) tables.  It contains none of the clustering method's arithmetic and
is the one piece both the FP64 oracle tests and the GPU path use.  Data are
FP32, generated with torch's generator on the requested device (CPU or GPU)
in chunks, so the same call gives the same array for a given device.

The paper's 23 real data sets are not available; these mixtures stand in
for them (Section 6.3 lists m from 7,797 to 10.5 million and 2 to 5,000
attributes; the scaling study of Section 6.8 uses Gaussian blobs plus
uniform noise).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch


@dataclass
class Mixture:
    X: torch.Tensor          # m x d float32
    comp: torch.Tensor       # m int64 component (-1 = noise)
    centres: torch.Tensor    # n_comp x d float64 (CPU)


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def gaussian_mixture(m: int, d: int, n_comp: int, *, seed: int, centre_box: float,
                     std: float | tuple[float, float] = 1.0, diag_std: bool = False,
                     dirichlet_weights: bool = False, rotate: bool = False,
                     log_uniform_std: bool = False, noise_frac: float = 0.0,
                     noise_box: float = 50.0, device="cpu", chunk: int = 1 << 22) -> Mixture:
    """m points in d dimensions from an n_comp-component mixture.

    centres ~ U[-centre_box, centre_box]^d; per-component standard
    deviation either fixed (``std`` a float), or drawn per component (and
    per dimension if ``diag_std``) uniformly / log-uniformly in the ``std``
    range; weights equal or Dirichlet(1); ``rotate`` applies a Haar-random
    rotation per component (anisotropic, rotated covariance); a fraction
    ``noise_frac`` of the points is uniform in [-noise_box, noise_box]^d."""
    gc = _gen(seed, "cpu")
    centres = (torch.rand(n_comp, d, generator=gc, dtype=torch.float64) * 2 - 1) * centre_box
    if isinstance(std, tuple):
        lo, hi = std
        shape = (n_comp, d) if diag_std else (n_comp, 1)
        u = torch.rand(*shape, generator=gc, dtype=torch.float64)
        sig = torch.exp(np.log(lo) + u * (np.log(hi) - np.log(lo))) if log_uniform_std else lo + u * (hi - lo)
        sig = sig.expand(n_comp, d).clone()
    else:
        sig = torch.full((n_comp, d), float(std), dtype=torch.float64)
    if dirichlet_weights:
        e = -torch.log(torch.rand(n_comp, generator=gc, dtype=torch.float64))
        w = e / e.sum()
    else:
        w = torch.full((n_comp,), 1.0 / n_comp, dtype=torch.float64)
    rots = None
    if rotate:
        A = torch.randn(n_comp, d, d, generator=gc, dtype=torch.float64)
        Q, R = torch.linalg.qr(A)
        Q = Q * torch.sign(torch.diagonal(R, dim1=1, dim2=2)).unsqueeze(1)
        rots = Q
    g = _gen(seed + 7919, device)
    X = torch.empty(m, d, dtype=torch.float32, device=device)
    comp = torch.empty(m, dtype=torch.int64, device=device)
    cen_d = centres.to(device=device, dtype=torch.float32)
    sig_d = sig.to(device=device, dtype=torch.float32)
    w_d = w.to(device=device, dtype=torch.float32)
    rot_d = rots.to(device=device, dtype=torch.float32) if rots is not None else None
    for a in range(0, m, chunk):
        b = min(m, a + chunk)
        n = b - a
        c = torch.multinomial(w_d, n, replacement=True, generator=g)
        z = torch.randn(n, d, generator=g, device=device, dtype=torch.float32) * sig_d[c]
        if rot_d is not None:
            # rotate each component's offsets by its own matrix (grouped, so
            # no per-point d x d matrix is ever materialised)
            zr = torch.empty_like(z)
            for q in range(n_comp):
                sel = (c == q).nonzero(as_tuple=True)[0]
                if sel.numel():
                    zr[sel] = z[sel] @ rot_d[q].T
            z = zr
        x = cen_d[c] + z
        if noise_frac > 0:
            is_noise = torch.rand(n, generator=g, device=device) < noise_frac
            nz = (torch.rand(n, d, generator=g, device=device) * 2 - 1) * noise_box
            x = torch.where(is_noise.unsqueeze(1), nz, x)
            c = torch.where(is_noise, torch.full_like(c, -1), c)
        X[a:b] = x
        comp[a:b] = c
    return Mixture(X, comp, centres)


# --------------------------------------------------------------------------
# The workloads (data shape, mixture recipe, per-sample sizes).
# --------------------------------------------------------------------------
def plain_small(device="cpu") -> Mixture:
    """m = 50,000, d = 8, 10 isotropic components, centres in [-10, 10]^8,
    sigma = 1, equal weights, seed 0 (k = 10, s = 2,000, 8 samples)."""
    return gaussian_mixture(50_000, 8, 10, seed=0, centre_box=10.0, std=1.0, device=device)


def plain_batched(m=10_000_000, device="cpu") -> Mixture:
    """m = 10^7, d = 16, 25 components, centres in [-20, 20]^16, diagonal std
    U[0.5, 3] per component and dimension, Dirichlet(1) weights."""
    return gaussian_mixture(m, 16, 25, seed=2, centre_box=20.0, std=(0.5, 3.0), diag_std=True,
                            dirichlet_weights=True, device=device)


def uneven(m=20_000_000, device="cpu") -> Mixture:
    """m = 2*10^7, d = 32: 95% from a 40-component mixture (centres in
    [-20, 20]^32, diagonal std U[0.5, 3], Dirichlet(1)), 5% uniform noise in
    [-50, 50]^32."""
    return gaussian_mixture(m, 32, 40, seed=3, centre_box=20.0, std=(0.5, 3.0), diag_std=True,
                            dirichlet_weights=True, noise_frac=0.05, noise_box=50.0, device=device)


def precision_set(m=100_000_000, device="cpu") -> Mixture:
    """m = 10^8, d = 64, 100 anisotropic rotated components, std
    log-uniform in [0.3, 5] per dimension, centres in [-20, 20]^64,
    Dirichlet(1) weights."""
    return gaussian_mixture(m, 64, 100, seed=4, centre_box=20.0, std=(0.3, 5.0), diag_std=True,
                            log_uniform_std=True, rotate=True, dirichlet_weights=True,
                            device=device)


def metric_set(m=10_000_000, device="cpu", seed=5) -> Mixture:
    """m = 10^7, d = 32 from one 25-component mixture with centres in
    [-20, 20]^32 and diagonal std U[0.5, 3] (k = 25, s = 10,000)."""
    return gaussian_mixture(m, 32, 25, seed=seed, centre_box=20.0, std=(0.5, 3.0), diag_std=True,
                            device=device)


def uneven_sizes(n: int, *, seed: int = 3, s_range=(1_000, 100_000), k_range=(2, 50)):
    """Per-sample (s, k), s ~ U[s_lo, s_hi] and k ~ U[k_lo, k_hi] (integers)."""
    rng = np.random.Generator(np.random.Philox(seed))
    s = rng.integers(s_range[0], s_range[1] + 1, size=n)
    k = rng.integers(k_range[0], k_range[1] + 1, size=n)
    return s.astype(np.int64), k.astype(np.int64)


def mixture_family(n_sets: int, s: int, *, d: int = 32, n_comp: int = 25, seed: int,
                   template: bool = False, template_seed: int = 0, device="cpu"):
    """n_sets independent point sets of s points, set i occupying rows
    [i*s, (i+1)*s) of the returned X (n_sets*s x d, float32).

    Each set is drawn from its own n_comp-component mixture with equal
    weights and diagonal std U[0.5, 3] per component and dimension.  With
    ``template`` False the centres of every set are fresh, U[-20, 20]^d (the
    learned initializer's training family).  With ``template`` True they
    are a shared random configuration T0 ~ U[-20, 20]^d (drawn from
    ``template_seed``, the same for every call), scaled by a ~
    U[0.5, 2], shifted by t ~ U[-20, 20]^d and jittered by N(0, 0.5^2) per
    coordinate: a family whose normalised structure repeats.
    Returns (X, centres as n_sets x n_comp x d float32)."""
    g = _gen(seed, device)
    kw = dict(generator=g, device=device, dtype=torch.float32)
    if template:
        gt = _gen(104729 + template_seed, device)
        T0 = (torch.rand(n_comp, d, generator=gt, device=device) * 2 - 1) * 20.0
        a = 0.5 + 1.5 * torch.rand(n_sets, 1, 1, **kw)
        t = (torch.rand(n_sets, 1, d, **kw) * 2 - 1) * 20.0
        cen = T0.unsqueeze(0) * a + t + 0.5 * torch.randn(n_sets, n_comp, d, **kw)
    else:
        cen = (torch.rand(n_sets, n_comp, d, **kw) * 2 - 1) * 20.0
    sig = 0.5 + 2.5 * torch.rand(n_sets, n_comp, d, **kw)
    lab = torch.randint(0, n_comp, (n_sets, s), generator=g, device=device)
    sets = torch.arange(n_sets, device=device).unsqueeze(1).expand(n_sets, s)
    X = cen[sets, lab] + sig[sets, lab] * torch.randn(n_sets, s, d, **kw)
    return X.reshape(n_sets * s, d).contiguous(), cen


def scaling_blobs(i: int, *, seed: int = 0, device="cpu") -> Mixture:
    """The scaling study's data (Section 6.8): m = 3^(i+7) points in 10
    dimensions from 10 Gaussian blobs with centres uniform in (-40, 40)^10
    and isotropic std uniform in (0, 10), plus 500 points uniform in
    (-50, 50)^10 as noise (appended after the blob points, component -1)."""
    m = 3 ** (i + 7)
    d, n_comp = 10, 10
    gc = _gen(seed, "cpu")
    centres = (torch.rand(n_comp, d, generator=gc, dtype=torch.float64) * 2 - 1) * 40.0
    sig = torch.rand(n_comp, 1, generator=gc, dtype=torch.float64) * 10.0
    g = _gen(seed + 7919, device)
    c = torch.randint(0, n_comp, (m,), generator=g, device=device)
    z = torch.randn(m, d, generator=g, device=device, dtype=torch.float32)
    X = centres.to(device=device, dtype=torch.float32)[c] + z * sig.to(device=device,
                                                                        dtype=torch.float32)[c]
    noise = (torch.rand(500, d, generator=g, device=device) * 2 - 1) * 50.0
    X = torch.cat([X, noise]).contiguous()
    comp = torch.cat([c, torch.full((500,), -1, dtype=c.dtype, device=device)])
    return Mixture(X, comp, centres)


def scaling_sample_size(m: int) -> int:
    """s = min(5000, m - 1000) (Section 6.8)."""
    return min(5000, m - 1000)
