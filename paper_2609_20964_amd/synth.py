"""Seeded synthetic inputs: oriented point clouds, query points and request streams.

This module only draws shapes and random numbers.  It holds none of the
reconstruction's arithmetic (no splat weights, divergence, solve, surface
extraction or distance), so both the HIP path and the FP64 CPU oracle can be
fed from it.  Every array is drawn in float64 with ``numpy.random.default_rng``
(PCG64) and rounded once to float32; the oracle promotes those float32 values
back to float64 exactly.

The paper's own clouds (fish, aircraft, vascular, ...) are not available, so
these shapes stand in for them with the sizes of its workloads:

* ``sphere``   radius 0.3 sphere, exact normals (plain forward, 32^3).
* ``torus``    R=0.3, r=0.1 torus with position / angular noise (forward at 128^3).
* ``star``     superellipsoid with a 16-coefficient azimuthal Fourier modulation
               (the differentiable case and the serving stream).
* ``flapping`` ellipsoid under a travelling-wave shear (moving boundary, 256^3).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

X0 = np.array([0.5, 0.5, 0.5])


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def unit_sphere_dirs(rng, n):
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def uniform_queries(n, seed):
    """``n`` query points uniform in [0,1)^3."""
    return _f32(np.random.default_rng(seed).random((n, 3)))


# ---------------------------------------------------------------------------
# sphere
# ---------------------------------------------------------------------------

def sphere(n_points=4096, radius=0.3, seed=101):
    u = unit_sphere_dirs(np.random.default_rng(seed), n_points)
    return _f32(X0 + radius * u), _f32(u)


# ---------------------------------------------------------------------------
# torus
# ---------------------------------------------------------------------------

def torus(n_points=200_000, R=0.3, r=0.1, pos_sigma=0.002, ang_sigma_deg=2.0,
          seeds=(201, 202, 203)):
    """Area-uniform torus about the z axis by rejection, then noise.

    Positions get isotropic Gaussian noise ``pos_sigma``; normals get a
    tangential Gaussian perturbation of angular size ``ang_sigma_deg`` and are
    renormalised.
    """
    rng = np.random.default_rng(seeds[0])
    us, vs = [], []
    have = 0
    while have < n_points:
        m = 2 * (n_points - have) + 1024
        u = rng.uniform(0, 2 * np.pi, m)
        v = rng.uniform(0, 2 * np.pi, m)
        acc = rng.random(m) < (R + r * np.cos(u)) / (R + r)
        us.append(u[acc]); vs.append(v[acc])
        have += int(acc.sum())
    u = np.concatenate(us)[:n_points]
    v = np.concatenate(vs)[:n_points]
    rr = R + r * np.cos(u)
    x = np.stack([rr * np.cos(v), rr * np.sin(v), r * np.sin(u)], 1) + X0
    nrm = np.stack([np.cos(u) * np.cos(v), np.cos(u) * np.sin(v), np.sin(u)], 1)
    x = x + np.random.default_rng(seeds[1]).normal(0.0, pos_sigma, x.shape)
    g = np.random.default_rng(seeds[2]).standard_normal(x.shape)
    g_t = g - np.sum(g * nrm, 1, keepdims=True) * nrm
    nrm = nrm + math.radians(ang_sigma_deg) * g_t
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    return _f32(x), _f32(nrm)


# ---------------------------------------------------------------------------
# star-shaped superellipsoid with a Fourier modulation
# ---------------------------------------------------------------------------

@dataclass
class StarShape:
    """Radial profile rho(u) = R_se(u) * (1 + sum_m c_{2m-1} Re w^m + c_{2m} Im w^m).

    ``u`` is a unit direction in the body frame, ``w = u_y + i u_z`` (azimuth
    about the body axis x) and R_se(u) = (sum |u_k / a_k|^p)^(-1/p).  The body
    frame is mapped to the world by ``rotation`` and centred at ``centre``.
    """
    coeffs: np.ndarray
    semi_axes: tuple = (0.30, 0.12, 0.15)
    p: float = 3.0
    rotation: np.ndarray = field(default_factory=lambda: np.eye(3))
    centre: np.ndarray = field(default_factory=lambda: X0.copy())

    def modulation(self, u, coeffs=None):
        c = self.coeffs if coeffs is None else coeffs
        w = u[..., 1] + 1j * u[..., 2]
        out = np.ones(u.shape[:-1])
        wm = np.ones_like(w)
        for m in range(1, len(c) // 2 + 1):
            wm = wm * w
            out = out + c[2 * m - 2] * wm.real + c[2 * m - 1] * wm.imag
        return out

    def rho(self, u):
        a = np.asarray(self.semi_axes, dtype=np.float64)
        rse = np.sum(np.abs(u / a) ** self.p, axis=-1) ** (-1.0 / self.p)
        return rse * self.modulation(u)


def draw_star_coeffs(seed, n_coeffs=16, amp=0.05, test_seed=None, band=(0.75, 1.25)):
    """Coefficients ~ U(-amp, amp); redrawn with seed+1, seed+2, ... until the
    modulation stays inside ``band`` on 1e5 test directions."""
    test_seed = (seed + 98) if test_seed is None else test_seed
    test_u = unit_sphere_dirs(np.random.default_rng(test_seed), 100_000)
    s = seed
    while True:
        c = np.random.default_rng(s).uniform(-amp, amp, n_coeffs)
        m = StarShape(c).modulation(test_u)
        if m.min() >= band[0] and m.max() <= band[1]:
            return c
        s += 1


def star_points_torch(shape: StarShape, dirs, coeffs_t):
    """Points and unit normals of ``shape`` along body-frame directions ``dirs``
    as differentiable torch functions of the coefficient vector ``coeffs_t``.

    Normals are grad G / |grad G| with G(x) = |x - x0| - rho((x - x0)/|x - x0|),
    taken with autograd (create_graph=True keeps them differentiable in the
    coefficients).  Returns float64 tensors (points [N,3], normals [N,3]).
    """
    import torch
    dt = coeffs_t.dtype
    a = torch.tensor(shape.semi_axes, dtype=dt)
    Rm = torch.tensor(shape.rotation, dtype=dt)
    x0 = torch.tensor(shape.centre, dtype=dt)

    def rho_t(u):
        rse = (torch.abs(u / a) ** shape.p).sum(-1) ** (-1.0 / shape.p)
        wr, wi = u[:, 1], u[:, 2]
        pr, pi = torch.ones_like(wr), torch.zeros_like(wr)
        mod = torch.ones_like(wr)
        for m in range(1, coeffs_t.shape[0] // 2 + 1):
            pr, pi = pr * wr - pi * wi, pr * wi + pi * wr
            mod = mod + coeffs_t[2 * m - 2] * pr + coeffs_t[2 * m - 1] * pi
        return rse * mod

    u = torch.as_tensor(dirs, dtype=dt)
    d_local = rho_t(u)[:, None] * u                   # body-frame offsets
    # normal: gradient of G at the surface point, evaluated in the body frame
    y = d_local.detach().clone().requires_grad_(True) if not d_local.requires_grad else d_local
    r = torch.linalg.norm(y, dim=1)
    G = r - rho_t(y / r[:, None])
    (gG,) = torch.autograd.grad(G.sum(), y, create_graph=True)
    n_local = gG / torch.linalg.norm(gG, dim=1, keepdim=True)
    pts = x0 + d_local @ Rm.T
    nrm = n_local @ Rm.T
    return pts, nrm


def star(coeffs, n_points, dir_seed, semi_axes=(0.30, 0.12, 0.15), p=3.0, rotation=None,
         centre=None):
    """float32 points and normals of a star shape (no autograd graph kept)."""
    import torch
    shape = StarShape(np.asarray(coeffs, np.float64), tuple(semi_axes), float(p),
                      np.eye(3) if rotation is None else np.asarray(rotation, np.float64),
                      X0.copy() if centre is None else np.asarray(centre, np.float64))
    dirs = unit_sphere_dirs(np.random.default_rng(dir_seed), n_points)
    with torch.enable_grad():
        pts, nrm = star_points_torch(shape, dirs, torch.tensor(shape.coeffs, dtype=torch.float64))
    return _f32(pts.detach().numpy()), _f32(nrm.detach().numpy())


def fish(n_points=200_000, seed=(811, 812), semi_axes=(0.40, 0.14, 0.18), p=2.5):
    """A fish-like body for bounding-box grids: an elongated star shape
    (semi-axes 0.40 x 0.14 x 0.18, exponent 2.5, 16 seeded Fourier
    coefficients) centred at (0.5, 0.5, 0.5): bounding box about 0.8 x 0.28 x
    0.36, the proportions of the paper's fish grid (338 x 120 x 151 cells).
    Returns float32 points and unit normals."""
    c = draw_star_coeffs(seed[0])
    return star(c, n_points, seed[1], semi_axes=semi_axes, p=p)


@dataclass
class DiffCase:
    """The differentiable workload: 16 coefficients, 100k points, 65,536 targets."""
    shape: StarShape
    dirs: np.ndarray
    targets: np.ndarray          # float32 [T,3]
    target_coeffs: np.ndarray


def diff_case(n_points=100_000, n_targets=65_536, seeds=(301, 302, 303, 304)):
    c = draw_star_coeffs(seeds[0])
    shape = StarShape(c)
    dirs = unit_sphere_dirs(np.random.default_rng(seeds[1]), n_points)
    delta = np.random.default_rng(seeds[2]).uniform(-0.02, 0.02, c.shape)
    ct = c + delta
    tdirs = unit_sphere_dirs(np.random.default_rng(seeds[3]), n_targets)
    tshape = StarShape(ct)
    tpts = X0 + tshape.rho(tdirs)[:, None] * tdirs
    return DiffCase(shape, dirs, _f32(tpts), ct)


# ---------------------------------------------------------------------------
# flapping ellipsoid (moving boundary)
# ---------------------------------------------------------------------------

@dataclass
class Flapping:
    """Ellipsoid (0.30, 0.12, 0.08) sheared by y += A sin(2 pi (xi/lam - t/T))."""
    n_points: int = 300_000
    semi_axes: tuple = (0.30, 0.12, 0.08)
    amp: float = 0.05
    lam: float = 0.6
    period: float = 100.0
    seed: int = 401

    def __post_init__(self):
        a = np.asarray(self.semi_axes)
        u = unit_sphere_dirs(np.random.default_rng(self.seed), self.n_points)
        self.x_base = X0 + u * a
        n0 = (self.x_base - X0) / a ** 2
        self.n_base = n0 / np.linalg.norm(n0, axis=1, keepdims=True)

    def step(self, t):
        xi = self.x_base[:, 0] - 0.5
        ph = 2 * np.pi * (xi / self.lam - t / self.period)
        f = self.amp * np.sin(ph)
        fp = self.amp * (2 * np.pi / self.lam) * np.cos(ph)
        x = self.x_base.copy()
        x[:, 1] += f
        n = np.stack([self.n_base[:, 0] - fp * self.n_base[:, 1], self.n_base[:, 1],
                      self.n_base[:, 2]], 1)
        n /= np.linalg.norm(n, axis=1, keepdims=True)
        return _f32(x), _f32(n)


# ---------------------------------------------------------------------------
# serving stream
# ---------------------------------------------------------------------------

@dataclass
class Request:
    index: int
    arrival_s: float
    n: int                       # cells per axis
    n_points: int
    want_grad: bool
    shape_seed: int

    def cloud(self):
        rng = np.random.default_rng([504, self.index])
        semi = rng.uniform(0.10, 0.30, 3)
        p = rng.uniform(2.0, 5.0)
        q, r = np.linalg.qr(rng.standard_normal((3, 3)))
        rot = q * np.sign(np.diag(r))
        if np.linalg.det(rot) < 0:
            rot[:, 0] = -rot[:, 0]
        coeffs = draw_star_coeffs(int(rng.integers(1, 2**31 - 1)))
        return star(coeffs, self.n_points, dir_seed=[507, self.index], semi_axes=semi, p=p,
                    rotation=rot)

    def queries(self, n_q=65_536):
        return uniform_queries(n_q, [506, self.index])


def request_stream(n_requests, rate_hz=50.0, sizes=(64, 128, 256), probs=(0.5, 0.3, 0.2),
                   grad_frac=0.3, seeds=(501, 502, 503, 505)):
    gaps = np.random.default_rng(seeds[0]).exponential(1.0 / rate_hz, n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    ns = np.random.default_rng(seeds[1]).choice(np.asarray(sizes), n_requests, p=probs)
    npts = np.random.default_rng(seeds[2]).lognormal(np.log(5e4), 1.0, n_requests)
    npts = np.clip(np.round(npts), 1e4, 2e6).astype(np.int64)
    grad = np.random.default_rng(seeds[3]).random(n_requests) < grad_frac
    return [Request(i, float(arrivals[i]), int(ns[i]), int(npts[i]), bool(grad[i]), i)
            for i in range(n_requests)]
