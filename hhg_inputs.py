"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the finite-element method itself: it only
produces macro meshes (vertex coordinates and triangles), random right-hand
side vectors and the random draws of a Gaussian random field.  Everything the
method computes from these inputs (refinement, numbering, stencils, solves) is
implemented separately by the oracle and by the HIP library.

Workloads (the paper shows its meshes only as figures, so these stand in):
  * unit square split into two macro-triangles (manufactured-solution case);
  * annulus r in [0.55, 1] with two radial layers of quads, each split into two
    triangles, vertex positions jittered by 5% from a seed (64 or 128 faces).
"""
import math

import numpy as np


def unit_square():
    """Unit square as two macro-triangles: (0,1,2) and (0,2,3)."""
    vxy = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    tri = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    return vxy, tri


def annulus(n_tan=16, n_rad=2, r_in=0.55, r_out=1.0, jitter=0.05, seed=0):
    """Jittered annulus macro mesh.

    Rings j = 0..n_rad at radii r_in + j*(r_out-r_in)/n_rad; vertex id
    j*n_tan + k sits at angle 2*pi*k/n_tan.  With generator default_rng(seed),
    drawn in vertex-id order: every vertex gets theta += jitter*dtheta*U(-1,1);
    vertices not on the two boundary rings then also get
    r += jitter*dr*U(-1,1).  Quad (ring j, sector k) with a=(j,k), b=(j,k+1),
    c=(j+1,k+1), d=(j+1,k) is split into (a,b,c) and (a,c,d).  These triangles
    are listed clockwise on purpose: a consumer must orient them.
    """
    rng = np.random.default_rng(seed)
    dth = 2.0 * math.pi / n_tan
    dr = (r_out - r_in) / n_rad
    vxy = np.zeros(((n_rad + 1) * n_tan, 2))
    for j in range(n_rad + 1):
        for k in range(n_tan):
            th = k * dth + jitter * dth * rng.uniform(-1.0, 1.0)
            r = r_in + j * dr
            if 0 < j < n_rad:
                r += jitter * dr * rng.uniform(-1.0, 1.0)
            vxy[j * n_tan + k] = (r * math.cos(th), r * math.sin(th))
    tri = []
    for j in range(n_rad):
        for k in range(n_tan):
            a = j * n_tan + k
            b = j * n_tan + (k + 1) % n_tan
            c = (j + 1) * n_tan + (k + 1) % n_tan
            d = (j + 1) * n_tan + k
            tri.append((a, b, c))
            tri.append((a, c, d))
    return vxy, np.array(tri, dtype=np.int32)


def mesh_by_name(name):
    """Named macro meshes of the workloads."""
    if name == "square":
        return unit_square()
    if name == "annulus64":
        return annulus(n_tan=16)
    if name == "annulus128":
        return annulus(n_tan=32)
    raise KeyError(name)


def face_viscosity(vxy, tri, r_jump=0.775, mu_in=1.0, mu_out=100.0):
    """Viscosity per macro-face with a radial jump: mu_in for faces whose
    centroid lies inside radius r_jump, mu_out outside (on the annulus: the
    inner and outer ring of quads, split along the jittered middle ring)."""
    c = np.asarray(vxy)[np.asarray(tri)].mean(axis=1)
    return np.where(np.hypot(c[:, 0], c[:, 1]) < r_jump, mu_in, mu_out)


def conductive_temperature(xy, r_in=0.55, r_out=1.0, t_in=1.0, t_out=0.0):
    """Initial temperature: the steady conductive profile between a hot inner
    wall (t_in at r_in) and a cold outer wall (t_out at r_out), linear in r."""
    r = np.hypot(np.asarray(xy)[:, 0], np.asarray(xy)[:, 1])
    return t_out + (t_in - t_out) * (r_out - r) / (r_out - r_in)


def uniform_rhs(n, seed):
    """n i.i.d. U[-1, 1] values from default_rng(seed), one per canonical point.

    Entries that land on Dirichlet points are ignored by the method."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def uniform_vector(n, seed, lo=-1.0, hi=1.0):
    """Generic seeded test vector."""
    return np.random.default_rng(seed).uniform(lo, hi, n)


def uniform_vector_device(n, seed, lo=-1.0, hi=1.0, device="cuda"):
    """n i.i.d. U[lo, hi] FP64 values drawn on the device by torch's seeded
    generator (for large training sets; reproducible on one device type)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    x = torch.rand(n, generator=gen, dtype=torch.float64, device=device)
    return lo + (hi - lo) * x


def grf_draws(seed, m=512, corr_len=0.1):
    """Random draws of a random-Fourier-feature Gaussian random field.

    Returns (omega[m,2], phi[m]) with omega ~ N(0, corr_len^-2 I) and
    phi ~ U[0, 2 pi), from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    omega = rng.normal(0.0, 1.0 / corr_len, size=(m, 2))
    phi = rng.uniform(0.0, 2.0 * math.pi, size=m)
    return omega, phi


def grf_eval(xy, seed, m=512, corr_len=0.1, sigma=1.0, chunk=1 << 16):
    """g(x) = sigma*sqrt(2/m)*sum_k cos(omega_k . x + phi_k) at points xy[N,2].

    Its covariance approximates sigma^2 exp(-|x-y|^2 / (2 corr_len^2))."""
    omega, phi = grf_draws(seed, m, corr_len)
    xy = np.asarray(xy, dtype=np.float64)
    out = np.empty(len(xy))
    scale = sigma * math.sqrt(2.0 / m)
    for s in range(0, len(xy), chunk):
        arg = xy[s:s + chunk] @ omega.T + phi
        out[s:s + chunk] = scale * np.cos(arg).sum(axis=1)
    return out


def grf_eval_device(xy, seed, m=512, corr_len=0.1, sigma=1.0, chunk=1 << 20, device="cuda"):
    """grf_eval on the GPU (torch, FP64) for large point sets: the same draws
    and formula, summed in another order (differences at rounding level)."""
    import torch
    omega, phi = grf_draws(seed, m, corr_len)
    om = torch.tensor(omega.T.copy(), dtype=torch.float64, device=device)
    ph = torch.tensor(phi, dtype=torch.float64, device=device)
    xy = torch.as_tensor(xy, dtype=torch.float64).to(device)
    out = torch.empty(len(xy), dtype=torch.float64, device=device)
    scale = sigma * math.sqrt(2.0 / m)
    for s in range(0, len(xy), chunk):
        arg = xy[s:s + chunk] @ om + ph
        out[s:s + chunk] = scale * torch.cos(arg).sum(dim=1)
    return out


def manufactured_u(xy):
    """u(x, y) = sin(pi x) sin(pi y)."""
    xy = np.asarray(xy)
    return np.sin(math.pi * xy[:, 0]) * np.sin(math.pi * xy[:, 1])


def manufactured_f(xy):
    """f = -Laplace(u) = 2 pi^2 sin(pi x) sin(pi y)."""
    return 2.0 * math.pi ** 2 * manufactured_u(xy)
