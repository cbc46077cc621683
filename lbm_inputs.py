"""Seeded synthetic inputs for the P-TRT workloads.

This module is shared by the tests, the benchmark and the smoke check.  It
only builds initial fields, masks and parameter sets; it holds none of the
lattice Boltzmann arithmetic, so the oracle and the GPU path stay
independent of each other.

The flows are the benchmark shapes of arXiv 2602.06686, Sec. 3: the double
shear layer (Sec. 3.1), the decaying Taylor-Green vortex (Sec. 3.2, Eq. TG),
the force-driven channel (Sec. 3.3) and a square obstacle (Sec. 3.4), plus
the three-dimensional Taylor-Green vortex used for the D3Q19 lattice.
All quantities are in lattice units (dx = dt = 1, c_s^2 = 1/3).
"""
import math

import numpy as np

BATCH_SEED = 260206686


def tau_plus_from_nu(nu):
    """Symmetric relaxation time for kinematic viscosity nu, Eq. viscosity."""
    return 0.5 + 3.0 * nu


def tau_minus_from_inverse(inv_tau_minus, tau_plus):
    """Lambda that yields a given 1/tau_minus for this tau_plus (Sec. 3.1 uses
    fixed 1/tau_minus values; the library takes Lambda)."""
    return (tau_plus - 0.5) * (1.0 / inv_tau_minus - 0.5)


# ---------------------------------------------------------------- 2D flows

def tgv2d(n, u0):
    """2D Taylor-Green vortex, Eq. TG at t = 0 on an n x n periodic lattice,
    node coordinates x_i = i, wavenumber k = 2 pi / n.
    Returns rho [1,n,n] and u [2,1,n,n] (component-major)."""
    k = 2 * np.pi / n
    y, x = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64),
                       indexing="ij")
    ux = -u0 * np.cos(k * x) * np.sin(k * y)
    uy = u0 * np.cos(k * y) * np.sin(k * x)
    rho = 1.0 - 3.0 * u0 * u0 / 4.0 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    return rho[None], np.stack([ux, uy])[:, None]


def double_shear_layer(n, U0, kappa=80.0, delta=0.05):
    """Double shear layer of Sec. 3.1 on an n x n periodic lattice with
    x = i/n, y = j/n.  Returns rho [1,n,n] (uniform 1) and u [2,1,n,n]."""
    y, x = np.meshgrid(np.arange(n, dtype=np.float64) / n, np.arange(n, dtype=np.float64) / n,
                       indexing="ij")
    ux = np.where(y <= 0.5, U0 * np.tanh(kappa * (y - 0.25)), U0 * np.tanh(kappa * (0.75 - y)))
    uy = U0 * delta * np.sin(2 * np.pi * (x + 0.25))
    return np.ones((1, n, n)), np.stack([ux, uy])[:, None]


def channel_mask(nx, ny):
    """Solid rows y = 0 and y = ny-1 (walls halfway to the fluid), uint8 [1,ny,nx]."""
    m = np.zeros((1, ny, nx), dtype=np.uint8)
    m[0, 0, :] = 1
    m[0, ny - 1, :] = 1
    return m


def square_obstacle_mask(nx, ny, side=None):
    """Centred solid square of side floor(min(nx, ny)/8) (at least 1), uint8 [1,ny,nx]."""
    D = max(1, min(nx, ny) // 8) if side is None else side
    m = np.zeros((1, ny, nx), dtype=np.uint8)
    x0 = (nx - D) // 2
    y0 = (ny - D) // 2
    m[0, y0:y0 + D, x0:x0 + D] = 1
    return m


# ---------------------------------------------------------------- 3D flows

def tgv3d(n, U0, nz=None, ny=None):
    """3D Taylor-Green vortex on a periodic n^3 box with x = 2 pi i / n:
    u = U0 sin x cos y cos z, v = -U0 cos x sin y cos z, w = 0 and
    rho = 1 + 3 (U0^2/16)(cos 2x + cos 2y)(cos 2z + 2).
    Returns rho [nz,ny,nx] and u [3,nz,ny,nx]."""
    nx = n
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    z, y, x = np.meshgrid(2 * np.pi * np.arange(nz) / nz, 2 * np.pi * np.arange(ny) / ny,
                          2 * np.pi * np.arange(nx) / nx, indexing="ij")
    u = U0 * np.sin(x) * np.cos(y) * np.cos(z)
    v = -U0 * np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(u)
    rho = 1.0 + 3.0 * (U0 * U0 / 16.0) * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
    return rho, np.stack([u, v, w])


def tgv3d_nu(n, U0=0.05, Re=1600.0):
    """Viscosity for the 3D Taylor-Green vortex, Re = U0 L / nu with L = n / (2 pi)."""
    return U0 * (n / (2 * np.pi)) / Re


def tgv3d_params(n, U0=0.05, Re=1600.0):
    nu = tgv3d_nu(n, U0, Re)
    return {"nu": nu, "tau_plus": tau_plus_from_nu(nu)}


# ------------------------------------------------------- random node states

def random_states(rng, w, n, amplitude=0.05):
    """n random population vectors near a rest state: f_i = w_i rho (1 + a r_i),
    rho in [0.9, 1.1], r_i uniform in [-1, 1].  Returns [n, Q]."""
    w = np.asarray(w, dtype=np.float64)
    rho = rng.uniform(0.9, 1.1, size=(n, 1))
    r = rng.uniform(-1.0, 1.0, size=(n, w.size))
    return w[None] * rho * (1.0 + amplitude * r)


def random_fields(rng, shape, umax=0.05):
    """Smooth-free random density [shape] near 1 and velocity [3, shape]."""
    rho = 1.0 + 0.02 * rng.uniform(-1, 1, size=shape)
    u = umax * rng.uniform(-1, 1, size=(3,) + tuple(shape))
    return rho, u


# ---------------------------------------------------------- batched lattices

def batch_specs(count=512, seed=BATCH_SEED, size_range=(32, 512)):
    """Independent D2Q9 lattices for the batched form.

    nx, ny uniform in [32, 512].  First half: force-driven channels (Sec. 3.3
    shape) with walls at y = 0 and y = ny-1, Lambda = 3/16, g_x log-uniform in
    [1e-7, 1e-5].  Second half: a periodic box around a centred solid square
    of side max(1, min(nx,ny)//8), Lambda = 3/16, nominal Reynolds number
    Re in [0.1, 1] based on the side length, driven by the body force that a
    Stokes drag coefficient of about 8.25 (Sec. 3.4) would balance.
    tau_plus uniform in [0.55, 2.0].  The channel centreline velocity
    g (ny-2)^2 / (8 nu) is capped at 0.1 by lowering g where needed.
    """
    rng = np.random.default_rng(seed)
    lo, hi = size_range
    specs = []
    half = count // 2
    for k in range(count):
        nx = int(rng.integers(lo, hi + 1))
        ny = int(rng.integers(lo, hi + 1))
        tau_plus = float(rng.uniform(0.55, 2.0))
        nu = (tau_plus - 0.5) / 3.0
        if k < half:
            gx = float(math.exp(rng.uniform(math.log(1e-7), math.log(1e-5))))
            N = ny - 2
            gx = min(gx, 0.1 * 8.0 * nu / (N * N))
            kind = "channel"
            mask = channel_mask(nx, ny)
        else:
            D = max(1, min(nx, ny) // 8)
            Re = float(rng.uniform(0.1, 1.0))
            U = Re * nu / D
            gx = 4.125 * U * nu / (nx * ny)
            kind = "obstacle"
            mask = square_obstacle_mask(nx, ny)
        specs.append({"kind": kind, "nx": nx, "ny": ny, "tau_plus": tau_plus,
                      "Lambda": 3.0 / 16.0, "g": (gx, 0.0, 0.0), "mask": mask})
    return specs
