"""Closed-form solutions used to pin the oracle.  Test infrastructure.

* Relative L2 norm, Sec. 3 (the norm defined before Sec. 3.1).
* 2D decaying Taylor-Green vortex, Eq. TG.  The velocity decays as
  exp(-t/t_d) with t_d = 1/(8 nu pi^2) on the unit square, i.e.
  exp(-2 nu k^2 t) for wavenumber k per axis; the kinetic energy decays at
  twice that rate.
* Force-driven Poiseuille flow with halfway bounce-back, Sec. 3.3: the
  discrete profile u(y_i) = 4 u_c y_i (N - y_i) / N^2, y_i = i - 1/2,
  with centreline velocity u_c = g N^2 / (8 nu).
"""
import numpy as np


def rel_l2(numeric, exact):
    numeric = np.asarray(numeric, dtype=np.float64)
    exact = np.asarray(exact, dtype=np.float64)
    return float(np.sqrt(((numeric - exact) ** 2).sum() / (exact ** 2).sum()))


def tgv2d_velocity(n, u0, nu, t, x=None, y=None):
    """Eq. TG on an n x n periodic lattice with node coordinates x_i = i:
    wavenumber k = 2 pi / n; returns (ux, uy) of shape [n, n] ([y, x])."""
    k = 2 * np.pi / n
    if x is None:
        y, x = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64),
                           indexing="ij")
    decay = np.exp(-2 * nu * k * k * t)
    ux = -u0 * np.cos(k * x) * np.sin(k * y) * decay
    uy = u0 * np.cos(k * y) * np.sin(k * x) * decay
    return ux, uy


def tgv2d_energy_rate(n, nu):
    """d ln E / dt of the 2D Taylor-Green vortex: -4 nu k^2 (two axes, k = 2 pi/n)."""
    k = 2 * np.pi / n
    return -2.0 * nu * (2 * k * k)


def poiseuille_profile(N, u_c):
    """Discrete halfway-bounce-back profile on N fluid rows, y_i = i - 1/2."""
    yi = np.arange(1, N + 1, dtype=np.float64) - 0.5
    return 4.0 * u_c * yi * (N - yi) / (N * N)


def poiseuille_acceleration(N, u_c, nu):
    """g with u_c = g N^2 / (8 nu)."""
    return 8.0 * nu * u_c / (N * N)
