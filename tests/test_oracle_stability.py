"""Stability of the double shear layer (Sec. 3.1) in the oracle.  CPU only.

The paper's criterion is that a run stays finite (it reports the runs that
reach t = 2 t_c without diverging).  Here the state is checked every 10
steps; the divergence step is the first checked step whose mass or kinetic
energy is not finite.  At the paper's resolution (128^2, kappa = 80,
delta = 0.05, U0 = 0.05) and Re = 1e4:

* with the configured Lambda = 1/4 (tau- = 130.7, so 1/tau- = 0.0077, far
  below the range of 1/tau- the paper tests) P-TRT diverges well before
  t_c = N / U0 = 2560 steps;
* at the paper's optimum 1/tau- = 1.6 the same flow stays finite for twice
  that divergence step, with mass conserved to round-off.

No step count is printed in the paper; the divergence step is a reported
result, bounded here so that a change in the oracle's arithmetic that moves
it shows up.
"""
import numpy as np

import lbm_inputs as I
from oracle import ptrt as O

N, U0, RE = 128, 0.05, 1e4


def dsl_lattice(inv_tau_minus=None):
    tp = I.tau_plus_from_nu(U0 * N / RE)
    lam = 0.25 if inv_tau_minus is None else I.tau_minus_from_inverse(inv_tau_minus, tp)
    rho, u = I.double_shear_layer(N, U0)
    L = O.Lattice(O.D2Q9, N, N, 1, tp, lam)
    L.init_equilibrium(rho, u[:2])
    return L


def divergence_step(L, limit, every=10):
    """First multiple of `every` (up to `limit`) at which the state is not
    finite, else None."""
    while L.t < limit:
        L.step(every)
        m, k = L.diagnostics()
        if not (np.isfinite(m) and np.isfinite(k)):
            return L.t
    return None


def test_dsl_diverges_at_lambda_quarter():
    step = divergence_step(dsl_lattice(), 2560)
    print(f"DSL 128^2 Re=1e4 Lambda=1/4: oracle diverges by step {step}", flush=True)
    assert step is not None and 1000 <= step <= 2500


def test_dsl_stays_finite_at_paper_optimum():
    L = dsl_lattice(1.6)
    m0, _ = L.diagnostics()
    assert divergence_step(L, 3500) is None
    m1, k1 = L.diagnostics()
    assert abs(m1 / m0 - 1) < 1e-12 and k1 > 0
