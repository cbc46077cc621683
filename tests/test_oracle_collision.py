"""Pins of the oracle's collision (Eq. PTRT) on independent node states.

* Theorems 2 and 3 / Remark on exactness: the P-TRT oracle (C) and the
  independently written TRT-RLB (NumPy, Hermite projection) give the same
  post-collision state on D2Q9 and D3Q19.
* Invariants: mass conserved, momentum gains exactly F, the post-collision
  non-equilibrium part has no ghost content (Theorem on ghost-mode
  annihilation).
* Eq. collision_PTRT / collision_TRT: spectrum of the linearised collision
  at rest, against a textbook TRT written out in this file.
* Special cases: tau+ = 1 reduces P-TRT to standard TRT; tau+ = tau- = 1 to
  the equilibrium; an equilibrium input without force is a fixed point.
CPU only.
"""
import numpy as np
import pytest

import lbm_inputs as I
from conftest import golden
from oracle import ptrt as O
from oracle import trt_rlb as R

LATS = [(O.D2Q9, "D2Q9", 2), (O.D3Q19, "D3Q19", 3)]
CS2 = 1.0 / 3.0


def _states(lat, n, seed, amp=0.05):
    _, w, _ = O.lattice(lat)
    return I.random_states(np.random.default_rng(seed), w, n, amp)


@pytest.mark.parametrize("lat,name,D", LATS)
@pytest.mark.parametrize("tau_plus,tau_minus", [(0.51, 1 / 1.6), (0.73, 1.9), (1.0, 3.0),
                                                (3.7, 0.55), (11503.0, 0.5 + 1e-3)])
@pytest.mark.parametrize("force", [False, True])
def test_ptrt_equals_trt_rlb(lat, name, D, tau_plus, tau_minus, force):
    f = _states(lat, 300, seed=int(tau_plus * 100) + D, amp=0.1)
    g = np.array([2e-3, -1e-3, 7e-4]) if force else np.zeros(3)
    a = O.collide(lat, f, g, tau_plus, tau_minus=tau_minus)
    b = R.collide(name, f, g[:D], tau_plus, tau_minus)
    # compare the deviation from the input, which carries all the physics
    scale = np.abs(b - f).max()
    assert np.abs(a - b).max() <= 1e-14 * max(scale, np.abs(f).max())


def test_d2q9_literal_third_order_is_the_projection():
    """On D2Q9 the printed tensor reconstruction is the orthogonal projection."""
    e, w = R.lattice("D2Q9")
    fneq = np.random.default_rng(3).normal(size=(50, 9))
    a = R.reconstruct_third_literal(e, w, fneq)
    b = R.reconstruct_third_projection(e, w, fneq)
    assert np.abs(a - b).max() < 1e-14 * np.abs(b).max()


def test_d3q19_literal_third_order_differs():
    """On D3Q19 the printed tensor contraction is not a projection (reading
    of the NumPy TRT-RLB): applying it twice does not give the same result."""
    e, w = R.lattice("D3Q19")
    fneq = np.random.default_rng(4).normal(size=(20, 19))
    once = R.reconstruct_third_literal(e, w, fneq)
    twice = R.reconstruct_third_literal(e, w, once)
    assert np.abs(once - twice).max() > 1e-3 * np.abs(once).max()
    p1 = R.reconstruct_third_projection(e, w, fneq)
    p2 = R.reconstruct_third_projection(e, w, p1)
    assert np.abs(p1 - p2).max() < 1e-14 * np.abs(p1).max()


@pytest.mark.parametrize("lat,name,D", LATS)
def test_conservation(lat, name, D):
    e, w, _ = O.lattice(lat)
    f = _states(lat, 500, seed=11 + D, amp=0.2)
    g = np.array([1e-3, 2e-3, -3e-3])
    g[D:] = 0
    fs = O.collide(lat, f, g, 0.61, Lambda=0.25)
    rho = f.sum(1)
    assert np.abs(fs.sum(1) - rho).max() < 4e-16 * 4
    F = rho[:, None] * g[None]
    assert np.abs(fs @ e - (f @ e + F)).max() < 1e-15 * 4


@pytest.mark.parametrize("lat,name,D", LATS)
def test_ghost_annihilation(lat, name, D):
    """The post-collision non-equilibrium part f* - f^eq(rho, u) carries no
    ghost content, for any tau+, tau- and force."""
    e, w, _ = O.lattice(lat)
    phi, _ = O.ghost_basis(lat)
    f = _states(lat, 400, seed=21 + D, amp=0.2)
    g = np.array([1e-3, -2e-3, 5e-4])
    g[D:] = 0
    for tp, tm in ((0.52, 7.0), (1.3, 0.8)):
        fs = O.collide(lat, f, g, tp, tau_minus=tm)
        rho, u = O.node_moments(lat, f, g)
        feq = O.equilibrium(lat, rho, u)
        ghost = (fs - feq) @ phi.T
        assert np.abs(ghost).max() < 1e-16 * 8
        # the same quantity before collision is not zero
        assert np.abs((f - feq) @ phi.T).max() > 1e-4


def _textbook_trt(e, w, opp, f, tau_plus, tau_minus):
    """Standard TRT without force: f* = f^eq + (1-1/tau+) f^{neq,+} + (1-1/tau-) f^{neq,-},
    with the second-order equilibrium, here only linearised at rest."""
    rho = f.sum(1)
    j = f @ e
    feq = w[None] * (rho[:, None] + (j @ e.T) / CS2)  # linear in the perturbation
    fneq = f - feq
    plus = 0.5 * (fneq + fneq[:, opp])
    minus = 0.5 * (fneq - fneq[:, opp])
    return feq + (1 - 1 / tau_plus) * plus + (1 - 1 / tau_minus) * minus


def _jacobian(fun, x0, h=1e-6):
    Q = x0.size
    J = np.zeros((Q, Q))
    for k in range(Q):
        d = np.zeros(Q)
        d[k] = h
        J[:, k] = (fun(x0 + d) - fun(x0 - d)) / (2 * h)
    return J


def _count(vals, target, tol=1e-7):
    return int(np.sum(np.abs(vals - target) < tol))


@pytest.mark.parametrize("lat,name,D", LATS)
def test_linearised_spectrum(lat, name, D):
    """Eq. collision_PTRT: eigenvalues of the collision linearised at rest are
    1 (conserved), 1-1/tau+ (stress), 1-1/tau- (third order), 0 (ghost); for
    standard TRT the ghost entry is 1-1/tau+ (Eq. collision_TRT)."""
    spec = golden("collision_spectrum.json")[name]
    e, w, opp = O.lattice(lat)
    tp, tm = 0.8, 2.5
    ap, am = 1 - 1 / tp, 1 - 1 / tm
    J = _jacobian(lambda x: O.collide(lat, x[None], None, tp, tau_minus=tm)[0], w.copy())
    ev = np.sort(np.linalg.eigvals(J).real)
    assert _count(ev, 1.0) == spec["one"]
    assert _count(ev, ap) == spec["a_plus"]
    assert _count(ev, am) == spec["a_minus"]
    assert _count(ev, 0.0) == spec["ghost"]
    Jt = _jacobian(lambda x: _textbook_trt(e.astype(float), w, opp, x[None], tp, tm)[0], w.copy())
    evt = np.sort(np.linalg.eigvals(Jt).real)
    assert _count(evt, ap) == spec["a_plus"] + spec["ghost"]
    assert _count(evt, 0.0) == 0


@pytest.mark.parametrize("lat,name,D", LATS)
def test_tau_plus_one_is_standard_trt(lat, name, D):
    """With tau+ = 1 the symmetric non-equilibrium part is discarded both by
    P-TRT and by standard TRT, so the two coincide (no force)."""
    e, w, opp = O.lattice(lat)
    f = _states(lat, 200, seed=31 + D, amp=0.1)
    tm = 1.7
    a = O.collide(lat, f, None, 1.0, tau_minus=tm)
    rho, u = O.node_moments(lat, f)
    feq = R.equilibrium(*R.lattice(name), rho, u[:, :D])
    fneq = f - feq
    b = feq + (1 - 1 / tm) * 0.5 * (fneq - fneq[:, opp])
    assert np.abs(a - b).max() < 1e-16 * 8


@pytest.mark.parametrize("lat,name,D", LATS)
def test_unit_relaxation_gives_equilibrium(lat, name, D):
    f = _states(lat, 100, seed=41 + D)
    a = O.collide(lat, f, None, 1.0, tau_minus=1.0)
    rho, u = O.node_moments(lat, f)
    assert np.abs(a - O.equilibrium(lat, rho, u)).max() < 1e-16 * 8


@pytest.mark.parametrize("lat,name,D", LATS)
def test_equilibrium_is_fixed_point(lat, name, D):
    rng = np.random.default_rng(51 + D)
    rho = rng.uniform(0.9, 1.1, 64)
    u = rng.uniform(-0.1, 0.1, (64, 3))
    u[:, D:] = 0
    feq = O.equilibrium(lat, rho, u)
    fs = O.collide(lat, feq, None, 0.57, Lambda=0.25)
    assert np.abs(fs - feq).max() < 1e-16 * 8


@pytest.mark.parametrize("lat,name,D", LATS)
def test_equilibrium_moments(lat, name, D):
    """Eq. feq_moments: sum f^eq = rho, sum e f^eq = rho u,
    sum e_a e_b f^eq = rho u_a u_b + rho c_s^2 d_ab."""
    e, w, _ = O.lattice(lat)
    rng = np.random.default_rng(61 + D)
    rho = rng.uniform(0.9, 1.1, 32)
    u = rng.uniform(-0.1, 0.1, (32, 3))
    u[:, D:] = 0
    feq = O.equilibrium(lat, rho, u)
    assert np.abs(feq.sum(1) - rho).max() < 1e-15
    assert np.abs(feq @ e - rho[:, None] * u).max() < 1e-15
    for a in range(D):
        for b in range(D):
            m2 = feq @ (e[:, a] * e[:, b])
            assert np.abs(m2 - rho * (u[:, a] * u[:, b] + CS2 * (a == b))).max() < 1e-15


def test_d2q9_ghost_moment_formula():
    """App. A.1: S_G = c_s^4 [f_0 - 2 sum_{1..4} f_j + 4 sum_{5..8} f_j]."""
    phi, _ = O.ghost_basis(O.D2Q9)
    x = np.random.default_rng(7).normal(size=(10, 9))
    sg = (x[:, 0] - 2 * x[:, 1:5].sum(1) + 4 * x[:, 5:9].sum(1)) / 9.0
    assert np.abs(x @ phi[0] - sg).max() < 1e-15


def test_force_terms_reading_matches_trt_rlb_not_literal():
    """Reading R1: with the printed source of Eq. PTRT (Scheme II added on
    top of the tau- force correction) the momentum gain per step would be
    F (3/2 - 1/(2 tau+)); the oracle's net source gives exactly F, which is
    also what TRT-RLB with tau+ on the first-order moment gives."""
    e, w, _ = O.lattice(O.D2Q9)
    f = _states(O.D2Q9, 50, seed=71)
    g = np.array([1e-3, 0.0, 0.0])
    tp = 0.9
    fs = O.collide(O.D2Q9, f, g, tp, Lambda=3 / 16)
    F = f.sum(1) * g[0]
    gain = (fs @ e)[:, 0] - (f @ e)[:, 0]
    assert np.abs(gain - F).max() < 1e-16 * 4
    literal_gain = F * (1.5 - 1 / (2 * tp))
    assert np.abs(gain - literal_gain).min() > 1e-5


@pytest.mark.parametrize("lat,name,D", LATS)
def test_oracle_trt_spectrum_and_ptrt_difference(lat, name, D):
    """The oracle's standard-TRT comparison model: its linearised collision has
    the ghost eigenvalue 1 - 1/tau+ (Eq. collision_TRT), it differs from
    P-TRT exactly by the ghost projection relaxed with tau+, and it coincides
    with P-TRT at tau+ = 1."""
    spec = golden("collision_spectrum.json")[name]
    e, w, opp = O.lattice(lat)
    phi, nrm = O.ghost_basis(lat)
    tp, tm = 0.8, 2.5
    J = _jacobian(lambda x: O.collide_trt(lat, x[None], None, tp, tm)[0], w.copy())
    ev = np.sort(np.linalg.eigvals(J).real)
    assert _count(ev, 1 - 1 / tp) == spec["a_plus"] + spec["ghost"]
    assert _count(ev, 0.0) == 0
    f = _states(lat, 100, seed=81 + D, amp=0.1)
    g = np.array([1e-3, -5e-4, 2e-4])
    g[D:] = 0
    a = O.collide(lat, f, g, tp, tau_minus=tm)
    b = O.collide_trt(lat, f, g, tp, tm)
    rho, u = O.node_moments(lat, f, g)
    fneq = f - O.equilibrium(lat, rho, u)
    pg = sum(w[None] * phi[k][None] / nrm[k] * (fneq @ phi[k])[:, None] for k in range(len(nrm)))
    assert np.abs((b - a) - (1 - 1 / tp) * pg).max() < 1e-15
    assert np.abs(O.collide_trt(lat, f, g, 1.0, tm) - O.collide(lat, f, g, 1.0, tau_minus=tm)).max() < 1e-15
