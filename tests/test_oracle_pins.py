"""Pins of two oracle functions that the collision and flow tests do not
reach on their own, each also checked against copies of the oracle with a
planted mistake.  CPU only.

* The third moment of the equilibrium, Eq. feq_moments (Sec. 2.6):
  sum_i e_ia e_ib e_ic f^eq_i = rho u_a u_b u_c + rho c_s^2 u_d Delta_abcd
  - Phi_abc / (3 c_s^2), with Phi_aaa = rho u_a^3 and zero otherwise (the
  definition after Eq. Gi, extended to z in 3D).  It is the only printed
  identity that reaches the third-order Hermite term of Eq. feq: the second
  moment, the channel flows (u_y = 0, no x dependence) and the spectra at
  rest do not.  D2Q9 and D3Q27 carry every component.  D3Q19 has no body
  diagonals, so sum_i w_i e_x^2 e_y^2 e_z^2 = 0 instead of c_s^6: there the
  aaa components hold as printed, and, written out from the D3Q19 weights,
  the aab components fall short by rho u_b u_c^2 / 2 (c the third axis)
  and the xyz component is 0.  In the plane u_z = 0 the printed form holds
  for the in-plane components (indices x and y).
* Mass and kinetic energy of the diagnostics.  At t = 0 the state is
  f = f^eq(rho0, u0) (equilibrium initialisation); Eq. macro then gives
  rho = rho0 and u = u0 + g/2, so M = sum over fluid nodes of rho0 and
  K = (1/2) sum over fluid nodes of rho0 |u0 + g/2|^2, a closed form of the
  initial fields (with a force and solid nodes present).

The planted mistakes (a wrong coefficient or sign of the third-order term,
the term dropped, one term of H^(3) dropped, the 1/2 of K dropped, solid
nodes counted, u without the half force) are compiled into copies of the
oracle's C source with oracle.build.build_variant; every one must turn a
pin red.
"""
import ctypes
import itertools

import numpy as np
import pytest

import lbm_inputs as I
from oracle import build as OB
from oracle import ptrt as O

CS2 = 1.0 / 3.0
LATS = [(O.D2Q9, 2), (O.D3Q19, 3), (O.D3Q27, 3)]


def _fields(n, D, seed, plane_axis=None):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.8, 1.2, n)
    u = np.zeros((n, 3))
    u[:, :D] = rng.uniform(-0.15, 0.15, (n, D))
    if plane_axis is not None:
        u[:, plane_axis] = 0.0
    return rho, u


def third_moment_error(lat, D, seed=11, plane_axis=None):
    """Largest deviation of the oracle's third equilibrium moments from
    Eq. feq_moments (with the D3Q19 lattice terms stated above) over every
    component and 64 random (rho, u)."""
    e, _, _ = O.lattice(lat)
    rho, u = _fields(64, D, seed, plane_axis)
    feq = O.equilibrium(lat, rho, u)
    worst = 0.0
    for a, b, c in itertools.combinations_with_replacement(range(D), 3):
        got = feq @ (e[:, a] * e[:, b] * e[:, c]).astype(float)
        want = rho * u[:, a] * u[:, b] * u[:, c] + rho * CS2 * (
            u[:, c] * (a == b) + u[:, b] * (a == c) + u[:, a] * (b == c))
        if a == b == c:
            want = want - rho * u[:, a] ** 3 / (3 * CS2)
        if lat == O.D3Q19 and len({a, b, c}) == 2:
            idx = (a, b, c)
            once = min(set(idx), key=idx.count)  # the axis that appears once
            third = ({0, 1, 2} - set(idx)).pop()
            want = want - 0.5 * rho * u[:, once] * u[:, third] ** 2
        if lat == O.D3Q19 and len({a, b, c}) == 3:
            want = np.zeros_like(rho)
        worst = max(worst, float(np.abs(got - want).max()))
    return worst


def energy_error(lat, shape, seed=5):
    """Relative deviation of the oracle's (mass, kinetic energy) at t = 0
    from the closed form, with a force and solid nodes."""
    nz, ny, nx = shape
    D = 2 if lat == O.D2Q9 else 3
    rng = np.random.default_rng(seed)
    rho, u = I.random_fields(rng, shape, umax=0.08)
    u = u[:D]
    solid = (rng.random(shape) < 0.15).astype(np.uint8)
    g = np.array([2e-2, -1.5e-2, 1e-2])[:D]
    L = O.Lattice(lat, nx, ny, nz, 0.8, 0.25, g=g, solid=solid)
    L.init_equilibrium(rho, u)
    m, k = L.diagnostics()
    fluid = solid == 0
    uh = u + 0.5 * g.reshape((D,) + (1,) * 3)
    m_ref = rho[fluid].sum()
    k_ref = 0.5 * (rho * (uh ** 2).sum(0))[fluid].sum()
    return max(abs(m / m_ref - 1), abs(k / k_ref - 1))


@pytest.mark.parametrize("lat,D", LATS)
def test_equilibrium_third_moment(lat, D):
    assert third_moment_error(lat, D) < 2e-15


def test_d3q19_third_moment_in_a_plane_is_as_printed():
    """In the plane u_z = 0 the printed identity holds on D3Q19 for the
    in-plane components with no lattice term (the moments they need are
    there)."""
    e, _, _ = O.lattice(O.D3Q19)
    rho, u = _fields(64, 3, 13, plane_axis=2)
    feq = O.equilibrium(O.D3Q19, rho, u)
    for a, b, c in itertools.combinations_with_replacement(range(2), 3):
        got = feq @ (e[:, a] * e[:, b] * e[:, c]).astype(float)
        want = rho * u[:, a] * u[:, b] * u[:, c] + rho * CS2 * (
            u[:, c] * (a == b) + u[:, b] * (a == c) + u[:, a] * (b == c))
        if a == b == c:
            want = want - rho * u[:, a] ** 3 / (3 * CS2)
        assert np.abs(got - want).max() < 2e-15, (a, b, c)


@pytest.mark.parametrize("lat,shape", [(O.D2Q9, (1, 13, 17)), (O.D3Q19, (6, 7, 9)),
                                       (O.D3Q27, (5, 6, 7))])
def test_mass_and_kinetic_energy_closed_form(lat, shape):
    assert energy_error(lat, shape) < 1e-13


# planted mistakes: (name, replacements, which pin must fail)
EQ_LINE = "t3 / (6.0 * cs6)"
MUTANTS = [
    ("third-order coefficient 1/2 instead of 1/6", [(EQ_LINE, "t3 / (2.0 * cs6)")], "moment"),
    ("third-order sign flipped", [("+ " + EQ_LINE, "- " + EQ_LINE)], "moment"),
    ("third-order term dropped", [("+ " + EQ_LINE, "")], "moment"),
    ("third-order over c_s^4", [(EQ_LINE, "t3 / (6.0 * cs4)")], "moment"),
    ("H3 without its last delta term",
     [("e[a] * kd(b, c) + e[b] * kd(c, a) + e[c] * kd(a, b)", "e[a] * kd(b, c) + e[b] * kd(c, a)")],
     "moment"),
    ("kinetic energy without 1/2", [("K += 0.5 * rho *", "K += rho *")], "energy"),
    ("solid nodes counted", [("        if (solid && solid[m]) continue;\n        double rho, u[3];",
                              "        double rho, u[3];")], "energy"),
    ("velocity without the half force", [("u[a] = (j[a] + 0.5 * r * g[a]) / r;",
                                          "u[a] = j[a] / r;")], "energy"),
]


@pytest.mark.parametrize("name,repl,pin", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistakes(name, repl, pin, tmp_path, monkeypatch):
    lib = OB.build_variant(repl, str(tmp_path))
    monkeypatch.setattr(O, "_lib", O.bind(ctypes.CDLL(lib)))
    if pin == "moment":
        worst = max(third_moment_error(lat, D) for lat, D in LATS)
        assert worst > 1e-6, name
    else:
        worst = max(energy_error(O.D2Q9, (1, 13, 17)), energy_error(O.D3Q19, (6, 7, 9)))
        assert worst > 1e-3, name


@pytest.mark.parametrize("lat,shape", [(O.D2Q9, (1, 11, 13)), (O.D3Q19, (6, 7, 9)),
                                       (O.D3Q27, (5, 5, 6))])
@pytest.mark.parametrize("nsteps", [1, 2, 4])
def test_sampled_steps_equal_whole_lattice_run(lat, shape, nsteps):
    """The sampled multi-step oracle (neighbourhoods collided level by
    level, for checks at sizes where no whole-lattice FP64 state fits)
    equals the whole-lattice oracle run exactly, also where the
    neighbourhood wraps around the periodic lattice."""
    nz, ny, nx = shape
    D = 2 if lat == O.D2Q9 else 3
    rng = np.random.default_rng(17 + nsteps)
    rho, u = I.random_fields(rng, shape, umax=0.05)
    u = u[:D]
    g = [1e-4, -2e-4, 3e-4][:D]
    L = O.Lattice(lat, nx, ny, nz, 0.7, 0.25, g=g)
    L.init_equilibrium(rho, u)
    L.step(nsteps)
    ref = L.populations().reshape(L.Q, -1).T
    nodes = rng.choice(nx * ny * nz, 25, replace=False)
    got = O.steps_from_fields_sampled(lat, rho, u, 0.7, 0.25, g, nodes, nsteps)
    assert np.array_equal(got, ref[nodes])
