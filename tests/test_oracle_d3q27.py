"""Pins of the oracle's D3Q27 path (App. A.3, Eq. PTRT_D3Q27), CPU only.

* Lattice: composition 1 + 6 + 12 + 8, weights fixed by the moment
  conditions up to sixth order (exact rationals).
* Modes: the seven printed ghost modes and the three fifth-order modes in
  exact rationals: mutually orthogonal, orthogonal to the hydrodynamic and
  third-order modes; the oracle's basis equals the printed one.  Reading R14:
  psi^(5,x) is not zero off the body diagonals.
* Collision: the hybrid R2 (tensor projection) equals the ghost subtraction
  of Eq. PTRT (Theorem 2); the exact variant equals TRT-RLB (NumPy);
  hybrid - exact = (1 - 1/tau-) P5 f^neq; invariants; linearised spectrum.
* Flows: exact variant vs TRT-RLB over 30 steps with walls and force;
  force-driven Poiseuille flow exact at Lambda = 3/16 (Sec. 3.3 setup on a
  two-layer periodic slab).
"""
from fractions import Fraction as Fr
import itertools

import numpy as np
import pytest

import lbm_inputs as I
from conftest import golden
from oracle import analytic as A
from oracle import ptrt as O
from oracle import trt_rlb as R

CS2 = Fr(1, 3)
LAT = O.D3Q27


def _exact_lattice():
    e, _, _ = O.lattice(LAT)
    ev = [tuple(int(c) for c in v) for v in e]
    w1 = {0: Fr(2, 3), 1: Fr(1, 6)}
    w = [w1[abs(a)] * w1[abs(b)] * w1[abs(c)] for a, b, c in ev]
    return ev, w


def _dot(w, p, q):
    return sum(wi * pi * qi for wi, pi, qi in zip(w, p, q))


def _printed_ghosts(ev):
    def h(v, a):
        return v[a] * v[a] - CS2
    return [[h(v, 0) * h(v, 1) for v in ev],
            [h(v, 1) * h(v, 2) for v in ev],
            [h(v, 2) * h(v, 0) for v in ev],
            [h(v, 0) * h(v, 1) * h(v, 2) / CS2 for v in ev],
            [v[0] * v[1] * h(v, 2) for v in ev],
            [v[1] * v[2] * h(v, 0) for v in ev],
            [v[2] * v[0] * h(v, 1) for v in ev]]


def _printed_fifth(ev):
    def h(v, a):
        return v[a] * v[a] - CS2
    return [[v[k] * h(v, (k + 1) % 3) * h(v, (k + 2) % 3) for v in ev] for k in range(3)]


def _hydro_and_third(ev):
    rows = [[Fr(1)] * len(ev)]
    rows += [[Fr(v[a]) for v in ev] for a in range(3)]
    for a in range(3):
        for b in range(a, 3):
            rows.append([v[a] * v[b] - CS2 * (a == b) for v in ev])
    for a, b in itertools.permutations(range(3), 2):
        rows.append([v[b] * (v[a] * v[a] - CS2) for v in ev])
    rows.append([Fr(v[0] * v[1] * v[2]) for v in ev])
    return rows


def test_composition_and_weights():
    """App. A.3: 1 rest, 6 axial, 12 face and 8 body diagonals; the weights
    satisfy sum w = 1, sum w e_a e_b = c_s^2 d_ab and the tensor-product
    moments up to sixth order (sum w e_x^2 e_y^2 e_z^2 = c_s^6)."""
    ev, w = _exact_lattice()
    e, wf, opp = O.lattice(LAT)
    n2 = sorted(np.bincount((e ** 2).sum(1)).tolist())
    assert n2 == sorted([1, 6, 12, 8])
    assert (e[opp] == -e).all()
    assert np.abs(wf - np.array([float(x) for x in w])).max() < 1e-17
    assert sum(w) == 1
    for a, b in itertools.product(range(3), repeat=2):
        assert sum(wi * v[a] * v[b] for wi, v in zip(w, ev)) == CS2 * (a == b)
        m4 = sum(wi * v[a] ** 2 * v[b] ** 2 for wi, v in zip(w, ev))
        assert m4 == (3 * CS2 ** 2 if a == b else CS2 ** 2)
    assert sum(wi * (v[0] * v[1] * v[2]) ** 2 for wi, v in zip(w, ev)) == CS2 ** 3
    # the first nineteen velocities are the D3Q19 set in its order
    e19, _, _ = O.lattice(O.D3Q19)
    assert (e[:19] == e19).all()


def test_printed_ghost_modes_are_orthogonal_and_oracle_keeps_them():
    """The seven ghost modes of App. A.3, exact rationals: orthogonal to the
    mass and stress modes and to each other, so the oracle's Gram-Schmidt
    leaves them as printed."""
    ev, w = _exact_lattice()
    gh = _printed_ghosts(ev)
    hyd = _hydro_and_third(ev)[:1] + _hydro_and_third(ev)[4:10]
    for k, p in enumerate(gh):
        for h in hyd:
            assert _dot(w, p, h) == 0
        for m, q in enumerate(gh):
            if m != k:
                assert _dot(w, p, q) == 0
    phi, nrm = O.ghost_basis(LAT)
    assert phi.shape == (7, 27)
    for k in range(7):
        ref = np.array([float(x) for x in gh[k]])
        assert np.abs(phi[k] - ref).max() < 1e-15
        assert abs(nrm[k] - float(_dot(w, gh[k], gh[k]))) < 1e-16


def test_fifth_order_modes_and_reading_r14():
    """The three fifth-order modes span the antisymmetric deficit: orthogonal
    to H1, the seven third-order modes and each other, norm 4/243.  They are
    not zero off the body diagonals (reading R14): psi^(5,x) = 1/9 at
    (1,0,0) and -2/9 at (1,1,0)."""
    ev, w = _exact_lattice()
    psi = _printed_fifth(ev)
    rows = _hydro_and_third(ev)
    odd = rows[1:4] + rows[10:]
    assert len(odd) == 3 + 7
    for k in range(3):
        for r in odd:
            assert _dot(w, psi[k], r) == 0
        for m in range(3):
            assert _dot(w, psi[k], psi[m]) == (Fr(4, 243) if k == m else 0)
    i100 = ev.index((1, 0, 0))
    i110 = ev.index((1, 1, 0))
    assert psi[0][i100] == Fr(1, 9) and psi[0][i110] == Fr(-2, 9)
    got = O.fifth_modes(LAT)
    assert np.abs(got - np.array([[float(x) for x in r] for r in psi])).max() < 4e-16


def _states(n, seed, amp=0.1):
    _, w, _ = O.lattice(LAT)
    return I.random_states(np.random.default_rng(seed), w, n, amp)


def _p5(f, g):
    _, w, _ = O.lattice(LAT)
    psi = O.fifth_modes(LAT)
    rho, u = O.node_moments(LAT, f, g)
    fneq = f - O.equilibrium(LAT, rho, u)
    return sum(w[None] * psi[k][None] / (w * psi[k] ** 2).sum() * (fneq @ psi[k])[:, None]
               for k in range(3))


@pytest.mark.parametrize("tau_plus,tau_minus", [(0.51, 1 / 1.6), (0.73, 1.9), (1.0, 3.0),
                                                (3.7, 0.55), (11503.0, 0.5 + 1e-3)])
@pytest.mark.parametrize("force", [False, True])
def test_hybrid_exact_and_trt_rlb(tau_plus, tau_minus, force):
    f = _states(300, seed=int(tau_plus * 100) + 27)
    g = np.array([2e-3, -1e-3, 7e-4]) if force else np.zeros(3)
    hyb = O.collide_model(LAT, O.PTRT, f, g, tau_plus, tau_minus)
    exact = O.collide_model(LAT, O.PTRT_EXACT, f, g, tau_plus, tau_minus)
    ghost = O.collide_model(LAT, O.PTRT_GHOST, f, g, tau_plus, tau_minus)
    rlb = R.collide("D3Q27", f, g, tau_plus, tau_minus)
    scale = max(np.abs(rlb - f).max(), np.abs(f).max())
    # exact variant == TRT-RLB (App. A.3 with the fifth-order projection removed)
    assert np.abs(exact - rlb).max() <= 2e-14 * scale
    # tensor-projection R2 == ghost subtraction (Theorem 2 on D3Q27)
    assert np.abs(hyb - ghost).max() <= 2e-14 * scale
    # the hybrid keeps the fifth-order part, relaxed with tau-
    d = hyb - exact
    assert np.abs(d - (1 - 1 / tau_minus) * _p5(f, g)).max() <= 1e-15 * scale
    if abs(1 - 1 / tau_minus) > 0.1:
        assert np.abs(d).max() > 1e-4 * scale
    # oracle P-TRT entry point is the hybrid
    assert np.array_equal(O.collide(LAT, f, g, tau_plus, tau_minus=tau_minus), hyb)


def test_d3q27_literal_third_order_is_the_projection():
    e, w = R.lattice("D3Q27")
    fneq = np.random.default_rng(5).normal(size=(40, 27))
    a = R.reconstruct_third_literal(e, w, fneq)
    b = R.reconstruct_third_projection(e, w, fneq)
    assert R.third_order_modes(e).shape[0] == 7
    assert np.abs(a - b).max() < 1e-14 * np.abs(b).max()


@pytest.mark.parametrize("model", [O.PTRT, O.PTRT_EXACT, O.TRT])
def test_conservation_and_fixed_point(model):
    e, w, _ = O.lattice(LAT)
    f = _states(400, seed=91, amp=0.2)
    g = np.array([1e-3, 2e-3, -3e-3])
    fs = O.collide_model(LAT, model, f, g, 0.61, 0.5 + 0.25 / 0.11)
    rho = f.sum(1)
    assert np.abs(fs.sum(1) - rho).max() < 1e-15 * 4
    assert np.abs(fs @ e - (f @ e + rho[:, None] * g[None])).max() < 1e-15 * 4
    rng = np.random.default_rng(92)
    r = rng.uniform(0.9, 1.1, 64)
    u = rng.uniform(-0.1, 0.1, (64, 3))
    feq = O.equilibrium(LAT, r, u)
    assert np.abs(O.collide_model(LAT, model, feq, None, 0.57, 1.3) - feq).max() < 1e-16 * 8
    # equilibrium moments (Eq. feq_moments)
    assert np.abs(feq.sum(1) - r).max() < 1e-15
    assert np.abs(feq @ e - r[:, None] * u).max() < 1e-15
    # unit relaxation gives the equilibrium
    rho1, u1 = O.node_moments(LAT, f)
    one = O.collide_model(LAT, model, f, None, 1.0, 1.0)
    assert np.abs(one - O.equilibrium(LAT, rho1, u1)).max() < 1e-16 * 8


def test_ghost_annihilation():
    phi, _ = O.ghost_basis(LAT)
    f = _states(300, seed=93, amp=0.2)
    g = np.array([1e-3, -2e-3, 5e-4])
    for model in (O.PTRT, O.PTRT_EXACT):
        for tp, tm in ((0.52, 7.0), (1.3, 0.8)):
            fs = O.collide_model(LAT, model, f, g, tp, tm)
            rho, u = O.node_moments(LAT, f, g)
            feq = O.equilibrium(LAT, rho, u)
            assert np.abs((fs - feq) @ phi.T).max() < 1e-16 * 8
    rho, u = O.node_moments(LAT, f, g)
    assert np.abs((f - O.equilibrium(LAT, rho, u)) @ phi.T).max() > 1e-4


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


def test_linearised_spectrum():
    spec = golden("collision_spectrum.json")["D3Q27"]
    _, w, _ = O.lattice(LAT)
    tp, tm = 0.8, 2.5
    ap, am = 1 - 1 / tp, 1 - 1 / tm
    for model, n_am, n_zero, n_ap in (
            (O.PTRT, spec["a_minus"] + spec["fifth"], spec["ghost"], spec["a_plus"]),
            (O.PTRT_EXACT, spec["a_minus"], spec["ghost"] + spec["fifth"], spec["a_plus"]),
            (O.TRT, spec["a_minus"] + spec["fifth"], 0, spec["a_plus"] + spec["ghost"])):
        J = _jacobian(lambda x: O.collide_model(LAT, model, x[None], None, tp, tm)[0], w.copy())
        ev = np.sort(np.linalg.eigvals(J).real)
        assert _count(ev, 1.0) == spec["one"]
        assert _count(ev, ap) == n_ap
        assert _count(ev, am) == n_am
        assert _count(ev, 0.0) == n_zero


def test_exact_variant_matches_trt_rlb_walls_force():
    rng = np.random.default_rng(27)
    nz, ny, nx = 5, 8, 6
    rho, u = I.random_fields(rng, (nz, ny, nx), umax=0.04)
    solid = np.zeros((nz, ny, nx), dtype=np.uint8)
    solid[:, 0, :] = 1
    solid[:, -1, :] = 1
    solid[2, 4, 3] = 1
    g = np.array([1e-4, 0.0, -5e-5])
    tp, lam = 0.7, 3 / 16
    L = O.Lattice(LAT, nx, ny, nz, tp, lam, g=g, solid=solid, model=O.PTRT_EXACT)
    L.init_equilibrium(rho, u)
    f0 = L.populations().copy()
    f0[:, solid.astype(bool)] = 0.0
    L.set_populations(f0)
    L.step(30)
    tm = 0.5 + lam / (tp - 0.5)
    f2 = R.run("D3Q27", f0, (nz, ny, nx), g, tp, tm, 30, solid=solid.astype(bool))
    fl = ~solid.astype(bool)
    f1 = L.populations()
    assert np.abs(f1[:, fl] - f2[:, fl]).max() <= 1e-13 * np.abs(f1).max()
    # the hybrid differs from it, a little, on the same run
    H = O.Lattice(LAT, nx, ny, nz, tp, lam, g=g, solid=solid)
    H.set_populations(f0)
    H.step(30)
    d = np.abs(H.populations()[:, fl] - f1[:, fl]).max()
    assert 1e-12 < d < 1e-3


@pytest.mark.parametrize("model", [O.PTRT, O.PTRT_EXACT])
def test_poiseuille_exact_at_magic_3_16(model):
    """Sec. 3.3 channel (N = 32, u_c = 0.1, tau+ = 10.1) as a two-layer
    periodic slab: the parabolic profile is exact at Lambda = 3/16 for both
    D3Q27 variants and slips at Lambda = 1/4."""
    gd = golden("poiseuille_l2.json")
    N, nx, uc = gd["N"], gd["nx"], gd["u_c"]
    tp = gd["cases"][0]["tau_plus"]
    nu = (tp - 0.5) / 3.0
    g = A.poiseuille_acceleration(N, uc, nu)
    steps = int(40 * N * N / (np.pi ** 2 * nu)) + 2000
    solid = np.repeat(I.channel_mask(nx, N + 2)[None], 2, axis=0).reshape(2, N + 2, nx)
    res = {}
    for lam in (gd["Lambda"], 0.25):
        L = O.Lattice(LAT, nx, N + 2, 2, tp, lam, g=[g, 0, 0], solid=solid, model=model)
        L.init_equilibrium()
        L.step(steps)
        _, u = L.moments()
        ux = u[0, :, 1:N + 1, :]
        assert np.abs(u[1:, :, 1:N + 1]).max() < 1e-12 * uc
        assert np.ptp(ux.reshape(2, N, nx).transpose(1, 0, 2).reshape(N, -1), axis=1).max() < 1e-12 * uc
        res[lam] = A.rel_l2(ux[0, :, 0], A.poiseuille_profile(N, uc))
    assert res[gd["Lambda"]] <= 10 * gd["cases"][0]["L2_ptrt"]
    assert res[0.25] > 1e-5
