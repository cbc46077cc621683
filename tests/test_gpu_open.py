"""GPU parity of the open boundaries and the momentum-exchange force (Sec.
3.4; D2Q9) against the FP64 oracle, through the C interface.

* Velocity inlet (moving halfway bounce-back) + Zou-He pressure outlet,
  walls, a square obstacle, ragged sizes: populations after 150 steps, FP64
  1e-12 relative; FP32 1e-5 on the velocity.
* Momentum-exchange force (Eq. Fx) on the obstacle: GPU (from the stored
  post-collision state of the last step) against the oracle (collision of
  the state one step earlier), 1e-12 relative; periodic force-driven flow
  around an obstacle: steady drag equals the total body force.
* Creeping flow past a square cylinder at the paper's setup (D = 21,
  L = 50 D, T = Ma^2 / Re = 0.1, Lambda = 3/16): C_d Re against
  Table tab_3 for Re = 1e-1 ... 1e-6.
"""
import numpy as np
import pytest

import lbm_inputs as I
from conftest import golden, print_case
from oracle import analytic as A
from oracle import ptrt as O

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2602_06686_amd.ptrt")


def _obstacle_channel(nx, ny, side, walls=True):
    mask = np.zeros((1, ny, nx), dtype=np.uint8)
    if walls:
        mask[0, 0, :] = 1
        mask[0, -1, :] = 1
    y0, x0 = ny // 2 - side // 2, nx // 3
    mask[0, y0:y0 + side, x0:x0 + side] = 1
    return mask


@pytest.mark.parametrize("nx,ny,walls", [(37, 21, True), (70, 33, False), (2, 5, False)])
def test_open_boundaries_fp64_match_oracle(nx, ny, walls):
    print_case("open x FP64 vs oracle", nx, ny, walls)
    uin, rho_out, tp, lam, steps = 0.04, 1.0, 0.7, 3 / 16, 150
    mask = _obstacle_channel(nx, ny, 3, walls) if nx > 2 else np.zeros((1, ny, nx), np.uint8)
    rng = np.random.default_rng(nx + ny)
    rho, u = I.random_fields(rng, (1, ny, nx), umax=0.02)
    u[0] += uin
    u[2] = 0
    with P.Lattice(0, nx, ny, 1, tp, lam, solid_mask=mask, storage="f64",
                   open_x=(uin, rho_out)) as G:
        G.init_equilibrium(rho, u)
        G.step(steps)
        fg = G.populations()
    ora = O.Lattice(O.D2Q9, nx, ny, 1, tp, lam, solid=mask, open_x=(uin, rho_out))
    ora.init_equilibrium(rho, u)
    ora.step(steps)
    fo = ora.populations()
    fluid = mask == 0
    err = float(np.abs(fg[:, fluid] - fo[:, fluid]).max() / np.abs(fo).max())
    print(f"open x {nx}x{ny}: max rel error {err:.3e}", flush=True)
    assert err < 1e-12


def test_open_boundaries_fp32_velocity():
    print_case("open x FP32 velocity")
    nx, ny, uin = 96, 40, 0.05
    mask = _obstacle_channel(nx, ny, 6)
    u = np.zeros((3, 1, ny, nx))
    u[0] = uin
    with P.Lattice(0, nx, ny, 1, 0.65, 3 / 16, solid_mask=mask, storage="f32",
                   open_x=(uin, 1.0)) as G:
        G.init_equilibrium(None, u)
        G.step(1000)
        _, ug = G.moments()
    ora = O.Lattice(O.D2Q9, nx, ny, 1, 0.65, 3 / 16, solid=mask, open_x=(uin, 1.0))
    ora.init_equilibrium(None, u)
    ora.step(1000)
    _, uo = ora.moments()
    err = A.rel_l2(ug[:2], uo[:2])
    print(f"open x FP32 1000 steps velocity rel L2 {err:.3e}", flush=True)
    assert err < 1e-5


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_momentum_exchange_matches_oracle(storage, tol):
    print_case("momentum exchange vs oracle", storage)
    nx, ny, uin, steps = 80, 41, 0.03, 300
    mask = _obstacle_channel(nx, ny, 7, walls=False)
    u = np.zeros((3, 1, ny, nx))
    u[0] = uin
    with P.Lattice(0, nx, ny, 1, 0.9, 3 / 16, solid_mask=mask, storage=storage,
                   open_x=(uin, 1.0)) as G:
        G.init_equilibrium(None, u)
        G.step(steps + 1)
        Fg = G.momentum_exchange()       # post-collision state of step `steps`
    ora = O.Lattice(O.D2Q9, nx, ny, 1, 0.9, 3 / 16, solid=mask, open_x=(uin, 1.0))
    ora.init_equilibrium(None, u)
    ora.step(steps)
    Fo = ora.momentum_exchange()
    print(f"{storage} force GPU {Fg} oracle {Fo}", flush=True)
    assert abs(Fg[0] - Fo[0]) < tol * abs(Fo[0])
    assert abs(Fg[1] - Fo[1]) < tol * abs(Fo[0])


def test_momentum_exchange_balances_body_force():
    """Periodic box, square obstacle, uniform acceleration: in the steady
    state the force on the obstacle equals the total body force."""
    print_case("momentum exchange = body force (periodic)")
    n, side, g = 48, 8, 2e-6
    mask = np.zeros((1, n, n), dtype=np.uint8)
    mask[0, n // 2 - side // 2:n // 2 + side // 2, n // 2 - side // 2:n // 2 + side // 2] = 1
    with P.Lattice(0, n, n, 1, 1.1, 3 / 16, force=[g, 0, 0], solid_mask=mask,
                   storage="f64") as G:
        G.init_equilibrium()
        G.step(30000)
        F = G.momentum_exchange()
        m, _ = G.diagnostics()
    print(f"drag {F[0]:.10e} body force {m * g:.10e}", flush=True)
    assert abs(F[0] - m * g) < 1e-6 * m * g
    assert abs(F[1]) < 1e-9 * m * g


def test_square_cylinder_stokes_drag_table():
    """Sec. 3.4 setup: D = 21, L = 50 D, inlet velocity u_c from
    Ma = u_c / c_s with Ma^2 / Re = 0.1, nu = u_c D / Re, Lambda = 3/16,
    rho_out = 1, started from the uniform stream; run until the drag changes
    by less than 1e-8 (relative) over 2000 steps (at large tau+ the pressure
    field relaxes at a rate of about c_s^2 / nu per step, hence up to 1.6e6
    steps).  C_d = 2 F_x / (u_c^2 D); C_d Re against the printed Table tab_3
    within 0.2 % (the paper leaves node placement and the domain's node
    count open; measured offsets are -0.15 % at Re = 0.1 and +0.03 % in the
    Stokes limit)."""
    gd = golden("square_cylinder_table3.json")
    D, K = gd["D"], gd["L_over_D"]
    n = D * K
    c0 = n // 2 - D // 2
    mask = np.zeros((1, n, n), dtype=np.uint8)
    mask[0, c0:c0 + D, c0:c0 + D] = 1
    res = {}
    for row in gd["rows"]:
        Re = row["Re"]
        Ma = np.sqrt(gd["T"] * Re)
        uc = Ma / np.sqrt(3.0)
        nu = uc * D / Re
        tp = 3 * nu + 0.5
        assert abs(tp - row["tau_plus"]) < 0.5 + 1e-3 * row["tau_plus"]
        print_case("square cylinder", Re, "tau+", tp)
        u = np.zeros((3, 1, n, n))
        u[0] = uc
        with P.Lattice(0, n, n, 1, tp, gd["Lambda"], solid_mask=mask, storage="f64",
                       open_x=(uc, 1.0)) as G:
            G.init_equilibrium(None, u)
            prev, steps = None, 0
            while steps < gd["max_steps"]:
                G.step(2000)
                steps += 2000
                cd = 2 * G.momentum_exchange()[0] / (uc * uc * D)
                if prev is not None and abs(cd - prev) < 1e-8 * abs(cd):
                    break
                prev = cd
        res[Re] = (cd * Re, steps)
        print(f"Re {Re:g}: C_d Re = {cd * Re:.5f} after {steps} steps "
              f"(printed {row['Cd_mu_ptrt']})", flush=True)
    for row in gd["rows"]:
        assert res[row["Re"]][1] < gd["max_steps"], ("not converged", row)
        assert abs(res[row["Re"]][0] / row["Cd_mu_ptrt"] - 1) < 2e-3, (row, res[row["Re"]])
