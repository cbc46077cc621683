"""GPU runs of the remaining configurations, with their errors reported.

* Precision form: D3Q19 Taylor-Green vortex at 64^3 (the FP64 oracle's copy
  of the 512^3 setup), FP32 / FP16 / BF16 storage against the oracle after
  500 steps: relative L2 of the velocity and of the vorticity (central
  differences).  Lambda = 1/4 as configured and 1/tau- = 1.6 (the paper's
  stability optimum, Sec. 3.1).
* Double shear layer at 2048^2 (Sec. 3.1 shape): one FP64 step checked
  against the oracle at sampled nodes; FP32 vs FP64 on the GPU and the
  divergence step, if any, at Re = 1e4, 1e6, 1e7 (Lambda = 1/4) and at
  1/tau- = 1.6.  No printed numbers pin this flow ("parity unpinned" beyond
  the FP64 step check).
* 3D Taylor-Green vortex at 256^3, FP32: kinetic energy from the FP64 GPU
  reduction; the early decay follows exp(-6 nu k^2 t) to within 2 %.
"""
import numpy as np
import pytest

import lbm_inputs as I
from conftest import print_case
from oracle import analytic as A
from oracle import ptrt as O

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2602_06686_amd.ptrt")


def _vorticity(u):
    """Central-difference vorticity of a periodic field u [3, nz, ny, nx]."""
    def d(f, axis):
        return 0.5 * (np.roll(f, -1, axis=axis) - np.roll(f, 1, axis=axis))
    ux, uy, uz = u
    return np.stack([d(uz, 1) - d(uy, 0), d(ux, 0) - d(uz, 2), d(uy, 2) - d(ux, 1)])


@pytest.mark.parametrize("setting", ["Lambda=1/4", "1/tau-=1.6"])
def test_precision_form_64cube(setting):
    n, steps = 64, 500
    prm = I.tgv3d_params(n)
    tp = prm["tau_plus"]
    lam = 0.25 if setting == "Lambda=1/4" else I.tau_minus_from_inverse(1.6, tp)
    rho, u = I.tgv3d(n, 0.05)
    ora = O.Lattice(O.D3Q19, n, n, n, tp, lam)
    ora.init_equilibrium(rho, u)
    ora.step(steps)
    _, uo = ora.moments()
    wo = _vorticity(uo)
    errs = {}
    # At 1/tau- = 1.6 the FP16 bar is the 1e-3 accuracy target.  At Lambda = 1/4
    # (tau- = 262 here) the third-order modes are almost undamped and the
    # FP64 run itself blows up after ~1000 steps, so low-precision rounding
    # noise is hardly damped: those errors are reported, with loose bounds.
    # FP32 at tau+ - 1/2 ~ 1e-3 accumulates more rounding than on the 2D
    # vortex (whose 1e-5 FP32 bar is tested in test_gpu_parity.py).
    bounds = {"Lambda=1/4": (("f32", 5e-5), ("f16", 0.2), ("bf16", 1.0)),
              "1/tau-=1.6": (("f32", 2e-5), ("f16", 1e-3), ("bf16", 2e-2))}[setting]
    for storage, bound in bounds:
        print_case("precision form 64^3", setting, storage)
        with P.Lattice(1, n, n, n, tp, lam, storage=storage) as G:
            G.init_equilibrium(rho, u)
            G.step(steps)
            _, ug = G.moments()
        eu = A.rel_l2(ug, uo)
        ew = A.rel_l2(_vorticity(ug), wo)
        errs[storage] = (eu, ew)
        print(f"precision form {setting} {storage} 64^3 {steps} steps: "
              f"velocity rel L2 {eu:.3e}, vorticity rel L2 {ew:.3e}", flush=True)
        assert eu < bound and ew < 5 * bound
    assert errs["f16"][0] < errs["bf16"][0]


def test_dsl_2048_fp64_step_sampled():
    print_case("DSL 2048^2 FP64 one step sampled")
    n, U0, Re = 2048, 0.05, 1e4
    tp = I.tau_plus_from_nu(U0 * n / Re)
    rho, u = I.double_shear_layer(n, U0)
    rng = np.random.default_rng(77)
    nodes = rng.choice(n * n, 2000, replace=False)
    ora = O.Lattice(O.D2Q9, n, n, 1, tp, 0.25)
    ora.init_equilibrium(rho, u)
    ref = ora.step_sampled(nodes)
    with P.Lattice(0, n, n, 1, tp, 0.25, storage="f64") as G:
        G.init_equilibrium(rho, u)
        G.step(1)
        got = G.populations().reshape(9, -1)[:, nodes].T
    assert np.abs(got - ref).max() < 1e-14


@pytest.mark.parametrize("Re,setting", [(1e4, "Lambda=1/4"), (1e6, "Lambda=1/4"),
                                        (1e7, "Lambda=1/4"), (1e6, "1/tau-=1.6")])
def test_dsl_2048_stability_and_fp32_error(Re, setting):
    n, U0, steps, chunk = 2048, 0.05, 20000, 2000
    tp = I.tau_plus_from_nu(U0 * n / Re)
    lam = 0.25 if setting == "Lambda=1/4" else I.tau_minus_from_inverse(1.6, tp)
    rho, u = I.double_shear_layer(n, U0)
    print_case("DSL 2048^2", Re, setting)
    res = {}
    with P.Lattice(0, n, n, 1, tp, lam, storage="f64") as G64, \
            P.Lattice(0, n, n, 1, tp, lam, storage="f32") as G32:
        G64.init_equilibrium(rho, u)
        G32.init_equilibrium(rho, u)
        m0, _ = G64.diagnostics()
        t = 0
        while t < steps:
            G64.step(chunk)
            G32.step(chunk)
            t += chunk
            m64, k64 = G64.diagnostics(raise_on_divergence=False)
            m32, k32 = G32.diagnostics(raise_on_divergence=False)
            if not (np.isfinite(m64) and np.isfinite(k64)):
                res["diverged_fp64_by_step"] = t
                break
            if not (np.isfinite(m32) and np.isfinite(k32)):
                res["diverged_fp32_by_step"] = t
                break
        if "diverged_fp64_by_step" not in res and "diverged_fp32_by_step" not in res:
            _, u64 = G64.moments()
            _, u32 = G32.moments()
            res["fp32_vs_fp64_velocity_rel_l2"] = A.rel_l2(u32[:2], u64[:2])
            res["max_speed_over_U0"] = float(np.sqrt((u64[:2] ** 2).sum(0)).max() / U0)
            res["mass_rel_change_fp64"] = abs(m64 - m0) / m0
    print(f"DSL 2048^2 Re={Re:g} {setting} tau+={tp:.8f}: {res}", flush=True)
    if Re == 1e4 or setting == "1/tau-=1.6":
        # laminar / paper-optimum settings stay finite over the run
        assert "fp32_vs_fp64_velocity_rel_l2" in res
        assert res["mass_rel_change_fp64"] < 1e-10


def test_tgv3d_256_kinetic_energy_decay():
    print_case("3D TGV 256^3 FP32 kinetic energy")
    n, U0 = 256, 0.05
    prm = I.tgv3d_params(n, U0)
    nu, tp = prm["nu"], prm["tau_plus"]
    rho, u = I.tgv3d(n, U0)
    k = 2 * np.pi / n
    with P.Lattice(1, n, n, n, tp, 0.25, storage="f32") as G:
        G.init_equilibrium(rho, u)
        m0, e0 = G.diagnostics()
        series = [(0, e0)]
        diverged = None
        for t in range(250, 5001, 250):
            G.step(250)
            m, e = G.diagnostics(raise_on_divergence=False)
            if not np.isfinite(e):
                diverged = t
                break
            series.append((t, e))
    print("3D TGV 256^3 E(t)/E0:", [(t, round(e / e0, 5)) for t, e in series],
          "diverged by step" if diverged else "", diverged or "", flush=True)
    # early decay against the viscous closed form exp(-6 nu k^2 t) (loose:
    # kinetic-acoustic exchange at Ma ~ 0.09)
    t1, e1 = series[2]
    assert abs(e1 / e0 - np.exp(-6 * nu * k * k * t1)) < 2e-2
    assert abs(m - m0) < 1e-5 * m0 if diverged is None else True
