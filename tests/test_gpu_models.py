"""GPU comparison models (NEXT step after the hot path): TRT-RLB with explicit
Hermite projection and standard TRT, against their oracles, and the paper's
equivalence result (Remark on exactness) checked on the GPU: P-TRT and
TRT-RLB kernels give the same populations to round-off."""
import numpy as np
import pytest

import lbm_inputs as I
from conftest import print_case
from oracle import analytic as A
from oracle import ptrt as O
from oracle import trt_rlb as R

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2602_06686_amd.ptrt")


def _case(lat):
    rng = np.random.default_rng(31 + lat)
    if lat == 0:
        shape = (1, 20, 33)
    else:
        shape = (8, 10, 12)
    nz, ny, nx = shape
    rho, u = I.random_fields(rng, shape, umax=0.04)
    if lat == 0:
        u[2] = 0
    mask = np.zeros(shape, dtype=np.uint8)
    mask[:, 0, :] = 1
    mask[:, -1, :] = 1
    mask[nz // 2, ny // 2, nx // 3] = 1
    g = [2e-5, -1e-5, 1e-5 if lat else 0.0]
    return shape, rho, u, mask, g


@pytest.mark.parametrize("lat", [0, 1])
def test_trt_rlb_kernel_matches_numpy_trt_rlb(lat):
    print_case("TRT-RLB kernel vs NumPy TRT-RLB", lat)
    (nz, ny, nx), rho, u, mask, g = _case(lat)
    tp, lam, steps = 0.7, 3 / 16, 25
    tm = 0.5 + lam / (tp - 0.5)
    name = "D2Q9" if lat == 0 else "D3Q19"
    with P.Lattice(lat, nx, ny, nz, tp, lam, force=g, solid_mask=mask, storage="f64",
                   model="trt-rlb") as G:
        G.init_equilibrium(rho, u)
        f0 = G.populations()
        G.step(steps)
        fg = G.populations()
    shape = (ny, nx) if lat == 0 else (nz, ny, nx)
    f0 = f0.reshape((f0.shape[0],) + shape)
    D = 2 if lat == 0 else 3
    fr = R.run(name, f0, shape, np.asarray(g)[:D], tp, tm, steps, solid=mask.reshape(shape).astype(bool))
    fluid = mask.reshape(shape) == 0
    fg = fg.reshape(fr.shape)
    assert np.abs(fg[:, fluid] - fr[:, fluid]).max() < 1e-12 * np.abs(fr).max()


@pytest.mark.parametrize("lat", [0, 1])
def test_trt_kernel_matches_oracle_trt(lat):
    print_case("TRT kernel vs oracle TRT", lat)
    (nz, ny, nx), rho, u, mask, g = _case(lat)
    tp, lam, steps = 0.62, 0.25, 40
    with P.Lattice(lat, nx, ny, nz, tp, lam, force=g, solid_mask=mask, storage="f64",
                   model="trt") as G:
        G.init_equilibrium(rho, u)
        G.step(steps)
        fg = G.populations()
    ora = O.Lattice(lat, nx, ny, nz, tp, lam, g=g, solid=mask, model=2)
    ora.init_equilibrium(rho, u)
    ora.step(steps)
    fo = ora.populations()
    fluid = mask == 0
    assert np.abs(fg[:, fluid] - fo[:, fluid]).max() < 1e-12 * np.abs(fo).max()


def test_ptrt_equals_trt_rlb_on_gpu_tgv64():
    """Remark on exactness, on the GPU: the two kernels agree over 1000 steps
    of the 64^2 vortex in FP64; standard TRT does not."""
    print_case("P-TRT vs TRT-RLB kernels, TGV 64^2")
    n, u0, nu = 64, 0.05, 0.01
    tp, lam = I.tau_plus_from_nu(nu), 0.25
    rho, u = I.tgv2d(n, u0)
    out = {}
    for model in ("ptrt", "trt-rlb", "trt"):
        with P.Lattice(0, n, n, 1, tp, lam, storage="f64", model=model) as G:
            G.init_equilibrium(rho, u)
            G.step(1000)
            out[model] = G.moments()[1][:2]
    d_rlb = A.rel_l2(out["trt-rlb"], out["ptrt"])
    d_trt = A.rel_l2(out["trt"], out["ptrt"])
    print(f"P-TRT vs TRT-RLB velocity rel L2 {d_rlb:.3e}; vs standard TRT {d_trt:.3e}")
    assert d_rlb < 1e-12
    assert d_trt > 1e-8


def test_model_switch_keeps_state():
    print_case("model switch mid-run")
    n = 32
    rho, u = I.tgv2d(n, 0.05)
    with P.Lattice(0, n, n, 1, 0.6, 0.25, storage="f64") as A1, \
            P.Lattice(0, n, n, 1, 0.6, 0.25, storage="f64") as A2:
        A1.init_equilibrium(rho, u)
        A2.init_equilibrium(rho, u)
        A1.step(30)
        P.ptrt_set_model(A1.h, "trt")
        A1.step(30)
        P.ptrt_set_model(A1.h, "ptrt")
        A1.step(30)
        A2.step(30)
        P.ptrt_set_model(A2.h, "trt")
        A2.step(30)
        P.ptrt_set_model(A2.h, "ptrt")
        A2.step(30)
        assert np.array_equal(A1.populations(), A2.populations())


@pytest.mark.parametrize("model", ["trt-rlb", "trt"])
@pytest.mark.parametrize("lat,storage,shape", [(0, "f32", (1, 40, 200)), (0, "f64", (1, 33, 130)),
                                               (1, "f32", (6, 10, 64)), (1, "f64", (5, 8, 128))])
def test_comparison_models_two_steps_per_pass_bitwise(model, lat, storage, shape):
    """The comparison models also run the two-step pass (first step kept in
    LDS) where P-TRT does, without solids: bit-identical to one step per
    pass, so the efficiency comparison can be made where the pass is bound
    by instruction issue rather than by HBM."""
    print_case("comparison model, steps per pass 2 vs 1", model, lat, storage, shape)
    nz, ny, nx = shape
    rng = np.random.default_rng(77 + lat)
    rho, u = I.random_fields(rng, shape, umax=0.04)
    if lat == 0:
        u[2] = 0
    g = [2e-6, -1e-6, 1e-6 if lat else 0.0]
    out, passes = [], []
    for spp in (1, 2):
        with P.Lattice(lat, nx, ny, nz, 0.62, 3 / 16, force=g, storage=storage, model=model,
                       steps_per_pass=spp) as G:
            G.init_equilibrium(rho, u)
            G.step(8)
            passes.append(G.last_pass()[0])
            out.append(G.populations())
    assert passes == [1, 2]
    assert np.array_equal(out[0], out[1])
