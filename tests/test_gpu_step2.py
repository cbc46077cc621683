"""Two steps per pass (temporal blocking through LDS, D3Q19 FP32): the
kernel must give the same populations, bit for bit, as one step per pass,
for odd and even step counts and through the graph-replay path of small
lattices; ineligible configurations (other storage types and lattices,
solids, force, nx not a multiple of 64) fall back to one step per pass.  One eligible case is also checked against the
FP64 oracle."""
import numpy as np
import pytest

import lbm_inputs as I
from conftest import print_case
from oracle import analytic as A
from oracle import ptrt as O

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2602_06686_amd.ptrt")


def _run(lat, shape, storage, steps, spp, mask=None, force=None, seed=5):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    rho, u = I.random_fields(rng, shape, umax=0.05)
    with P.Lattice(lat, nx, ny, nz, 0.61, 0.25, storage=storage, solid_mask=mask, force=force,
                   steps_per_pass=spp) as G:
        G.init_equilibrium(rho, u)
        G.step(steps)
        return G.populations()


@pytest.mark.parametrize("lat,storage,shape", [
    (1, "f32", (6, 8, 64)), (1, "f32", (7, 16, 128)), (1, "f32", (2, 8, 64)),
    (1, "f32", (3, 12, 64)),
    (1, "f16", (5, 16, 64)), (1, "bf16", (9, 8, 128)),
    (2, "f16", (9, 8, 64)), (2, "bf16", (4, 12, 64))])
@pytest.mark.parametrize("steps", [1, 2, 7, 40])
def test_two_steps_per_pass_bitwise(lat, storage, shape, steps):
    print_case("steps per pass 2 vs 1", lat, storage, shape, steps)
    a = _run(lat, shape, storage, steps, 1)
    b = _run(lat, shape, storage, steps, 2)
    assert np.array_equal(a, b)


def test_two_steps_per_pass_large_bitwise():
    print_case("steps per pass 2 vs 1, 256x64x64 FP32, 10 steps")
    shape = (64, 64, 256)
    assert np.array_equal(_run(1, shape, "f32", 10, 1), _run(1, shape, "f32", 10, 2))


def test_ineligible_configurations_fall_back():
    print_case("steps per pass: ineligible configurations")
    shape = (4, 8, 64)
    mask = np.zeros(shape, dtype=np.uint8)
    mask[:, 0, :] = 1
    assert np.array_equal(_run(1, shape, "f32", 6, 1, mask=mask), _run(1, shape, "f32", 6, 2, mask=mask))
    assert np.array_equal(_run(1, (4, 8, 48), "f32", 6, 1), _run(1, (4, 8, 48), "f32", 6, 2))
    assert np.array_equal(_run(1, shape, "f64", 6, 1), _run(1, shape, "f64", 6, 2))
    assert np.array_equal(_run(1, shape, "f32", 6, 1, force=[1e-5, 0, 0]),
                          _run(1, shape, "f32", 6, 2, force=[1e-5, 0, 0]))


def test_two_steps_per_pass_matches_oracle():
    print_case("steps per pass 2, D3Q19 FP32 64x8x8 vs oracle, 100 steps")
    n = (8, 8, 64)
    nz, ny, nx = n
    rng = np.random.default_rng(9)
    rho, u = I.random_fields(rng, n, umax=0.04)
    with P.Lattice(1, nx, ny, nz, 0.7, 0.25, storage="f32") as G:
        G.init_equilibrium(rho, u)
        G.step(100)
        _, ug = G.moments()
    ora = O.Lattice(O.D3Q19, nx, ny, nz, 0.7, 0.25)
    ora.init_equilibrium(rho, u)
    ora.step(100)
    _, uo = ora.moments()
    err = A.rel_l2(ug, uo)
    print(f"two steps per pass, 100 steps, velocity rel L2 {err:.3e}", flush=True)
    assert err < 1e-5
