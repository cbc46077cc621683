"""ptrt_momentum_exchange_noalloc (the entry point for callers that cannot
allocate device memory) against ptrt_momentum_exchange: the same kernels on
the same state, so the same force bit for bit, on two calls in a row, the
second on a smaller lattice (the fixed scratch still holds the first call's
partials, of which the second must read none)."""
import numpy as np
import pytest

import lbm_inputs as I
from conftest import print_case

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2602_06686_amd.ptrt")


def _force_pair(lattice, shape, storage, mask, g, steps=30, open_x=None):
    nz, ny, nx = shape
    D = 2 if lattice == P.PTRT_D2Q9 else 3
    rng = np.random.default_rng(nx + ny)
    rho, u = I.random_fields(rng, shape, umax=0.03)
    with P.Lattice(lattice, nx, ny, nz, 0.8, 3 / 16, force=g, solid_mask=mask, storage=storage,
                   open_x=open_x) as G:
        G.init_equilibrium(rho, u[:D])
        G.step(steps)
        f_noalloc = P.ptrt_momentum_exchange_noalloc(G.h)
        f_ref = P.ptrt_momentum_exchange(G.h)
        f_noalloc2 = P.ptrt_momentum_exchange_noalloc(G.h)
    return f_noalloc, f_ref, f_noalloc2


def test_noalloc_momentum_exchange_equals_allocating_one():
    # first call: D3Q19 256 x 96 x 80 with walls and a block (7680 blocks of
    # 64 x 4 nodes); second call: a smaller D2Q9 cylinder with open x
    m3 = np.zeros((80, 96, 256), np.uint8)
    m3[:, 0, :] = m3[:, -1, :] = 1
    m3[30:50, 40:60, 100:140] = 1
    print_case("noalloc momentum exchange, D3Q19 256x96x80 FP64")
    a, ref, a2 = _force_pair(P.PTRT_D3Q19, m3.shape, "f64", m3, [1e-6, 0, 0])
    print("D3Q19:", a, ref, flush=True)
    assert np.array_equal(a, ref) and np.array_equal(a2, ref)
    assert np.abs(ref).max() > 0
    m2 = I.square_obstacle_mask(210, 150)
    print_case("noalloc momentum exchange, D2Q9 210x150 FP32 open x")
    b, ref2, b2 = _force_pair(P.PTRT_D2Q9, m2.shape, "f32", m2, None, open_x=(0.02, 1.0))
    print("D2Q9:", b, ref2, flush=True)
    assert np.array_equal(b, ref2) and np.array_equal(b2, ref2)
    assert np.abs(ref2).max() > 0
