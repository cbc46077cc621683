"""Two steps per pass (temporal blocking through LDS: D3Q19 in FP32 and
FP64, D2Q9 in FP32 and FP64): the kernel must give the same populations, bit for
bit, as one step per pass, for odd and even step counts, ragged strips and
row chunks, with solids and open boundaries, and through the graph-replay
path of small lattices; ineligible configurations (other storage types and
lattices, solids near most rows, nx not a multiple of 64 in 3D) fall back
to one step per pass.  Eligible cases are also checked against the FP64
oracle."""
import numpy as np
import pytest

import lbm_inputs as I
from conftest import print_case
from oracle import analytic as A
from oracle import ptrt as O

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2602_06686_amd.ptrt")


def _run(lat, shape, storage, steps, spp, mask=None, force=None, seed=5, passes=None):
    """Populations after `steps` steps; `passes`, if a list, receives the
    steps covered by the last kernel pass."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    rho, u = I.random_fields(rng, shape, umax=0.05)
    with P.Lattice(lat, nx, ny, nz, 0.61, 0.25, storage=storage, solid_mask=mask, force=force,
                   steps_per_pass=spp) as G:
        G.init_equilibrium(rho, u)
        G.step(steps)
        if passes is not None:
            passes.append(G.last_pass()[0])
        return G.populations()


# FP32 D3Q19: where ny is a multiple of the rows per layout tile (16 at
# nx = 64, 8 at 128, 4 at 192 and 256) the pass forms each task's source
# offsets once (7x16x128, 4x32x64, 3x64x128, 2x16x192); elsewhere it takes
# the general pulls
@pytest.mark.parametrize("lat,storage,shape", [
    (1, "f32", (6, 8, 64)), (1, "f32", (7, 16, 128)), (1, "f32", (2, 8, 64)),
    (1, "f32", (3, 12, 64)), (1, "f32", (4, 10, 64)), (1, "f32", (3, 13, 128)), (1, "f32", (5, 6, 64)),
    (1, "f32", (4, 32, 64)), (1, "f32", (3, 64, 128)), (1, "f32", (2, 16, 192)),
    (1, "f64", (4, 8, 64)), (1, "f64", (3, 10, 128)),
    # FP64 keeps two planes of loads in flight (its loop unrolled by two):
    # chunks of 1, 2, 5 and 7 planes, and several chunks per column
    (1, "f64", (1, 8, 64)), (1, "f64", (2, 8, 64)), (1, "f64", (5, 6, 64)), (1, "f64", (7, 16, 128)),
    (1, "f64", (128, 128, 128)), (1, "f64", (99, 64, 64)),
    # more whole-depth columns than one round of resident workgroups (on
    # MI355X 512 in FP32, 256 in FP64): one launch per round's worth of
    # workgroup rows, the last one short (600 rows as 512 + 88, 300 as
    # 256 + 44)
    (1, "f32", (4, 2400, 64)), (1, "f64", (4, 1200, 64)),
    (1, "f16", (5, 16, 64)), (1, "bf16", (9, 8, 128)),
    (2, "f16", (9, 8, 64)), (2, "bf16", (4, 12, 64))])
@pytest.mark.parametrize("steps", [1, 2, 7, 40])
def test_two_steps_per_pass_bitwise(lat, storage, shape, steps):
    print_case("steps per pass 2 vs 1", lat, storage, shape, steps)
    a = _run(lat, shape, storage, steps, 1)
    last = []
    b = _run(lat, shape, storage, steps, 2, passes=last)
    assert np.array_equal(a, b)
    if lat == 1 and storage in ("f32", "f64") and steps % 2 == 0:
        assert last == [2]          # the two-step kernel ran


# D2Q9 (two steps per pass in FP32 and FP64): strips of 62 columns (the
# last partial when nx is not a multiple), chunks of 1 to 9 rows chosen by
# size (the last partial; the chunk height of each case in the comment),
# the periodic wrap crossing both, and the degenerate widths 1, 2 and 3 and
# heights 1, 2 and 4
D2_CASES = [
    ("f32", (1, 523, 1010)),  # 6 rows
    ("f32", (1, 1, 600000)), ("f32", (1, 2, 300000)),
    ("f32", (1, 200000, 3)),  # 9
    ("f32", (1, 9000, 62)),  # 6
    ("f32", (1, 64, 64)), ("f32", (1, 37, 130)), ("f32", (1, 5, 1)),  # 1
    ("f32", (1, 333, 500)),  # 2
    ("f32", (1, 517, 530)),  # 3
    ("f32", (1, 2049, 2048)),  # 7
    ("f64", (1, 515, 520)),  # 6
    ("f64", (1, 200000, 2)), ("f64", (1, 4, 70000)),
    ("f64", (1, 64, 64)),  # 1
    ("f64", (1, 301, 390)),  # 3
    ("f64", (1, 453, 400)),  # 5 (4 is skipped)
    ("f64", (1, 1023, 1000))]  # 9 (8 is skipped)


@pytest.mark.parametrize("storage,shape", D2_CASES)
@pytest.mark.parametrize("steps", [1, 2, 7, 40])
def test_two_steps_per_pass_d2q9_bitwise(storage, shape, steps):
    print_case("D2Q9 steps per pass 2 vs 1", storage, shape, steps)
    a = _run(0, shape, storage, steps, 1)
    b = _run(0, shape, storage, steps, 2)
    assert np.array_equal(a, b)


def _last_pass(shape, storage, mask=None):
    nz, ny, nx = shape
    with P.Lattice(0, nx, ny, nz, 0.6, 0.25, storage=storage, solid_mask=mask) as G:
        G.init_equilibrium(np.ones(shape), np.zeros((2,) + shape))
        G.step(4)
        return G.last_pass()


def test_two_steps_per_pass_d2q9_used_where_it_pays():
    """The pass covers two steps at every size in FP32 and FP64 only, with
    or without a body force; with solids from 2^20 nodes on while few rows
    are near them."""
    print_case("D2Q9 last pass: sizes, storage types, force, solids")
    assert _last_pass((1, 512, 1024), "f32") == (2, 2.0 * 1024 * 512 * 9 * 4)
    assert _last_pass((1, 3, 5), "f32") == (2, 2.0 * 5 * 3 * 9 * 4)
    assert _last_pass((1, 512, 512), "f64") == (2, 2.0 * 512 * 512 * 9 * 8)
    assert _last_pass((1, 64, 64), "f64")[0] == 2
    for st in ("f16", "bf16"):
        assert _last_pass((1, 1024, 1024), st)[0] == 1
        assert _last_pass((1, 64, 64), st)[0] == 1
    mask = np.zeros((1, 1024, 1024), dtype=np.uint8)
    mask[0, 0, :] = 1
    # with solids: the state and the mask bytes
    assert _last_pass((1, 1024, 1024), "f64", mask=mask) == (2, (2.0 * 9 * 8 + 1) * 1024 * 1024)
    assert _last_pass((1, 1024, 1024), "f32", mask=mask) == (2, (2.0 * 9 * 4 + 1) * 1024 * 1024)
    assert _last_pass((1, 1024, 1024), "f16", mask=mask)[0] == 1
    # below 2^20 nodes with solids: one step per pass
    assert _last_pass((1, 1023, 1024), "f64", mask=mask[:, :1023])[0] == 1
    assert _last_pass((1, 64, 64), "f32", mask=mask[:, :64, :64])[0] == 1
    for m in _d2_masks():
        for st in ("f32", "f64"):
            assert _last_pass(m.shape, st, mask=m)[0] == 2
    # solids near most rows: one step per pass
    dense = (np.random.default_rng(4).random((1, 1024, 1024)) < 0.01).astype(np.uint8)
    assert _last_pass((1, 1024, 1024), "f64", mask=dense)[0] == 1
    f = [2e-5, -1e-5, 0]
    shape = (1, 600, 1000)
    assert np.array_equal(_run(0, shape, "f32", 9, 1, force=f), _run(0, shape, "f32", 9, 2, force=f))


def _d2_masks():
    """Solid layouts of at least 2^20 nodes with few rows near solids (where
    two steps per pass are used): channel walls on the periodic y seam, a
    band of random solids (some next to each other, across chunk and strip
    borders), a square obstacle, a solid column on the periodic x seam with
    blocks at a strip border and in the last, partial strip, and a tall
    block (masked rows in chunks of several rows)."""
    rng = np.random.default_rng(21)
    out = []
    m = np.zeros((1, 1050, 1000), dtype=np.uint8)
    m[0, 0, :] = m[0, -1, :] = 1
    out.append(m)
    m = np.zeros((1, 1030, 1030), dtype=np.uint8)
    m[0, 200:241, :] = rng.random((41, 1030)) < 0.05
    out.append(m)
    m = np.zeros((1, 2060, 520), dtype=np.uint8)
    m[0, 1000:1033, 240:273] = 1
    out.append(m)
    m = np.zeros((1, 1400, 801), dtype=np.uint8)
    m[0, 300:321, 0] = 1
    m[0, 300:310, 700:800] = 1
    m[0, 7:9, 61:63] = 1
    out.append(m)
    m = np.zeros((1, 1100, 1000), dtype=np.uint8)
    m[0, 100:301, 400:600] = 1
    out.append(m)
    return out


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("case", range(5))
@pytest.mark.parametrize("steps", [2, 7, 40])
def test_two_steps_per_pass_d2q9_solids_bitwise(storage, case, steps):
    mask = _d2_masks()[case]
    print_case("D2Q9 with solids, steps per pass 2 vs 1", storage, mask.shape, steps)
    a = _run(0, mask.shape, storage, steps, 1, mask=mask, force=[1e-6, 0, 0])
    b = _run(0, mask.shape, storage, steps, 2, mask=mask, force=[1e-6, 0, 0])
    fluid = np.broadcast_to(mask == 0, a.shape)
    assert np.array_equal(a[fluid], b[fluid])


def test_two_steps_per_pass_d2q9_channel_matches_oracle():
    print_case("D2Q9 channel, steps per pass 2, FP64 1020x1030 vs oracle, 40 steps")
    nz, ny, nx = n = (1, 1030, 1020)
    mask = np.zeros(n, dtype=np.uint8)
    mask[0, 0, :] = mask[0, -1, :] = 1
    mask[0, 400:420, 100:130] = 1
    rng = np.random.default_rng(17)
    rho, u = I.random_fields(rng, n, umax=0.03)
    u = u[:2]
    g = [2e-5, 0, 0]
    with P.Lattice(0, nx, ny, nz, 0.62, 3 / 16, storage="f64", force=g, solid_mask=mask) as G:
        G.init_equilibrium(rho, u)
        G.step(40)
        assert G.last_pass()[0] == 2
        rg, ug = G.moments()
    ora = O.Lattice(O.D2Q9, nx, ny, nz, 0.62, 3 / 16, g=g, solid=mask, nthreads=8)
    ora.init_equilibrium(rho, u)
    ora.step(40)
    ro, uo = ora.moments()
    fl = mask == 0
    err = np.abs(ug[:2][:, fl] - uo[:2][:, fl]).max() / np.abs(uo[:2][:, fl]).max()
    print(f"D2Q9 channel two steps per pass, 40 steps, max rel velocity error {err:.3e}", flush=True)
    assert err < 1e-12
    assert np.abs(rg[fl] - ro[fl]).max() < 1e-12


def test_two_steps_per_pass_d2q9_matches_oracle():
    print_case("D2Q9 steps per pass 2, FP64 520x510 with force vs oracle, 60 steps")
    nz, ny, nx = n = (1, 510, 520)
    rng = np.random.default_rng(13)
    rho, u = I.random_fields(rng, n, umax=0.05)
    u = u[:2]
    with P.Lattice(0, nx, ny, nz, 0.58, 0.25, storage="f64", force=[1e-5, 2e-6, 0]) as G:
        G.init_equilibrium(rho, u)
        G.step(60)
        assert G.last_pass()[0] == 2
        hg = G.populations()
    ora = O.Lattice(O.D2Q9, nx, ny, nz, 0.58, 0.25, g=[1e-5, 2e-6, 0], nthreads=8)
    ora.init_equilibrium(rho, u)
    ora.step(60)
    ho = ora.populations()
    err = np.abs(hg - ho).max() / np.abs(ho).max()
    print(f"D2Q9 two steps per pass, 60 steps, max rel population error {err:.3e}", flush=True)
    assert err < 1e-12


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


def _run_open(shape, storage, steps, spp, mask=None, seed=8):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    rho, u = I.random_fields(rng, shape, umax=0.02)
    u[0] += 0.03
    with P.Lattice(0, nx, ny, nz, 0.7, 3 / 16, storage=storage, solid_mask=mask,
                   open_x=(0.03, 1.0), steps_per_pass=spp) as G:
        G.init_equilibrium(rho, u[:2])
        G.step(steps)
        return G.populations(), G.last_pass()[0]


def _open_masks():
    """Open-x layouts of at least 2^20 nodes: no solids (last strip partial),
    a square cylinder (the benchmark's shape), channel walls at y = 0 and
    ny - 1, and a width that is a multiple of 62 (the last strip's halo
    column wraps onto the inlet)."""
    out = [((1, 1030, 1040), None)]
    n = 1050
    m = np.zeros((1, n, n), dtype=np.uint8)
    c0 = n // 2 - 10
    m[0, c0:c0 + 21, c0:c0 + 21] = 1
    out.append(((1, n, n), m))
    m = np.zeros((1, 1030, 1040), dtype=np.uint8)
    m[0, 0, :] = m[0, -1, :] = 1
    out.append(((1, 1030, 1040), m))
    out.append(((1, 1000, 1054), None))
    return out


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("case", range(4))
@pytest.mark.parametrize("steps", [2, 7, 40])
def test_two_steps_per_pass_d2q9_open_bitwise(storage, case, steps):
    """Open x (velocity inlet, Zou-He outlet): the boundary strips run the
    open kernel in the special launch; bit for bit against one step per
    pass on every fluid node."""
    shape, mask = _open_masks()[case]
    print_case("D2Q9 open x, steps per pass 2 vs 1", storage, shape, steps)
    a, pa = _run_open(shape, storage, steps, 1, mask)
    b, pb = _run_open(shape, storage, steps, 2, mask)
    assert pa == 1 and pb == (2 if steps % 2 == 0 else 1)
    fluid = np.broadcast_to(True if mask is None else mask == 0, a.shape)
    assert np.array_equal(a[fluid], b[fluid])


def test_two_steps_per_pass_d2q9_open_floor():
    print_case("D2Q9 open x below 2^20 nodes: one step per pass")
    _, p = _run_open((1, 1000, 1000), "f64", 4, 2)
    assert p == 1


def _d3_masks():
    """D3Q19 solid layouts of 2^24 nodes with few near-solid column chunks
    (where two steps per pass are used): channel walls at y = 0 and ny - 1
    (the y seam); a cube, a band of random solids in z and a block on the
    x seam, in a lattice whose y extent is not a multiple of 4."""
    rng = np.random.default_rng(31)
    out = []
    m = np.zeros((256, 1024, 64), dtype=np.uint8)
    m[:, 0, :] = m[:, -1, :] = 1
    out.append(m)
    m = np.zeros((256, 1030, 64), dtype=np.uint8)
    m[100:104, 500:504, 20:24] = 1
    m[30:33, 200:203] = rng.random((3, 3, 64)) < 0.2
    m[5:9, 12:15, 0] = 1
    m[5:9, 12:15, 63] = 1
    out.append(m)
    return out


@pytest.mark.parametrize("storage", ["f32", "f64"])
@pytest.mark.parametrize("case", range(2))
def test_two_steps_per_pass_d3q19_solids_bitwise(storage, case):
    """D3Q19 with solids: mask-free column chunks in one launch, the chunks
    near solids (short z chunks, bounce-back in both steps) in a second;
    7 steps (three passes and a single step), bit for bit against one step
    per pass on every fluid node."""
    mask = _d3_masks()[case]
    print_case("D3Q19 with solids, steps per pass 2 vs 1", storage, mask.shape)
    a = _run(1, mask.shape, storage, 7, 1, mask=mask, force=[1e-6, 0, 0])
    b = _run(1, mask.shape, storage, 7, 2, mask=mask, force=[1e-6, 0, 0])
    fluid = np.broadcast_to(mask == 0, a.shape)
    assert np.array_equal(a[fluid], b[fluid])
    del a, b


def _last_pass_3d(m, st):
    nz, ny, nx = m.shape
    with P.Lattice(1, nx, ny, nz, 0.6, 0.25, storage=st, solid_mask=m) as G:
        G.init_equilibrium(np.ones(m.shape), np.zeros((3,) + m.shape))
        G.step(4)
        return G.last_pass()


def test_two_steps_per_pass_d3q19_solids_used_where_it_pays():
    """From 2^24 nodes with at most 5 % of the column chunks near solids."""
    print_case("D3Q19 with solids: last pass")
    m = _d3_masks()[0]
    for st in ("f32", "f64"):
        assert _last_pass_3d(m, st) == (2, (2.0 * 19 * (4 if st == "f32" else 8) + 1) * m.size)
    # below 2^24 nodes, or solids near many chunks: one step per pass
    assert _last_pass_3d(m[:, :1020], "f32")[0] == 1
    cube = np.zeros((128, 512, 256), dtype=np.uint8)
    cube[48:80, 240:272, 112:144] = 1
    assert _last_pass_3d(cube, "f32")[0] == 1


def _random_shapes(seed, n):
    """Seeded lattice shapes for the two-step pass: D3Q19 with nx a multiple
    of 64 (the pass's requirement) and any ny >= 4, nz >= 1; D2Q9 of any
    size from one row up, so that strips, row chunks and z chunks end
    ragged in every way."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        if k % 2 == 0:
            out.append((1, (int(rng.integers(1, 40)), int(rng.integers(4, 41)),
                            64 * int(rng.integers(1, 5)))))
        else:
            out.append((0, (1, int(rng.integers(1, 300)), int(rng.integers(2, 300)))))
    return out


@pytest.mark.parametrize("storage", ["f32", "f64"])
@pytest.mark.parametrize("lat,shape", _random_shapes(2602, 16))
def test_two_steps_per_pass_random_shapes_bitwise(storage, lat, shape):
    """Seeded random shapes, 9 steps (four two-step passes and one single
    step): bit-identical to one step per pass."""
    print_case("steps per pass 2 vs 1, random shape", lat, storage, shape)
    a = _run(lat, shape, storage, 9, 1, seed=11)
    b = _run(lat, shape, storage, 9, 2, seed=11)
    assert np.array_equal(a, b)
