"""GPU tests of the batched form: every instance evolves bit for bit like a
single lattice with the same parameters (fused graph launch, per-lattice
launches and any tile plan), and matches the FP64 oracle."""
import numpy as np
import pytest

import lbm_inputs as I
from conftest import print_case
from oracle import analytic as A
from oracle import ptrt as O

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2602_06686_amd.ptrt")


def _small_specs(seed=1):
    rng = np.random.default_rng(seed)
    specs = []
    for k, (nx, ny) in enumerate([(37, 23), (64, 64), (100, 41), (32, 200), (257, 9), (5, 70)]):
        kind = k % 3
        if kind == 0:
            mask = I.channel_mask(nx, ny)
            g = (float(rng.uniform(1e-6, 1e-5)), 0.0, 0.0)
        elif kind == 1:
            mask = I.square_obstacle_mask(nx, ny)
            g = (float(rng.uniform(1e-6, 1e-5)), float(rng.uniform(-1e-6, 1e-6)), 0.0)
        else:
            mask = None
            g = (0.0, 0.0, 0.0)
        specs.append({"nx": nx, "ny": ny, "tau_plus": float(rng.uniform(0.55, 2.0)),
                      "Lambda": [3 / 16, 0.25, 0.1][kind], "g": g, "mask": mask})
    return specs


def _init_fields(spec, seed):
    rng = np.random.default_rng(seed)
    rho, u = I.random_fields(rng, (1, spec["ny"], spec["nx"]), umax=0.03)
    return rho, u[:2]


def _single(spec, storage, rho, u, steps):
    with P.Lattice(0, spec["nx"], spec["ny"], 1, spec["tau_plus"], spec["Lambda"],
                   force=spec["g"], solid_mask=spec["mask"], storage=storage) as L:
        L.init_equilibrium(rho, u)
        L.step(steps)
        return L.populations()


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16sr"])
def test_batch_bitwise_equals_single(storage):
    print_case("batch bitwise vs single", storage)
    specs = _small_specs()
    b = P.ptrt_batch_create(specs, storage)
    try:
        fields = [_init_fields(s, 100 + k) for k, s in enumerate(specs)]
        for k, (rho, u) in enumerate(fields):
            P.ptrt_batch_init_equilibrium(b, k, rho, u)
        P.ptrt_batch_set_plan(b, 64, 4, 0, 0)
        P.ptrt_batch_step(b, 13)            # one graph replay of 10 steps + 3 launches
        P.ptrt_batch_set_plan(b, 32, 8, 7, 1)
        P.ptrt_batch_step(b, 5)              # persistent grid, XCD ordering
        P.ptrt_batch_set_plan(b, 512, 1, 0, 0)
        P.ptrt_batch_step(b, 3)              # whole short rows packed per workgroup
        P.ptrt_batch_set_plan(b, 64, 1, 5, 1)
        P.ptrt_batch_step(b, 3)              # one-wave row segments, persistent, XCD order
        P.ptrt_batch_step_separate(b, 4)     # one launch per lattice
        plan = P.ptrt_batch_autotune(b)      # must leave the state as it was
        P.ptrt_batch_step(b, 2)
        print("autotuned plan", plan)
        for k, s in enumerate(specs):
            ref = _single(s, storage, *fields[k], 30)
            got = P.ptrt_batch_get_populations(b, k)
            assert np.array_equal(got, ref), f"instance {k}"
    finally:
        P.ptrt_batch_destroy(b)


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_batch_two_step_plans_bitwise(storage):
    """Every two-step plan computes the same values: rows per chunk, rows
    per masked chunk, waves per workgroup, one wave per task or a
    persistent grid (down to one workgroup), the masked launch after or
    beside the other; odd step counts (two-step passes, then a one-step
    launch) and graph replays; then the autotuned plan.  Each instance
    equals the single lattice bit for bit after all of them."""
    print_case("batch two-step plans bitwise", storage)
    specs = _small_specs(seed=3)
    b = P.ptrt_batch_create(specs, storage)
    try:
        fields = [_init_fields(s, 300 + k) for k, s in enumerate(specs)]
        for k, (rho, u) in enumerate(fields):
            P.ptrt_batch_init_equilibrium(b, k, rho, u)
        plans = [(1, 1, 2, 0, 0), (2, 1, 4, 0, 1), (3, 2, 8, 0, 0), (5, 3, 4, 64, 1),
                 (7, 7, 2, 16, 0), (64, 64, 8, 0, 1), (3, 1, 4, 1, 1)]
        total = 0
        for plan in plans:
            P.ptrt_batch_set_plan2(b, *plan)
            assert P.ptrt_batch_get_plan2(b) == plan
            P.ptrt_batch_step(b, 7)          # three two-step passes and one step
            total += 7
        assert P.ptrt_batch_last_pass(b)[0] == 1
        P.ptrt_batch_step(b, 12)             # a graph replay of ten steps, one pass
        total += 12
        assert P.ptrt_batch_last_pass(b)[0] == 2
        P.ptrt_batch_autotune(b)             # must leave the state as it was
        print("autotuned two-step plan", P.ptrt_batch_get_plan2(b))
        P.ptrt_batch_step(b, 5)
        total += 5
        for k, s in enumerate(specs):
            ref = _single(s, storage, *fields[k], total)
            got = P.ptrt_batch_get_populations(b, k)
            assert np.array_equal(got, ref), f"instance {k}"
        with pytest.raises(P.PtrtError):
            P.ptrt_batch_set_plan2(b, 0, 1)
        with pytest.raises(P.PtrtError):
            P.ptrt_batch_set_plan2(b, 3, 3, 16)
    finally:
        P.ptrt_batch_destroy(b)


def test_batch_fp64_matches_oracle():
    print_case("batch FP64 vs oracle")
    specs = _small_specs(seed=2)
    b = P.ptrt_batch_create(specs, "f64")
    try:
        fields = [_init_fields(s, 200 + k) for k, s in enumerate(specs)]
        for k, (rho, u) in enumerate(fields):
            P.ptrt_batch_init_equilibrium(b, k, rho, u)
        P.ptrt_batch_step(b, 30)
        mg, kg = P.ptrt_batch_diagnostics(b)
        for k, s in enumerate(specs):
            ora = O.Lattice(O.D2Q9, s["nx"], s["ny"], 1, s["tau_plus"], s["Lambda"], g=s["g"],
                            solid=s["mask"])
            ora.init_equilibrium(*fields[k])
            ora.step(30)
            fo = ora.populations()
            fg = P.ptrt_batch_get_populations(b, k)
            fluid = np.ones((1, s["ny"], s["nx"]), bool) if s["mask"] is None else s["mask"] == 0
            assert np.abs(fg[:, fluid] - fo[:, fluid]).max() < 1e-12 * np.abs(fo).max(), k
            mo, ko = ora.diagnostics()
            assert abs(mg[k] - mo) < 1e-12 * mo and abs(kg[k] - ko) < 1e-12 * ko
            rho_g, u_g = P.ptrt_batch_moments(b, k)
            rho_o, u_o = ora.moments()
            assert np.abs(u_g - u_o).max() < 1e-13
    finally:
        P.ptrt_batch_destroy(b)


def test_batch_poiseuille_instance_reaches_closed_form():
    """A channel instance of the batch (Lambda = 3/16) converges to the exact
    halfway-bounce-back profile, like the single lattice."""
    print_case("batch Poiseuille instance")
    N, nx, uc, tp = 32, 4, 0.1, 2.42
    nu = (tp - 0.5) / 3
    g = A.poiseuille_acceleration(N, uc, nu)
    specs = [{"nx": nx, "ny": N + 2, "tau_plus": tp, "Lambda": 3 / 16, "g": (g, 0, 0),
              "mask": I.channel_mask(nx, N + 2)},
             {"nx": 48, "ny": 16, "tau_plus": 0.8, "Lambda": 0.25, "g": (0, 0, 0), "mask": None}]
    b = P.ptrt_batch_create(specs, "f64")
    try:
        P.ptrt_batch_step(b, int(40 * N * N / (np.pi ** 2 * nu)) + 2000)
        _, u = P.ptrt_batch_moments(b, 0)
        err = A.rel_l2(u[0, 0, 1:N + 1, 0], A.poiseuille_profile(N, uc))
        assert err < 1e-11
    finally:
        P.ptrt_batch_destroy(b)


def test_full_batch_sampled_instances_vs_oracle():
    """The benchmark batch (512 lattices, seed 260206686) with the autotuned
    plan: 20 fused steps, then 6 sampled instances against the FP64 oracle
    (FP32 bar 1e-5 on the populations' deviation from the weights), plus the
    mass of every instance conserved."""
    print_case("full 512-lattice batch, sampled")
    specs = I.batch_specs()
    b = P.ptrt_batch_create(specs, "f32")
    try:
        m0, _ = P.ptrt_batch_diagnostics(b)
        P.ptrt_batch_autotune(b)
        P.ptrt_batch_step(b, 20)
        m1, _ = P.ptrt_batch_diagnostics(b)
        assert np.abs(m1 - m0).max() < 1e-6 * m0.max()
        w = O.lattice(O.D2Q9)[1][:, None, None, None]
        for k in (0, 17, 255, 256, 400, 511):
            s = specs[k]
            ora = O.Lattice(O.D2Q9, s["nx"], s["ny"], 1, s["tau_plus"], s["Lambda"], g=s["g"],
                            solid=s["mask"])
            ora.init_equilibrium()
            ora.step(20)
            fo = ora.populations() - w
            fg = P.ptrt_batch_get_populations(b, k) - w
            fluid = s["mask"] == 0
            scale = max(np.abs(fo[:, fluid]).max(), 1e-12)
            err = np.abs(fg[:, fluid] - fo[:, fluid]).max()
            # populations start at rest: compare to the forcing-driven deviation
            assert err <= 1e-5 * scale + 1e-9, (k, err, scale)
    finally:
        P.ptrt_batch_destroy(b)


def _batch_run(specs, storage, spp, schedule, seed0=300):
    """Populations of every instance after the step counts in schedule
    (calls of ptrt_batch_step), with spp steps per pass."""
    b = P.ptrt_batch_create(specs, storage)
    try:
        P.ptrt_batch_set_steps_per_pass(b, spp)
        for k, s in enumerate(specs):
            P.ptrt_batch_init_equilibrium(b, k, *_init_fields(s, seed0 + k))
        for n in schedule:
            P.ptrt_batch_step(b, n)
        return [P.ptrt_batch_get_populations(b, k) for k in range(len(specs))], P.ptrt_batch_last_pass(b)
    finally:
        P.ptrt_batch_destroy(b)


@pytest.mark.parametrize("storage", ["f32", "f64"])
@pytest.mark.parametrize("schedule", [[1], [2], [7], [13], [10, 10, 3], [25, 1, 14]])
def test_batch_two_steps_per_pass_bitwise(storage, schedule):
    """Two steps per pass (task table of strips and one-row chunks; channels,
    obstacles and a solid-free instance, widths 5 ... 257) against one step
    per pass: bit for bit, through graph replays (odd parity change) and odd
    remainders."""
    print_case("batch steps per pass 2 vs 1", storage, schedule)
    specs = _small_specs(seed=3)
    a, pa = _batch_run(specs, storage, 1, schedule)
    c, pc = _batch_run(specs, storage, 2, schedule)
    for k, s in enumerate(specs):
        fluid = np.broadcast_to(True if s["mask"] is None else s["mask"] == 0, a[k].shape)
        assert np.array_equal(a[k][fluid], c[k][fluid]), f"instance {k}"
    # the last call: graphs of ten steps, then pairs, then an odd step
    assert pa[0] == 1
    assert pc[0] == (2 if schedule[-1] % 10 % 2 == 0 else 1)
    assert pc[1] == pa[1] > 0


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_batch_two_steps_per_pass_larger_chunks_bitwise(storage):
    """48 lattices of the benchmark's kinds and sizes (chunks of several
    rows, partial strips and chunks, masked and mask-free tasks): two steps
    per pass against one, bit for bit."""
    print_case("batch 48 lattices steps per pass 2 vs 1", storage)
    specs = I.batch_specs(count=48, seed=5)
    a, _ = _batch_run(specs, storage, 1, [12, 3])
    c, pc = _batch_run(specs, storage, 2, [12, 3])
    assert pc[0] == 1
    for k in range(len(specs)):
        fluid = np.broadcast_to(specs[k]["mask"] == 0, a[k].shape)
        assert np.array_equal(a[k][fluid], c[k][fluid]), f"instance {k}"


def test_batch_two_steps_per_pass_half_precision_falls_back():
    print_case("batch steps per pass 2, FP16 / BF16: one step per pass")
    specs = _small_specs(seed=4)[:3]
    for st in ("f16", "bf16"):
        a, _ = _batch_run(specs, st, 1, [6])
        c, pc = _batch_run(specs, st, 2, [6])
        assert pc[0] == 1
        for k in range(len(specs)):
            assert np.array_equal(a[k], c[k])
