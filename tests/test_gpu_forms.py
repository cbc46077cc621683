"""GPU runs of the remaining configurations, with their errors reported.

* Precision form: D3Q19 Taylor-Green vortex at 64^3 (the FP64 oracle's copy
  of the 512^3 setup), FP64 / FP32 / FP16 / BF16 storage against the oracle
  at steps 500 and 1000: relative L2 of the velocity and of the vorticity
  (central differences).  At 1/tau- = 1.6 (the paper's stability optimum,
  Sec. 3.1) with the accuracy bars; at the configured Lambda = 1/4 at step
  500, reported.
* Double shear layer at 2048^2 (Sec. 3.1 shape): one FP64 step checked
  against the oracle at sampled nodes; FP32 vs FP64 on the GPU and the
  divergence step, if any, at Re = 1e4, 1e6, 1e7 (Lambda = 1/4) and at
  1/tau- = 1.6.  No printed numbers pin this flow ("parity unpinned" beyond
  the FP64 step check).
* 3D Taylor-Green vortex at 256^3, FP32: kinetic energy from the FP64 GPU
  reduction; the early decay follows exp(-6 nu k^2 t) to within 2 %, and at
  1/tau- = 1.6 the whole 5000-step energy history equals that of the
  FP64-storage run to 1e-4.
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


def _precision_errors(n, tp, lam, rho, u, checkpoints, storages):
    """Relative L2 errors of velocity and vorticity of each storage type
    against the FP64 oracle at each checkpoint step."""
    ora = O.Lattice(O.D3Q19, n, n, n, tp, lam)
    ora.init_equilibrium(rho, u)
    ref, done = {}, 0
    for t in checkpoints:
        ora.step(t - done)
        done = t
        ref[t] = ora.moments()[1]
    del ora
    errs = {}
    for storage in storages:
        print_case("precision form", f"{n}^3", storage, checkpoints)
        with P.Lattice(1, n, n, n, tp, lam, storage=storage) as G:
            G.init_equilibrium(rho, u)
            done = 0
            for t in checkpoints:
                G.step(t - done)
                done = t
                ug = G.moments()[1]
                errs[(storage, t)] = (A.rel_l2(ug, ref[t]),
                                      A.rel_l2(_vorticity(ug), _vorticity(ref[t])))
                print(f"precision form {n}^3 {storage} step {t}: velocity rel L2 "
                      f"{errs[(storage, t)][0]:.3e}, vorticity rel L2 {errs[(storage, t)][1]:.3e}",
                      flush=True)
    return errs


def test_precision_form_64cube_stable():
    """At the paper's 1/tau- = 1.6 (Sec. 3.1): the accuracy bars at steps 500
    and 1000 (nx = 64, so FP64 and FP32 run two steps per pass): FP64 within
    1e-12 of the oracle, FP32 within 1e-5 and FP16 within 1e-3 in relative
    L2 of the velocity; BF16 reported (bounded loosely)."""
    n = 64
    tp = I.tgv3d_params(n)["tau_plus"]
    lam = I.tau_minus_from_inverse(1.6, tp)
    rho, u = I.tgv3d(n, 0.05)
    errs = _precision_errors(n, tp, lam, rho, u, (500, 1000), ("f64", "f32", "f16", "bf16"))
    bars = {"f64": 1e-12, "f32": 1e-5, "f16": 1e-3, "bf16": 5e-2}
    for (storage, t), (eu, ew) in errs.items():
        assert eu < bars[storage], (storage, t, eu)
        assert ew < 5 * bars[storage], (storage, t, ew)
    for t in (500, 1000):
        assert errs[("f16", t)][0] < errs[("bf16", t)][0]


def test_precision_form_64cube_lambda_quarter():
    """At the configured Lambda = 1/4 (tau- = 262 at this tau+) the
    third-order modes are almost undamped (1 - 1/tau- = 0.996) and the FP64
    run itself blows up after about 1000 steps, so rounding noise of the
    storage is hardly damped: errors at step 500, reported with loose
    bounds (FP32 5e-5: the reading that 1e-5 does not hold at this Lambda is
    stated with the measured values in the design notes)."""
    n = 64
    tp = I.tgv3d_params(n)["tau_plus"]
    rho, u = I.tgv3d(n, 0.05)
    errs = _precision_errors(n, tp, 0.25, rho, u, (500,), ("f32", "f16", "bf16"))
    bounds = {"f32": 5e-5, "f16": 0.2, "bf16": 1.0}
    for (storage, t), (eu, ew) in errs.items():
        assert eu < bounds[storage] and ew < 5 * bounds[storage], (storage, eu, ew)
    assert errs[("f16", 500)][0] < errs[("bf16", 500)][0]


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
        # the library's divergence check every 100 steps
        G64.set_divergence_check(100)
        G32.set_divergence_check(100)
        t = 0
        while t < steps:
            try:
                G64.step(chunk)
                G32.step(chunk)
            except P.PtrtError as e:
                assert e.code == -5, e
                break
            t += chunk
        for key, G in (("fp64", G64), ("fp32", G32)):
            d = G.divergence_step()
            if d >= 0:
                res[f"diverged_{key}_at_step"] = d
        if not any(k.startswith("diverged") for k in res):
            m64, _ = G64.diagnostics()
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


def test_divergence_check_reports_the_first_non_finite_step():
    """The library's divergence check on the double shear layer at 128^2,
    Re = 1e4, Lambda = 1/4 (Sec. 3.1 shape), checked every 10 steps:
    ptrt_step returns PTRT_EDIVERGED (naming the step) once a check has seen
    a non-finite population, and the step ptrt_divergence_step reports is
    the first checked one at which the state is not finite: a fresh run of
    the same deterministic kernels is finite (ptrt_diagnostics) 10 steps
    earlier and not at that step.  The oracle's divergence step for the same
    flow is reported beside it: FP64 kernel and oracle agree to 1e-12 on
    stable flows, but here the unstable modes amplify their different
    rounding orders, so the two blow up within 10 % of each other, not at
    the same step."""
    from test_oracle_stability import N, RE, U0, divergence_step, dsl_lattice
    print_case("divergence check DSL 128^2 oracle")
    ref = divergence_step(dsl_lattice(), 2560)
    tp = I.tau_plus_from_nu(U0 * N / RE)
    rho, u = I.double_shear_layer(N, U0)
    got = {}
    for storage in ("f64", "f32"):
        print_case("divergence check DSL 128^2", storage)
        with P.Lattice(0, N, N, 1, tp, 0.25, storage=storage) as G:
            G.init_equilibrium(rho, u[:2])
            G.set_divergence_check(10)
            err = None
            try:
                for _ in range(400):
                    G.step(10)
            except P.PtrtError as e:
                err = e
            d = G.divergence_step()
        got[storage] = d
        print(f"DSL 128^2 Lambda=1/4 {storage}: library divergence step {d} (oracle {ref}); "
              f"ptrt_step raised: {err}", flush=True)
        assert err is not None and err.code == -5 and str(d) in str(err)
        assert d > 0 and d % 10 == 0
        with P.Lattice(0, N, N, 1, tp, 0.25, storage=storage) as G:
            G.init_equilibrium(rho, u[:2])
            G.step(d - 10)
            m, k = G.diagnostics()
            assert np.isfinite(m) and np.isfinite(k)
            G.step(10)
            with pytest.raises(P.PtrtError) as ei:
                G.diagnostics()
            assert ei.value.code == -5
    assert abs(got["f64"] - ref) <= 0.1 * ref


def _tgv3d_256_energy_series(storage, lam, n=256, U0=0.05):
    """E(t) every 250 steps up to 5000 (FP64 GPU reduction), the final mass
    and the divergence step from the library's check (every 50 steps)."""
    prm = I.tgv3d_params(n, U0)
    rho, u = I.tgv3d(n, U0)
    with P.Lattice(1, n, n, n, prm["tau_plus"], lam, storage=storage) as G:
        G.init_equilibrium(rho, u)
        del rho, u
        G.set_divergence_check(50)
        m0, e0 = G.diagnostics()
        series, m = [(0, e0)], m0
        for t in range(250, 5001, 250):
            try:
                G.step(250)
            except P.PtrtError as e:
                assert e.code == -5, e
                break
            m, e = G.diagnostics(raise_on_divergence=False)
            if not np.isfinite(e):
                break
            series.append((t, e))
        return series, m0, m, G.divergence_step()


@pytest.mark.parametrize("setting", ["Lambda=1/4", "1/tau-=1.6"])
def test_tgv3d_256_kinetic_energy_decay(setting):
    """3D vortex at 256^3, FP32, 5000 steps (configured length): the kinetic
    energy from the FP64 GPU reduction every 250 steps, the divergence step
    from the library's check (every 50 steps).  The early decay follows the
    viscous closed form exp(-6 nu k^2 t) within 2 % (kinetic-acoustic
    exchange at Ma ~ 0.09 keeps it from being closer).  At the configured
    Lambda = 1/4 the run diverges; at the paper's optimum 1/tau- = 1.6
    (Sec. 3.1) it stays finite, and its whole energy history, into the
    nonlinear stage, equals that of the same run in FP64 storage (whose
    update matches the oracle to 1e-12 elsewhere) to 1e-4."""
    print_case("3D TGV 256^3 FP32 kinetic energy", setting)
    n, U0 = 256, 0.05
    prm = I.tgv3d_params(n, U0)
    nu, tp = prm["nu"], prm["tau_plus"]
    lam = 0.25 if setting == "Lambda=1/4" else I.tau_minus_from_inverse(1.6, tp)
    k = 2 * np.pi / n
    series, m0, m, diverged = _tgv3d_256_energy_series("f32", lam)
    e0 = series[0][1]
    print(f"3D TGV 256^3 {setting} E(t)/E0:", [(t, round(e / e0, 5)) for t, e in series],
          f"diverged at step {diverged}" if diverged >= 0 else "finite through 5000 steps",
          flush=True)
    t1, e1 = series[2]
    assert abs(e1 / e0 - np.exp(-6 * nu * k * k * t1)) < 2e-2
    if setting == "Lambda=1/4":
        assert 0 < diverged <= 5000
        return
    assert diverged < 0 and len(series) == 21
    assert abs(m - m0) < 1e-5 * m0
    ref, _, _, d64 = _tgv3d_256_energy_series("f64", lam)
    assert d64 < 0 and len(ref) == 21
    dev = max(abs(e / er - 1) for (_, e), (_, er) in zip(series, ref))
    print(f"3D TGV 256^3 1/tau-=1.6: E(t) in FP32 vs FP64 storage, largest relative "
          f"difference over 5000 steps {dev:.2e}; E(5000)/E0 = {ref[-1][1] / ref[0][1]:.5f}",
          flush=True)
    assert dev < 1e-4


def test_precision_form_512_against_fp64_storage():
    """The precision form at its own size: the 512^3 vortex at the paper's
    1/tau- = 1.6, 1000 steps in FP32, FP16 and BF16 storage against the same
    run in FP64 storage on the GPU (whose update matches the oracle to
    1e-12 on the 64^3 copy).  FP32 stays within its 1e-5 bar.  With round
    to nearest the FP16 and BF16 errors are reported: the 1e-3 bar is
    defined on the 64^3 copy, and at 512^3 the change of a population per
    step is eight times smaller against the same storage resolution, so
    more of it is lost to rounding (measured 1.4e-3 for FP16 here against
    7.7e-4 at 64^3).  With stochastic rounding of the stores the loss is
    no longer systematic: FP16 meets the 1e-3 bar at this size."""
    print_case("precision form 512^3 against FP64 storage, 1000 steps")
    n, steps = 512, 1000
    tp = I.tgv3d_params(n)["tau_plus"]
    lam = I.tau_minus_from_inverse(1.6, tp)
    rho, u = I.tgv3d(n, 0.05)

    def run(storage):
        with P.Lattice(1, n, n, n, tp, lam, storage=storage) as G:
            G.init_equilibrium(rho, u)
            G.step(steps)
            return G.moments()[1]

    ref = run("f64")
    norm = np.sqrt(np.sum(ref * ref))
    bounds = {"f32": 1e-5, "f16": 5e-3, "bf16": 5e-2, "f16sr": 1e-3, "bf16sr": 1e-2}
    errs = {}
    for storage in ("f32", "f16", "bf16", "f16sr", "bf16sr"):
        ug = run(storage)
        ug -= ref
        errs[storage] = float(np.sqrt(np.sum(ug * ug)) / norm)
        del ug
        print(f"precision form 512^3 {storage} step {steps}: velocity rel L2 vs FP64 storage "
              f"{errs[storage]:.3e}", flush=True)
    for storage, e in errs.items():
        assert e < bounds[storage], (storage, e)
    assert errs["f32"] < errs["f16"] < errs["bf16"]
    assert errs["f16sr"] < errs["f16"] and errs["bf16sr"] < errs["bf16"]


def test_stochastic_rounding_is_reproducible():
    """Stochastic rounding draws its random bits from the stored value itself:
    two runs give the same bits, and the result differs from round to
    nearest; the initial state is rounded to nearest in both."""
    print_case("stochastic rounding reproducible")
    n = 32
    tp = I.tgv3d_params(n)["tau_plus"]
    rho, u = I.tgv3d(n, 0.05)
    out = {}
    for key, storage, steps in (("a", "f16sr", 50), ("b", "f16sr", 50), ("rne", "f16", 50),
                                ("sr0", "f16sr", 0), ("rne0", "f16", 0)):
        with P.Lattice(1, n, n, n, tp, 0.25, storage=storage) as G:
            G.init_equilibrium(rho, u)
            G.step(steps)
            out[key] = G.populations()
    assert np.array_equal(out["a"], out["b"])
    assert not np.array_equal(out["a"], out["rne"])
    assert np.array_equal(out["sr0"], out["rne0"])


def _ordered16(bits):
    """FP16 / BF16 bit patterns as integers in the order of their values:
    neighbouring representable values are one apart, both zeros are 0."""
    b = bits.astype(np.int32)
    mag = b & 0x7FFF
    return np.where(b & 0x8000, -mag, mag)


def _stored_bits(f, storage):
    """The stored 16-bit patterns of the shifted populations h = f - w (the
    FP64 read-back is h + w in FP64, so the nearest 16-bit value of f - w is
    h exactly)."""
    _, w = P.ptrt_velocity_set(P.PTRT_D3Q19)
    h = f - w[:, None, None, None]
    if storage.startswith("f16"):
        return h.astype(np.float16).view(np.uint16)
    return (h.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


@pytest.mark.parametrize("rne,sr", [("f16", "f16sr"), ("bf16", "bf16sr")])
def test_stochastic_rounding_picks_a_neighbour(rne, sr):
    """One step from the same state with round to nearest and with
    stochastic rounding: the collision is the same FP32 code, so every
    stochastically rounded value is the round-to-nearest result or the
    representable value next to it, across binade boundaries and zero too;
    the two differ in about a quarter of the values (the mean of min(p, 1 -
    p) for a uniform position p between the neighbours), and the
    stochastic choice moves up and down about equally often."""
    print_case("stochastic rounding picks a neighbour", rne, sr)
    n = 32
    tp = I.tgv3d_params(n)["tau_plus"]
    rho, u = I.tgv3d(n, 0.05)
    bits = {}
    for st in (rne, sr):
        with P.Lattice(1, n, n, n, tp, 0.25, storage=st) as G:
            G.init_equilibrium(rho, u)
            G.step(1)
            bits[st] = _stored_bits(G.populations(), st)
    d = _ordered16(bits[sr]) - _ordered16(bits[rne])
    differ = float(np.mean(d != 0))
    up = float(np.mean(d[d != 0] > 0))
    print(f"{sr}: {differ:.3f} of the values differ from {rne}, {up:.3f} of those upwards",
          flush=True)
    assert np.abs(d).max() <= 1
    assert 0.15 < differ < 0.35
    assert 0.45 < up < 0.55
