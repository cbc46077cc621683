"""Throughput of the P-TRT hot path on one MI355X.

Headline (``value``): MLUPS of the fused D3Q19 FP32 step on the 256^3
triply periodic Taylor-Green vortex (U0 = 0.05, Re = 1600, Lambda = 1/4),
inputs resident in HBM, timed with HIP events on the stream the kernels run
on.  The same JSON line carries the other forms of the metric:
D3Q19 512^3 with FP32 vs FP16 vs BF16 shifted storage (round to nearest and
stochastic rounding), the batched D2Q9
form (512 uneven lattices, graph-replayed two-step passes, one step per
pass with the autotuned tile plan, and the one-launch-per-lattice
comparison), and the two D2Q9 single-lattice
configurations (2048^2 double shear layer FP32, 64^2 Taylor-Green FP64),
the collision-model comparison (P-TRT, TRT-RLB, TRT with one and with two
steps per pass), D3Q27 (hybrid P-TRT, FP32 / FP16, and
its comparison models) on the 256^3 vortex, the forcing schemes (Scheme II
with the cubic correction, Scheme I) against the default, a 4096^2 FP64
channel with walls (one and two steps per pass), and the square cylinder
with open boundaries and the momentum-exchange force.

``roofline`` describes the dominant kernel of the headline: the pass that
runs two D3Q19 FP32 steps per launch (first step over each workgroup's
column and halo, kept in LDS; second step written back).  Its algorithmic
HBM bytes per launch (reported by the library: the state read once and
written once, 2 * 19 * 4 bytes per node for two steps) over the average
launch time, against the 8 TB/s HBM peak; beside it the MLUPS as a fraction
of the one-step roofline (8 TB/s over 2 * 19 * 4 bytes per node and step),
and a plain streaming kernel's bandwidth measured beside it.  ``traffic`` is
read from the committed rocprofv3 counter summary when it was taken on the
current kernel sources, else null.  ``cpu_baseline`` times the FP64 C oracle
on twelve steps of the same 256^3 lattice on the host cores (and on one
thread), and under ``other_workloads`` on bounded samples of the D2Q9
forms (the 64^2 vortex in full, 10 steps of the 2048^2 shear layer, 2
steps of each batch lattice).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--only FORM]
                       [--no-cpu] [--copy-calibration]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "k_step_d3q19_f32_256_traffic.json")
KERNEL_SOURCES = ["paper_2602_06686_amd/csrc/kernels.hpp", "paper_2602_06686_amd/csrc/collide.hpp",
                  "paper_2602_06686_amd/csrc/codec.hpp", "paper_2602_06686_amd/csrc/lattice.hpp",
                  "paper_2602_06686_amd/csrc/trt_rlb.hpp", "paper_2602_06686_amd/csrc/step_launch.hpp",
                  "paper_2602_06686_amd/csrc/step2.hpp",
                  "paper_2602_06686_amd/csrc/step_d3q19.hip", "paper_2602_06686_amd/csrc/ptrt_single.hip"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the kernel sources' code: comments and whitespace are left
    out, so that a counter summary stays valid across edits of comments."""
    import re
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as fh:
            code = re.sub(r"/\*.*?\*/|//[^\n]*", " ", fh.read(), flags=re.S)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()[:16]


WARM_MS = 300.0  # device time of the warm-up before each timed region (default)
WARM = [WARM_MS]  # the value in use (--warm-ms)


def warm_for(torch, stream, step_fn, ms=None, chunk=20, max_steps=None):
    """Run chunks of steps until `ms` of device time have passed (or
    max_steps are done).  After a change of load the clocks settle over tens
    of milliseconds; a fixed step count covers too little of that on large
    lattices and too much on small ones.  Returns (steps run, ms)."""
    ms = WARM[0] if ms is None else ms
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    done, el = 0, 0.0
    while el < ms and (max_steps is None or done < max_steps):
        step_fn(chunk)
        done += chunk
        e1.record(stream)
        e1.synchronize()
        el = e0.elapsed_time(e1)
    return done, el


WARM_MAX_STEPS = 400  # the 256^3 vortex at Lambda = 1/4 turns non-finite at step 1050


def self_warm(torch, stream, step_fn, ms=None, record=None):
    """Warm-up function: the measured lattice itself stepped for `ms` of
    device time (at most WARM_MAX_STEPS steps), right before the warm-up
    steps and the timed region, with no idle time in between.  After the
    device has idled for a few milliseconds (a host-to-device upload, or the
    one-time load of a kernel at its first launch, about 6 ms) the next
    passes speed up and then slow down for about a hundred passes (kernel
    trace of the 256^3 vortex: 0.61 ms for the first two-step pass, 0.78 ms
    by the sixth, back to 0.59 ms after about 100), so a short timed region
    must not follow such a gap.  One single step runs first: it loads the
    one-step kernel that an odd warm-up count launches just before the
    timed steps."""
    def fn():
        if (WARM[0] if ms is None else ms) <= 0:
            return
        step_fn(1)
        done, el = warm_for(torch, stream, step_fn, ms, max_steps=WARM_MAX_STEPS)
        if record is not None:
            record["steps"], record["ms"] = done + 1, el
    return fn


def timed_steps(torch, stream, step_fn, steps, warmup, warm_fn=None):
    """Run warm_fn (a time-based warm-up) if given and `warmup` steps, then
    time exactly `steps` steps with HIP events on `stream` (bracketed by
    device synchronisation).  Returns (event ms, wall s)."""
    if warm_fn is not None:
        warm_fn()
    if warmup:
        step_fn(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    step_fn(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1), wall


def pass_accounting(res, nodes):
    """Bandwidth figures of a timed run whose passes cover res["steps_per_pass"]
    steps and move res["pass_bytes"] (the library's algorithmic bytes: the
    state read once and written once per pass).  hbm_frac is the pass's own
    bytes over its time against the 8 TB/s peak; the one-step-equivalent
    figures (2 Q s bytes per node per step, what one step per pass would have
    to move at this node-update rate) are named as such: with two steps per
    pass they are not traffic and may exceed the peak."""
    res["pass_ms"] = res["ms_per_step"] * res["steps_per_pass"]
    res["pass_gbs"] = res["pass_bytes"] / (res["pass_ms"] * 1e-3) / 1e9
    res["hbm_frac"] = res["pass_gbs"] / HBM_PEAK_GBS
    res["one_step_equiv_gbs"] = res["bytes_per_node"] * nodes / (res["ms_per_step"] * 1e-3) / 1e9
    res["mlups_over_one_step_roofline"] = res["one_step_equiv_gbs"] / HBM_PEAK_GBS
    return res


def bench_single(P, torch, stream, lattice, shape, storage, init, tau_plus, Lambda, steps, warmup,
                 force=None, mask=None, diag=False, steps_per_pass=2, warm_ms=None):
    nz, ny, nx = shape

    def make():
        return P.Lattice(lattice, nx, ny, nz, tau_plus, Lambda, force=force, solid_mask=mask,
                         storage=storage, stream=stream, steps_per_pass=steps_per_pass)

    warm = {}
    warm_ms = WARM[0] if warm_ms is None else warm_ms
    with make() as L:
        rho, u = init()
        L.init_equilibrium(rho, u)
        del rho, u
        e0 = None
        if diag:
            m0, e0 = L.diagnostics(raise_on_divergence=False)
        ms, wall = timed_steps(torch, stream, L.step, steps, warmup,
                               self_warm(torch, stream, L.step, warm_ms, warm))
        nodes = nx * ny * nz
        res = {
            "shape": [nx, ny, nz], "storage": storage, "steps": steps, "warmup": warmup,
            "warm_up": warm,
            "ms_per_step": ms / steps, "mlups": nodes * steps / (ms * 1e-3) / 1e6,
            "wall_mlups": nodes * steps / wall / 1e6,
            "bytes_per_node": L.bytes_per_node,
        }
        # the kernel pass actually run (two steps per pass where allowed)
        res["steps_per_pass"], res["pass_bytes"] = L.last_pass()
        pass_accounting(res, nodes)
        if diag:
            m1, e1 = L.diagnostics(raise_on_divergence=False)
            res["mass_rel_change"] = abs(m1 - m0) / m0
            res["kinetic_energy_ratio"] = e1 / e0 if e0 else None
            res["steps_total"] = L.t
    return res


def form_d3q19(P, torch, stream, n, storage, steps, warmup, diag=False, inv_tau_minus=None,
               steps_per_pass=2):
    """D3Q19 3D Taylor-Green vortex; Lambda = 1/4, or the Lambda giving a
    fixed 1/tau- (the paper's stability optimum 1.6, used for the precision
    form, where Lambda = 1/4 makes the flow itself unstable)."""
    import lbm_inputs as I
    prm = I.tgv3d_params(n)
    tp = prm["tau_plus"]
    lam = 0.25 if inv_tau_minus is None else I.tau_minus_from_inverse(inv_tau_minus, tp)
    r = bench_single(P, torch, stream, P.PTRT_D3Q19, (n, n, n), storage,
                     lambda: I.tgv3d(n, 0.05), tp, lam, steps, warmup, diag=diag,
                     steps_per_pass=steps_per_pass)
    setting = "Lambda=1/4" if inv_tau_minus is None else f"1/tau-={inv_tau_minus}"
    r["workload"] = (f"D3Q19 P-TRT {storage.upper()} {n}^3 periodic 3D Taylor-Green vortex "
                     f"(U0=0.05, Re=1600, {setting})")
    return r


def form_dsl(P, torch, stream, steps, warmup):
    import lbm_inputs as I
    n, U0, Re = 2048, 0.05, 1e4
    tp = I.tau_plus_from_nu(U0 * n / Re)
    r = bench_single(P, torch, stream, P.PTRT_D2Q9, (1, n, n), "f32",
                     lambda: I.double_shear_layer(n, U0), tp, 0.25, steps, warmup)
    r["workload"] = "D2Q9 P-TRT FP32 2048^2 doubly periodic double shear layer (kappa=80, delta=0.05, U0=0.05, Re=1e4, Lambda=1/4)"
    r["note"] = "302 MB working set, partly resident in the 256 MB Infinity Cache: no HBM roofline claim"
    return r


def form_tgv64(P, torch, stream, steps, warmup):
    import lbm_inputs as I
    n = 64
    r = bench_single(P, torch, stream, P.PTRT_D2Q9, (1, n, n), "f64",
                     lambda: I.tgv2d(n, 0.05), I.tau_plus_from_nu(0.01), 0.25, steps, warmup)
    r["workload"] = "D2Q9 P-TRT FP64 64^2 Taylor-Green vortex (u0=0.05, nu=0.01, Lambda=1/4); launch-bound"
    return r


def form_batch(P, torch, stream, steps, warmup):
    import lbm_inputs as I
    specs = I.batch_specs()
    b = P.ptrt_batch_create(specs, "f32")
    try:
        P.ptrt_batch_set_stream(b, stream)
        # tile plan of the one-step launches (odd steps, one step per pass)
        plan = P.ptrt_batch_autotune(b)
        plan2 = P.ptrt_batch_get_plan2(b)
        nodes = P.ptrt_batch_nodes(b)
        bps = P.ptrt_batch_bytes_per_step(b)
        # two steps per pass (the default), then one step per pass; the
        # batch's flows are steady or creeping, so it warms up on itself
        step = lambda k: P.ptrt_batch_step(b, k)  # noqa: E731
        ms_f, _ = timed_steps(torch, stream, step, steps, warmup,
                              lambda: warm_for(torch, stream, step))
        spp, pass_bytes = P.ptrt_batch_last_pass(b)
        P.ptrt_batch_set_steps_per_pass(b, 1)
        ms_1, _ = timed_steps(torch, stream, step, steps, warmup,
                              lambda: warm_for(torch, stream, step))
        P.ptrt_batch_set_steps_per_pass(b, 2)
        sep_steps = max(10, steps // 10)
        ms_s, _ = timed_steps(torch, stream, lambda k: P.ptrt_batch_step_separate(b, k),
                              sep_steps, 2)
        fluid = nodes - sum(int(s["mask"].sum()) for s in specs)
    finally:
        P.ptrt_batch_destroy(b)
    mf = ms_f / steps
    m1 = ms_1 / steps
    return {
        "workload": "512 independent D2Q9 P-TRT FP32 lattices (nx, ny in [32, 512], seed 260206686): "
                    "256 force-driven channels + 256 periodic boxes with a square obstacle, per-instance tau+, Lambda=3/16",
        "instances": len(specs), "nodes": nodes, "fluid_nodes": fluid,
        "plan": {"tile_x": plan[0], "tile_y": plan[1], "blocks": plan[2], "xcd_order": plan[3]},
        "plan2": dict(zip(("rows", "masked_rows", "waves", "blocks", "concurrent"), plan2)),
        "steps": steps, "ms_per_step": mf,
        "mlups": nodes / (mf * 1e-3) / 1e6, "mflups": fluid / (mf * 1e-3) / 1e6,
        # the pass actually run: two steps per pass move the bytes of one step
        "steps_per_pass": spp, "pass_bytes": pass_bytes, "pass_ms": mf * spp,
        "pass_gbs": pass_bytes / (mf * spp * 1e-3) / 1e9,
        "hbm_frac": pass_bytes / (mf * spp * 1e-3) / 1e9 / HBM_PEAK_GBS,
        # what one step per pass would have to move at this rate (2 Q s + 1
        # bytes per node per step): not traffic, may exceed the peak
        "one_step_equiv_gbs": bps / (mf * 1e-3) / 1e9,
        "mlups_over_one_step_roofline": bps / (mf * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "one_step_per_pass": {"ms_per_step": m1, "mlups": nodes / (m1 * 1e-3) / 1e6,
                              "pass_gbs": bps / (m1 * 1e-3) / 1e9,
                              "hbm_frac": bps / (m1 * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "separate_launches": {"steps": sep_steps, "ms_per_step": ms_s / sep_steps,
                              "mlups": nodes / (ms_s / sep_steps * 1e-3) / 1e6},
        "speedup_vs_separate": (ms_s / sep_steps) / mf,
    }


def form_models(P, torch, stream, steps, warmup):
    """P-TRT against TRT-RLB (Hermite projection) and standard TRT kernels in
    the same harness: the paper's efficiency comparison (Table efficiency)
    on this GPU, for the D2Q9 shear layer and the D3Q19 vortex (FP32).  One
    step per pass, where every model is bound by HBM bandwidth, and two
    steps per pass, where the pass is bound by instruction issue and the
    models' arithmetic shows."""
    import lbm_inputs as I
    out = {}
    n2, U0 = 2048, 0.05
    tp2 = I.tau_plus_from_nu(U0 * n2 / 1e4)
    n3 = 256
    tp3 = I.tgv3d_params(n3)["tau_plus"]
    for lat, shape, tp, init, key in (
            (P.PTRT_D2Q9, (1, n2, n2), tp2, lambda: I.double_shear_layer(n2, U0), "d2q9_2048_dsl"),
            (P.PTRT_D3Q19, (n3, n3, n3), tp3, lambda: I.tgv3d(n3, U0), "d3q19_256_tgv")):
        nz, ny, nx = shape
        rho, u = init()
        res = {}
        for spp in (1, 2):
            sub = {}
            for model in ("ptrt", "trt-rlb", "trt"):
                with P.Lattice(lat, nx, ny, nz, tp, 0.25, storage="f32", stream=stream,
                               model=model, steps_per_pass=spp) as L:
                    L.init_equilibrium(rho, u)
                    ms, _ = timed_steps(torch, stream, L.step, steps, warmup,
                                        self_warm(torch, stream, L.step))
                    sub[model] = {"ms_per_step": ms / steps,
                                  "mlups": nx * ny * nz * steps / (ms * 1e-3) / 1e6,
                                  "steps_per_pass": L.last_pass()[0]}
            sub["trt_rlb_time_over_ptrt"] = sub["trt-rlb"]["ms_per_step"] / sub["ptrt"]["ms_per_step"]
            sub["trt_time_over_ptrt"] = sub["trt"]["ms_per_step"] / sub["ptrt"]["ms_per_step"]
            res["one_step_per_pass" if spp == 1 else "two_steps_per_pass"] = sub
        out[key] = res
    return out


def form_d3q27(P, torch, stream, steps, warmup):
    """D3Q27 (App. A.3) on the 256^3 vortex at 1/tau- = 1.6: the hybrid P-TRT
    in FP32 and FP16 storage, and the FP32 collision models (exact variant,
    TRT-RLB, standard TRT) in the same harness."""
    import lbm_inputs as I
    n = 256
    tp = I.tgv3d_params(n)["tau_plus"]
    lam = I.tau_minus_from_inverse(1.6, tp)
    rho, u = I.tgv3d(n, 0.05)
    out = {"workload": "D3Q27 256^3 periodic 3D Taylor-Green vortex (U0=0.05, Re=1600, 1/tau-=1.6)"}
    for storage, model in (("f32", "ptrt"), ("f16", "ptrt"), ("f32", "ptrt-exact"),
                           ("f32", "trt-rlb"), ("f32", "trt")):
        def make():
            return P.Lattice(P.PTRT_D3Q27, n, n, n, tp, lam, storage=storage, stream=stream,
                             model=model)
        with make() as L:
            L.init_equilibrium(rho, u)
            ms, _ = timed_steps(torch, stream, L.step, steps, warmup,
                                self_warm(torch, stream, L.step))
            bpn = L.bytes_per_node
        mps = ms / steps
        gbs = bpn * n ** 3 / (mps * 1e-3) / 1e9
        out[f"{model}_{storage}"] = {"ms_per_step": mps, "mlups": n ** 3 / (mps * 1e-3) / 1e6,
                                     "bytes_per_node": bpn, "achieved_gbs": gbs,
                                     "hbm_frac": gbs / HBM_PEAK_GBS}
    base = out["ptrt_f32"]["ms_per_step"]
    out["fp16_over_fp32"] = out["ptrt_f16"]["mlups"] / out["ptrt_f32"]["mlups"]
    for m in ("ptrt-exact", "trt-rlb", "trt"):
        out[f"{m}_time_over_ptrt"] = out[f"{m}_f32"]["ms_per_step"] / base
    return out


def form_forcing(P, torch, stream, steps, warmup):
    """Forcing schemes (Sec. 2.1) in the same harness, FP32: Scheme II
    (default), Scheme II with the cubic correction G_i (a Phi pass of Q reads
    and D writes per node before the fused step, which also reads Phi at the
    2D axis neighbours) and Scheme I (Guo), on the 256^3 D3Q19 vortex and
    the 2048^2 D2Q9 shear layer, each with a uniform acceleration of 1e-6."""
    import lbm_inputs as I
    out = {}
    n3, n2, U0 = 256, 2048, 0.05
    cases = ((P.PTRT_D3Q19, (n3, n3, n3), I.tgv3d_params(n3)["tau_plus"],
              lambda: I.tgv3d(n3, U0), 19, 3, "d3q19_256_tgv"),
             (P.PTRT_D2Q9, (1, n2, n2), I.tau_plus_from_nu(U0 * n2 / 1e4),
              lambda: I.double_shear_layer(n2, U0), 9, 2, "d2q9_2048_dsl"))
    for lat, shape, tp, init, Q, D, key in cases:
        nz, ny, nx = shape
        nodes = nx * ny * nz
        rho, u = init()
        res = {}
        for forcing in ("scheme2", "scheme2+g", "guo"):
            def make():
                return P.Lattice(lat, nx, ny, nz, tp, 0.25, force=[1e-6, 0, 0], storage="f32",
                           stream=stream, forcing=forcing, steps_per_pass=1)
            with make() as L:
                L.init_equilibrium(rho, u)
                ms, _ = timed_steps(torch, stream, L.step, steps, warmup,
                                    self_warm(torch, stream, L.step))
            mps = ms / steps
            alg = 2 * Q * 4 + (Q * 4 + 2 * D * 4 if forcing == "scheme2+g" else 0)
            res[forcing] = {"ms_per_step": mps, "mlups": nodes / (mps * 1e-3) / 1e6,
                            "algorithmic_bytes_per_node": alg,
                            "achieved_gbs": alg * nodes / (mps * 1e-3) / 1e9}
        res["g_time_over_scheme2"] = res["scheme2+g"]["ms_per_step"] / res["scheme2"]["ms_per_step"]
        res["guo_time_over_scheme2"] = res["guo"]["ms_per_step"] / res["scheme2"]["ms_per_step"]
        out[key] = res
    return out


def form_channel(P, torch, stream, steps, warmup):
    """Force-driven channel (the Sec. 3.3 geometry, at a bandwidth-sized
    lattice): D2Q9 FP64 4096^2, halfway bounce-back walls at y = 0 and
    ny - 1, Lambda = 3/16, tau+ = 0.8, g_x = 1e-8; one step per pass and
    two steps per pass (the wall rows' tasks through the masked kernel)."""
    import numpy as np
    n = 4096
    mask = np.zeros((1, n, n), dtype=np.uint8)
    mask[0, 0, :] = mask[0, -1, :] = 1
    out = {"workload": "D2Q9 P-TRT FP64 4096^2 channel (walls at y = 0 and 4095, g_x = 1e-8, "
                       "tau+ = 0.8, Lambda = 3/16), from rest"}

    def init():
        return np.ones((1, n, n)), np.zeros((2, 1, n, n))

    for spp in (1, 2):
        r = bench_single(P, torch, stream, P.PTRT_D2Q9, (1, n, n), "f64", init, 0.8, 3 / 16,
                         steps, warmup, force=[1e-8, 0, 0], mask=mask, steps_per_pass=spp)
        out[f"steps_per_pass_{spp}"] = r
    out["two_over_one"] = out["steps_per_pass_2"]["mlups"] / out["steps_per_pass_1"]["mlups"]
    return out


def form_cylinder(P, torch, stream, steps, warmup):
    """Creeping flow past a square cylinder (Sec. 3.4): D2Q9, D = 21,
    L = 50 D (1050^2 nodes), moving-wall inlet, Zou-He outlet, periodic y,
    Re = 0.1, T = 0.1, Lambda = 3/16; two steps per pass (open-boundary
    strips in the special launch) in FP64 and FP32 and the
    momentum-exchange reduction, from the uniform stream."""
    import numpy as np
    D, K, Re, T = 21, 50, 0.1, 0.1
    n = D * K
    uc = (T * Re) ** 0.5 / 3 ** 0.5
    tp = 3 * uc * D / Re + 0.5
    mask = np.zeros((1, n, n), dtype=np.uint8)
    c0 = n // 2 - D // 2
    mask[0, c0:c0 + D, c0:c0 + D] = 1
    u = np.zeros((3, 1, n, n))
    u[0] = uc
    out = {"workload": "D2Q9 P-TRT square cylinder 1050^2 (D=21, L=50D, Re=0.1, Ma=0.1, "
                       "velocity inlet + Zou-He outlet, Lambda=3/16)"}
    for storage in ("f64", "f32"):
        def make():
            return P.Lattice(0, n, n, 1, tp, 3 / 16, solid_mask=mask, storage=storage,
                             stream=stream, open_x=(uc, 1.0))
        with make() as L:
            L.init_equilibrium(None, u)
            ms, _ = timed_steps(torch, stream, L.step, steps, warmup,
                                self_warm(torch, stream, L.step))
            spp, pass_bytes = L.last_pass()
            t0 = time.perf_counter()
            for _ in range(10):
                F = L.momentum_exchange()
            mx = (time.perf_counter() - t0) / 10 * 1e3
            bpn = L.bytes_per_node
        mps = ms / steps
        out[storage] = {"ms_per_step": mps, "mlups": n * n / (mps * 1e-3) / 1e6,
                        "steps_per_pass": spp,
                        # the pass's own bytes over its time; the one-step
                        # figure is what one step per pass would have to
                        # move at this rate (not traffic, may exceed the peak)
                        "pass_gbs": pass_bytes / (mps * spp * 1e-3) / 1e9,
                        "one_step_equiv_gbs": bpn * n * n / (mps * 1e-3) / 1e9,
                        "momentum_exchange_ms_host": mx,
                        "cd_after_timed_steps": 2 * F[0] / (uc * uc * D)}
    return out


def cpu_baseline(n=256, steps=12):
    """The FP64 C oracle, as it is, on `steps` steps of the headline lattice."""
    import lbm_inputs as I
    from oracle import ptrt as O
    prm = I.tgv3d_params(n)
    rho, u = I.tgv3d(n, 0.05)
    L = O.Lattice(O.D3Q19, n, n, n, prm["tau_plus"], 0.25)
    L.init_equilibrium(rho, u)
    del rho, u
    cores = O.max_threads()
    t0 = time.perf_counter()
    L.step(steps)
    dt = time.perf_counter() - t0
    del L
    # the same oracle on one thread: two steps of a 96^3 lattice after one
    # untimed step (which also touches the memory)
    n1, s1 = 96, 2
    prm1 = I.tgv3d_params(n1)
    rho, u = I.tgv3d(n1, 0.05)
    L1 = O.Lattice(O.D3Q19, n1, n1, n1, prm1["tau_plus"], 0.25, nthreads=1)
    L1.init_equilibrium(rho, u)
    L1.step(1)
    t1 = time.perf_counter()
    L1.step(s1)
    dt1 = time.perf_counter() - t1
    return {"value": n ** 3 * steps / dt / 1e6, "unit": "MLUPS", "cores": cores,
            "kind": "oracle",
            "sample": f"{steps} steps of the same {n}^3 D3Q19 lattice (FP64 C oracle, OpenMP over nodes), {dt:.1f} s",
            "value_one_core": n1 ** 3 * s1 / dt1 / 1e6,
            "sample_one_core": f"{s1} steps of a {n1}^3 D3Q19 lattice on one thread, {dt1:.1f} s",
            "other_workloads": cpu_baseline_2d(cores)}


def cpu_baseline_2d(cores):
    """The same oracle on bounded samples of the D2Q9 workloads (all host
    threads): the 64^2 FP64 vortex in full (1000 steps), 10 steps of the
    2048^2 double shear layer, and 2 steps of every lattice of the
    512-lattice batch (walls, obstacles and forces as in the batch), one
    lattice after the other.  The thread count is passed explicitly: the
    one-thread run before leaves OpenMP's default at one thread."""
    import lbm_inputs as I
    from oracle import ptrt as O
    out = {}
    n = 64
    rho, u = I.tgv2d(n, 0.05)
    L = O.Lattice(O.D2Q9, n, n, 1, I.tau_plus_from_nu(0.01), 0.25, nthreads=cores)
    L.init_equilibrium(rho, u)
    t0 = time.perf_counter()
    L.step(1000)
    dt = time.perf_counter() - t0
    out["d2q9_64_f64_tgv"] = {"value": n * n * 1000 / dt / 1e6, "unit": "MLUPS", "cores": cores,
                              "sample": f"1000 steps of the 64^2 vortex (in full), {dt:.2f} s"}
    n, U0, steps = 2048, 0.05, 10
    rho, u = I.double_shear_layer(n, U0)
    L = O.Lattice(O.D2Q9, n, n, 1, I.tau_plus_from_nu(U0 * n / 1e4), 0.25, nthreads=cores)
    L.init_equilibrium(rho, u[:2])
    del rho, u
    t0 = time.perf_counter()
    L.step(steps)
    dt = time.perf_counter() - t0
    del L
    out["d2q9_2048_dsl"] = {"value": n * n * steps / dt / 1e6, "unit": "MLUPS", "cores": cores,
                            "sample": f"{steps} steps of the 2048^2 double shear layer, {dt:.1f} s"}
    steps, nodes, dt = 2, 0, 0.0
    for sp in I.batch_specs():
        L = O.Lattice(O.D2Q9, sp["nx"], sp["ny"], 1, sp["tau_plus"], sp["Lambda"], g=sp["g"],
                      solid=sp["mask"], nthreads=cores)
        L.init_equilibrium()
        t0 = time.perf_counter()
        L.step(steps)
        dt += time.perf_counter() - t0
        nodes += sp["nx"] * sp["ny"]
        del L
    out["batched_d2q9"] = {"value": nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": cores,
                           "sample": f"{steps} steps of each of the 512 batch lattices ({nodes} nodes), "
                                     f"one lattice at a time, {dt:.1f} s"}
    return out


def copy_calibration(torch, stream, nbytes=1 << 30):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    with torch.cuda.stream(stream):
        for _ in range(3):
            b.copy_(a)
    torch.cuda.synchronize()
    return {"copy_bytes_read": nbytes, "copy_bytes_written": nbytes}


def stream_rate(torch, stream, nbytes=1 << 30, reps=10):
    """Read + write bytes per second of a plain streaming kernel, PyTorch's
    elementwise multiply by 1 over a 1 GiB FP32 tensor (its vectorised
    kernel streams faster than the runtime's copy): the bandwidth a simple
    HBM-bound kernel reaches here, beside the 8 TB/s peak."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    with torch.cuda.stream(stream):
        ms, _ = timed_steps(torch, stream,
                            lambda n: [torch.mul(a, 1.0, out=b) for _ in range(n)], reps, 2)
    del a, b
    return 2.0 * nbytes * reps / (ms * 1e-3) / 1e9


def traffic_from_profile():
    """Per-launch HBM bytes of the headline kernel from the committed counter
    summary, if it was taken on the current kernel sources."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return None, "no counter summary"
    with open(PROFILE_TRAFFIC) as fh:
        prof = json.load(fh)
    if prof.get("kernel_source_hash") != kernel_source_hash():
        return None, "kernel changed since the counters were taken"
    return prof.get("bytes_per_launch"), "rocprofv3 FETCH_SIZE + WRITE_SIZE scaled by a device copy"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--only", default=None,
                    help="run one form: d3q19_256_f32, d3q19_512, batch, dsl2048, models, "
                         "d3q27, forcing, channel, cylinder, tgv64")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--warm-ms", type=float, default=WARM_MS,
                    help="device time of the warm-up before each timed region (0: none; "
                         "for counter collection, where every launch is profiled)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not a build)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2602_06686_amd import ptrt as P

    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    K, W = args.steps, args.warmup
    only = args.only
    WARM[0] = args.warm_ms

    if args.copy_calibration:
        log("copy calibration", copy_calibration(torch, stream))

    forms = {}
    head = None
    if only in (None, "d3q19_256_f32"):
        log("D3Q19 FP32 256^3")
        head = form_d3q19(P, torch, stream, 256, "f32", K, W, diag=True)
        log(json.dumps(head))
    if only in (None, "d3q19_512"):
        # the precision form compares storage types on the one-step kernel
        # (two steps per pass is built for FP32 only); the FP32 two-step
        # pass is reported beside it
        for st, spp, key in (("f32", 1, "d3q19_512_f32"), ("f16", 2, "d3q19_512_f16"),
                             ("bf16", 2, "d3q19_512_bf16"), ("f16sr", 2, "d3q19_512_f16sr"),
                             ("bf16sr", 2, "d3q19_512_bf16sr"),
                             ("f32", 2, "d3q19_512_f32_two_steps")):
            log(f"D3Q19 {st} 512^3 (steps per pass {spp})")
            forms[key] = form_d3q19(P, torch, stream, 512, st, max(20, K // 2), max(2, W // 2),
                                    inv_tau_minus=1.6, steps_per_pass=spp)
            log(json.dumps(forms[key]))
        f32 = forms["d3q19_512_f32"]["mlups"]
        forms["fp16_over_fp32_512"] = forms["d3q19_512_f16"]["mlups"] / f32
        forms["bf16_over_fp32_512"] = forms["d3q19_512_bf16"]["mlups"] / f32
        forms["fp16sr_over_fp32_512"] = forms["d3q19_512_f16sr"]["mlups"] / f32
        best = forms["d3q19_512_f32_two_steps"]["mlups"]
        forms["fp16_over_fp32_two_steps_512"] = forms["d3q19_512_f16"]["mlups"] / best
    if only in (None, "batch"):
        log("batched D2Q9")
        forms["batched_d2q9"] = form_batch(P, torch, stream, K, W)
        log(json.dumps(forms["batched_d2q9"]))
    if only in (None, "dsl2048"):
        log("D2Q9 FP32 2048^2")
        forms["d2q9_2048_f32"] = form_dsl(P, torch, stream, K, W)
    if only in (None, "models"):
        log("collision models")
        forms["models_fp32"] = form_models(P, torch, stream, max(20, K // 2), max(2, W // 2))
        log(json.dumps(forms["models_fp32"]))
    if only in (None, "d3q27"):
        log("D3Q27 256^3")
        forms["d3q27_256"] = form_d3q27(P, torch, stream, max(20, K // 2), max(2, W // 2))
        log(json.dumps(forms["d3q27_256"]))
    if only in (None, "forcing"):
        log("forcing schemes")
        forms["forcing_fp32"] = form_forcing(P, torch, stream, max(20, K // 2), max(2, W // 2))
        log(json.dumps(forms["forcing_fp32"]))
    if only in (None, "channel"):
        log("D2Q9 FP64 channel 4096^2")
        forms["channel_d2q9_4096_f64"] = form_channel(P, torch, stream, max(20, K // 2),
                                                      max(2, W // 2))
        log(json.dumps(forms["channel_d2q9_4096_f64"]))
    if only in (None, "cylinder"):
        log("square cylinder")
        forms["cylinder_d2q9"] = form_cylinder(P, torch, stream, K, W)
        log(json.dumps(forms["cylinder_d2q9"]))
    if only in (None, "tgv64"):
        log("D2Q9 FP64 64^2")
        forms["d2q9_64_f64"] = form_tgv64(P, torch, stream, 1000, 50)

    if head is None:
        print(json.dumps({"forms": forms}))
        return

    traffic, traffic_note = traffic_from_profile()
    n_nodes = 256 ** 3
    two = head["steps_per_pass"] == 2
    one_step_roof_mlups = HBM_PEAK_GBS * 1e9 / head["bytes_per_node"] / 1e6
    roof = {"bound": "hbm", "achieved": head["pass_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": head["pass_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": ("k_step2<D3Q19, float> (two steps per launch)" if two
                       else "k_step<D3Q19, float, MASK=false>"),
            "bytes_per_launch": head["pass_bytes"], "avg_launch_ms": head["pass_ms"],
            "steps_per_launch": head["steps_per_pass"],
            "one_step_bytes_per_node": head["bytes_per_node"],
            "one_step_roofline_mlups": one_step_roof_mlups,
            "mlups_over_one_step_roofline": head["mlups"] / one_step_roof_mlups,
            "traffic_source": traffic_note}
    ref = stream_rate(torch, stream)
    roof["stream_reference_gbs"] = ref
    roof["stream_reference"] = ("torch.mul(a, 1.0, out=b) over 1 GiB FP32 on the same stream, "
                                "read + write bytes per second")
    roof["achieved_over_stream_reference"] = head["pass_gbs"] / ref
    roof["one_step_roofline_at_stream_reference_mlups"] = ref * 1e9 / head["bytes_per_node"] / 1e6
    cpu = None
    if not args.no_cpu:
        log("CPU baseline (oracle)")
        cpu = cpu_baseline()
        log(json.dumps(cpu))
    line = {
        "metric": "MLUPS & % HBM roofline: D3Q19 P-TRT FP32 vs FP16-storage; batched D2Q9 MLUPS",
        "value": head["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": head["workload"], "lattice": "D3Q19", "nodes": n_nodes,
                   "storage": "f32", "layout": "SoA two-buffer pull", "parallelism": "single GPU"},
        "roofline": roof, "cpu_baseline": cpu, "forms": forms,
        "headline_detail": head,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
