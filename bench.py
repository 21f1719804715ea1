"""Benchmark: FP64 RK4 grid-point updates per second of the BSSN + radiation
fluid hot path on one MI355X, on the 256^3 periodic configuration (box 16/H0,
Gaussian curvature perturbation mu = 0.6, sigma = 2.0, CFL 0.25).

One step = one classic RK4 step = 4 stages of the stage kernel (k_bssn_stage_lds), inputs
resident in HBM; the K timed steps are one library call (cosmos_rk4_steps), in which every stage
kernel writes the point fluxes of the state it produces beside it, for the next stage, so the
flux pre-pass (k_fluid_flux) runs once per call.
Prints one JSON line with the roofline of a stage (algorithmic bytes per stage /
average stage time, measured with HIP events on the launch stream around the
timed steps), the CPU oracle timed on a bounded sample of the same workload, and
the other forms of the metric as sub-objects: "batched" (runs/s of the 64-run
scan), "adjoint" (cost of the gradient relative to the forward run), "kt" (the
headline workload with the Kurganov-Tadmor fluid scheme), "scalar" (with the
massless scalar field) and "c2" (the 128^3 run with constraint norms every 10 steps).

Extra modes:
  --headline-only  skip the batched, adjoint, kt, scalar and c2 sub-objects
  --batched      only the 64-run threshold-scan workload (grid sizes drawn from
                 {48, 64, 80, 96}^3, mu in [0.3, 0.8], sigma in [0.8, 1.6], box 12/H0,
                 300 RK4 steps per run): runs/s of the batched, hipGraph-replayed form
                 against the same runs advanced one after another by the plain solver
  --adjoint      only the differentiation workload: 96^3, box 12/H0, mu = 0.55,
                 sigma = 1.2, 200 RK4 steps, checkpoint every 20; gradient of the centre
                 lapse in (mu, sigma) by the discrete adjoint, its cost relative to the
                 plain forward run, and central finite differences (h = 1e-6)
  --threshold    only the threshold search (32^3, box 12/H0, sigma = 1.2, 24 RK4 steps):
                 batched multisection + Newton with the adjoint derivative for the amplitude
                 whose centre lapse equals that of mu = 0.4371, against serial bisection
  --kt           only the headline workload with the Kurganov-Tadmor fluid scheme
                 (fluid_scheme 1), against the centred scheme on the same configuration
  --scalar       only the headline workload with the massless scalar field (iso-curvature mode
                 0.1 x Gaussian of width 2), against the plain run on the same configuration
  --c2           only the 128^3 evolution (box 12/H0, mu = 0.5, sigma = 1.5, 500 RK4 steps) with
                 the constraint norms every 10 steps, timed with and without the norms, and the
                 HBM roofline of one constraint evaluation
  --fmr          only the three-layer refined run (128^3 layer 0, two nested children at h/2 and
                 h/4 over central 64^3 cell boxes), against the same RK4 steps without refinement
  --triad-probe  only the STREAM triad probe (16 B read, 8 B written per element; a second
                 calibration point for the counters)
  --copy-probe   only a plain device-to-device copy of known size (calibrates
                 rocprofv3 FETCH_SIZE / WRITE_SIZE counters)
  --no-cpu       skip the CPU baseline leg
  --config K     fixed configuration (lds|direct:BXxBYxBZ:xcd|linear|blocked) instead of the autotuner

roofline.achievable holds this device's measured peaks (STREAM triad bandwidth and FP64 FMA
rate, libcosmos_probe.so) beside the published ones that roofline.frac uses.
roofline.traffic is the HBM bytes per stage launch from committed rocprofv3 counters
(profiles/k_bssn_stage_lds_256cubed_traffic.txt), reported only while the stage-kernel
sources, the configuration and the grid are the ones those counters were taken on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import torch

METRIC = "grid-point RK4 updates/sec FP64 at 256^3 (+ batched runs/sec, adjoint cost)"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# algorithmic HBM bytes per point per RK4 step: 16 passes over the 25 FP64 fields
# (stage 1 reads u, writes acc and U2; stages 2-3 read U_s, u, acc and write acc, U_{s+1};
#  stage 4 reads U4, acc and writes u): 16 * 25 * 8
BYTES_PER_POINT_STEP = 3200.0
LAUNCHES_PER_STEP = 4
# with the scalar field, per point and RK4 step: the plain 3200 B; the scalar stage reads 12
# geometry fields (chi, gt_ij, K, alpha, beta^i) and (phi, Pi) in every stage (112 B), acc and u_n
# of (phi, Pi) as its mode needs (0 / 32 / 32 / 16 B), and writes the 11 source arrays and the
# field's acc and next state (120 / 120 / 120 / 104 B): 992 B; the stage kernel reads 10 source
# arrays per stage (320 B)
SCALAR_BYTES_PER_POINT_STEP = 3200.0 + 992.0 + 320.0


def step_roofline(point_updates_per_s, bytes_per_point_step, kernels):
    """HBM roofline of whole RK4 steps from algorithmic bytes per point and step."""
    gbs = point_updates_per_s * bytes_per_point_step / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": kernels,
            "algorithmic_bytes_per_point_step": bytes_per_point_step}
HERE = os.path.dirname(os.path.abspath(__file__))
# sources that define the stage kernel; the committed counters apply only while they are unchanged
ORDER_NAMES = ("xcd", "linear", "blocked")
STAGE_SOURCES = ["bssn_device.hpp", "bssn_lds.hpp", "stage.hip.inc"]
TRAFFIC_FILE = os.path.join(HERE, "profiles", "k_bssn_stage_lds_256cubed_traffic.txt")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--triad-probe", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--no-tune", action="store_true", help="use the default tile instead of the autotuned one")
    ap.add_argument("--batched", action="store_true")
    ap.add_argument("--headline-only", action="store_true", help="no batched / adjoint / kt / scalar / c2 sub-objects")
    ap.add_argument("--batched-steps", type=int, default=30, help="timed steps (runs/s is scaled to 300 steps)")
    ap.add_argument("--adjoint", action="store_true")
    ap.add_argument("--threshold", action="store_true")
    ap.add_argument("--kt", action="store_true", help="only the Kurganov-Tadmor fluid-scheme leg")
    ap.add_argument("--scalar", action="store_true", help="only the massless-scalar-field leg")
    ap.add_argument("--c2", action="store_true", help="only the 128^3 run with constraint norms every 10 steps")
    ap.add_argument("--fmr", action="store_true", help="only the three-layer refined run")
    ap.add_argument("--adjoint-steps", type=int, default=200, help="RK4 steps of the differentiated run")
    ap.add_argument("--no-fd", action="store_true", help="skip the finite-difference check of the adjoint")
    ap.add_argument("--config", default=None,
                    help="fixed kernel configuration instead of autotuning, e.g. lds:16x4x4:blocked or direct:32x4x2:xcd")
    ap.add_argument("--source-hash", action="store_true", help="print the stage-kernel source hash and exit")
    return ap.parse_args()


def parse_config(text):
    kind, tile, order = text.split(":")
    kv = {"lds": 0, "direct": 1}[kind]
    return kv, tuple(int(x) for x in tile.split("x")), ORDER_NAMES.index(order)


def config_name(kv, tile, order):
    return f"{'lds' if kv == 0 else 'direct'}:{'x'.join(map(str, tile))}:{ORDER_NAMES[order]}"


def stage_source_hash():
    h = hashlib.sha256()
    for name in STAGE_SOURCES:
        with open(os.path.join(HERE, "paper_2606_02053_amd", "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def measured_counters(cfg, npts):
    """From the committed rocprofv3 counters of the stage kernel (TRAFFIC_FILE): HBM bytes per
    stage launch (FETCH_SIZE / WRITE_SIZE in KiB per dispatch, averaged over the four RK4 stages,
    each scaled by what the same counter reads for plain copy and triad kernels of known size)
    and the FP64 operations executed per point and stage (SQ_INSTS_VALU_{FMA,ADD,MUL}_F64 x 64
    lanes, an FMA counted as 2). (None, None) when the counters were taken on other kernel
    sources, another configuration or grid."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith(("#", " ", "|")))
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        if kv["source_hash"] != stage_source_hash() or kv["config"] != cfg or int(kv["points"]) != npts:
            return None, None
        fetch = float(kv["fetch_kib_per_dispatch"]) * float(kv["fetch_scale"])
        write = float(kv["write_kib_per_dispatch"]) * float(kv["write_scale"])
        return round((fetch + write) * 1024.0), float(kv["fp64_flop_per_point"])
    except (OSError, KeyError, ValueError):
        return None, None


def measured_traffic(cfg, npts):
    return measured_counters(cfg, npts)[0]


def machine_probes():
    """Achievable peaks of this device, beside the published ones the fractions use:
    STREAM triad a = b + s c over three 2 GiB FP64 arrays (24 B per element) and FP64
    FMA throughput (16 independent chains per thread, 1 M threads), each timed with HIP
    events over 20 launches on the launch stream (libcosmos_probe.so, cosmos_probe.h)."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(HERE, "paper_2606_02053_amd", "libcosmos_probe.so"))
    lib.cosmos_probe_triad.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                       ctypes.c_size_t, ctypes.c_void_p]
    lib.cosmos_probe_fma64.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    lib.cosmos_probe_fma64_flops.argtypes = [ctypes.c_size_t, ctypes.c_int]
    lib.cosmos_probe_fma64_flops.restype = ctypes.c_double
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)

    def timed(call, reps=20):
        for _ in range(3):
            call()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            call()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    n = 1 << 28
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.full((n,), 1.0, dtype=torch.float64, device="cuda")
    c = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")

    def triad():
        if lib.cosmos_probe_triad(a.data_ptr(), b.data_ptr(), c.data_ptr(), 3.0, n, sp) != 0:
            raise RuntimeError("cosmos_probe_triad failed")
    t_triad = timed(triad)
    if not bool((a == 7.0).all()):
        raise RuntimeError("triad probe produced wrong values")
    del a, b, c
    nthreads, iters = 1 << 20, 4096
    out = torch.empty(nthreads, dtype=torch.float64, device="cuda")

    def fma():
        if lib.cosmos_probe_fma64(out.data_ptr(), nthreads, iters, sp) != 0:
            raise RuntimeError("cosmos_probe_fma64 failed")
    t_fma = timed(fma)
    if not bool(torch.isfinite(out).all()):
        raise RuntimeError("FMA probe produced non-finite values")
    gbs = 24.0 * n / t_triad / 1e9
    tfl = lib.cosmos_probe_fma64_flops(nthreads, iters) / t_fma / 1e12
    return {"hbm_triad_gbs": round(gbs, 1), "hbm_triad_frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "fp64_fma_tflops": round(tfl, 2), "fp64_fma_frac_of_peak": round(tfl / FP64_PEAK_TFLOPS, 4),
            "triad_ms": round(t_triad * 1e3, 4), "fma_ms": round(t_fma * 1e3, 4)}


def copy_probe():
    nbytes = 1 << 30
    x = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": nbytes, "copy_probe_bytes_written": nbytes, "launches": 5}))


def triad_probe():
    """The STREAM triad of libcosmos_probe.so over three 2 GiB arrays, 5 launches: 16 bytes read
    and 8 written per element, a second known-byte point (beside the copy) for scaling the
    FETCH_SIZE / WRITE_SIZE counters."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(HERE, "paper_2606_02053_amd", "libcosmos_probe.so"))
    lib.cosmos_probe_triad.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                       ctypes.c_size_t, ctypes.c_void_p]
    n = 1 << 28
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.full((n,), 1.0, dtype=torch.float64, device="cuda")
    c = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for _ in range(5):
        if lib.cosmos_probe_triad(a.data_ptr(), b.data_ptr(), c.data_ptr(), 3.0, n, sp) != 0:
            raise RuntimeError("cosmos_probe_triad failed")
    torch.cuda.synchronize()
    print(json.dumps({"triad_probe_bytes_read": 16 * n, "triad_probe_bytes_written": 8 * n, "launches": 5}))


def op_counts():
    """Algorithmic FP64 operation counts (tests/golden/op_counts.json, written from the
    oracle's operation-counting scalar by tests/golden/make_golden.py):
    step_per_point (one RK4 step, centred scheme) and kt_prepass_per_point."""
    with open(os.path.join(HERE, "tests", "golden", "op_counts.json")) as f:
        return json.load(f)


def flops_per_point_step():
    return op_counts()["step_per_point"]


def cpu_baseline(n_steps: int, form: str = "plain"):
    """The oracle (serial FP64 C++, OpenMP over z-planes) on a bounded sample of
    the workload: RK4 steps on a 64^3 periodic grid with the benchmark's grid
    spacing h = 1/16 and perturbation parameters; its cost per point is the
    same as on the full grid. form: "plain", "kt" (fluid_scheme 1) or "scalar"
    (with the scalar field's iso-curvature mode 0.1 x Gaussian of width 2)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    s = oracle.Setup(n=(64, 64, 64), L=(4.0, 4.0, 4.0), fluid_scheme=1 if form == "kt" else 0)
    ini = oracle.Init(mu=0.6, sigma=2.0)
    dt = 0.25 * s.h[0]
    if form == "scalar":
        u, sc = oracle.init_fields_sc(s, ini, 0.1, 2.0)
        run = lambda k: oracle.rk4_sc(s, u, sc, 0.0, dt, k, parallel=True)  # noqa: E731
    else:
        u = oracle.init_fields(s, ini)
        run = lambda k: oracle.rk4(s, u, 0.0, dt, k, parallel=True)  # noqa: E731
    run(1)  # warm-up
    t0 = time.perf_counter()
    run(n_steps)
    el = time.perf_counter() - t0
    what = {"plain": "", "kt": ", Kurganov-Tadmor fluxes", "scalar": ", with the scalar field"}[form]
    out = {"value": 64 ** 3 * n_steps / el, "unit": "point-updates/s", "cores": threads, "kind": "oracle",
           "sample": f"{n_steps} RK4 steps of the CPU oracle on a 64^3 periodic grid (h = 1/16, mu = 0.6, "
                     f"sigma = 2.0{what}), OpenMP over z-planes, {el:.1f} s"}
    if form == "plain":
        # one core: 2 steps of a 32^3 grid with the same spacing (the cost per point does not depend on N)
        s1 = oracle.Setup(n=(32, 32, 32), L=(2.0, 2.0, 2.0))
        u1 = oracle.init_fields(s1, ini)
        t0 = time.perf_counter()
        oracle.rk4(s1, u1, 0.0, dt, 2, parallel=False)
        out["serial_value"] = 32 ** 3 * 2 / (time.perf_counter() - t0)
        out["host"] = host_cpu()
    return out


def host_cpu():
    """The host the CPU legs ran on: model name, logical CPUs, physical cores."""
    model, phys = None, set()
    try:
        cur = {}
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "model name" and model is None:
                model = v
            if k in ("physical id", "core id"):
                cur[k] = v
            if not line.strip() and cur:
                phys.add((cur.get("physical id"), cur.get("core id")))
                cur = {}
    except OSError:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "physical_cores": len(phys) or None,
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def batched_bench(a):
    import paper_2606_02053_amd as P
    from paper_2606_02053_amd import autotune
    from paper_2606_02053_amd.batch import Batch, draw_scan
    runs = draw_scan(64, seed=2606)
    total_steps = 300
    tile = (16, 4, 4)
    if not a.no_tune:  # untimed: the batched stage kernel's brick for this batch (cached)
        tile, _ = autotune.tune_batch(runs)
    b = Batch(runs, autotune.with_tile(P.make_params(), 0, tile, 1))
    b.init()
    b.capture(steps=10)  # 10 steps per replay: one flux pre-pass per 10 steps
    b.run(10)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.run(a.batched_steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / a.batched_steps
    st = b.status()
    if any(x["nonfinite"] for x in st):
        raise RuntimeError("non-finite values in the batched run")
    # the same runs, one after another, on the plain solver (its default configuration)
    plain_ms = 0.0
    for spec in runs:
        s = P.Solver(spec.n, spec.L, P.make_params())
        s.init(mu=spec.mu, sigma=spec.sigma)
        dt = 0.25 * spec.L / spec.n
        s.step(dt)
        torch.cuda.synchronize()
        e0.record(stream)
        s.run(3, dt)
        e1.record(stream)
        torch.cuda.synchronize()
        plain_ms += e0.elapsed_time(e1) / 3
    pts = sum(r.n ** 3 for r in runs)
    out = {"metric": "batched runs/sec (64-run threshold scan, 300 RK4 steps per run)",
           "value": len(runs) / (ms_step * total_steps / 1e3), "unit": "runs/s",
           "serial_plain_value": len(runs) / (plain_ms * total_steps / 1e3), "speedup_vs_serial": plain_ms / ms_step,
           "ms_per_batched_step": ms_step, "ms_per_serial_step_sum": plain_ms, "points_per_step": pts,
           "point_updates_per_s": pts / (ms_step / 1e3), "timed_steps": a.batched_steps,
           "roofline": step_roofline(pts / (ms_step / 1e3), BYTES_PER_POINT_STEP,
                                     "k_batch_stage over the (run, brick) work list + flux pre-pass, whole RK4 steps"),
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "64 runs, n from {48,64,80,96} (numpy default_rng(2606)), mu U[0.3,0.8], "
                                  "sigma U[0.8,1.6], L = 12/H0, CFL 0.25, hipGraph replays of 10 RK4 steps",
                      "brick": "x".join(map(str, tile))}}
    if not a.no_cpu:
        # the oracle's point-update rate on a 64^3 sample with the scan's box, as runs of the scan per second
        cb = cpu_baseline_scan(16)
        per_run = pts * total_steps / len(runs)
        out["cpu_baseline"] = {"value": cb["value"] / per_run, "unit": "runs/s", "cores": cb["cores"], "kind": "oracle",
                               "sample": cb["sample"] + f"; runs/s = point-updates/s / ({per_run:.4g} point-updates "
                                                       "per average run of the scan)"}
    return out


def cpu_baseline_scan(n_steps: int):
    """The oracle on a bounded sample of the scan: RK4 steps of one 64^3 run of box 12 (the
    scan's spacing at its middle size) at the middle of its mu, sigma ranges."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    s = oracle.Setup(n=(64, 64, 64), L=(12.0, 12.0, 12.0))
    u = oracle.init_fields(s, oracle.Init(mu=0.55, sigma=1.2))
    dt = 0.25 * s.h[0]
    oracle.rk4(s, u, 0.0, dt, 1, parallel=True)  # warm-up
    t0 = time.perf_counter()
    oracle.rk4(s, u, 0.0, dt, n_steps, parallel=True)
    el = time.perf_counter() - t0
    return {"value": 64 ** 3 * n_steps / el, "cores": threads,
            "sample": f"{n_steps} RK4 steps of the CPU oracle on one 64^3 run (L = 12, mu = 0.55, sigma = 1.2), "
                      f"OpenMP over z-planes, {el:.1f} s"}


def kt_bench(a, kv=0, tile=(16, 4, 4), order=2):
    """The headline workload with the Kurganov-Tadmor fluid scheme (fluid_scheme 1): RK4
    steps per second on 256^3, each stage a k_fluid_kt pre-pass (interface fluxes and their
    divergence) plus the stage kernel; timed like the headline, on the same kernel
    configuration, against the centred scheme measured back to back."""
    import paper_2606_02053_amd as P
    from paper_2606_02053_amd import autotune
    n, L = a.n, 16.0
    ms = {}
    for scheme in (1, 0):
        sol = P.Solver(n, L, autotune.with_tile(P.make_params(fluid_scheme=scheme), kv, tile, order))
        sol.init(mu=0.6, sigma=2.0)
        dt = sol.default_dt()
        for _ in range(a.warmup):
            sol.step(dt)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sol.run(a.steps, dt)
        e1.record(stream)
        torch.cuda.synchronize()
        ms[scheme] = e0.elapsed_time(e1) / a.steps
        st = sol.status()
        if st["nonfinite"] or st["prim_fail"]:
            raise RuntimeError(f"KT benchmark run (scheme {scheme}) went bad: {st}")
        del sol
    # the pre-pass alone (cosmos_kt_divergence: one k_fluid_kt launch), timed with HIP events
    # on the launch stream; algorithmic bytes: 15 fields read + 4 written per point
    g = P.make_grid(n, L)
    u = torch.empty((25, n, n, n), dtype=torch.float64, device="cuda")
    P.cosmos_init_fields(g, P.make_params(), P.make_init(mu=0.6, sigma=2.0), u)
    div = torch.empty((4, n, n, n), dtype=torch.float64, device="cuda")
    kp = P.make_params(fluid_scheme=1)
    for _ in range(3):
        P.cosmos_kt_divergence(g, kp, u, div)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 4 * a.steps
    e0.record(stream)
    for _ in range(reps):
        P.cosmos_kt_divergence(g, kp, u, div)
    e1.record(stream)
    torch.cuda.synchronize()
    pre_s = e0.elapsed_time(e1) / 1e3 / reps
    flops = op_counts()["kt_prepass_per_point"] * n ** 3
    byts = 19 * 8 * n ** 3
    del u, div
    roof = {"bound": "alu", "achieved": round(flops / pre_s / 1e12, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(flops / pre_s / 1e12 / FP64_PEAK_TFLOPS, 4), "traffic": None,
            "kernel": "k_fluid_kt (interface fluxes + divergence, one launch per stage)",
            "avg_launch_ms": round(pre_s * 1e3, 4), "algorithmic_flops_per_launch": round(flops),
            "algorithmic_bytes_per_launch": byts, "hbm_achieved_gbs": round(byts / pre_s / 1e9, 1),
            "hbm_frac": round(byts / pre_s / 1e9 / HBM_PEAK_GBS, 4)}
    return {"metric": "grid-point RK4 updates/sec FP64 at 256^3, Kurganov-Tadmor fluid fluxes",
            "value": n ** 3 / (ms[1] / 1e3), "unit": "point-updates/s", "ms_per_step": ms[1],
            "centred_ms_per_step": ms[0], "cost_vs_centred": ms[1] / ms[0], "steps": a.steps, "roofline": roof,
            **({} if a.no_cpu else {"cpu_baseline": cpu_baseline(5, "kt")}),
            "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"as the headline ({n}^3, L = 16/H0, mu = 0.6, sigma = 2.0, CFL 0.25) with "
                                   "fluid_scheme 1 (minmod reconstruction, characteristic-speed bound, no KO on "
                                   "the fluid)", "kernel_config": config_name(kv, tile, order)}}


def scalar_bench(a, kv=0, tile=(16, 4, 4), order=2):
    """The headline workload with the massless scalar field (iso-curvature mode Upsilon =
    0.1 x Gaussian of width 2 on the same zeta): RK4 steps per second on 256^3, each stage
    k_scalar_stage_lds (the field's stage update and its 11 source arrays) + the stage kernel
    with the sources (the flux pre-pass before the first stage); timed like the headline,
    against the plain run on the same configuration."""
    import paper_2606_02053_amd as P
    from paper_2606_02053_amd import autotune
    n, L = a.n, 16.0
    ms = {}
    for scalar in (True, False):
        sol = P.Solver(n, L, autotune.with_tile(P.make_params(), kv, tile, order), scalar=scalar)
        if scalar:
            sol.init(mu=0.6, sigma=2.0, sc_mu=0.1, sc_sigma=2.0)
        else:
            sol.init(mu=0.6, sigma=2.0)
        dt = sol.default_dt()
        for _ in range(a.warmup):
            sol.step(dt)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sol.run(a.steps, dt)
        e1.record(stream)
        torch.cuda.synchronize()
        ms[scalar] = e0.elapsed_time(e1) / a.steps
        st = sol.status()
        if st["nonfinite"] or st["prim_fail"]:
            raise RuntimeError(f"scalar benchmark run (scalar={scalar}) went bad: {st}")
        if scalar and not torch.isfinite(sol.s).all():
            raise RuntimeError("non-finite scalar field in the benchmark run")
        del sol
    return {"metric": "grid-point RK4 updates/sec FP64 at 256^3 with the massless scalar field",
            "value": n ** 3 / (ms[True] / 1e3), "unit": "point-updates/s", "ms_per_step": ms[True],
            "plain_ms_per_step": ms[False], "cost_vs_plain": ms[True] / ms[False], "steps": a.steps,
            "roofline": step_roofline(n ** 3 / (ms[True] / 1e3), SCALAR_BYTES_PER_POINT_STEP,
                                      "k_scalar_stage_lds + stage kernel with the sources (+ one flux pre-pass), "
                                      "whole RK4 steps"),
            **({} if a.no_cpu else {"cpu_baseline": cpu_baseline(5, "scalar")}),
            "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"as the headline ({n}^3, L = 16/H0, zeta mu = 0.6, sigma = 2.0, CFL 0.25) with "
                                   "the massless scalar field, iso-curvature Upsilon mu = 0.1, sigma = 2.0",
                       "kernel_config": config_name(kv, tile, order)}}


def c2_bench(a):
    """The 128^3 evolution (box 12/H0, Gaussian zeta mu = 0.5, sigma = 1.5, CFL 0.25, KO 0.1,
    500 RK4 steps) with the Hamiltonian/momentum constraint norms every 10 steps (51
    evaluations, t = 0 included, kept on the device until the end), timed with HIP events on
    the launch stream, and the same 500 steps without the norms; plus the roofline of one
    constraint evaluation (k_constraints + k_reduce_partials: every field read once, 200 B per
    point) timed over repeated evaluations of the final state."""
    import paper_2606_02053_amd as P
    n, L, nsteps, every = 128, 12.0, 500, 10
    npts = n ** 3
    ms = {}
    for with_norms in (True, False):
        sol = P.Solver(n, L)
        sol.init(mu=0.5, sigma=1.5)
        dt = sol.default_dt()
        hist = torch.empty((nsteps // every + 1, 8), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        if with_norms:
            P.cosmos_constraints(sol.grid, sol.params, sol.u, hist[0], ws=sol.ws)
        for i in range(nsteps // every):
            sol.run(every, dt)
            if with_norms:
                P.cosmos_constraints(sol.grid, sol.params, sol.u, hist[i + 1], ws=sol.ws)
        e1.record(stream)
        torch.cuda.synchronize()
        ms[with_norms] = e0.elapsed_time(e1)
        st = sol.status()
        if st["nonfinite"] or st["prim_fail"]:
            raise RuntimeError(f"128^3 run (norms: {with_norms}) went bad: {st}")
        if with_norms:
            h = hist.cpu().numpy()
            norms = {"H_rms_first": float(h[0, 0]), "H_rms_last": float(h[-1, 0]),
                     "H_rms_max": float(h[:, 0].max()), "M_rms_max": float(h[:, 2].max()),
                     "alpha_min_last": float(h[-1, 6])}
            # one constraint evaluation alone, repeated on the final state
            reps = 50
            P.cosmos_constraints(sol.grid, sol.params, sol.u, hist[0], ws=sol.ws)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(reps):
                P.cosmos_constraints(sol.grid, sol.params, sol.u, hist[0], ws=sol.ws)
            e1.record(stream)
            torch.cuda.synchronize()
            cons_s = e0.elapsed_time(e1) / 1e3 / reps
        del sol
    byts = 25 * 8 * npts
    roof = {"bound": "hbm", "achieved": round(byts / cons_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(byts / cons_s / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_constraints + k_reduce_partials (one constraint evaluation)",
            "avg_launch_ms": round(cons_s * 1e3, 4), "algorithmic_bytes_per_launch": byts}
    out = {"metric": "grid-point RK4 updates/sec FP64 at 128^3, constraint norms every 10 steps",
           "value": npts * nsteps / (ms[True] / 1e3), "unit": "point-updates/s",
           "value_without_norms": npts * nsteps / (ms[False] / 1e3),
           "ms_total": ms[True], "ms_total_without_norms": ms[False], "steps": nsteps,
           "norm_evaluations": nsteps // every + 1, "norms": norms, "roofline": roof,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "BSSN + radiation fluid classic RK4, 128^3 periodic grid, L = 12/H0, Gaussian "
                                  "zeta mu = 0.5 sigma = 1.5, CFL 0.25, KO eps 0.1, 500 steps, constraint "
                                  "norms every 10 steps"}}
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline_c2()
    return out


def cpu_baseline_c2():
    """The oracle on a bounded sample of the 128^3 cadence: 10 RK4 steps and one constraint
    evaluation on a 64^3 grid with the same spacing (h = 0.09375) and perturbation parameters."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    s = oracle.Setup(n=(64, 64, 64), L=(6.0, 6.0, 6.0))
    u = oracle.init_fields(s, oracle.Init(mu=0.5, sigma=1.5))
    dt = 0.25 * s.h[0]
    oracle.rk4(s, u, 0.0, dt, 1, parallel=True)  # warm-up
    t0 = time.perf_counter()
    u1, _ = oracle.rk4(s, u, 0.0, dt, 10, parallel=True)
    oracle.constraints(s, u1, parallel=True)
    el = time.perf_counter() - t0
    return {"value": 64 ** 3 * 10 / el, "unit": "point-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"10 RK4 steps + 1 constraint evaluation of the CPU oracle on a 64^3 periodic grid "
                      f"(h = 0.09375, mu = 0.5, sigma = 1.5), OpenMP over z-planes, {el:.1f} s"}


def adjoint_bench(a):
    from paper_2606_02053_amd.adjoint import RunConfig, central_lapse
    import paper_2606_02053_amd as P
    numel = P.NFIELDS * 96 ** 3
    keep_all = 4 * a.adjoint_steps * numel * 8 < 0.6 * torch.cuda.mem_get_info()[0]
    cfg = RunConfig(n=96, L=12.0, nsteps=a.adjoint_steps, checkpoint_every=20, keep_all=keep_all)
    t64 = lambda x, g=False: torch.tensor(x, dtype=torch.float64, requires_grad=g)  # noqa: E731
    # plain forward run (same steps, no checkpoints)
    s = P.Solver(cfg.n, cfg.L, cfg.params)
    s.init(mu=0.55, sigma=1.2)
    s.step(cfg.dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.init(mu=0.55, sigma=1.2)
    s.run(cfg.nsteps, cfg.dt)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    mu, sigma = t64(0.55, True), t64(1.2, True)
    t0 = time.perf_counter()
    J = central_lapse(mu, sigma, cfg)
    J.backward()
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    g = [mu.grad.item(), sigma.grad.item()]
    h = 1e-6
    fd = [None, None]
    if not a.no_fd:
        fd = []
        for dm, ds in ((h, 0.0), (0.0, h)):
            jp = central_lapse(t64(0.55 + dm), t64(1.2 + ds), cfg).item()
            jm = central_lapse(t64(0.55 - dm), t64(1.2 - ds), cfg).item()
            fd.append((jp - jm) / (2 * h))
    out = {"metric": "adjoint cost (forward + backward wall time / plain forward wall time)",
           "value": t_grad / t_fwd, "unit": "x forward", "higher_is_better": False,
           "forward_s": t_fwd, "forward_plus_adjoint_s": t_grad, "J": J.item(),
           "dJ_dmu": g[0], "dJ_dsigma": g[1], "fd_dJ_dmu": fd[0], "fd_dJ_dsigma": fd[1],
           "rel_diff_vs_fd": None if a.no_fd else [abs(g[i] - fd[i]) / abs(fd[i]) for i in range(2)],
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"96^3 periodic, L = 12/H0, Gaussian zeta mu = 0.55 sigma = 1.2, {cfg.nsteps} RK4 "
                                  "steps, CFL 0.25, J = centre lapse at the final time",
                      "states": (f"every step's start and stage states kept ({4 * cfg.nsteps * numel * 8 / 1e9:.0f} GB)"
                                 if keep_all else "checkpoint every 20 steps, segments recomputed")}}
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline_adjoint()
    return out


def c3b_bench(a, kv, tile, order):
    """The headline workload on the 384^3 grid (same box L = 16/H0 and perturbation, h = 1/24):
    whole RK4 steps timed with HIP events on the launch stream, in the headline's kernel
    configuration."""
    import paper_2606_02053_amd as P
    from paper_2606_02053_amd import autotune
    n, L, steps = 384, 16.0, max(1, min(a.steps, 10))
    sol = P.Solver(n, L)
    sol.init(mu=0.6, sigma=2.0)
    dt = sol.default_dt()
    sol.params = autotune.with_tile(sol.params, kv, tile, order)
    for _ in range(max(1, a.warmup)):
        sol.step(dt)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    sol.run(steps, dt)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    if sol.status()["nonfinite"]:
        raise RuntimeError("non-finite values in the 384^3 run")
    value = n ** 3 * steps / (ms / 1e3)
    out = {"metric": "grid-point RK4 updates/sec FP64 at 384^3", "value": value, "unit": "point-updates/s",
           "ms_per_step": ms / steps, "timed_steps": steps, "higher_is_better": True, "dtype": "f64",
           "data": "synthetic",
           "roofline": step_roofline(value, BYTES_PER_POINT_STEP, "k_bssn_stage_lds + k_fluid_flux, whole RK4 steps"),
           "config": {"workload": "BSSN + radiation fluid classic RK4, 384^3 periodic grid, L = 16/H0, Gaussian zeta "
                                  "mu = 0.6 sigma = 2.0, CFL 0.25, KO eps 0.1",
                      "kernel_config": config_name(kv, tile, order)}}
    del sol
    torch.cuda.empty_cache()
    return out


def fmr_bench(a):
    """Three refinement layers on the headline data (zeta Gaussian mu 0.6, sigma 2.0, box 16/H0):
    layer 0 a 128^3 periodic grid, layer 1 over its central 64^3 cells (h/2), layer 2 over the
    central 64^3 cells of layer 1 (h/4); Berger-Oliger sub-cycling (1, 2, 4 steps per layer-0
    step). Timed with HIP events on the launch stream; beside it the same RK4 steps of the three
    padded grids run alone, whose difference is the cost of the refinement (interpolation in
    space and time, injection, the parents' start-of-step copies)."""
    import paper_2606_02053_amd as P
    n, L = 128, 16.0
    boxes = [((32, 32, 32), (64, 64, 64)), ((44, 44, 44), (64, 64, 64))]
    steps = max(1, min(a.steps, 5))
    run = P.RefinedRun((n, n, n), (L, L, L), boxes)
    run.init(mu=0.6, sigma=2.0)
    dt = run.default_dt()
    run.step(dt)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        run.step(dt)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    st = run.status(0)
    if st["nonfinite"]:
        raise RuntimeError(f"non-finite values in the refined run: {st}")
    # the same RK4 steps of the three padded grids alone
    ev0.record(stream)
    for _ in range(steps):
        for k, reps in ((0, 1), (1, 2), (2, 4)):
            for _ in range(reps):
                P.cosmos_rk4_step(run.grids[k], run.params, 0.0, dt / reps, run.u0[k] if k < 2 else run.u[k],
                                  run.ws[k])
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_plain = ev0.elapsed_time(ev1) / steps
    interior = n ** 3 + 2 * 128 ** 3 + 4 * 128 ** 3
    padded = n ** 3 + 2 * 152 ** 3 + 4 * 152 ** 3
    value = interior / (ms / 1e3)
    out = {"metric": "refined-run point-updates/sec (interior points of all layers)", "value": value,
           "unit": "point-updates/s", "higher_is_better": True, "ms_per_layer0_step": ms,
           "ms_plain_rk4_steps": ms_plain, "refinement_overhead_frac": (ms - ms_plain) / ms,
           "uniform_equivalent_point_updates_per_s": (4 * n) ** 3 * 4 / (ms / 1e3),
           "timed_steps": steps, "dtype": "f64", "data": "synthetic",
           "roofline": step_roofline(padded / (ms / 1e3), BYTES_PER_POINT_STEP,
                                     "k_bssn_stage_lds + k_fluid_flux on the padded layers, k_fmr_pass_*, "
                                     "k_fmr_restrict"),
           "config": {"workload": "3 layers: 128^3 periodic, L = 16/H0, Gaussian zeta mu = 0.6 sigma = 2.0; layer 1 "
                                  "= central 64^3 cells at h/2 (152^3 padded), layer 2 = central 64^3 cells of layer 1 "
                                  "at h/4 (152^3 padded); buffer 12; CFL 0.25 on every layer"}}
    del run
    torch.cuda.empty_cache()
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline_fmr()
    return out


def cpu_baseline_fmr():
    """The oracle's refined run (oracle/fmr.py) on a bounded sample: a 24^3 periodic grid with one
    child over its central 16^3 cells (56^3 padded), eight layer-0 steps, OpenMP inside each step."""
    import oracle
    from oracle import fmr
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    s = oracle.Setup(n=(24, 24, 24), L=(3.0, 3.0, 3.0))  # h = 1/8 as layer 0 of the GPU run
    H = fmr.Hierarchy(s, [fmr.Box((4, 4, 4), (16, 16, 16))])
    st = H.init(oracle.init_fields(s, oracle.Init(mu=0.6, sigma=2.0)))
    dt = 0.25 * s.h[0]
    steps = 8
    t0 = time.perf_counter()
    for m in range(steps):
        H.step(st, m * dt, dt)
    sec = time.perf_counter() - t0
    interior = steps * (24 ** 3 + 2 * 32 ** 3)
    return {"value": interior / sec, "unit": "point-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} layer-0 steps of a 24^3 grid with one child over its central 16^3 cells (56^3 "
                      f"padded), {sec:.1f} s; interior points of both layers"}


def cpu_baseline_adjoint():
    """The oracle's discrete adjoint (taped reverse mode through one RK4 step) on a 24^3 grid with
    the differentiated run's grid spacing and data, beside its forward step: the CPU cost ratio
    (forward + adjoint) / forward, the unit of the adjoint leg (24^3: about 10 s of serial work on
    the GPU host)."""
    import numpy as np
    import oracle
    n = 24
    s = oracle.Setup(n=(n, n, n), L=(3.0, 3.0, 3.0))  # h = 12/96, as in the 96^3 run
    u = oracle.init_fields(s, oracle.Init(mu=0.55, sigma=1.2))
    lam = np.random.default_rng(5).standard_normal(u.shape)
    dt = 0.25 * s.h[0]
    t0 = time.perf_counter()
    for _ in range(20):
        oracle.rk4(s, u.copy(), 0.0, dt, 1)
    t_fwd = (time.perf_counter() - t0) / 20
    t0 = time.perf_counter()
    oracle.vjp(s, u, lam, "step", t=0.0, dt=dt)
    t_adj = time.perf_counter() - t0
    return {"value": (t_fwd + t_adj) / t_fwd, "unit": "x forward", "cores": 1, "kind": "oracle",
            "sample": f"one RK4 step and its taped reverse-mode adjoint on a 24^3 grid (h = 1/8, mu = 0.55, "
                      f"sigma = 1.2), serial: forward {t_fwd * 1e3:.1f} ms, adjoint {t_adj:.1f} s; "
                      f"{n ** 3 / t_adj:.1f} adjoint point-steps/s"}


def threshold_bench(a):
    """Time to locate the collapse threshold mu* in [0.3, 0.6] to 1e-10, with alpha_th the centre
    lapse after T of the run with mu = 0.4371 (so that mu* = 0.4371): batched multisection on the
    device collapse counters (3 rounds of 16 runs) + Newton with the adjoint derivative, against
    serial bisection with the plain solver (one run per bisection step, its cost measured). T is 24
    steps: up to there the lapse falls monotonically and is lowest at the centre, so the collapse
    test and the centre-lapse surrogate share their root (later the centre lapse rebounds after a
    minimum near step 30, and the two would part). A 32^3 run fills half the GPU, so 16 of them in
    one batch cost little more than one."""
    import math
    import paper_2606_02053_amd as P
    from paper_2606_02053_amd.threshold import find_threshold, find_threshold_interpolated
    n, L, sigma, nsteps, mu_ref, lo, hi, tol = 32, 12.0, 1.2, 24, 0.4371, 0.3, 0.6, 1e-10
    dt = 0.25 * L / n
    s = P.Solver(n, L)

    def plain_run(mu):
        s.init(mu=mu, sigma=sigma)
        for m in range(nsteps):
            P.cosmos_rk4_step(s.grid, s.params, m * dt, dt, s.u, s.ws)
        torch.cuda.synchronize()
        return float(s.u[17, n // 2, n // 2, n // 2])

    target = plain_run(mu_ref)
    t0 = time.perf_counter()
    plain_run(mu_ref)
    t_run = time.perf_counter() - t0
    t0 = time.perf_counter()
    res = find_threshold(sigma, lo, hi, target, n=n, L=L, nsteps=nsteps, K=16, rounds=3, tol=tol)
    torch.cuda.synchronize()
    t_search = time.perf_counter() - t0
    # batched rounds alone, each fitting the runs' centre lapse (no adjoint)
    t0 = time.perf_counter()
    res_i = find_threshold_interpolated(sigma, lo, hi, target, n=n, L=L, nsteps=nsteps, K=16, rounds=2, tol=tol)
    torch.cuda.synchronize()
    t_interp = time.perf_counter() - t0
    bisect_runs = math.ceil(math.log2((hi - lo) / tol))
    return {"metric": "threshold search time (batched multisection + adjoint Newton)", "value": t_search,
            "unit": "s", "higher_is_better": False, "mu_found": res.mu, "mu_reference": mu_ref,
            "abs_error": abs(res.mu - mu_ref), "J_at_mu": res.J, "dJ_dmu": res.dJ_dmu,
            "batched_runs": res.batched_runs, "newton_steps": res.newton_steps,
            "serial_bisection_runs": bisect_runs, "serial_run_s": t_run,
            "serial_bisection_s_estimate": bisect_runs * t_run,
            "interpolated_search": {"s": t_interp, "mu_found": res_i.mu, "abs_error": abs(res_i.mu - mu_ref),
                                    "batched_runs": res_i.batched_runs,
                                    "note": "batched rounds alone, the cubic through the runs' centre lapse"},
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"{n}^3 periodic, L = 12/H0, Gaussian zeta sigma = 1.2, {nsteps} RK4 steps, "
                                   f"CFL 0.25; mu* in [{lo}, {hi}] with alpha_centre(T; mu*) = alpha_centre(T; "
                                   f"{mu_ref}), tolerance {tol}"}}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU (the library has no multi-GPU path); got --gpus {a.gpus}",
              file=sys.stderr)
        sys.exit(2)
    if a.source_hash:
        print(stage_source_hash())
        return
    if a.copy_probe:
        copy_probe()
        return
    if a.triad_probe:
        triad_probe()
        return
    if a.batched:
        print(json.dumps(batched_bench(a)), flush=True)
        return
    if a.adjoint:
        print(json.dumps(adjoint_bench(a)), flush=True)
        return
    if a.threshold:
        print(json.dumps(threshold_bench(a)), flush=True)
        return
    if a.c2:
        print(json.dumps(c2_bench(a)), flush=True)
        return
    if a.fmr:
        print(json.dumps(fmr_bench(a)), flush=True)
        return
    if a.kt:
        kv, tile, order = parse_config(a.config) if a.config else (0, (16, 4, 4), 2)
        print(json.dumps(kt_bench(a, kv, tile, order)), flush=True)
        return
    if a.scalar:
        kv, tile, order = parse_config(a.config) if a.config else (0, (16, 4, 4), 2)
        print(json.dumps(scalar_bench(a, kv, tile, order)), flush=True)
        return
    import paper_2606_02053_amd as P
    from paper_2606_02053_amd import autotune
    n, L = a.n, 16.0
    sol = P.Solver(n, L)
    sol.init(mu=0.6, sigma=2.0)
    dt = sol.default_dt()
    kv, tile, order = 0, (16, 4, 4), 2
    if a.config:
        kv, tile, order = parse_config(a.config)
    elif not a.no_tune:  # untimed: picks kernel variant and brick (cached per arch and grid)
        (kv, tile, order), _ = autotune.tune(sol.grid, sol.params, sol.u, dt)
    sol.params = autotune.with_tile(sol.params, kv, tile, order)
    for _ in range(a.warmup):
        sol.step(dt)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()  # the library launches on this stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    sol.run(a.steps, dt)  # one library call: the fluid fluxes carried from step to step
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    st = sol.status()
    if st["nonfinite"]:
        raise RuntimeError(f"non-finite values during the benchmark: {st}")
    npts = n ** 3
    ms_step = ms / a.steps
    value = npts * a.steps / (ms / 1e3)
    launch_s = ms / 1e3 / (a.steps * LAUNCHES_PER_STEP)
    bytes_launch = BYTES_PER_POINT_STEP / LAUNCHES_PER_STEP * npts
    achieved = bytes_launch / launch_s / 1e9
    fl = flops_per_point_step()
    traffic, xfl = measured_counters(config_name(kv, tile, order), npts)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_unit": "bytes per launch", "algorithmic_bytes_per_launch": round(bytes_launch),
            "kernel": (f"k_bssn_stage_lds<{tile[0]},{tile[1]},{tile[2]}> (one RK4 stage; its point fluxes "
                       "written by the stage before, one k_fluid_flux pre-pass per call of K steps)"
                       if kv == 0 and tile == (16, 4, 4) else
                       (f"k_bssn_stage_lds<{tile[0]},{tile[1]},{tile[2]}>" if kv == 0 else "k_bssn_stage") +
                       " + k_fluid_flux pre-pass (one RK4 stage)"),
            "avg_launch_ms": round(launch_s * 1e3, 4),
            "fp64_tflops_algorithmic": round(fl * npts * a.steps / (ms / 1e3) / 1e12, 2),
            "fp64_frac": round(fl * npts * a.steps / (ms / 1e3) / 1e12 / FP64_PEAK_TFLOPS, 4)}
    # what the stage kernel executes (counters), beside the oracle's operation count above
    roof["fp64_flop_per_point_stage_executed"] = xfl
    roof["fp64_tflops_executed"] = None if xfl is None else round(xfl * npts / launch_s / 1e12, 2)
    roof["fp64_executed_frac"] = None if xfl is None else round(xfl * npts / launch_s / 1e12 / FP64_PEAK_TFLOPS, 4)
    ach = machine_probes()
    roof["achievable"] = ach
    roof["frac_of_achievable_hbm"] = round(achieved / ach["hbm_triad_gbs"], 4)
    out = {"metric": METRIC, "value": value, "unit": "point-updates/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"BSSN + radiation fluid (P = rho/3) classic RK4, {n}^3 periodic grid, L = 16/H0, "
                                  f"Gaussian zeta mu = 0.6 sigma = 2.0, CFL 0.25, KO eps 0.1",
                      "grid": n, "dt": dt, "kernel_variant": "lds-staged" if kv == 0 else "direct",
                      "tile": list(tile), "tile_order": ORDER_NAMES[order],
                      "kernel_config": config_name(kv, tile, order),
                      "parallelism": "single GPU"},
           "roofline": roof}
    if not a.headline_only:
        out["batched"] = batched_bench(a)
        out["adjoint"] = adjoint_bench(a)
        out["kt"] = kt_bench(a, kv, tile, order)
        # the LDS-staged kernel takes the scalar sources with the 16x4x4 brick only
        out["scalar"] = scalar_bench(a, kv, (16, 4, 4) if kv == 0 else tile, order)
        out["c2"] = c2_bench(a)
        out["c3b"] = c3b_bench(a, kv, tile, order)
        out["fmr"] = fmr_bench(a)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(a.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
