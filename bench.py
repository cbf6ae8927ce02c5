"""Benchmark of the FP64 structured-grid Euler hot path on one MI355X.

Workload (default): 3D Euler, one 256^3 block on a seeded smoothly jittered
periodic grid (node jitter <= 5 % of the spacing), Mach 0.8 free stream with
2 % random-phase velocity perturbations, MUSCL + van Albada, Roe flux,
4-stage Runge-Kutta with the global CFL step recomputed on the device.

A "step" is one full Runge-Kutta step (4 stages; each stage: ghost pack +
physical patches, unpack, fused residual/update kernel; the last stage also
reduces the next time step).  Inputs are resident in HBM before timing.

Prints one JSON line:
  value      FP64 cell-updates per second per RK stage (cells * stages * steps / time),
             the median over --repeats timed regions of exactly --steps steps
             (captured step graph; each region bracketed by synchronisation)
  roofline   the fused stage kernel against HBM bandwidth: algorithmic bytes
             per launch (190 B per cell-stage in 3D, 128 B in 2D, see the
             design notes) / mean launch time from HIP events recorded on the
             library's stream around every stage launch of the timed region
  fp64       the same launches against the FP64 vector peak, with the FP64
             operations per launch counted by rocprofv3 (FMA = 2) for this
             kernel source, when such a count is on record
  copy_gbs   a 1 GiB device-to-device copy on the same GPU (for context)
  stream_ceiling  a plain streaming kernel with the stage kernel's traffic per
             cell (20 doubles read, 5 written), the practical HBM ceiling the
             roofline also reports its fraction of
  cpu_baseline  the CPU oracle timed on a bounded sample of the same workload,
             with all host threads and with one
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
BYTES_PER_CELL_STAGE = {2: 128.0, 3: 190.0}  # mean over the 4 stages, metrics stored


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("stage_kernel.h", "device_math.h", "cfd_internal.h"):
        with open(os.path.join(ROOT, "paper_2012_02925_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(name, sha):
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % name)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha") != sha:
        return None
    return t


def copy_ceiling_gbs(nbytes=1 << 30, reps=5):
    """Read+write bandwidth of a plain device copy (torch's copy kernel)."""
    import torch

    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def make_case(workload, n):
    import synth

    if workload == "jittered_periodic_box":
        return synth.jittered_periodic_box(n=n, seed=0)
    if workload == "compression_ramp":
        return synth.compression_ramp(n, n)
    if workload == "patchwork":
        return synth.patchwork(seed=0)
    if workload == "gaussian_bump_periodic":
        return synth.gaussian_bump_periodic(n, n)
    raise SystemExit("unknown workload %s" % workload)


def cpu_baseline(workload, target_s=10.0):
    """The oracle, as it is, on a reduced copy of the workload: RK steps until
    at least target_s seconds of CPU work, once with all of torch's host
    threads and once with one thread; returns cell-stages/s for both."""
    import torch

    import oracle
    import synth

    if workload == "jittered_periodic_box":
        n = 64
        case = synth.jittered_periodic_box(n=n, seed=0)
        sample = "jittered_periodic_box %d^3 (same generator, reduced size)" % n
    else:
        case = make_case(workload, 128) if workload != "patchwork" else synth.patchwork(seed=0, side_lo=16, side_hi=64)
        sample = case.name + " (reduced size)"

    def timed(threads):
        old = torch.get_num_threads()
        torch.set_num_threads(threads)
        try:
            P = oracle.Problem(case)
            Q = P.initial_state()
            met = P.metrics()
            steps = 0
            t0 = time.perf_counter()
            while True:
                Q, _ = P.rk_step(Q, met)
                steps += 1
                el = time.perf_counter() - t0
                if el >= target_s:
                    break
            return case.ncells * P.stages * steps / el, steps, el
        finally:
            torch.set_num_threads(old)

    cores = torch.get_num_threads()
    rate, steps, el = timed(cores)
    rate1, steps1, el1 = timed(1)
    return {"value": rate, "unit": "cell-updates/s per RK stage", "cores": cores, "kind": "oracle",
            "sample": "%s, %d RK steps in %.1f s on %d threads" % (sample, steps, el, cores),
            "single_thread": {"value": rate1, "cores": 1,
                              "sample": "%s, %d RK steps in %.1f s on 1 thread" % (sample, steps1, el1)},
            "host_logical_cpus": os.cpu_count()}


def stream_ceiling(cells, reps=10):
    """Practical HBM ceiling for the stage kernel's traffic: a plain streaming
    kernel (cfd_stream_probe) reading 20 and writing 5 arrays of `cells`
    doubles (the 3D stage kernel's per-cell traffic after the first stage),
    with 8-byte and with 16-byte accesses; GB/s of each."""
    import ctypes

    import torch

    from paper_2012_02925_amd import capi

    lib = capi.load()
    src = torch.ones(20 * cells, dtype=torch.float64, device="cuda:0")
    dst = torch.empty(5 * cells, dtype=torch.float64, device="cuda:0")
    st = torch.cuda.current_stream()
    out = {"reads": 20, "writes": 5, "cells": cells}
    for vec in (1, 2):
        ms = ctypes.c_double()
        capi.check(lib.cfd_stream_probe(20, 5, vec, capi.dptr(src), capi.dptr(dst), cells, reps,
                                        ctypes.c_void_p(st.cuda_stream), ctypes.byref(ms)))
        out["gbs_%dB_access" % (8 * vec)] = 25.0 * 8 * cells / (ms.value * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    out["gbs"] = max(out["gbs_8B_access"], out["gbs_16B_access"])
    return out


def bench_batching(steps=20, warmup=2, repeats=3):
    """64-block patchwork (block sides uniform in [64, 512], all faces
    connected): one launch per block per phase (no graph) vs. batched launches
    over the tile list of every block -- one workgroup per tile, or persistent
    (as many workgroups as the GPU holds, walking the list) -- without and with
    the captured hipGraph of one RK step; tile shape autotuned for the batched
    launch.  Same kernels, bitwise-identical results.  Median over `repeats`
    timed regions each."""
    import statistics

    import torch

    import synth
    from paper_2012_02925_amd.solver import Solver

    case = synth.patchwork(seed=0)
    out = {"workload": case.name, "blocks": len(case.blocks), "cells": case.ncells}
    results = {}
    variant = None
    for mode, graph, label in (("batched", False, "batched"), ("batched", True, "batched_graph"),
                               ("persistent", False, "persistent"), ("persistent", True, "persistent_graph"),
                               ("per_block", False, "per_block")):
        s = Solver.from_case(case, device="cuda:0")
        if variant is None:
            variant = s.autotune(reps=3)
            out["tile_variant"] = variant
        else:
            s.set_variant(variant)
        s.set_exec(mode, graph)
        s.rk_step(warmup)
        torch.cuda.synchronize()
        times = []
        for _ in range(repeats):
            t0 = time.perf_counter()
            s.rk_step(steps)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        el = statistics.median(times)
        results[label] = case.ncells * case.scheme.rk_stages * steps / el
        out[label + "_ms_per_step"] = el * 1e3 / steps
        s.close()
    for label, rate in results.items():
        out[label + "_value"] = rate
    out["speedup_batching"] = results["batched"] / results["per_block"]
    out["speedup_persistent"] = results["persistent"] / results["per_block"]
    out["speedup_batching_and_graph"] = max(results["batched_graph"], results["persistent_graph"]) / results["per_block"]
    out["per_block_mode"] = "one launch per block per phase, no graph"
    out["unit"] = "cell-updates/s per RK stage"
    return out


def bench_flux_variants(workload, n, variant, steps=5, warmup=2):
    """Same workload and tile variant with each face flux (Roe, van Leer and
    Steger-Warming flux-vector splitting): mean stage-kernel time from HIP
    events and the resulting cell-updates/s per stage (the paper compares Roe
    with van Leer's splitting in Sec. 7.2)."""
    import torch

    from paper_2012_02925_amd.solver import Solver

    out = {}
    for flux in ("roe", "vanleer_fvs", "steger_warming"):
        case = make_case(workload, n)
        case.scheme.flux = flux
        s = Solver.from_case(case, device="cuda:0")
        s.set_variant(variant)
        s.rk_step(warmup)
        s.profile(True)
        torch.cuda.synchronize()
        s.rk_step(steps)
        kms, launches = s.kernel_time()
        s.profile(False)
        ms = kms / max(launches, 1)
        out[flux] = {"stage_kernel_ms": ms, "cell_updates_per_s": case.ncells / (ms * 1e-3),
                     "hbm_frac": BYTES_PER_CELL_STAGE[case.dim] * case.ncells / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        s.close()
        del s
        torch.cuda.empty_cache()
    return out


def bench_ramp(n=1024, steps=10, warmup=3):
    """The 2D 1024^2 compression ramp (supersonic inflow, extrapolated outflow,
    slip wall; van Leer + Roe, RK4): autotuned tiles, captured steps timed
    with events on the library stream, and the stage kernel's mean launch
    time from HIP events with its algorithmic HBM fraction."""
    import torch

    from paper_2012_02925_amd.solver import Solver

    case = make_case("compression_ramp", n)
    s = Solver.from_case(case, device="cuda:0")
    v = s.autotune(reps=3)
    s.rk_step(warmup)
    st = s.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    s.rk_step(steps)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    s.profile(True)
    s.rk_step(steps)
    kms, launches = s.kernel_time()
    s.profile(False)
    kms /= max(launches, 1)
    out = {"workload": case.name, "cells": case.ncells, "tile_variant": v, "ms_per_step": ms,
           "cell_updates_per_s": case.ncells * case.scheme.rk_stages / (ms * 1e-3),
           "stage_kernel_ms": kms,
           "stage_kernel_hbm_frac": BYTES_PER_CELL_STAGE[2] * case.ncells / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    s.close()
    del s
    torch.cuda.empty_cache()
    return out


def bench_navier_stokes(workload, n, variant, steps=20, warmup=5, reynolds=1.0e4):
    """Same workload and tiles as the headline with the laminar viscous terms
    switched on (mu = M / Re per unit length): whole RK steps timed with
    events on the library stream (captured step), against the Euler step; the
    paper reports the Navier-Stokes/Euler throughput ratio (about 0.7)."""
    import torch

    from paper_2012_02925_amd.solver import Solver

    out = {"workload": "%s_%d" % (workload, n), "reynolds_per_unit_length": reynolds}
    for label, visc in (("euler", False), ("navier_stokes", True)):
        case = make_case(workload, n)
        if visc:
            mach = float(case.meta.get("mach", 0.8))
            case.scheme.viscosity = mach / reynolds
            out["viscosity"] = case.scheme.viscosity
        s = Solver.from_case(case, device="cuda:0")
        s.set_variant(variant)
        s.rk_step(warmup)
        st = s.stream  # the library's stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(st)
        s.rk_step(steps)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out[label + "_ms_per_step"] = ms
        out[label + "_cell_updates_per_s"] = case.ncells * case.scheme.rk_stages / (ms * 1e-3)
        s.close()
        del s
        torch.cuda.empty_cache()
    out["ns_over_euler_throughput"] = out["euler_ms_per_step"] / out["navier_stokes_ms_per_step"]
    return out


def bench_adjoint(n=512, steps=50, every=10):
    """2D ramp n x n, van Albada (eps 1e-2), Roe, RK4 with the CFL step of the
    initial state held fixed; objective = integrated wall pressure after
    `steps` steps.  Forward: the unrolled steps with checkpoints; backward:
    segment replay + reverse steps with the hand-written VJP."""
    import torch

    import synth
    from paper_2012_02925_amd.autograd import unrolled_wall_pressure
    from paper_2012_02925_amd.solver import Solver

    probe = Solver.from_case(synth.compression_ramp(n, n, limiter="vanalbada"), device="cuda:0")
    dt = probe.time_step().item()
    probe.close()
    eps = 1e-2
    case = synth.compression_ramp(n, n, limiter="vanalbada", lim_eps=[eps, eps, eps, eps / 1.4], dt_fixed=dt)
    s = Solver.from_case(case, device="cuda:0", adjoint=True)
    theta = torch.tensor(case.meta["inflow"], requires_grad=True)
    nodes = torch.tensor(case.blocks[0].nodes).reshape(2, -1).to("cuda:0").requires_grad_(True)
    # warm-up passes of the same length (graph capture, allocator, stage-record buffer)
    for _ in range(2):
        J = unrolled_wall_pressure(s, theta, nodes, steps, every)
        J.backward()
        del J
        theta.grad = None
        nodes.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = unrolled_wall_pressure(s, theta, nodes, steps, every)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    # one residual vs one residual VJP
    Rb = torch.ones((s.nvar, s.ncells), dtype=torch.float64, device="cuda:0")
    s.residual()
    s.residual_vjp(Rb)
    torch.cuda.synchronize()
    reps = 20
    a0 = time.perf_counter()
    for _ in range(reps):
        s.residual()
    torch.cuda.synchronize()
    a1 = time.perf_counter()
    for _ in range(reps):
        s.residual_vjp(Rb)
    torch.cuda.synchronize()
    a2 = time.perf_counter()
    fwd, bwd = t1 - t0, t2 - t1
    return {"workload": "compression_ramp_%dx%d adjoint, %d steps, checkpoint every %d" % (n, n, steps, every),
            "dt_fixed": dt, "J": J.item(), "forward_ms": fwd * 1e3, "backward_ms": bwd * 1e3,
            "ratio": bwd / fwd, "residual_ms": (a1 - a0) * 1e3 / reps, "residual_vjp_ms": (a2 - a1) * 1e3 / reps,
            "vjp_over_residual": (a2 - a1) / (a1 - a0),
            "grad_theta": [float(x) for x in theta.grad], "grad_nodes_norm": float(nodes.grad.norm())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--repeats", type=int, default=5, help="timed regions of --steps steps; value = median")
    ap.add_argument("--workload", default="jittered_periodic_box")
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--variant", type=int, default=-1)
    ap.add_argument("--no-extras", action="store_true", help="skip the batching and adjoint measurements")
    ap.add_argument("--viscosity", type=float, default=0.0,
                    help="profiling aid: run the measured workload with the laminar viscous terms (mu)")
    ap.add_argument("--only-adjoint", action="store_true",
                    help="run only the adjoint measurement and print its JSON object")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of 1 GiB (torch copy kernel) to scale HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: cfdhip runs the whole workload on one GPU; --gpus %d is not supported "
              "(multi-GPU sharding is described in the design notes only)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2012_02925_amd.solver import Solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        n = (1 << 30) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))
        return
    if args.only_adjoint:
        print(json.dumps(bench_adjoint()))
        return
    case = make_case(args.workload, args.n)
    if args.viscosity > 0.0:
        case.scheme.viscosity = args.viscosity
        case.name += "_navier_stokes"
    print("[bench] workload %s, %d cells, building" % (case.name, case.ncells), file=sys.stderr, flush=True)
    s = Solver.from_case(case, device="cuda:0")
    chosen = None
    if args.variant >= 0:
        s.set_variant(args.variant)
    elif not args.no_autotune:
        chosen = s.autotune(reps=3)
    print("[bench] variant %d (tile %dx%d)" % (s.query("variant"), s.query("tile_x"), s.query("tile_y")),
          file=sys.stderr, flush=True)
    s.rk_step(args.warmup)
    torch.cuda.synchronize()

    # timed regions: `repeats` times exactly K steps (captured step graph),
    # each bracketed by synchronisation; the value is the median
    import statistics

    st = s.stream
    reps = []
    for _ in range(args.repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(st)
        s.rk_step(args.steps)
        e1.record(st)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        reps.append({"wall_s": t1 - t0, "event_ms": e0.elapsed_time(e1)})
    walls = [r["wall_s"] for r in reps]
    elapsed = statistics.median(walls)

    # kernel timing: K more steps with HIP events around every stage launch
    s.profile(True)
    torch.cuda.synchronize()
    s.rk_step(args.steps)
    torch.cuda.synchronize()
    kms, launches = s.kernel_time()
    s.profile(False)

    stages = case.scheme.rk_stages
    cells = case.ncells
    value = cells * stages * args.steps / elapsed
    dim = case.dim
    per_launch_bytes = BYTES_PER_CELL_STAGE[dim] * cells
    mean_launch_s = kms / 1e3 / max(launches, 1)
    achieved = per_launch_bytes / mean_launch_s / 1e9
    sha = kernel_source_sha()
    kname = "stage_kernel_%s" % case.name
    traffic = load_traffic(kname, sha)
    Q = s.get_state()
    finite = bool(torch.isfinite(Q).all().item())
    variant = s.query("variant")
    s.close()
    del s, Q
    torch.cuda.empty_cache()
    copy_gbs = copy_ceiling_gbs()
    ceiling = stream_ceiling(cells) if dim == 3 else None

    out = {
        "metric": "FP64 cell-updates/s per RK stage + % HBM roofline; adjoint/forward time ratio",
        "value": value,
        "unit": "cell-updates/s per RK stage",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": case.name, "cells": cells, "dim": dim, "limiter": case.scheme.limiter,
                   "flux": "roe", "rk_stages": stages, "dt": "global CFL 0.5, device-side",
                   "tile_variant": variant, "autotuned": chosen is not None},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None if traffic is None else traffic["bytes_per_launch"],
                     "kernel": "cfd::stage_kernel", "bytes_per_cell_stage": BYTES_PER_CELL_STAGE[dim],
                     "mean_launch_ms": mean_launch_s * 1e3, "launches": launches,
                     "practical_ceiling_gbs": None if ceiling is None else ceiling["gbs"],
                     "frac_of_practical_ceiling": None if ceiling is None else achieved / ceiling["gbs"],
                     # the counters' bytes (reads + writes) over the same launch time
                     "traffic_gbs": None if traffic is None else traffic["bytes_per_launch"] / mean_launch_s / 1e9,
                     "traffic_frac": None if traffic is None else
                     traffic["bytes_per_launch"] / mean_launch_s / 1e9 / HBM_PEAK_GBS},
        "timing": {"repeats": args.repeats, "steps_per_repeat": args.steps,
                   "ms_per_step_each": [w * 1e3 / args.steps for w in walls],
                   "event_ms_per_step_each": [r["event_ms"] / args.steps for r in reps],
                   "median_ms_per_step": elapsed * 1e3 / args.steps,
                   "spread": (max(walls) - min(walls)) / elapsed,
                   "captured_step_graph": True},
        "copy_gbs": copy_gbs,
        "stream_ceiling": ceiling,
        "state_finite": finite,
        "kernel_source_sha": sha,
    }
    if traffic is not None and traffic.get("fp64_flops_per_launch"):
        fl = traffic["fp64_flops_per_launch"] / mean_launch_s / 1e12
        out["fp64"] = {"achieved": fl, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                       "frac": fl / FP64_VECTOR_PEAK_TFLOPS,
                       "flops_per_cell_stage": traffic["fp64_flops_per_launch"] / cells}
    if not args.no_extras:
        print("[bench] batching: 64-block patchwork, per-block vs batched+graph", file=sys.stderr, flush=True)
        out["batching"] = bench_batching()
        print("[bench] adjoint: 512^2 ramp, 50 unrolled steps", file=sys.stderr, flush=True)
        out["adjoint"] = bench_adjoint()
        print("[bench] face-flux variants on the same workload", file=sys.stderr, flush=True)
        out["flux_variants"] = bench_flux_variants(args.workload, args.n, out["config"]["tile_variant"])
        print("[bench] 2D 1024^2 compression ramp", file=sys.stderr, flush=True)
        out["ramp_2d"] = bench_ramp()
        print("[bench] laminar Navier-Stokes vs Euler on the same workload", file=sys.stderr, flush=True)
        out["navier_stokes"] = bench_navier_stokes(args.workload, args.n, out["config"]["tile_variant"])
        out["navier_stokes_2d"] = bench_navier_stokes("compression_ramp", 1024, 2, steps=50, warmup=10)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
