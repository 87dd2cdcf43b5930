"""Benchmark: rays per second of the full per-ray pipeline (emit -> index-grid integration ->
thick lens -> sensor deposit) on one MI355X.

Default workload (tomo_piv_512): a Tomo-PIV image through a normal shock, 512^3 grid over
10 x 10 x 3 cm (tanh density step 1.2 -> 3.0 kg/m^3 over 0.2 mm), 1e5 particles inside the box
x 1e4 rays = 1e9 rays per image, f = 105 mm f/11 lens focused on the mid-plane, 2048^2 sensor of
10 um pixels read out as 16-bit, ds = 0.1 mm, FP32 integration; the same image again with FP64
steps in the bricks the precision calibration flags (at 1e-3 px).  The BOS-through-turbulence
workload (128^3 field, 5e7 rays) is reported beside it.

One step = one pbr_emit_and_trace call over the whole image (sensor cleared on the device first)
plus the 16-bit readout; the density field, sources and buffers are resident in HBM before timing
starts.  Prints one JSON line.  The CPU baseline is the FP64 oracle timed on a bounded prefix of
the same sources, on all host threads and on one.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP32 operations of one Runge-Kutta step of the method (eqs. 3, 5, 6), per field layout.  Three
# evaluations of D = n grad n, each a trilinear interpolation of four quantities plus n = 1 + dn
# and D = n grad n (4 operations), and 69 for the stage points and updates: A, B, C = h D (9),
# stage B point (15), stage C point (12), R update (18), T update (15).
#   cells: the interpolant from the cell's polynomial coefficients, 7 multiply-adds (14 operations)
#          per quantity: 3 * (4 * 14 + 4) + 69 = 249;
#   nodes: from the eight corner values, 7 linear interpolations a + t (b - a) (3 operations) per
#          quantity: 3 * (4 * 21 + 4) + 69 = 333.
FLOPS_PER_STEP = {"cells": 249, "nodes": 333}
PEAK_FP32_TFLOPS = 157.3  # MI355X vector FP32, published
PMC_FILES = {"turbulence_bos_128": os.path.join(ROOT, "profiles", "trace_turbulence_bos_128_pmc.json"),
             "tomo_piv_512": os.path.join(ROOT, "profiles", "tomo_piv_512_pmc.json")}
PMC_FILE = PMC_FILES["turbulence_bos_128"]


def _kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("trace.hip", "pbr_internal.h"):
        with open(os.path.join(ROOT, "paper_1812_05902_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profile(workload="turbulence_bos_128"):
    """The committed rocprofv3 counter summary of the workload's integration kernel, if it was taken
    on the current kernel source; else None."""
    try:
        with open(PMC_FILES[workload]) as fh:
            d = json.load(fh)
    except (OSError, ValueError, KeyError):
        return None
    return d if d.get("kernel_source_hash") == _kernel_source_hash() else None


def _traffic_from_profile(workload="turbulence_bos_128"):
    """HBM bytes per trace launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) or None."""
    d = _profile(workload)
    return d.get("hbm_bytes_per_launch") if d else None


HBM_PEAK_GBS = 8000.0
GATHER_BYTES_PER_STEP = 384  # the method's field reads per step: 3 evaluations x 8 corners x float4


def memory_roofline(steps_per_launch, kernel_ms, workload="turbulence_bos_128", peaks=None):
    """Memory-side view of the integration kernel: HBM and L2 traffic per launch from the committed
    counters (when current) over the live kernel time, and the method's algorithmic gather rate
    against the measured L2 read peak."""
    g = steps_per_launch * GATHER_BYTES_PER_STEP / (kernel_ms * 1e-3) / 1e9
    out = {"algorithmic_gather_bytes_per_step": GATHER_BYTES_PER_STEP, "algorithmic_gather_GBps": g}
    if peaks and peaks.get("l2_read_GBps"):
        out["algorithmic_gather_over_measured_l2_peak"] = g / peaks["l2_read_GBps"]
    d = _profile(workload)
    if d:
        hbm = d["hbm_bytes_per_launch"] / (kernel_ms * 1e-3) / 1e9
        out.update({"hbm_GBps": hbm, "hbm_frac": hbm / HBM_PEAK_GBS})
        if "l2_read_bytes_per_launch" in d:
            out["l2_read_GBps"] = d["l2_read_bytes_per_launch"] / (kernel_ms * 1e-3) / 1e9
    return out


def measured_peaks():
    """The device's ceilings measured by the library's probes (a few ms each)."""
    from paper_1812_05902_amd import pbr
    return {"fp32_fma_TFLOPs": pbr.pbr_probe_fma_rate(0, False) / 1e12,
            "fp64_fma_TFLOPs": pbr.pbr_probe_fma_rate(0, True) / 1e12,
            "l2_read_GBps": pbr.pbr_probe_read_bandwidth(0, 1 << 20, 1 << 35, False) / 1e9,
            "l2_scattered_read_GBps": pbr.pbr_probe_read_bandwidth(0, 1 << 20, 1 << 33, True) / 1e9,
            "hbm_read_GBps": pbr.pbr_probe_read_bandwidth(0, 1 << 33, 1 << 33, False) / 1e9,
            "lds_read_GBps": pbr.pbr_probe_lds_bandwidth(0) / 1e9,
            "u64_atomics_per_s": pbr.pbr_probe_u64_atomics(0, 1 << 22, 1 << 28)}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(o, scene, src, threads, target_s):
    """Rays/s of the oracle over the first sources of src on `threads` threads, about target_s of work:
    renders of growing prefixes (at most 8x per step, aiming at 0.8 target_s) until one takes at least
    half the target; the last one is the measurement."""
    def timed(n):
        t0 = time.perf_counter()
        o.render(src[:n], scene.rays_per_src, n_threads=threads, want_float=False)
        return time.perf_counter() - t0
    n = min(len(src), max(1, threads))
    while True:
        dt = timed(n)
        if dt >= 0.5 * target_s or n >= len(src):
            break
        n = min(len(src), max(n + 1, int(n * min(8.0, 0.8 * target_s / max(dt, 1e-3)))))
    rays = n * scene.rays_per_src
    return rays / dt, (f"first {n} of {len(src)} sources x {scene.rays_per_src} rays ({rays} rays, {dt:.1f} s, "
                       f"{threads} thread{'s' if threads > 1 else ''})")


def cpu_baseline(scene, rho, src, target_s: float = 15.0, single_s: float = 10.0):
    """FP64 oracle on a prefix of the sources: all host threads (OpenMP over sources), then one."""
    import oracle
    o = oracle.scene_oracle(scene, rho=rho)
    threads = oracle.num_threads()
    v, sample = _oracle_rate(o, scene, src, threads, target_s)
    v1, sample1 = _oracle_rate(o, scene, src, 1, single_s)
    return {"value": v, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": sample + "; FP64 oracle, same scene and sources as the GPU step",
            "single_core": {"value": v1, "sample": sample1},
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="tomo_piv_512",
                    choices=["tomo_piv_512", "turbulence_bos_128", "batch64", "surrogate256", "bos_fig4",
                             "piv_pair_512"],
                    help="tomo_piv_512 (default): the 1e9-ray Tomo-PIV image through a 512^3 shock field, with "
                         "the 128^3 BOS workload reported beside it; turbulence_bos_128: that BOS workload alone; "
                         "batch64: the 64 uneven images of inputs.batch_scenes in one graph-captured batch; "
                         "surrogate256: train the ray surrogate on a 256^3 turbulence field, then 1e9 rays "
                         "with and without it; bos_fig4: the BOS displacement check of sec. 4 (two renders, "
                         "per-dot displacement map, eq. 9 map); piv_pair_512: both frames of a Tomo-PIV pair "
                         "(particles moved by a vortex between them)")
    ap.add_argument("--epochs", type=int, default=8, help="surrogate256: training epochs")
    ap.add_argument("--field-layout", choices=["auto", "cells", "nodes"], default="auto",
                    help="field stored per cell (128 B) or per node (16 B); auto takes the faster measured "
                         "one per workload")
    ap.add_argument("--rays-per-chunk", type=int, default=1 << 24,
                    help="rays per trace chunk (64 bytes of ray state each; the bos_fig4 renders use one chunk)")
    ap.add_argument("--source-order", choices=["morton", "index"], default="morton",
                    help="tomo_piv_512: trace the particles in Morton order of their positions (computed in "
                         "every step; same image bit for bit) or in index order")
    ap.add_argument("--no-extra", action="store_true",
                    help="tomo_piv_512: leave out the shock-FP64 leg, the 128^3 BOS workload and the peak probes "
                         "(for profiling runs; the headline value is unchanged)")
    ap.add_argument("--mlp-forward", action="store_true",
                    help="only the surrogate network's forward pass (k_mlp_infer) over 2^22 rows of a randomly "
                         "initialised network, five timed passes (for counter runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy a 1 GiB device buffer 4 times (calibrates HBM byte counters)")
    ap.add_argument("--atomic-probe", action="store_true",
                    help="only measure the device's rate of 64-bit atomic additions (sensor-sized buffer)")
    ap.add_argument("--peaks", action="store_true", help="only run the library's peak probes")
    args = ap.parse_args()
    if args.atomic_probe:
        from paper_1812_05902_amd import pbr
        out = {}
        for slots in (1 << 20, 1 << 22):  # 1024^2 and 2048^2 sensors
            out[f"u64_atomics_per_s_{slots}_slots"] = pbr.pbr_probe_u64_atomics(0, slots, 1 << 28)
        print(json.dumps(out))
        return
    if args.mlp_forward:
        print(json.dumps(bench_mlp_forward()), flush=True)
        return
    if args.copy_probe:
        import torch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": a.numel() * 4, "copy_probe_bytes_written": b.numel() * 4,
                          "launches": 4}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the renderer has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.peaks:
        print(json.dumps(measured_peaks()), flush=True)
        return

    if args.workload == "batch64":
        return bench_batch(args)
    if args.workload == "surrogate256":
        return bench_surrogate(args)
    if args.workload == "tomo_piv_512":
        return bench_tomo(args)
    if args.workload == "bos_fig4":
        return bench_bos_fig4(args)
    if args.workload == "piv_pair_512":
        return bench_piv_pair(args)
    out = bench_turbulence(args)
    if not args.no_cpu_baseline:
        from paper_1812_05902_amd import inputs
        scene = inputs.turbulence_bos()
        out["cpu_baseline"] = cpu_baseline(scene, inputs.density(scene), inputs.sources(scene))
    print(json.dumps(out), flush=True)


def bench_turbulence(args, steps=None, warmup=None, peaks=None):
    """The BOS-through-turbulence workload: 128^3 k^-5/3 random-phase field (ratio 1.05) over a
    10 cm box, 50 000 dots x 1000 rays (5e7 rays per image), f = 105 mm f/11, 1024^2 sensor of
    10 um pixels, ds = 0.1 mm, per-cell field records.  Returns the bench record (no CPU baseline)."""
    import torch
    from paper_1812_05902_amd import inputs, pbr
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    layout = "nodes" if args.field_layout == "nodes" else "cells"
    scene = inputs.turbulence_bos()
    rho = inputs.density(scene)
    src = inputs.sources(scene)
    r = pbr.Renderer.from_scene(scene, rho=rho, rays_per_chunk=args.rays_per_chunk, nodes=layout == "nodes")
    src_dev = torch.as_tensor(src, device=r.device).contiguous()
    torch.cuda.synchronize()

    def step(stats):
        return r.emit_and_trace(src_dev, scene.rays_per_src, scene.ray_seed, scene.ds,
                                pbr.PBR_CLEAR_FIRST, stats=stats)

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    box_ms, box_launches, trace_ms, steps_total = 0.0, 0, 0.0, 0
    t0 = time.perf_counter()
    for _ in range(steps):
        # HIP events on the launch stream around each integration launch and around the trace
        st = step(True)
        box_ms += st["box_ms"]
        box_launches += st["box_launches"]
        trace_ms += st["trace_ms"]
        steps_total += st["rkn_steps"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    r.close()

    n_rays = scene.n_rays
    value = n_rays * steps / wall
    avg_ms = box_ms / box_launches
    fps = FLOPS_PER_STEP[layout]
    achieved = steps_total * fps / box_launches / (avg_ms * 1e-3) / 1e12
    return {
        "metric": "rays/sec on 1 MI355X (trace+lens+sensor)",
        "value": value,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "turbulence_bos_128", "grid": "128^3", "n_src": scene.n_src,
                   "rays_per_src": scene.rays_per_src, "rays_per_image": n_rays,
                   "sensor": f"{scene.width}x{scene.height}", "ds_m": scene.ds,
                   "rays_per_chunk": args.rays_per_chunk, "field_layout": layout,
                   "mean_rkn_steps_per_ray": steps_total / steps / n_rays},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": _traffic_from_profile("turbulence_bos_128"),
                     "kernel": f"k_box32<{'true' if layout == 'nodes' else 'false'}>",
                     "kernel_ms_per_launch": avg_ms,
                     "launches_per_step": box_launches / steps,
                     "trace_ms_per_step": trace_ms / steps,
                     "flops_per_rkn_step": fps},
        "memory": memory_roofline(steps_total / box_launches, avg_ms, "turbulence_bos_128", peaks),
    }


def bench_batch(args):
    """64 images of uneven particle counts, rays per particle, grids (64^3 / 128^3 / 256^3) and
    sensors (512^2 .. 2048^2) in one graph-captured batch, tuned by the library's autotuner."""
    import tempfile

    import torch
    from paper_1812_05902_amd import inputs, pbr

    scenes = inputs.batch_scenes(64)
    # field layout per image: "nodes" for all; "cells" and "auto" per-cell records for all (measured
    # faster here: with nodes for the 22 images of 256^3 the batch ran at 4.4e8 rays/s, cells 5.0e8)
    use_nodes = [args.field_layout == "nodes" for _ in scenes]
    t0 = time.perf_counter()
    rs, srcs = [], []
    for sc, nodes in zip(scenes, use_nodes):
        r = pbr.Renderer(rays_per_chunk=1 << 8)
        r.set_density_field(inputs.density(sc), sc.origin, sc.spacing, sc.K, sc.rho_inf, nodes=nodes)
        r.set_optics(sc.z_lens, sc.focal_length, sc.f_number, sc.thickness, sc.n_glass, sc.clear_radius,
                     sc.z_focus)
        r.set_sensor(sc.width, sc.height, sc.pitch, sc.z_sensor, sc.wavelength, sc.sigma_px, sc.dtau_with_pi)
        rs.append(r)
        srcs.append(inputs.sources(sc))
        torch.cuda.synchronize()
        del r._rho_keepalive
        if len(rs) % 8 == 0:
            print(f"set up {len(rs)}/{len(scenes)} images ({time.perf_counter() - t0:.1f} s)", file=sys.stderr,
                  flush=True)
    setup_s = time.perf_counter() - t0
    b = pbr.Batch(rs, srcs, [sc.rays_per_src for sc in scenes], [sc.ray_seed for sc in scenes],
                  [sc.ds for sc in scenes], round_rays=1 << 24)
    cache = os.path.join(tempfile.gettempdir(), "pbr_batch_tune.txt")
    cfg, rate = b.autotune(cache_path=cache, probe_rounds=2)
    for _ in range(args.warmup):
        b.run(stats=False)
    torch.cuda.synchronize()
    steps, steps_nodes, run_ms = 0, 0, 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = b.run(stats=True)
        run_ms += st["run_ms"]
        steps += st["rkn_steps"]
        steps_nodes += st["rkn_steps_nodes"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n_rays = sum(sc.n_rays for sc in scenes)
    flops = (steps - steps_nodes) * FLOPS_PER_STEP["cells"] + steps_nodes * FLOPS_PER_STEP["nodes"]
    achieved = flops / (run_ms * 1e-3) / 1e12
    out = {
        "metric": "rays/sec on 1 MI355X (trace+lens+sensor)", "value": n_rays * args.steps / wall,
        "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch64", "images": len(scenes), "rays_per_batch": n_rays,
                   "node_layout_images": int(sum(use_nodes)),
                   "rounds": st["rounds"], "autotuned": cfg, "probe_rays_per_ms": rate,
                   "mean_rkn_steps_per_ray": steps / args.steps / n_rays, "setup_s": setup_s},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "whole batch graph (emit + persistent k_box_batch + finish)",
                     "graph_ms_per_step": run_ms / args.steps, "flops_per_rkn_step": flops / max(steps, 1),
                     "rkn_steps_on_nodes": steps_nodes / max(steps, 1)},
    }
    print(json.dumps(out), flush=True)


def bench_tomo(args):
    """Tomo-PIV scale (the default): 512^3 shock field, 1e5 particles x 1e4 rays = 1e9 rays, 2048^2
    sensor with 16-bit readout inside the step; FP32 integration (the value), and again with FP64
    steps in the bricks the calibration flags (1e-3 px).  The dominant kernel is the integration of
    the FP32 leg: its average launch duration comes from HIP events recorded on the launch stream
    around every launch of the timed steps."""
    import torch
    from paper_1812_05902_amd import inputs, pbr

    extra = not args.no_extra
    sc = inputs.tomo_piv_shock()
    t0 = time.perf_counter()
    rho = inputs.density(sc)
    # the node layout unless told otherwise (faster on this fine grid); the shock-FP64 legs use the
    # same field after the precision calibration
    layout = "cells" if args.field_layout == "cells" else "nodes"
    rn = pbr.Renderer.from_scene(sc, rho=rho, nodes=layout == "nodes", rays_per_chunk=args.rays_per_chunk)
    rc = rn if extra else None
    rho_cpu = rho if not args.no_cpu_baseline else None
    del rho
    src_np = inputs.sources(sc)
    src = torch.as_tensor(src_np, device=rn.device).contiguous()
    out16 = torch.empty(sc.height, sc.width, dtype=torch.int16, device=rn.device)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    cal = rc.calibrate_precision(sc.ds, tol_px=1e-3) if extra else None
    print(f"set up in {setup_s:.1f} s; calibration {cal}", file=sys.stderr, flush=True)

    # sources traced in Morton order of their positions (the order is computed inside every step;
    # rays keep their keys, so the image is the same bit for bit)
    morton = args.source_order == "morton"
    n_src = src.shape[0]
    order = torch.empty(n_src, dtype=torch.int64, device=rn.device)
    order_ws = torch.empty(max(pbr.pbr_source_order_morton_workspace_bytes(n_src), 8) // 8, dtype=torch.int64,
                           device=rn.device)
    for r in {id(x): x for x in (rn, rc) if x is not None}.values():
        pbr.pbr_set_source_order(r.ctx, order, n_src)

    def step(r, flags, stats):
        if morton:
            pbr.pbr_source_order_morton(r.ctx, src, n_src, order, order_ws)
            flags |= pbr.PBR_SOURCE_ORDER
        st = r.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds, pbr.PBR_CLEAR_FIRST | flags, stats=stats)
        pbr.pbr_read_image(r.ctx, pbr.PBR_FMT_U16, out16, 0.0)
        return st

    legs = [("fp32", rn, 0)] + ([("shock_fp64", rc, pbr.PBR_PREC_SHOCK_FP64),
                                 ("shock_fp64_tight", rc, pbr.PBR_PREC_SHOCK_FP64)] if extra else [])
    res = {}
    cal_tight = None
    for name, r, flags in legs:
        if name == "shock_fp64_tight":
            # a tolerance below FP32's error in the steep bricks: some bricks take FP64 steps
            cal_tight = r.calibrate_precision(sc.ds, tol_px=1e-7)
            print(f"calibration at 1e-7 px: {cal_tight}", file=sys.stderr, flush=True)
        for _ in range(args.warmup):
            step(r, flags, False)
        torch.cuda.synchronize()
        box_ms, launches, steps_total = 0.0, 0, 0
        t1 = time.perf_counter()
        for _ in range(args.steps):
            st = step(r, flags, True)
            box_ms += st["box_ms"]
            launches += st["box_launches"]
            steps_total += st["rkn_steps"]
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t1, box_ms, launches, steps_total, st)
        print(f"{name}: {res[name][0] / args.steps * 1e3:.1f} ms per image", file=sys.stderr, flush=True)
    wall, box_ms, launches, steps_total, st = res["fp32"]
    for r in {id(x): x for x in (rn, rc) if x is not None}.values():
        r.close()
    del rn, rc
    torch.cuda.empty_cache()
    fps = FLOPS_PER_STEP[layout]
    avg_ms = box_ms / launches
    achieved = steps_total * fps / launches / (avg_ms * 1e-3) / 1e12
    peaks = measured_peaks() if extra else None
    out = {
        "metric": "rays/sec on 1 MI355X (trace+lens+sensor)", "value": sc.n_rays * args.steps / wall,
        "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "tomo_piv_512", "grid": "512^3 over 10 x 10 x 3 cm, tanh shock 1.2 -> 3.0 kg/m^3",
                   "rays_per_chunk": args.rays_per_chunk, "n_src": sc.n_src, "rays_per_src": sc.rays_per_src,
                   "rays_per_image": sc.n_rays, "sensor": f"{sc.width}x{sc.height} u16", "ds_m": sc.ds,
                   "mean_rkn_steps_per_ray": steps_total / args.steps / sc.n_rays, "setup_s": setup_s,
                   "field_layout": layout, "source_order": args.source_order},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": _traffic_from_profile("tomo_piv_512"),
                     "kernel": f"k_box32<{'true' if layout == 'nodes' else 'false'}>",
                     "kernel_ms_per_launch": avg_ms, "launches_per_step": launches / args.steps,
                     "rkn_steps_per_launch": steps_total / launches, "flops_per_rkn_step": fps},
        "memory": memory_roofline(steps_total / launches, avg_ms, "tomo_piv_512", peaks),
    }
    if extra:
        out["shock_fp64"] = {"rays_per_s": sc.n_rays * args.steps / res["shock_fp64"][0],
                             "field_layout": layout, "fp64_bricks": cal["n_fp64"], "steep_bricks": cal["n_steep"],
                             "calibration_max_err_px": cal["max_err_px"],
                             "rkn_steps_fp64": res["shock_fp64"][4]["rkn_steps_fp64"]}
        st_t = res["shock_fp64_tight"][4]
        out["shock_fp64_tight"] = {"rays_per_s": sc.n_rays * args.steps / res["shock_fp64_tight"][0],
                                   "field_layout": layout, "calibration_tol_px": 1e-7,
                                   "fp64_bricks": cal_tight["n_fp64"], "steep_bricks": cal_tight["n_steep"],
                                   "rkn_steps_fp64": st_t["rkn_steps_fp64"], "rkn_steps": st_t["rkn_steps"]}
        out["measured_peaks"] = peaks
        out["roofline"]["frac_of_measured_fp32_fma_rate"] = achieved / peaks["fp32_fma_TFLOPs"]
        tb = bench_turbulence(args, steps=10, warmup=2, peaks=peaks)
        out["turbulence_bos_128"] = {"rays_per_s": tb["value"], "ms_per_step": tb["ms_per_step"],
                                     "config": tb["config"], "roofline": tb["roofline"], "memory": tb["memory"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, rho_cpu, src_np)
    print(json.dumps(out), flush=True)


def bench_bos_fig4(args):
    """The BOS experiment of sec. 4 (Fig. 4): a 257 x 257 x 81 z-stacked slice field with the
    Table 1 geometry, 5200 dots x 1000 rays rendered through the field and through the ambient
    medium with per-dot hit sums, then the bilinear map of the dot displacements and the eq. 9 map
    on a 64 x 64 grid.  One step = the whole experiment; value = rays of both renders per second."""
    import numpy as np
    import torch
    from paper_1812_05902_amd import inputs, pbr

    sc = inputs.bos_slice()
    sc0 = sc.replace(field="uniform", field_params=dict(rho0=sc.rho_inf))
    grid = inputs.map_grid(sc)
    # one trace chunk holds a whole render (no ragged second launch)
    nodes = args.field_layout != "cells"
    r1 = pbr.Renderer.from_scene(sc, rays_per_chunk=1 << 23, nodes=nodes)
    r0 = pbr.Renderer.from_scene(sc0, rays_per_chunk=1 << 23, nodes=nodes)
    src = torch.as_tensor(inputs.sources(sc), device=r1.device).contiguous()
    s1 = r1.set_source_sums(sc.n_src)
    s0 = r0.set_source_sums(sc.n_src)
    torch.cuda.synchronize()
    flags = pbr.PBR_CLEAR_FIRST | pbr.PBR_SOURCE_SUMS

    def step(stats):
        s1.zero_()
        s0.zero_()
        a = r1.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds, flags, stats=stats)
        b = r0.emit_and_trace(src, sc.rays_per_src, sc.ray_seed, sc.ds, flags, stats=stats)
        sim = r1.dot_displacement_map(s1, s0, src, grid)
        th = r1.bos_theory_map(grid)
        return a, b, sim, th

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    box_ms, launches, steps_total = 0.0, 0, 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a, b, sim, th = step(True)
        for st in (a, b):
            box_ms += st["box_ms"]
            launches += st["box_launches"]
            steps_total += st["rkn_steps"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim, th = sim.cpu().numpy().astype(np.float64), th.cpu().numpy().astype(np.float64)
    f = np.isfinite(sim[:, :, 0])
    x, y = sim[f].ravel(), th[f].ravel()
    achieved = steps_total * FLOPS_PER_STEP["nodes" if nodes else "cells"] / (box_ms * 1e-3) / 1e12
    n_rays = 2 * sc.n_rays
    out = {
        "metric": "rays/sec on 1 MI355X (trace+lens+sensor)", "value": n_rays * args.steps / wall,
        "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "bos_fig4", "grid": f"{sc.nx}x{sc.ny}x{sc.nz} z-stacked slice",
                   "n_src": sc.n_src, "rays_per_src": sc.rays_per_src, "renders_per_step": 2,
                   "rays_per_step": n_rays, "sensor": f"{sc.width}x{sc.height}", "ds_m": sc.ds,
                   "map": f"{grid[4]}x{grid[5]} nodes, {grid[2] * 1e3:.3f} mm",
                   "field_layout": "nodes" if nodes else "cells"},
        "fig4": {"corr_simulated_vs_eq9": float(np.corrcoef(x, y)[0, 1]),
                 "rms_simulated_over_eq9": float(np.sqrt((x * x).mean() / (y * y).mean())),
                 "eq9_max_px": float(np.abs(y).max()), "nodes_filled": int(f.sum())},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None, "kernel": "k_box32",
                     "kernel_ms_per_launch": box_ms / launches,
                     "flops_per_rkn_step": FLOPS_PER_STEP["nodes" if nodes else "cells"],
                     "mean_rkn_steps_per_ray": steps_total / args.steps / n_rays},
    }
    print(json.dumps(out), flush=True)


def bench_piv_pair(args):
    """A Tomo-PIV frame pair: the 512^3 shock field, 1e5 particles x 1e4 rays per frame, the second
    frame's particles moved by a Lamb-Oseen vortex in a uniform stream over 0.5 ms (RK4, 4 steps),
    both frames rendered with one seed and read out as 16-bit images.  One step = displacement +
    two renders + two readouts; value = rays of both frames per second."""
    import torch
    from paper_1812_05902_amd import inputs, pbr

    sc = inputs.tomo_piv_shock()
    t0 = time.perf_counter()
    rho = inputs.density(sc)
    nodes = args.field_layout != "cells"
    r = pbr.Renderer.from_scene(sc, rho=rho, nodes=nodes, rays_per_chunk=args.rays_per_chunk)
    del rho
    src = torch.as_tensor(inputs.sources(sc), device=r.device).contiguous()
    vel, org, sp, dt = inputs.piv_pair_flow()
    vel = torch.as_tensor(vel, device=r.device).contiguous()
    src_b = torch.empty_like(src)
    img = [torch.empty(sc.height, sc.width, dtype=torch.int16, device=r.device) for _ in range(2)]
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0

    def step(stats):
        pbr.pbr_displace_sources(r.ctx, src, src_b, vel, org, sp, dt, 4)
        out = []
        for k, s in enumerate((src, src_b)):
            out.append(r.emit_and_trace(s, sc.rays_per_src, sc.ray_seed, sc.ds, pbr.PBR_CLEAR_FIRST, stats=stats))
            pbr.pbr_read_image(r.ctx, pbr.PBR_FMT_U16, img[k], 0.0)
        return out

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    box_ms, launches, steps_total = 0.0, 0, 0
    t1 = time.perf_counter()
    for _ in range(args.steps):
        for st in step(True):
            box_ms += st["box_ms"]
            launches += st["box_launches"]
            steps_total += st["rkn_steps"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    moved = (src_b[:, :2] - src[:, :2]).abs().max().item()
    achieved = steps_total * FLOPS_PER_STEP["nodes" if nodes else "cells"] / (box_ms * 1e-3) / 1e12
    n_rays = 2 * sc.n_rays
    out = {
        "metric": "rays/sec on 1 MI355X (trace+lens+sensor)", "value": n_rays * args.steps / wall,
        "unit": "rays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "piv_pair_512", "grid": "512^3", "rays_per_chunk": args.rays_per_chunk, "n_src": sc.n_src, "rays_per_src": sc.rays_per_src,
                   "frames_per_step": 2, "rays_per_step": n_rays, "sensor": f"{sc.width}x{sc.height} u16",
                   "flow": "Lamb-Oseen vortex (0.05 m^2/s, core 1 cm) in a 0.2 m/s stream, 65^3 grid",
                   "frame_interval_s": dt, "max_particle_move_mm": moved * 1e3, "setup_s": setup_s,
                   "field_layout": "nodes" if nodes else "cells"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None, "kernel": "k_box32",
                     "kernel_ms_per_launch": box_ms / launches,
                     "flops_per_rkn_step": FLOPS_PER_STEP["nodes" if nodes else "cells"],
                     "mean_rkn_steps_per_ray": steps_total / args.steps / n_rays},
    }
    print(json.dumps(out), flush=True)


MLP_FLOPS_PER_ROW = 2 * (6 * 256 + 3 * 256 * 256 + 256 * 6)  # forward pass, multiply-adds x 2
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense bfloat16 matrix cores, published


def mlp_forward_rate(s, rows, device):
    """Average time of five forward passes of surrogate s over `rows` uniform inputs in [-1, 1)
    (one warm-up pass first), timed with events on torch's current stream, which the surrogate
    uses.  Returns (ms per pass, TFLOP/s)."""
    import torch
    from paper_1812_05902_amd import pbr
    x = torch.rand(rows, 6, device=device) * 2 - 1
    y = torch.empty_like(x)
    pbr.pbr_surrogate_forward(s.h, x, y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        pbr.pbr_surrogate_forward(s.h, x, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    return ms, MLP_FLOPS_PER_ROW * rows / (ms * 1e-3) / 1e12


def bench_mlp_forward():
    """The surrogate network's forward pass alone (the matrix-core kernel of the surrogate path)."""
    from paper_1812_05902_amd import pbr
    s = pbr.Surrogate(init_seed=3, max_rows=1024, ray_chunk=0)
    rows = 1 << 22
    ms, achieved = mlp_forward_rate(s, rows, "cuda")
    return {"kernel": "k_mlp_infer", "rows": rows, "ms_per_pass": ms, "achieved_TFLOPs": achieved,
            "peak_TFLOPs": PEAK_BF16_TFLOPS, "frac": achieved / PEAK_BF16_TFLOPS, "flops_per_row": MLP_FLOPS_PER_ROW}


def bench_surrogate(args):
    """Surrogate workload: train on 1e7 tracer rays (1e6 validation rays fix the fallback tiles),
    then render the same 1e9 evaluation rays with the plain tracer and with the surrogate, and
    compare a sample of their sensor hits ray by ray."""
    import numpy as np
    import torch
    from paper_1812_05902_amd import inputs, pbr

    ev, tr, va = inputs.surrogate_turbulence()
    t0 = time.perf_counter()
    rho = inputs.density(ev)
    r = pbr.Renderer.from_scene(ev, rho=rho, rays_per_chunk=args.rays_per_chunk)
    src_ev = torch.as_tensor(inputs.sources(ev), device=r.device).contiguous()
    src_tr = inputs.sources(tr)
    src_va = inputs.sources(va)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    s = pbr.Surrogate(init_seed=7, max_rows=1 << 18, ray_chunk=args.rays_per_chunk)
    rep = s.train(r, src_tr, tr.rays_per_src, src_va, va.rays_per_src, tr.ray_seed, va.ray_seed, ev.ds, batch=4096,
                  epochs=args.epochs, lr_max=1e-3, lr_min=1e-5, tol_px=0.01, tiles=64, min_tile_samples=8)
    print(json.dumps({"surrogate_training": rep}), flush=True)

    def render(flags, stats=True):
        return r.emit_and_trace(src_ev, ev.rays_per_src, ev.ray_seed, ev.ds, pbr.PBR_CLEAR_FIRST | flags,
                                stats=stats)

    s.attach(r)
    for _ in range(args.warmup):
        render(pbr.PBR_SURROGATE, stats=False)
    torch.cuda.synchronize()
    res = {}
    for name, flags in (("tracer", 0), ("surrogate", pbr.PBR_SURROGATE)):
        t1 = time.perf_counter()
        st = None
        for _ in range(args.steps):
            st = render(flags)
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t1, st)
        print(f"{name}: {res[name][0] / args.steps:.3f} s per image", file=sys.stderr, flush=True)
    # exit error on a sample of the rays: every 1000th ray of the image, both ways
    stride = 1000
    r.set_exit_recording(0, stride, ev.n_rays // stride)
    render(pbr.PBR_RECORD_EXITS, stats=False)
    rec_t = r.read_ray_exits()
    render(pbr.PBR_RECORD_EXITS | pbr.PBR_SURROGATE, stats=False)
    rec_s = r.read_ray_exits()
    surr = (rec_s["entered"] == 1) & (rec_s["n_steps"] == 0) & (rec_t["n_steps"] > 0)
    both = surr & (rec_s["status"] == 0) & (rec_t["status"] == 0)
    e = np.hypot(*(rec_s["sensor_px"][both] - rec_t["sensor_px"][both]).T) if both.any() else np.zeros(1)
    # matrix-core rate of the network alone: forward passes over 2^22 rows
    fwd_rows = 1 << 22
    fwd_ms, achieved = mlp_forward_rate(s, fwd_rows, r.device)
    wall_t, st_t = res["tracer"]
    wall_s, st_s = res["surrogate"]
    out = {
        "metric": "rays/sec on 1 MI355X (trace+lens+sensor); surrogate vs tracer at <=0.01 px",
        "value": ev.n_rays * args.steps / wall_s, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall_s / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f32", "data": "synthetic",
        "config": {"workload": "surrogate256", "grid": "256^3", "rays_per_chunk": args.rays_per_chunk, "rays_per_image": ev.n_rays,
                   "train_rays": tr.n_rays, "val_rays": va.n_rays, "tiles": "64x64", "tol_px": 0.01,
                   "epochs": args.epochs, "setup_s": setup_s},
        "tracer_rays_per_s": ev.n_rays * args.steps / wall_t,
        "speedup_vs_tracer": wall_t / wall_s,
        "surrogate_ray_fraction": st_s["surrogate_rays"] / ev.n_rays,
        "eligible_tiles": rep["eligible_tiles"],
        "exit_error_px_vs_tracer": {"rays_compared": int(both.sum()), "median": float(np.median(e)),
                                    "p99": float(np.quantile(e, 0.99)), "max": float(e.max())},
        "training": dict({k: rep[k] for k in ("train_samples", "steps", "loss_first_epoch", "loss_last_epoch",
                                              "train_ms", "val_median_px", "val_p99_px")},
                         us_per_adam_step=rep["train_ms"] / max(rep["steps"], 1) * 1e3, batch=4096),
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_BF16_TFLOPS, "traffic": None,
                     "kernel": "surrogate forward (all layers)", "rows": fwd_rows,
                     "ms_per_pass": fwd_ms, "flops_per_row": MLP_FLOPS_PER_ROW},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
