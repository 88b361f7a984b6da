#!/usr/bin/env python
"""Throughput of the Monte Carlo dust transport and the ray-tracer on one MI355X.

One step runs the whole hot path on the clumpy AGN torus (256^3 cells, 2000
clumps, 100 wavelengths, 1e8 packets, FP32 walk): packet transport with
immediate Bjorkman & Wood re-emission, Lucy estimator, modified random walk
in cells with Rosseland depth > 50, HG scattering events for 8 views, the
PAH second stage, Eq. 4 temperatures (FP64), then the ray-tracer forward
(512x512 pixels, 16 wavelengths, 8 views) and its adjoint. Inputs are
resident on the GPU before the timed region.

Prints one JSON line (see the keys below); the CPU oracle is timed on a
bounded sample of the same model as the reference baseline.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "photon packets/s & cell-crossings/s (256^3 torus); ray-trace px/s fwd+bwd"
HBM_PEAK = 8.0e12  # B/s, MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def walk_bytes(st, ns_thermal, rs=4):
    """Bytes the walk kernel must move for one run, for walk values of rs
    bytes (4: FP32, 8: FP64): rs per cell crossing (density gather); per
    flight the queued packet is read (positions, direction, density, depth:
    8 x rs; cell and wavelength: 4 x 4 B; id 8 B; RNG position and
    interaction count 2 x 4 B: 64 B in FP32) and, when it ends in an
    interaction, written back; rs per escape to free its entry; 16 per Lucy
    deposit and thermal species (read-modify-write of the FP64 path
    energy)."""
    inter = st["scatters"] + st["absorptions"]
    flights = inter + st["escaped"]
    pk = 8 * rs + 32
    return (rs * st["crossings"] + pk * flights + pk * inter + rs * st["escaped"]
            + 16 * ns_thermal * st["lucy_deposits"])


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packets", type=int, default=100_000_000)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--npix", type=int, default=512)
    ap.add_argument("--cpu-sample", type=int, default=600_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--queue-depth", type=int, default=0,
                    help="packets per wavefront queue (0: the library default)")
    ap.add_argument("--walk-blocks-per-cu", type=int, default=0,
                    help="walk-kernel blocks per CU (0: the library default)")
    ap.add_argument("--blocks-per-cu", type=int, default=0,
                    help="emission/interaction blocks per CU (0: the library default)")
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32",
                    help="walk precision of the context (the benchmark line is fp32)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one elementwise copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the method is not sharded here); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import mcrt_inputs as mi
    import paper_1203_2941_amd as mc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)  # reads and writes calib_copy_mib MiB each
        torch.cuda.synchronize()
        del a, b
        log(f"calibration copy: {args.calib_copy_mib} MiB read + written")
    N = args.packets
    m = mi.torus(n=args.grid, n_packets=N)
    views, idx = mi.image_views(n_views=8, n_img=16, nl=m.nl)
    D = 15.0 * mi.MPC_CM
    log(f"setup: torus {args.grid}^3, {N} packets, views {len(views)}, imaged {len(idx)}")
    fp64 = args.precision == "fp64"
    ctx = mc.Context(0, args.precision).from_inputs(m, views=views, img_idx=idx, distance=D)
    npx = npy = args.npix
    rng = np.random.default_rng(5)
    fdt = torch.float64 if fp64 else torch.float32
    w_img = torch.tensor(rng.random((len(views), len(idx), npy, npx)).astype(np.float64 if fp64 else np.float32),
                         device="cuda")
    img = torch.empty_like(w_img)
    sed = torch.empty((len(views), len(idx)), dtype=torch.float64, device="cuda")
    grad = torch.empty(ctx.ncells, dtype=fdt, device="cuda")
    opts = dict(mode="bw_ticket", n_total=N, mrw_tau=50.0, mrw_gamma=2.0, lucy_tau=1e-2,
                max_interactions=10_000_000, sed_theta_bins=10, queue_depth=args.queue_depth,
                walk_blocks_per_cu=args.walk_blocks_per_cu, blocks_per_cu=args.blocks_per_cu)

    def step(seed):
        ctx.reset()
        st = ctx.run_packets(0, N, seed, **opts)
        ph = ctx.phase_timings()
        sp = ctx.run_pah(seed, **opts)
        ph2 = ctx.phase_timings()
        ctx.finalize_temperatures()
        ctx.raytrace_device(npx, npy, img=img, sed=sed)
        t = ctx.timings()
        ctx.raytrace_adjoint_device(npx, npy, w_img=w_img, out=grad)
        t2 = ctx.timings()
        phases = {k: ph[k] + ph2[k] for k in ("emit_ms", "walk_ms", "interact_ms", "rounds")}
        return st, sp, t["rt_fwd_ms"], t2["rt_adj_ms"], phases

    for w in range(args.warmup):
        t0 = time.perf_counter()
        step(1000 + w)
        torch.cuda.synchronize()
        log(f"warmup {w}: {time.perf_counter() - t0:.2f} s")
    times, rec = [], []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, sp, fwd_ms, adj_ms, phases = step(k)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        times.append(dt)
        rec.append((st, sp, fwd_ms, adj_ms, phases))
        log(f"step {k}: {dt:.3f} s, transport {st['kernel_ms']:.1f} ms, pah {sp['kernel_ms']:.1f} ms,"
            f" rt fwd {fwd_ms:.2f} ms, adj {adj_ms:.2f} ms, crossings {st['crossings']}")
    ms = 1000.0 * float(np.mean(times))
    st0 = rec[-1][0]
    cross = np.mean([r[0]["crossings"] + r[1]["crossings"] for r in rec])
    t_tr = np.mean([r[0]["kernel_ms"] for r in rec]) / 1e3
    t_pah = np.mean([r[1]["kernel_ms"] for r in rec]) / 1e3
    fwd = np.mean([r[2] for r in rec]) / 1e3
    adj = np.mean([r[3] for r in rec]) / 1e3
    rays = len(views) * npx * npy
    ns_th = m.ns - (1 if m.pah_species >= 0 else 0)
    # roofline of the walk kernel (the largest share of the step): its
    # algorithmic bytes over its device time, both summed over the source
    # and PAH runs of a step; launches = rounds
    rs = 8 if fp64 else 4
    b_alg = np.mean([walk_bytes(r[0], ns_th, rs) + walk_bytes(r[1], ns_th, rs) for r in rec])
    t_walk = np.mean([r[4]["walk_ms"] for r in rec]) / 1e3
    t_emit = np.mean([r[4]["emit_ms"] for r in rec]) / 1e3
    t_int = np.mean([r[4]["interact_ms"] for r in rec]) / 1e3
    n_walk = float(np.mean([r[4]["rounds"] for r in rec]))
    # bytes per launch measured by the committed counter runs, reported only
    # for the workload they were taken on and while the kernel is unchanged
    traffic = traffic_step = None
    if (N == 100_000_000 and args.grid == 256 and not fp64 and not args.queue_depth
            and not args.walk_blocks_per_cu and not args.blocks_per_cu):
        from paper_1203_2941_amd import profiling
        tr = profiling.read_traffic()
        if tr is not None:
            traffic, traffic_step = tr["per_launch"], tr["per_step"]
    out = {
        "metric": METRIC,
        "value": N / (ms / 1e3),
        "unit": "packets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if fp64 else "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"clumpy AGN torus {args.grid}^3, 2000 clumps r=0.02 r_out, contrast 100, "
                         f"100 wavelengths, {N} packets, immediate B&W, MRW tau_R>50, PAH; "
                         f"ray-tracer {npx}x{npy} px x 16 wavelengths x 8 views fwd+adjoint"),
            "packets": N, "grid": args.grid, "wavelengths": int(m.nl), "views": len(views),
            "imaged_wavelengths": len(idx), "pixels": [npx, npy],
            "precision": ("fp64" if fp64 else "fp32 walk, fp64 Eq. 4"),
        },
        "cell_crossings_per_s": cross / (ms / 1e3),
        "transport_packets_per_s": N / t_tr,
        "transport_crossings_per_s": st0["crossings"] / t_tr,
        "raytrace_px_per_s_fwd_bwd": rays / (fwd + adj),
        "raytrace_px_per_s_fwd": rays / fwd,
        "raytrace_fwd_ms": fwd * 1e3,
        "raytrace_adj_ms": adj * 1e3,
        "transport_ms": t_tr * 1e3,
        "pah_pass_ms": t_pah * 1e3,
        "events_per_step": {k: int(v) for k, v in st0.items() if k != "kernel_ms"},
        "phase_ms": {"emit": t_emit * 1e3, "walk": t_walk * 1e3, "interact": t_int * 1e3,
                     "rounds": n_walk},
        "roofline": {
            "bound": "hbm",
            "kernel": f"k_wf_walk<{'double' if fp64 else 'float'}, false, true>",
            "achieved": b_alg / t_walk / 1e9,
            "peak": HBM_PEAK / 1e9,
            "unit": "GB/s",
            "frac": b_alg / t_walk / HBM_PEAK,
            "traffic": traffic,
            "traffic_unit": "bytes per launch (L2 <-> memory, rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                            "each over the walk launches of its own counter run)",
            "traffic_per_step": traffic_step,
            "launches_per_step": n_walk,
            "avg_launch_ms": t_walk * 1e3 / n_walk,
            "algorithmic_bytes_per_step": b_alg,
            "algorithmic_bytes_per_launch": b_alg / n_walk,
        },
    }
    if not args.no_cpu_baseline:
        from oracle import oracle
        oracle.build(force=False)
        n = args.cpu_sample
        log(f"cpu baseline: oracle on {n} packets of the same torus (FP64, one core)")
        o = oracle.Oracle(m)
        t0 = time.perf_counter()
        o.run(n=n, mode=oracle.BW_EPOCH, epoch=1 << 30, mrw_tau=50.0, n_total=N)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": n / dt, "unit": "packets/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} source packets of the 256^3 torus (no PAH stage, no ray-tracing), "
                      f"FP64 Bjorkman & Wood with one epoch, {o.stats['crossings']} crossings in {dt:.1f} s",
            "crossings_per_s": o.stats["crossings"] / dt,
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
