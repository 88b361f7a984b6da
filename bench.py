#!/usr/bin/env python
"""Throughput of the Monte Carlo dust transport and the ray-tracer on one MI355X.

One step runs the whole hot path on the clumpy AGN torus (256^3 cells, 2000
clumps, 100 wavelengths, 1e8 packets, FP32 walk): packet transport with
immediate Bjorkman & Wood re-emission, Lucy estimator, modified random walk
in cells with Rosseland depth > 50, HG scattering events for 8 views, the
PAH second stage, Eq. 4 temperatures (FP64), then the ray-tracer forward
(source functions, 512x512 pixels, 16 wavelengths, 8 views) and its adjoint.
Inputs are resident on the GPU before the timed region.

Prints one JSON line. Besides throughput it reports the roofline of the walk
kernel (algorithmic bytes: 4 B of density per cell crossing plus 16 B per
Lucy deposit and thermal species), rooflines of the ray-tracer kernels, the
FP64 path's rate and the FP32 path's difference from it per output, and the
CPU oracle timed on a bounded sample of the same model.
"""
import argparse
import json
import os
import subprocess
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "photon packets/s & cell-crossings/s (256^3 torus); ray-trace px/s fwd+bwd"
HBM_PEAK = 8.0e12  # B/s, MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def walk_alg_bytes(st, ns_thermal, rs=4):
    """Bytes the method must move in the voxel walk: rs (4 FP32, 8 FP64) of
    density per cell crossing, and a 16-byte read-modify-write of the FP64
    path energy per Lucy deposit and thermal species."""
    return rs * st["crossings"] + 16 * ns_thermal * st["lucy_deposits"]


def walk_queue_bytes(st, rs=4):
    """Packet-state traffic of the wavefront design around the walk (not part
    of the method), for the record-free walk of the benchmark: per flight the
    walk reads position, direction and depth (7 x rs) with the word holding
    cell and wavelength (8 B); a flight that ends in an interaction writes
    back position and density (4 x rs) with that word (8 B); an escape marks
    that word free (8 B)."""
    inter = st["scatters"] + st["absorptions"]
    flights = inter + st["escaped"]
    return (7 * rs + 8) * flights + (4 * rs + 8) * inter + 8 * st["escaped"]


def cpu_worker(args):
    """One oracle process on a packet range (used by the CPU baseline)."""
    first, n, lib_path, rho_path, n_total = args.cpu_worker
    from oracle import oracle
    import mcrt_inputs as mi
    oracle.use_library(lib_path)
    m = mi.torus(n=args.grid, n_packets=int(n_total))
    rho = np.load(rho_path, mmap_mode="r")
    o = oracle.Oracle(m, rho=rho)
    t0 = time.perf_counter()
    o.run(first=int(first), n=int(n), mode=oracle.BW_EPOCH, epoch=1 << 40, mrw_tau=50.0,
          n_total=int(n_total))
    dt = time.perf_counter() - t0
    print(json.dumps({"packets": int(n), "crossings": int(o.stats["crossings"]), "seconds": dt}))


def cpu_baseline(args, N):
    """The FP64 oracle on the same torus: one process on a single core for
    each of two builds (-O2; -O3 -march=native for this host), then one
    process per core of the share (at most 16) with the faster build on
    disjoint packet ranges. With a single B&W epoch
    every packet sees the same (initial) temperatures, so packets are
    independent and the ranges add up to one run."""
    from oracle import oracle
    import mcrt_inputs as mi
    tmp = tempfile.mkdtemp(prefix="mcrt_cpu_")
    libs = {"gcc -O2": oracle.build(force=True, out=os.path.join(tmp, "liboracle_o2.so")),
            "gcc -O3 -march=native": oracle.build(force=True, out=os.path.join(tmp, "liboracle_native.so"),
                                                  native=True)}
    m = mi.torus(n=args.grid, n_packets=N)
    rho_path = os.path.join(tmp, "rho.npy")
    np.save(rho_path, oracle.density(m))
    try:
        cores = min(16, len(os.sched_getaffinity(0)))
    except AttributeError:
        cores = min(16, os.cpu_count() or 1)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass

    def launch(first, n, lib):
        cmd = [sys.executable, os.path.abspath(__file__), "--grid", str(args.grid),
               "--cpu-worker", str(first), str(n), lib, rho_path, str(N)]
        return subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True)

    def collect(procs):
        out = []
        for p in procs:
            so, _ = p.communicate()
            if p.returncode != 0:
                raise RuntimeError("cpu baseline worker failed")
            out.append(json.loads(so.strip().splitlines()[-1]))
        return out

    n1 = args.cpu_sample
    single = {}
    for name, lib in libs.items():
        log(f"cpu baseline: oracle ({name}) on {n1} packets, one core")
        single[name] = collect([launch(0, n1, lib)])[0]
    # the all-core run uses the faster of the two builds on this host
    best = min(single, key=lambda k: single[k]["seconds"])
    r1 = single[best]
    per = args.cpu_sample_per_core
    log(f"cpu baseline: {cores} processes x {per} packets ({best})")
    t0 = time.perf_counter()
    rs = collect([launch(n1 + i * per, per, libs[best]) for i in range(cores)])
    wall_all = time.perf_counter() - t0
    # the processes start together; the longest transport loop bounds the
    # time all of them ran side by side (interpreter start-up left out)
    wall = max(r["seconds"] for r in rs)
    pk = sum(r["packets"] for r in rs)
    cr = sum(r["crossings"] for r in rs)
    return {
        "value": pk / wall, "unit": "packets/s", "cores": cores, "kind": "oracle",
        "sample": (f"{pk} source packets of the {args.grid}^3 torus in {cores} processes on "
                   f"disjoint id ranges ({per} each; FP64 Bjorkman & Wood, one epoch, MRW armed; "
                   f"no PAH stage, no ray-tracing), {cr} crossings; longest process loop "
                   f"{wall:.1f} s ({wall_all:.1f} s with interpreter start-up)"),
        "crossings_per_s": cr / wall,
        "single_core_packets_per_s": r1["packets"] / r1["seconds"],
        "single_core_crossings_per_s": r1["crossings"] / r1["seconds"],
        "single_core_sample": f"{n1} packets, {r1['crossings']} crossings in {r1['seconds']:.1f} s",
        "single_core_packets_per_s_by_build": {k: v["packets"] / v["seconds"]
                                               for k, v in single.items()},
        "build": f"{best} -ffp-contract=off -fno-fast-math (faster of -O2 and -O3 -march=native "
                 f"on this host)",
        "cpu_model": model, "nproc": os.cpu_count(),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--packets", type=int, default=100_000_000)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--npix", type=int, default=512)
    ap.add_argument("--cpu-sample", type=int, default=150_000,
                    help="packets of the single-core oracle run")
    ap.add_argument("--cpu-sample-per-core", type=int, default=150_000,
                    help="packets per process of the all-core oracle run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--accuracy-packets", type=int, default=10_000_000,
                    help="packets of the FP32-against-FP64 comparison (0: skip it)")
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
    ap.add_argument("--workload", choices=("torus", "replica", "batch", "shell"), default="torus",
                    help="torus: the benchmark step (default); replica: the sect. 3.6 run-time "
                         "comparison (Table 1) on its constant-density envelope; batch: 64 "
                         "uneven torus models in one batched launch against per-model launches; "
                         "shell: the 128^3 r^-2 shell at tau_V 1, 10, 100, FP32 against FP64")
    ap.add_argument("--cpu-worker", nargs=5, default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker:
        cpu_worker(args)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the method is not sharded here); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "replica":
        replica(args)
        return
    if args.workload == "batch":
        batch(args)
        return
    if args.workload == "shell":
        shell(args)
        return

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
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def step(seed):
        ctx.reset()
        st = ctx.run_packets(0, N, seed, **opts)
        ph = ctx.phase_timings()
        sp = ctx.run_pah(seed, **opts)
        ph2 = ctx.phase_timings()
        ctx.finalize_temperatures()
        # the library launches on torch's current stream: these events
        # bracket the forward call (source functions, pixel rays, SED, point
        # sources) and the adjoint call
        ev[0].record()
        ctx.raytrace_device(npx, npy, img=img, sed=sed)
        ev[1].record()
        t = ctx.timings()
        ctx.raytrace_adjoint_device(npx, npy, w_img=w_img, out=grad)
        ev[2].record()
        t2 = ctx.timings()
        phases = {k: ph[k] + ph2[k] for k in ("emit_ms", "walk_ms", "interact_ms", "rounds")}
        rt = {"fwd_kernel_ms": t["rt_fwd_ms"], "adj_kernel_ms": t2["rt_adj_ms"],
              "build_S_ms": t["build_S_ms"]}
        return st, sp, rt, phases

    def rt_calls_ms():
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])

    for w in range(args.warmup):
        t0 = time.perf_counter()
        step(1000 + w)
        torch.cuda.synchronize()
        log(f"warmup {w}: {time.perf_counter() - t0:.2f} s")
    times, rec = [], []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, sp, rt, phases = step(k)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rt["fwd_call_ms"], rt["adj_call_ms"] = rt_calls_ms()
        times.append(dt)
        rec.append((st, sp, rt, phases))
        log(f"step {k}: {dt:.3f} s, transport {st['kernel_ms']:.1f} ms, pah {sp['kernel_ms']:.1f} ms,"
            f" rt S {rt['build_S_ms']:.2f} ms fwd {rt['fwd_call_ms']:.2f} ms"
            f" (kernel {rt['fwd_kernel_ms']:.2f}), adj {rt['adj_call_ms']:.2f} ms"
            f" (kernel {rt['adj_kernel_ms']:.2f}), crossings {st['crossings']}")
    ms = 1000.0 * float(np.mean(times))
    st0 = rec[-1][0]
    cross = np.mean([r[0]["crossings"] + r[1]["crossings"] for r in rec])
    t_tr = np.mean([r[0]["kernel_ms"] for r in rec]) / 1e3
    t_pah = np.mean([r[1]["kernel_ms"] for r in rec]) / 1e3

    def rtm(key):
        return float(np.mean([r[2][key] for r in rec])) / 1e3

    fwd_call, adj_call = rtm("fwd_call_ms"), rtm("adj_call_ms")
    t_S, t_fk, t_ak = rtm("build_S_ms"), rtm("fwd_kernel_ms"), rtm("adj_kernel_ms")
    rays = len(views) * npx * npy
    ns_th = m.ns - (1 if m.pah_species >= 0 else 0)
    # roofline of the walk kernel (the largest share of the step): the
    # method's bytes over its device time, both summed over the source and
    # PAH runs of a step (the finishing kernel's flights included in both)
    rs = 8 if fp64 else 4
    b_alg = np.mean([walk_alg_bytes(r[0], ns_th, rs) + walk_alg_bytes(r[1], ns_th, rs) for r in rec])
    b_q = np.mean([walk_queue_bytes(r[0], rs) + walk_queue_bytes(r[1], rs) for r in rec])
    t_walk = np.mean([r[3]["walk_ms"] for r in rec]) / 1e3
    t_emit = np.mean([r[3]["emit_ms"] for r in rec]) / 1e3
    t_int = np.mean([r[3]["interact_ms"] for r in rec]) / 1e3
    n_walk = float(np.mean([r[3]["rounds"] for r in rec]))
    # bytes per launch measured by the committed counter runs, reported only
    # for the workload they were taken on and while the kernel is unchanged
    traffic = traffic_step = None
    default_shape = (N == 100_000_000 and args.grid == 256 and not args.queue_depth
                     and not args.walk_blocks_per_cu and not args.blocks_per_cu)
    from paper_1203_2941_amd import profiling
    if default_shape and not fp64:
        tr = profiling.read_traffic()
        if tr is not None:
            traffic, traffic_step = tr["per_launch"], tr["per_step"]
    # ray-tracer: compulsory bytes per call (each array once)
    nc, nv, nq = ctx.ncells, len(views), len(idx)
    img_b = nv * nq * npx * npy * rs
    b_fwd = nv * nc * (rs + nq * rs) + img_b          # density and S per view, image out
    b_adj = nv * nc * (rs + nq * rs) + img_b + nc * rs  # the same, weights in, gradient out
    b_S = nc * (8 * ns_th + rs) + 2 * nv * nc * nq * rs  # T, density, sums in; S out
    rt_traffic = profiling.read_rt_traffic() if (default_shape and not fp64) else None

    def roof(kernel, b, t, key):
        d = {"kernel": kernel, "bound": "hbm", "achieved": b / t / 1e9, "peak": HBM_PEAK / 1e9,
             "unit": "GB/s", "frac": b / t / HBM_PEAK, "bytes_per_launch": b, "launch_ms": t * 1e3,
             "traffic": None}
        if rt_traffic and key in rt_traffic:
            d["traffic"] = rt_traffic[key]
        return d

    tn = "double" if fp64 else "float"
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
        "raytrace_px_per_s_fwd_bwd": rays / (fwd_call + adj_call),
        "raytrace_px_per_s_fwd": rays / fwd_call,
        "raytrace_fwd_ms": fwd_call * 1e3,
        "raytrace_adj_ms": adj_call * 1e3,
        "raytrace_build_S_ms": t_S * 1e3,
        "raytrace_fwd_kernel_ms": t_fk * 1e3,
        "raytrace_adj_kernel_ms": t_ak * 1e3,
        "transport_ms": t_tr * 1e3,
        "pah_pass_ms": t_pah * 1e3,
        "events_per_step": {k: int(v) for k, v in st0.items() if k != "kernel_ms"},
        "phase_ms": {"emit": t_emit * 1e3, "walk": t_walk * 1e3, "interact": t_int * 1e3,
                     "rounds": n_walk},
        "roofline": {
            "bound": "hbm",
            "kernel": f"k_wf_walk<{tn}, false, true, false, false>",
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
            "algorithmic_bytes_rule": f"{rs} B per cell crossing + 16 B per Lucy deposit and "
                                      f"thermal species",
            "design_overhead_bytes_per_launch": b_q / n_walk,
            "design_overhead_rule": "queued packet state read per flight and written back per "
                                    "interaction (wavefront queues; not the method's bytes)",
        },
        "roofline_raytrace": {
            "build_S": roof(f"k_build_S<{tn}, false, false>", b_S, t_S, "k_build_S"),
            "forward": roof(f"k_rt_fwd<{tn}, false, false>", b_fwd, t_fk, "k_rt_fwd"),
            "adjoint": roof(f"k_rt_adj<{tn}, false, false>", b_adj, t_ak, "k_rt_adj"),
            "bytes_rule": "compulsory: each array once per launch (density and source "
                          "functions per view, images, weights, gradient; for S: temperatures, "
                          "density, scattering sums in and S out)",
        },
    }
    if args.accuracy_packets and not fp64:
        out["fp64_path"], out["fp32_vs_fp64"] = accuracy(args, m, views, idx, D, ctx, opts)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, N)
    print(json.dumps(out), flush=True)


def accuracy(args, m, views, idx, D, ctx32, opts):
    """FP64 path's rate on the same torus, and the FP32 path's outputs against
    it at args.accuracy_packets packets. Trajectories diverge chaotically
    between precisions after a few events, so each difference is stated
    beside the same quantity between two FP64 runs with different seeds (the
    Monte Carlo noise at this packet count)."""
    import ctypes as C

    import torch

    import paper_1203_2941_amd as mc
    from paper_1203_2941_amd import _lib as L
    n = args.accuracy_packets
    npx = npy = args.npix
    o = dict(opts, n_total=n)
    log(f"accuracy: FP64 context, {n} packets")
    c64 = mc.Context(0, "fp64").from_inputs(m, views=views, img_idx=idx, distance=D)

    def run(c, seed):
        c.reset()
        st = c.run_packets(0, n, seed, **o)
        sp = c.run_pah(seed, **o)
        T, E = c.temperatures(with_energy=True)
        f, cnt = c.sed()
        im, sd = c.raytrace_device(npx, npy)
        full = torch.empty((len(views), len(idx), c.ncells), dtype=torch.float64, device="cuda")
        c._chk(c.lib.mcrt_scattering(c.h, C.c_void_p(full.data_ptr()), L.DEVICE, None))
        ss = full.sum(dim=2)
        del full
        torch.cuda.synchronize()
        return {"st": st, "sp": sp, "T": T, "E": E, "sed": cnt.astype(np.float64),
                "img": im.double().cpu().numpy(), "ssca": ss.cpu().numpy()}

    r64 = run(c64, 11)
    t64 = r64["st"]["kernel_ms"] / 1e3
    r64b = run(c64, 12)
    r32 = run(ctx32, 11)
    t32 = r32["st"]["kernel_ms"] / 1e3
    del c64
    torch.cuda.empty_cache()

    def diffs(a, b):
        k = (a["E"][:2] > 0) & (b["E"][:2] > 0)
        w = a["E"][:2][k]
        dT = np.abs(a["T"][:2][k] / b["T"][:2][k] - 1.0)
        sed_a, sed_b = a["sed"], b["sed"]
        ok = (sed_a + sed_b) > 50
        chi = float(np.sum((sed_a[ok] - sed_b[ok]) ** 2 / (sed_a[ok] + sed_b[ok])) / ok.sum())
        ia, ib = a["img"], b["img"]
        rel_img = [float(np.linalg.norm(ia[v, q] - ib[v, q]) / max(np.linalg.norm(ib[v, q]), 1e-300))
                   for v in range(ia.shape[0]) for q in range(ia.shape[1])]
        sa, sb = a["ssca"], b["ssca"]
        ok2 = sb > 0
        return {
            "T_rel_energy_weighted": float(np.sum(w * dT) / np.sum(w)),
            "T_rel_median": float(np.median(dT)),
            "E_total_rel": [float(a["E"][s].sum() / b["E"][s].sum() - 1.0) for s in range(2)],
            "sed_counts_chi2_per_bin": chi,
            "sed_total_rel": float(sed_a.sum() / sed_b.sum() - 1.0),
            "scattering_totals_rel_rms": float(np.sqrt(np.mean((sa[ok2] / sb[ok2] - 1.0) ** 2))),
            "image_rel_l2_median": float(np.median(rel_img)),
            "image_rel_l2_max": float(np.max(rel_img)),
            "crossings_per_packet_rel": float(a["st"]["crossings"] / b["st"]["crossings"] - 1.0),
        }

    fp64_path = {"packets": n, "transport_ms": t64 * 1e3, "transport_packets_per_s": n / t64,
                 "fp32_transport_ms_same_packets": t32 * 1e3,
                 "fp32_speedup_transport": t64 / t32}
    err = {"packets": n, "seed": 11,
           "fp32_vs_fp64_same_seed": diffs(r32, r64),
           "fp64_vs_fp64_other_seed": diffs(r64b, r64),
           "note": "per output: FP32 path against the FP64 path on the benchmark torus; the "
                   "second block is the Monte Carlo noise at this packet count"}
    return fp64_path, err


# Table 1 of the paper (minutes for 1e7 packets on the sect. 3.6 envelope,
# 1e6 cells; 2012 hardware: one 3 GHz core, 8 threads, a 256-core GPU).
TABLE1_MIN = {"Lucy, 1 thread": 180, "B&W, 1 thread": 60, "Lucy, 8 threads": 45,
              "B&W, 8 threads": 20, "GPU (iterative)": 3, "GPU+Lucy": 4, "GPU+B&W": 2,
              "GPU+B&W+Lucy": 2}


def replica(args):
    """The run-time comparison of sect. 3.6 on its own model: a 2500 K, 1 L_sun
    star in a constant-density envelope (0.7-700 AU, tau_V = 10, 100^3 cells),
    1e7 packets per pass. The GPU runs the variants of Table 1 (iterative
    scheme with three passes from the thin-limit temperatures, with and
    without Lucy's estimator; immediate B&W with and without Lucy); the FP64
    oracle (serial B&W, Lucy off and on) is timed on one core on a sample and
    scaled to 1e7 packets. Prints one JSON line."""
    import torch

    import mcrt_inputs as mi
    import paper_1203_2941_amd as mc
    from oracle import oracle

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    N = args.packets if args.packets != 100_000_000 else 10_000_000
    m = mi.replica(n=100, n_packets=N)
    ctx = mc.Context(0, args.precision).from_inputs(m)
    variants = {
        "GPU (iterative)": dict(mode="frozen", n_iter=3, lucy_tau=0.0),
        "GPU+Lucy": dict(mode="frozen", n_iter=3, lucy_tau=1e-2),
        "GPU+B&W": dict(mode="bw_ticket", lucy_tau=0.0),
        "GPU+B&W+Lucy": dict(mode="bw_ticket", lucy_tau=1e-2),
    }
    out_v = {}
    for name, kw in variants.items():
        times, stats = [], None
        for k in range(args.warmup + args.steps):
            ctx.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if kw["mode"] == "frozen":
                ctx.init_temperatures()
            st = ctx.run_packets(0, N, 100 + k, n_total=N, mrw_tau=0.0, **kw)
            ctx.finalize_temperatures()
            torch.cuda.synchronize()
            if k >= args.warmup:
                times.append(time.perf_counter() - t0)
                stats = st
        sec = float(np.median(times))
        passes = kw.get("n_iter", 1) if kw["mode"] == "frozen" else 1
        out_v[name] = {"seconds": sec, "passes": passes, "packets_per_pass": N,
                       "packets_per_s": passes * N / sec,
                       "crossings": int(stats["crossings"]),
                       "paper_minutes": TABLE1_MIN[name],
                       "speedup_vs_paper": TABLE1_MIN[name] * 60.0 / sec}
        log(f"replica {name}: {sec:.3f} s ({passes} x {N} packets)")
    # CPU oracle, one core, serial B&W (one packet per epoch), scaled
    cpu = {}
    n_cpu = max(1000, min(args.cpu_sample, 20000))
    if not args.no_cpu_baseline:
        o = oracle.Oracle(m)
        for name, lt in (("B&W, 1 thread", 0.0), ("Lucy+B&W, 1 thread", 1e-2)):
            o.reset()
            t0 = time.perf_counter()
            o.run(n=n_cpu, mode=oracle.BW_EPOCH, epoch=1, lucy_tau=lt, n_total=N)
            dt = time.perf_counter() - t0
            cpu[name] = {"sample_packets": n_cpu, "seconds": dt,
                         "scaled_minutes_1e7": dt * (N / n_cpu) / 60.0,
                         "paper_minutes": TABLE1_MIN.get(name)}
            log(f"replica cpu {name}: {dt:.2f} s for {n_cpu} packets")
    best = min(out_v.values(), key=lambda v: v["seconds"])
    print(json.dumps({
        "metric": "run time of the sect. 3.6 comparison (Table 1 replica)",
        "value": best["seconds"], "unit": "s", "higher_is_better": False,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "dtype": "f64" if args.precision == "fp64" else "f32", "data": "synthetic",
        "config": {"workload": (f"constant-density envelope 0.7-700 AU, tau_V = 10, "
                                f"{m.nx}^3 cells, 2500 K 1 L_sun star, Ivezic 1D dust law, "
                                f"{m.nl} wavelengths, {N} packets per pass")},
        "variants": out_v, "cpu_oracle": cpu,
        "paper_table1_minutes": TABLE1_MIN,
        "note": "paper times are for 2012 hardware (context, not a target)",
    }), flush=True)


def batch(args):
    """64 uneven clumpy-torus models (grids 64^3-192^3, 200-1e4 clumps, 40-100
    wavelengths, 1e6-1e7 packets each, about 2.5e8 in all): one batched
    launch (every model in each wavefront round, rounds replayed from a HIP
    graph) against the same models launched one after the other. FP32 walk,
    immediate B&W, MRW armed. Prints one JSON line."""
    import torch

    import mcrt_inputs as mi
    import paper_1203_2941_amd as mc

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    specs = mi.batch_specs(64, seed=4)
    ctxs, npk, seeds = [], [], []
    t0 = time.perf_counter()
    for s in specs:
        m = mi.torus(n=s["n"], n_clumps=s["n_clumps"], nl=s["nl"], n_packets=s["n_packets"],
                     seed=s["seed"], geo_seed=s["geo_seed"])
        ctxs.append(mc.Context(0, args.precision).from_inputs(m))
        npk.append(s["n_packets"])
        seeds.append(s["seed"])
    torch.cuda.synchronize()
    log(f"batch: 64 models set up in {time.perf_counter() - t0:.1f} s, {sum(npk)} packets")
    opts = dict(mode="bw_ticket", mrw_tau=50.0, mrw_gamma=2.0, lucy_tau=1e-2,
                queue_depth=args.queue_depth or (1 << 20))
    times = []
    for k in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = mc.run_batch(ctxs, npk, [s + 1000 * k for s in seeds], **opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert all(x["escaped"] + x["killed"] + x["pah_stopped"] == n for x, n in zip(st, npk))
        if k >= args.warmup:
            times.append(dt)
        log(f"batched run {k}: {dt:.3f} s")
    seq = []
    for k in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c, n, s in zip(ctxs, npk, seeds):
            c.reset()
            c.run_packets(0, n, s + 1000 * k, n_total=n, **opts)
            c.finalize_temperatures()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if k >= args.warmup:
            seq.append(dt)
        log(f"per-model runs {k}: {dt:.3f} s")
    tb, ts = float(np.median(times)), float(np.median(seq))
    total = sum(npk)
    print(json.dumps({
        "metric": "photon packets/s, 64-model batch", "value": total / tb, "unit": "packets/s",
        "higher_is_better": True, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": tb * 1e3, "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": ("64 clumpy-torus models: grids 64^3-192^3, 200-1e4 clumps, "
                                "40-100 wavelengths, 1e6-1e7 packets each; immediate B&W, "
                                "MRW tau_R > 50, PAH"),
                   "packets": total, "queue_depth": opts["queue_depth"]},
        "batched_s": tb, "per_model_s": ts, "per_model_packets_per_s": total / ts,
        "batch_speedup": ts / tb,
        "note": "per-model runs include a tally reset and Eq. 4 per model, as the batch does",
    }), flush=True)


def tally_diffs(a, b, nth):
    """Temperature, absorbed-energy and SED differences of run a against run b
    (thermal species 0..nth-1; SED counts by polar bin and wavelength)."""
    k = (a["E"][:nth] > 0) & (b["E"][:nth] > 0)
    w = a["E"][:nth][k]
    dT = np.abs(a["T"][:nth][k] / b["T"][:nth][k] - 1.0)
    sa, sb = a["sed"], b["sed"]
    ok = (sa + sb) > 50
    return {
        "T_rel_energy_weighted": float(np.sum(w * dT) / np.sum(w)),
        "T_rel_median": float(np.median(dT)),
        "E_total_rel": [float(a["E"][s].sum() / b["E"][s].sum() - 1.0) for s in range(nth)],
        "sed_counts_chi2_per_bin": float(np.sum((sa[ok] - sb[ok]) ** 2 / (sa[ok] + sb[ok]))
                                         / max(ok.sum(), 1)),
        "crossings_per_packet_rel": float(a["st"]["crossings"] / b["st"]["crossings"] - 1.0),
    }


def shell(args):
    """The r^-2 shell of the sect. 3.6 and 5.1 comparisons on 128^3 cells
    (R_in = 1 AU to 1000 R_in, 2500 K 1 L_sun star, two species) at radial
    tau_V = 1, 10 and 100 with 1e7 packets each: FP32 and FP64 transport rates
    (immediate B&W, Lucy and diffusion steps armed, Eq. 4 included), the FP32
    outputs against FP64 beside the FP64 seed-to-seed noise, and the oracle's
    rate (serial B&W) on a sample of about 10 s per optical depth. Prints one
    JSON line; `value` is the FP32 rate at tau_V = 10."""
    import torch

    import mcrt_inputs as mi
    import paper_1203_2941_amd as mc
    from oracle import oracle

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    N = args.packets if args.packets != 100_000_000 else 10_000_000
    n = args.grid if args.grid != 256 else 128
    opts = dict(mode="bw_ticket", n_total=N, mrw_tau=50.0, mrw_gamma=2.0, lucy_tau=1e-2,
                max_interactions=10_000_000, sed_theta_bins=10)
    res = {}
    for tau in (1.0, 10.0, 100.0):
        m = mi.shell(n=n, tau_v=tau, n_packets=N)
        ctx = {p: mc.Context(0, p).from_inputs(m) for p in ("fp32", "fp64")}

        def run(c, seed):
            c.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = c.run_packets(0, N, seed, **opts)
            c.finalize_temperatures()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            T, E = c.temperatures(with_energy=True)
            _, cnt = c.sed()
            return {"st": st, "s": dt, "T": T, "E": E, "sed": cnt.astype(np.float64)}

        for p in ctx:
            run(ctx[p], 1)  # warm-up
        r32, r64, r64b = run(ctx["fp32"], 11), run(ctx["fp64"], 11), run(ctx["fp64"], 12)
        del ctx
        torch.cuda.empty_cache()
        log(f"shell tau_V {tau:g}: FP32 {r32['s']:.3f} s, FP64 {r64['s']:.3f} s for {N} packets")
        cpu = None
        if not args.no_cpu_baseline:
            o = oracle.Oracle(m)
            done, t0 = 0, time.perf_counter()
            while time.perf_counter() - t0 < 10.0 and done < N:
                k = min(500, N - done)
                o.run(first=done, n=k, seed=11, mode=oracle.BW_EPOCH, epoch=1, n_total=N,
                      lucy_tau=1e-2, mrw_tau=50.0, mrw_gamma=2.0, max_int=10_000_000)
                done += k
            dt = time.perf_counter() - t0
            cpu = {"kind": "oracle", "cores": 1, "sample_packets": done, "seconds": dt,
                   "packets_per_s": done / dt,
                   "crossings_per_s": o.stats["crossings"] / dt}
            log(f"shell tau_V {tau:g}: oracle {done} packets in {dt:.1f} s")
        res[f"{tau:g}"] = {
            "fp32": {"seconds": r32["s"], "packets_per_s": N / r32["s"],
                     "crossings_per_s": r32["st"]["crossings"] / r32["s"],
                     "events": {k: int(v) for k, v in r32["st"].items() if k != "kernel_ms"}},
            "fp64": {"seconds": r64["s"], "packets_per_s": N / r64["s"],
                     "crossings_per_s": r64["st"]["crossings"] / r64["s"]},
            "fp32_vs_fp64_same_seed": tally_diffs(r32, r64, m.ns),
            "fp64_vs_fp64_other_seed": tally_diffs(r64b, r64, m.ns),
            "cpu_oracle": cpu,
        }
    v = res["10"]["fp32"]["packets_per_s"]
    print(json.dumps({
        "metric": "photon packets/s, r^-2 shell", "value": v, "unit": "packets/s",
        "higher_is_better": True, "n_gpus": 1, "steps": 1, "warmup": 1,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"r^-2 shell {n}^3, R_in 1 AU to 1000 R_in, 2500 K 1 L_sun star, "
                                f"two species, 100 wavelengths, {N} packets per optical depth; "
                                f"immediate B&W, Lucy 1e-2, diffusion steps above 50"),
                   "value_at_tau_v": 10},
        "tau_v": res,
        "note": "timed: reset, transport and Eq. 4 per run (FP32 walk or FP64 walk); the FP64 "
                "second seed gives the Monte Carlo noise the FP32 differences stand beside",
    }), flush=True)


if __name__ == "__main__":
    main()
