#!/usr/bin/env python
"""Throughput of the graph-based FEM fracture step on one MI355X.

Workload: the ductile ellipsoid of 619,830 tets (111,912 nodes, 748,579
edges), split precision (FP32 element pass and SpMV, FP64 dot products,
residual and refinement), one backward-Euler step per timestep accepted at
FP64 |b - A dv| <= 1e-6 |b|.  A "step" is one whole timestep: damage update,
element pass with plasticity, assembly, preconditioner (network inference
every 4 steps, factor build every step), PCG with iterative refinement,
integration.  All inputs are resident in HBM before timing.

`value` is the learned-preconditioner leg (trained weights shipped in
paper_2103_14870_amd/weights); the same K steps from the same start state
are timed again with block-Jacobi PCG and reported beside it.  Prints one
JSON line.  Extra legs: the dominant kernel's roofline (SpMV, HIP events on
the library's stream) and the FP64 CPU oracle timed on a two-step sample of
the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "pcg_ellipsoid620k_hbm_counters.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2103_14870_amd", "csrc", f) for f in ("kernels.hip", "kernels.hpp", "gfem.hip")]


def kernel_sources_digest():
    """SHA-256 over the kernel sources and the launch configuration."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic(path=COUNTERS):
    """HBM bytes per SpMV launch from the committed rocprofv3 counter summary,
    or None when the kernel source changed since the counters were taken."""
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    kv = dict(ln.split(None, 1) for ln in lines if ln and not ln.startswith("#") and len(ln.split(None, 1)) == 2)
    if kv.get("kernel_sources_sha256", "").strip() != kernel_sources_digest():
        return None
    try:
        return float(kv["spmv_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def kernel_short_name(name):
    import re

    m = re.search(r"(k_[a-z0-9_]+)(<[^>(]*>)?", name)
    return (m.group(1) + (m.group(2) or "")) if m else name.split("(")[0][-60:]


def write_counter_summary(fetch_csv, write_csv, calib_mb, command_f, command_w, out_path=COUNTERS):
    """Per-kernel HBM traffic from two rocprofv3 counter runs of
    `bench.py --calib-copy-mb calib_mb` (FETCH_SIZE, then WRITE_SIZE, KiB per
    dispatch), each scaled by what the same counter reads for the cache-cold
    calibration sum (reads calib_mb MiB) and copy (writes calib_mb MiB) that
    the bench runs first.  Writes the summary that measured_traffic() reads."""
    import collections
    import csv

    def per_kernel(path, counter):
        agg = collections.defaultdict(list)
        full = []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                v = float(r["Counter_Value"])
                agg[kernel_short_name(r["Kernel_Name"])].append(v)
                full.append((r["Kernel_Name"], v))
        return agg, full

    fetch, ffull = per_kernel(fetch_csv, "FETCH_SIZE")
    write, wfull = per_kernel(write_csv, "WRITE_SIZE")
    calib_kib = calib_mb * 1024.0
    red = max(v for n, v in ffull if "reduce_kernel" in n)
    cpy = max(v for n, v in wfull if "copyBuffer" in n)
    fr, fw = calib_kib / red, calib_kib / cpy
    mean = lambda xs: sum(xs) / len(xs) if xs else 0.0
    spmv = next(k for k in fetch if k.startswith("k_pcg_spmv_p<"))
    spmv_bytes = (mean(fetch[spmv]) * fr + mean(write[spmv]) * fw) * 1024.0
    digest = kernel_sources_digest()
    lines = [
        "# HBM traffic per dispatch from rocprofv3 counters: 619,830-tet ellipsoid bench (learned leg, kernel",
        "# timing leg and block-Jacobi leg), one MI355X.  Commands (repository root):",
        f"#   {command_f}",
        f"#   {command_w}",
        f"#   python bench.py --counter-summary <fetch counter_collection.csv> <write counter_collection.csv> "
        f"--calib-copy-mb {calib_mb}",
        f"# calibration: the {calib_mb} MiB cache-cold sum reads FETCH_SIZE {red:.0f} KiB (x{fr:.3f}); "
        f"the {calib_mb} MiB copy reads WRITE_SIZE {cpy:.0f} KiB (x{fw:.3f})",
        "# table: dispatches, mean FETCH_SIZE KiB, mean WRITE_SIZE KiB, calibrated MB per dispatch",
        f"kernel_sources_sha256 {digest}",
        f"calib_read_factor {fr:.4f}",
        f"calib_write_factor {fw:.4f}",
        f"spmv_hbm_bytes_per_launch {spmv_bytes:.0f}",
    ]
    names = sorted(set(fetch) | set(write), key=lambda k: -sum(fetch.get(k, [0.0])))
    for k in names:
        if not k.startswith("k_"):
            continue
        f_, w_ = mean(fetch.get(k, [])), mean(write.get(k, []))
        lines.append(f"#  {len(fetch.get(k, [])):6d} {f_:12.1f} {w_:12.1f} {(f_ * fr + w_ * fw) * 1024 / 1e6:10.2f}  {k}")
    open(out_path, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


STATS = os.path.join(ROOT, "profiles", "pcg_learned_ellipsoid620k_kernel_stats.txt")


ELLIPSOID_TITLE = ("# rocprofv3 kernel statistics: bench.py on the 619,830-tet ductile ellipsoid, one MI355X\n"
                   "# (learned-preconditioner leg, kernel timing leg and block-Jacobi leg, 10 timed steps after "
                   "5 warm-up each)")


def write_stats_summary(stats_csv, command, out_path=STATS, title=ELLIPSOID_TITLE):
    """Per-kernel table from a rocprofv3 --kernel-trace --stats run of
    bench.py (run_kernel_stats.csv), with the command that made it."""
    import csv

    rows = list(csv.DictReader(open(stats_csv)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [
        *title.split("\n"),
        "#",
        "# command (repository root):",
        f"#   {command}",
        "#",
        "# rows of run_kernel_stats.csv (names shortened to the kernel and its template arguments);",
        "# durations are per-dispatch GPU begin/end timestamps in microseconds",
        "#",
        "#  calls    avg_us    min_us    max_us  total_ms      %  kernel",
    ]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        tot = float(r["TotalDurationNs"])
        lines.append(f"{int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:9.2f} {float(r['MinNs']) / 1e3:9.2f} "
                     f"{float(r['MaxNs']) / 1e3:9.2f} {tot / 1e6:9.2f} {100 * tot / total:6.2f}  "
                     f"{kernel_short_name(r['Name'])}")
    open(out_path, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def profile_avg_us(kernel_prefix, path=STATS):
    """Average duration of a kernel in the committed rocprofv3 statistics, or
    None when absent or when the kernel source changed since (the counter
    summary records the source hash of the same profiling session)."""
    try:
        kv = dict(ln.split(None, 1) for ln in open(COUNTERS).read().splitlines()
                  if ln and not ln.startswith("#") and len(ln.split(None, 1)) == 2)
        if kv.get("kernel_sources_sha256", "").strip() != kernel_sources_digest():
            return None
        for ln in open(path):
            f = ln.split()
            if len(f) >= 7 and not ln.startswith("#") and f[6].startswith(kernel_prefix):
                return float(f[1])
    except (OSError, ValueError):
        return None
    return None


def cpu_baseline(prob, n_threads=1):
    """FP64 oracle, the first two steps of the same workload from rest, on host cores."""
    from threadpoolctl import threadpool_limits

    from oracle import gfem_oracle as O

    with threadpool_limits(n_threads):
        mesh = O.setup(prob.X, prob.tets, prob.params)
        st = O.initial_state(mesh)
        O.break_pairs(mesh, st, prob.broken_pairs)
        t0 = time.perf_counter()
        iters = []
        for _ in range(2):
            st, h = O.step(mesh, st, prob.dir_nodes, prob.dir_vel)
            iters.append(h["iters"])
        dt = time.perf_counter() - t0
    return dict(value=2.0 / dt, unit="timesteps/s", cores=n_threads, kind="oracle",
                sample=f"first 2 steps from rest of the same {prob.n_tets}-tet workload "
                       f"(FP64 NumPy/SciPy oracle, block-Jacobi PCG, {iters} iterations, {dt:.1f} s)")


def cpu_baseline_qs(prob, rtol, n_threads=1):
    """FP64 oracle, the first quasi-static load step of the same block from rest, on host cores."""
    from threadpoolctl import threadpool_limits

    from oracle import gfem_oracle as O

    with threadpool_limits(n_threads):
        mesh = O.setup(prob.X, prob.tets, prob.params)
        st = O.initial_state(mesh)
        O.break_pairs(mesh, st, prob.broken_pairs)
        t0 = time.perf_counter()
        st, h = O.quasi_static_step(mesh, st, prob.dir_nodes, prob.dir_vel, newton_rtol=rtol)
        dt = time.perf_counter() - t0
    return dict(value=1.0 / dt, unit="load steps/s", cores=n_threads, kind="oracle",
                sample=f"first load step from rest of the same {prob.n_tets}-tet block (FP64 NumPy/SciPy "
                       f"oracle, {h['newton_iters']} Newton iterations, {h['inner_iters']} PCG iterations, "
                       f"{dt:.1f} s)")


def quasi_static_leg(m, steps, warmup, rtol, window, log):
    """Load steps of a quasi-static block (Newton with a line search, Eq. 36),
    one call per load step: per-window wall time, Newton and PCG iterations,
    line-search halvings and broken edges."""
    import torch

    for _ in range(warmup):
        m.quasi_static_step(1, newton_rel_tol=rtol)
    torch.cuda.synchronize()
    from paper_2103_14870_amd import gfem

    rows, cur, tot, failed = [], None, dict(newton=0, inner=0, halvings=0), None
    t_start = t0 = time.perf_counter()
    for i in range(steps):
        if cur is None:
            cur = dict(first=warmup + i + 1, steps=0, newton=0, inner=0, halvings=0, broken=0)
        s = m.quasi_static_step(1, newton_rel_tol=rtol, raise_on_error=False)
        if s["status"] != gfem.GF_OK:
            failed = dict(load_step=warmup + i + 1, status=gfem.STATUS_NAMES.get(s["status"], s["status"]),
                          error=(gfem.load().gf_last_error() or b"").decode())
            log(f"load step {warmup + i + 1} failed: {failed['error']}")
        else:
            cur["steps"] += 1
            cur["newton"] += s["newton_iters"]
            cur["inner"] += s["inner_iters"]
            cur["halvings"] += s["line_search_halvings"]
            cur["broken"] = s["total_broken"]
        if failed or (i + 1) % window == 0 or i + 1 == steps:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if not cur["steps"]:
                break
            cur.update(last=cur["first"] + cur["steps"] - 1, seconds=t1 - t0,
                       ms_per_load_step=1000.0 * (t1 - t0) / cur["steps"])
            for k in tot:
                tot[k] += cur[k]
            rows.append(cur)
            log(f"load steps {cur['first']}-{cur['last']}: {cur['ms_per_load_step']:.1f} ms/step, "
                f"{cur['newton'] / cur['steps']:.1f} Newton, {cur['inner'] / max(cur['newton'], 1):.0f} PCG it/Newton, "
                f"{cur['halvings']} halvings, broken {cur['broken']}")
            cur, t0 = None, t1
        if failed:
            break
    elapsed = sum(r["seconds"] for r in rows)
    return dict(windows=rows, elapsed=elapsed, done=sum(r["steps"] for r in rows), failed=failed, **tot)


def host_cpu_model():
    """The host CPU's model name (Linux), or the platform's processor string."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def timed_steps(m, steps, warmup):
    """The K timed steps are one gf_step(K) call (one host round trip per
    step fewer than K calls of one step); the stats are summed over them."""
    import torch

    if warmup > 0:
        m.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = m.step(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert s["steps_done"] == steps
    return dict(value=steps / elapsed, elapsed=elapsed, iters=s["inner_iters"] / steps,
                outer=s["outer_iters"] / steps, fallback=s["used_fallback"])


def per_call_steps(m, steps, warmup, readback):
    """The same step window as the timed leg as one gf_step(1) call per step;
    with readback, each step is followed by gf_get_positions and
    gf_get_edge_damage into host buffers (the boundary's output path, over
    PCIe)."""
    import torch

    if warmup > 0:
        m.step(warmup)
    torch.cuda.synchronize()
    nbytes = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        m.step(1)
        if readback:
            x, z = m.positions(), m.edge_damage()
            nbytes = x.nbytes + z.nbytes
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return dict(value=steps / elapsed, ms_per_step=1000.0 * elapsed / steps, bytes_per_step=nbytes)


def kernel_times(m, steps, warmup):
    """Per-kernel device time over the same step window as the timed leg, on a
    fresh mesh (event timing adds host work, so it is kept out of that leg)."""
    import torch

    for _ in range(warmup):
        m.step(1)
    m.set_timing(True)
    kus, kn = {}, {}
    for _ in range(steps):
        s = m.step(1)
        for k, v in s["kernel_us"].items():
            kus[k] = kus.get(k, 0.0) + v
        for k, v in s["n_launch"].items():
            kn[k] = kn.get(k, 0) + v
    torch.cuda.synchronize()
    m.set_timing(False)
    return kus, kn


def trajectory(make_mesh, n_steps, window, learned, log):
    """n_steps from rest, one gf_step call per step, with per-window totals:
    steps/s (wall clock, synchronised at window ends), PCG iterations per
    step, learned attempts re-solved with block-Jacobi, steps re-run in FP64,
    broken edges at the window's end.  Stops at the first step that does not
    converge and reports it."""
    import torch

    from paper_2103_14870_amd import gfem

    m = make_mesh(learned)
    rows, cur, failed = [], None, None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_steps):
        if cur is None:
            cur = dict(first=i + 1, steps=0, iters=0, fallback=0, fp64=0)
        s = m.step(1, raise_on_error=False)
        if s["status"] != gfem.GF_OK:
            failed = dict(step=i + 1, status=gfem.STATUS_NAMES.get(s["status"], s["status"]),
                          rel_residual=s["rel_residual"], iters=s["inner_iters"])
        else:
            cur["steps"] += 1
            cur["iters"] += s["inner_iters"]
            cur["fallback"] += s["used_fallback"]
            cur["fp64"] += s["fp64_steps"]
            cur["broken"] = s["total_broken"]
        if failed or (i + 1) % window == 0 or i + 1 == n_steps:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if cur["steps"]:
                cur.update(last=cur["first"] + cur["steps"] - 1, seconds=t1 - t0,
                           steps_per_s=cur["steps"] / (t1 - t0), iters_per_step=cur["iters"] / cur["steps"])
                rows.append(cur)
                log(f"{'learned' if learned else 'block-Jacobi'} steps {cur['first']}-{cur['last']}: "
                    f"{cur['iters_per_step']:.1f} it/step {cur['steps_per_s']:.1f} steps/s "
                    f"fb {cur['fallback']} fp64 {cur['fp64']} broken {cur['broken']}")
            cur, t0 = None, t1
        if failed:
            log(f"step {failed['step']} did not converge: {failed}")
            break
    m.close()
    return dict(windows=rows, failed=failed)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ellipsoid", choices=["ellipsoid", "beam", "block"],
                    help="ellipsoid: the 619,830-tet ductile ellipsoid (the metric's workload); beam: the "
                         "122,880-tet notched beam in three-point bending, with --crack-fraction pre-broken edges; "
                         "block: a 168,432-tet block pulled from both ends in quasi-static load steps "
                         "(--material; --steps load steps, one JSON line of its own)")
    ap.add_argument("--material", default="stone", choices=["stone", "wood", "cheese"],
                    help="block workload: stone, wood or cheese (kernel support R_d 0, 0.1, 0.5 m)")
    ap.add_argument("--newton-rtol", type=float, default=1e-4, help="block workload: Newton force tolerance")
    ap.add_argument("--cg-max-iter", type=int, default=None, help="block workload: PCG iteration cap per solve")
    ap.add_argument("--pull", type=float, default=None, help="block workload: m each end moves per load step")
    ap.add_argument("--energy", default="stable_neo_hookean", choices=["stable_neo_hookean", "stvk"],
                    help="element energy of the dynamic workloads")
    ap.add_argument("--visual", action="store_true",
                    help="after the timed leg, time the split visualisation mesh (gf_get_visual_mesh)")
    ap.add_argument("--readback", action="store_true",
                    help="after the legs, time the same window as one gf_step(1) call per step, without and with "
                         "the positions and damage labels read back to the host after every step")
    ap.add_argument("--crack-fraction", type=float, default=0.0)
    ap.add_argument("--dt", type=float, default=None, help="time step (default: 1e-2 ellipsoid, 1e-4 beam)")
    ap.add_argument("--precond", default="learned", choices=["learned", "block_jacobi"])
    ap.add_argument("--net-every", type=int, default=4, help="network inference every N steps (factor every step)")
    ap.add_argument("--reorder", default="none", choices=["none", "rcm"],
                    help="internal node numbering: the generator's order or reverse Cuthill-McKee")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2103_14870_amd", "weights", "precond_net.npy"))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="before the legs, one device-to-device copy of this many MiB from a cache-cold "
                         "source (calibrates the HBM byte counters)")
    ap.add_argument("--trajectory", type=int, default=0, metavar="N",
                    help="instead of the metric: N steps from rest with each preconditioner, one call per step, "
                         "printing per-window iterations and steps/s (one JSON line)")
    ap.add_argument("--window", type=int, default=25, help="window length of --trajectory")
    ap.add_argument("--stats-summary", metavar="STATS_CSV",
                    help="write the kernel statistics summary from a rocprofv3 --kernel-trace --stats run and exit")
    ap.add_argument("--counter-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the HBM counter summary from two rocprofv3 --pmc runs and exit (no GPU)")
    args = ap.parse_args()
    if args.stats_summary:
        if args.workload == "block":
            write_stats_summary(
                args.stats_summary,
                "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/statsQ -o run -- "
                f"python bench.py --workload block --material {args.material} --steps 10 --warmup 0 --no-cpu-baseline",
                os.path.join(ROOT, "profiles", f"qs_{args.material}_block168k_kernel_stats.txt"),
                f"# rocprofv3 kernel statistics: bench.py on the 168,432-tet {args.material} block pulled from both "
                "ends, one MI355X\n# (10 quasi-static load steps from rest: Newton with a line search, "
                "block-Jacobi PCG)")
            return
        write_stats_summary(args.stats_summary,
                            "rocprofv3 --kernel-trace --stats --output-format csv -d gpurun_out/statsL -o run -- "
                            "python bench.py --steps 10 --warmup 5 --no-cpu-baseline")
        return
    if args.counter_summary:
        cmd = ("timeout -s KILL 280 rocprofv3 --pmc {} --output-format csv -d gpurun_out/pmc{} -o run -- "
               "python bench.py --steps 10 --warmup 5 --no-cpu-baseline --calib-copy-mb {}")
        write_counter_summary(*args.counter_summary, args.calib_copy_mb or 512,
                              cmd.format("FETCH_SIZE", "F", args.calib_copy_mb or 512),
                              cmd.format("WRITE_SIZE", "W", args.calib_copy_mb or 512))
        return
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding a mesh over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2103_14870_amd import gfem, meshgen

    if args.calib_copy_mb > 0:
        # The source is evicted from the 256 MB last-level cache by filling a
        # 1 GiB buffer after it, so the copy reads all of it from HBM.
        nel = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        evict = torch.full(((1 << 30) // 4,), 2.0, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        float(src.sum())  # read calibration: args.calib_copy_mb MiB read from HBM
        evict.fill_(3.0)
        torch.cuda.synchronize()
        dst.copy_(src)  # copy calibration: the same size read and written
        torch.cuda.synchronize()
        del src, dst, evict

    log = lambda msg: print(f"bench: {msg}", file=sys.stderr, flush=True)
    if args.workload == "block":
        kw = {} if args.pull is None else {"pull": args.pull}
        if args.dt is not None:
            kw["dt"] = args.dt
        if args.cg_max_iter is not None:
            kw["cg_max_iter"] = args.cg_max_iter
        prob = meshgen.pulled_block(args.material, **kw)
        nu, thr, radius = meshgen.BLOCK_MATERIALS[args.material]
        workload = (f"{args.material} block {prob.n_tets} tets / {prob.n_nodes} nodes pulled from both ends, "
                    f"quasi-static load steps (Newton + line search to {args.newton_rtol:g} of the first force), "
                    f"R_d={radius:g} m, Green-strain threshold {thr:g}, block-Jacobi PCG to 1e-6")
        log(f"quasi-static leg ({args.material})")
        t0 = time.perf_counter()
        m = gfem.mesh_from_problem(prob)
        create_s = time.perf_counter() - t0
        stream = torch.cuda.Stream()
        m.set_stream(stream.cuda_stream)
        leg = quasi_static_leg(m, args.steps, args.warmup, args.newton_rtol, max(1, min(args.steps, 5)), log)
        n_edges = m.n_edges
        m.close()
        steps = max(leg["done"], 1)
        out = {"mode": "quasi_static", "workload": workload, "material": args.material,
               "tets": prob.n_tets, "nodes": prob.n_nodes, "edges": n_edges, "damage_radius": radius,
               "load_steps": leg["done"], "warmup": args.warmup, "failed": leg["failed"],
               "load_steps_per_s": leg["done"] / max(leg["elapsed"], 1e-12),
               "ms_per_load_step": 1000.0 * leg["elapsed"] / steps,
               "newton_per_load_step": leg["newton"] / steps,
               "pcg_iters_per_newton": leg["inner"] / max(leg["newton"], 1),
               "line_search_halvings": leg["halvings"], "broken": leg["windows"][-1]["broken"] if leg["windows"] else 0,
               "create_s": create_s, "windows": leg["windows"], "dtype": "f32+f64", "data": "synthetic"}
        if not args.no_cpu_baseline:
            log("CPU oracle sample")
            out["cpu_baseline"] = cpu_baseline_qs(prob, args.newton_rtol)
            out["cpu_baseline"]["cpu_model"] = host_cpu_model()
        print(json.dumps(out), flush=True)
        return
    if args.workload == "ellipsoid":
        args.dt = args.dt or 1e-2
        prob = meshgen.ellipsoid(dt=args.dt)
        workload = (f"ellipsoid {prob.n_tets} tets / {prob.n_nodes} nodes, ductile (yield 0.05, damage 0.3), "
                    f"end caps pulled 1 cm/step, dt={args.dt:g}, PCG to 1e-6 FP64 rel. residual")
    else:
        args.dt = args.dt or 1e-4
        prob = meshgen.notched_beam(crack_fraction=args.crack_fraction, dt=args.dt)
        workload = (f"notched beam {prob.n_tets} tets / {prob.n_nodes} nodes, three-point bending, "
                    f"{100 * args.crack_fraction:g} % pre-broken edges, dt={args.dt:g}, PCG to 1e-6 FP64 rel. residual")
    prob.params["net_every_n_steps"] = args.net_every
    prob.params["reorder"] = args.reorder
    prob.params["energy"] = args.energy
    if args.energy != "stable_neo_hookean":
        workload += f", {args.energy} energy"
    stream = torch.cuda.Stream()
    net = None
    if args.precond == "learned":
        net = gfem.Net(seed=0)
        net.set_weights(np.load(args.weights))

    def make_mesh(learned):
        m = gfem.mesh_from_problem(prob)
        m.set_stream(stream.cuda_stream)
        if learned:
            gfem.attach_net(m, net)
        return m

    if args.trajectory > 0:
        out = {"mode": "trajectory", "workload": workload, "steps": args.trajectory, "window": args.window,
               "net_every_n_steps": args.net_every}
        legs = (("learned", True), ("block_jacobi", False)) if net is not None else (("block_jacobi", False),)
        for name, learned in legs:
            log(f"trajectory leg ({name})")
            out[name] = trajectory(make_mesh, args.trajectory, args.window, learned, log)
        print(json.dumps(out), flush=True)
        return
    log(f"timed leg ({args.precond})")
    m = make_mesh(net is not None)
    main_leg = timed_steps(m, args.steps, args.warmup)
    visual = None
    if args.visual:
        log("visualisation mesh")
        m.visual_mesh()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            xyz, grp = m.visual_mesh()
        visual = dict(ms_per_call=1000.0 * (time.perf_counter() - t0) / 5, bytes_out=xyz.nbytes + grp.nbytes,
                      split_tets=int(np.count_nonzero(grp.max(axis=1) > 0)))
    m.close()
    log("kernel timing leg")
    m = make_mesh(net is not None)
    kus, kn = kernel_times(m, args.steps, args.warmup)
    n_edges, n_blocks = m.n_edges, m.n_blocks
    if net is not None:
        # k_pcg_spmv_p: 36 B values + 4 B column per block; per block row the
        # row pointer (4 B), p read once (12 B) and q written (12 B)
        spmv_bytes = n_blocks * 40.0 + prob.n_nodes * 28.0
        spmv_name = "k_pcg_spmv_p (BSR 3x3 FP32 SpMV q = A p, partial p.q; factorised-preconditioner path)"
    else:
        _, spmv_bytes = m.bench_spmv(10)
        spmv_name = "k_pcg_spmv (BSR 3x3 FP32 SpMV fused with the direction update and p.q)"
    spmv_us = kus["spmv"] / max(kn["spmv"], 1)
    achieved = spmv_bytes / (spmv_us * 1e-6) / 1e9
    m.close()
    jac = None
    if net is not None:
        log("block-Jacobi leg")
        mj = make_mesh(False)
        jac = timed_steps(mj, args.steps, args.warmup)
        mj.close()
    readback = None
    if args.readback:
        readback = {}
        for key, rb in (("per_step_calls", False), ("with_readback", True)):
            log(f"per-call leg ({key})")
            mr = make_mesh(net is not None)
            readback[key] = per_call_steps(mr, args.steps, args.warmup, rb)
            mr.close()

    out = {
        "metric": "timesteps/s @620k tets: learned-PCG vs Jacobi-PCG at 1e-6 rel. residual",
        "value": main_leg["value"],
        "unit": "timesteps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * main_leg["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64 (bf16 network and factor)" if net is not None else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": workload,
            "tets": prob.n_tets, "nodes": prob.n_nodes, "edges": n_edges, "blocks": n_blocks,
            "precond": args.precond, "net_every_n_steps": args.net_every if net is not None else None,
            "dt": args.dt, "reorder": args.reorder, "parallelism": "single GPU",
        },
        "pcg_iters_per_step": main_leg["iters"],
        "outer_iters_per_step": main_leg["outer"],
        "fallback_steps": main_leg["fallback"],
        "kernel_us_per_step": {k: v / args.steps for k, v in kus.items()},
        "kernel_avg_us_per_launch": {k: kus[k] / kn[k] for k in kus if kn.get(k)},
        "roofline": {
            "kernel": spmv_name,
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
            "avg_launch_us": spmv_us, "launches": kn["spmv"], "bytes_per_launch": spmv_bytes,
            "timing": "HIP events recorded by each SpMV dispatch over the timed step window",
        },
    }
    prof_us = profile_avg_us("k_pcg_spmv_p<") if net is not None else None
    if prof_us:
        # the same kernel's mean duration in the committed rocprofv3 statistics
        out["roofline"]["profile_avg_launch_us"] = prof_us
        out["roofline"]["profile_frac"] = spmv_bytes / (prof_us * 1e-6) / 1e9 / HBM_PEAK_GBS
    if visual is not None:
        out["visual_mesh"] = visual
    if readback is not None:
        out["readback"] = readback
    if jac is not None:
        out["block_jacobi"] = {"value": jac["value"], "pcg_iters_per_step": jac["iters"],
                               "ms_per_step": 1000.0 * jac["elapsed"] / args.steps}
        out["speedup_vs_block_jacobi"] = main_leg["value"] / jac["value"]
    if not args.no_cpu_baseline:
        log("CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(prob)
        out["cpu_baseline"]["host_cpus"] = os.cpu_count()
        out["cpu_baseline"]["cpu_model"] = host_cpu_model()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
