"""Benchmark of the explicit octree-SBFEM hot path on one MI355X.

Workload (default): one GPU's share of a paper-scale run -- a unit box with
three random ellipsoidal inclusions (E ratio 5, rho ratio 2), octree levels
8/9, ~3.0e8 dofs in ~9.9e7 cells, Ricker patch load, base fixed.  A step is
one pass of the whole hot path: load, element-by-element internal force of
every cell, central-difference update of every dof.

Timed: K steps after W warm-up steps, bracketed by torch.cuda.synchronize(),
with HIP events on the stream the library launches on.  The headline value
is the FP32-product / FP64-state path; the plain FP64 path (and the colour
assembly) are timed beside it.  HIP events that the library records around
each launch on the same stream, in the same timed region, give the average
duration per launch of each kernel class for the roofline figure; the
algorithmic bytes per launch come from the library's layout report.

Serving (reported beside the throughput): a Poisson stream of 256 requests
(mean 20/s) of seeded inclusion meshes of 1e4-5e6 dofs (log-uniform) with
200-3000 steps each, built before the clock.  Requests are admitted in
arrival order while their device footprint fits a 4 GB budget, then again
with the whole free HBM; p50/p99 latency is arrival -> result on the host.
A seeded subset is re-run alone and compared with its served result.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config cfg3|cfg2]
                       [--serve N] [--serve-only]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF-steps/s vs FP64 plain at ≤1e-5 rel err; % HBM roofline; p99 solve latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(mesh):
    """Bytes the method must move per step (FP64 state): per dof u_n, u_{n-1}, M^-1 read and
    u_{n+1} written (8 B each); per cell its node ids (4 B each) and orientation, level,
    material (1 B each); per load entry index + value (16 B).  The library reports the same
    count per pass, for the mesh's state storage."""
    return 32 * mesh.n_dof + 4 * int(mesh.conn.shape[0]) + 3 * mesh.n_cells + 16 * len(mesh.load_dof)


def owner_kernel_name(prod, state="fp64"):
    """rocprofv3's short name of the owner-tile kernel instance for a product / state form."""
    from paper_2103_09100_amd.binding import PROD, STATE
    return f"tiled_step8<{PROD[prod]}, {STATE[state]}>"


def hang_kernel_name(prod, state="fp64"):
    from paper_2103_09100_amd.binding import PROD, STATE
    return f"tiled_hang_mma<{PROD[prod]}, {STATE[state]}>"


COUNTERS = {"cfg3": os.path.join(ROOT, "profiles", "cfg3_owner_tiles_hbm_counters.txt"),
            "cfg4": os.path.join(ROOT, "profiles", "cfg4_pattern_rich_hbm_counters.txt")}


def roofline_block(r, copy_gbs, prod, state="fp64", config="cfg3"):
    """Roofline of the owner-tile kernel (the dominant one) and of the whole step, from the
    library's algorithmic bytes per pass and the per-launch HIP events of the timed region."""
    k8 = r["kernels"]["element_8node"]
    kh = r["kernels"]["element_larger"]
    lay = r["layout"]
    alg8, algo = lay["alg_bytes_8node"], lay["alg_bytes_other"]
    achieved = alg8 / (k8["ms_avg"] * 1e-3) / 1e9 if k8["ms_avg"] > 0 else 0.0
    step_bytes = alg8 + algo
    kname = owner_kernel_name(prod, state)
    return {"bound": "hbm", "kernel": f"{kname}: owner-tile pass (regular 8-node cells, hanging-cell row forces, update)",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": counter_traffic(kname, COUNTERS.get(config, "")),
            "step_achieved": step_bytes / (r["ms_per_step"] * 1e-3) / 1e9,
            "step_frac": step_bytes / (r["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs if copy_gbs else None,
            "alg_bytes_per_launch": alg8, "alg_bytes_other_kernel": algo, "alg_bytes_per_step": step_bytes,
            "avg_launch_ms": k8["ms_avg"], "launches": k8["launches"],
            "timing": "step time from a region with events around the whole region only; kernel durations "
                      "from HIP events around each launch, on the launch stream, in a second region of as "
                      "many steps",
            "hang_kernel": hang_kernel_name(prod, state), "hang_avg_launch_ms": kh["ms_avg"]}


def kernel_sources_hash():
    """SHA-256 over the library's kernel and host sources (names and contents)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2103_09100_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".h", ".hip", ".cpp")):
            h.update(f.encode())
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def _kernel_short(name):
    import re
    m = re.search(r"sbfem::(\w+(?:<[^>]*>)?)\(", name)
    return m.group(1) if m else name.split("(")[0][:60]


def summarise_counters(fetch_dir, write_dir, out, header):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of every kernel in two rocprofv3 --pmc runs,
    with the scale factors that a plain 1 GiB read + 1 GiB write elementwise kernel gives."""
    import csv
    import glob
    from collections import defaultdict

    def per_kernel(d, counter):
        acc = defaultdict(lambda: defaultdict(float))
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r.get("Counter_Name") != counter:
                    continue
                acc[r["Kernel_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
        return {k: sum(v.values()) / len(v) for k, v in acc.items()}

    fetch, write = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    copy = [k for k in fetch if "AUnaryFunctor" in k]
    if not copy:
        raise SystemExit("no copy kernel in the fetch run (run the bench with --copy-probe)")
    copy_bytes = 1 << 30
    lines = [f"# {l}" for l in header] + [
        f"kernel_sources_sha256: {kernel_sources_hash()}",
        f"copy_kernel: elementwise y = 1.0 * x over 2^28 floats (reads {copy_bytes} B, writes {copy_bytes} B)",
        f"copy_fetch_kib: {fetch[copy[0]]:.1f}",
        f"copy_write_kib: {write[copy[0]]:.1f}",
        f"fetch_scale: {copy_bytes / 1024 / fetch[copy[0]]:.6f}",
        f"write_scale: {copy_bytes / 1024 / write[copy[0]]:.6f}",
    ]
    for k in sorted(fetch):
        if "sbfem::" in k:
            lines.append(f"fetch_kib[{_kernel_short(k)}]: {fetch[k]:.1f}")
    for k in sorted(write):
        if "sbfem::" in k:
            lines.append(f"write_kib[{_kernel_short(k)}]: {write[k]:.1f}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarise_trace(trace_dir, out, header):
    """Kernel statistics of a rocprofv3 --kernel-trace --stats run (per kernel: dispatches,
    average and total duration)."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True):
        rows += list(csv.DictReader(open(f)))
    lines = [f"# {l}" for l in header] + [f"kernel_sources_sha256: {kernel_sources_hash()}",
                                          "kernel | calls | average ns | total ns | percent"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"{_kernel_short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']):.0f} | "
                     f"{float(r['TotalDurationNs']):.0f} | {float(r['Percentage']):.2f}")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def counter_traffic(kernel, path):
    """HBM bytes per dispatch of `kernel` from the committed counter summary, scaled by the copy
    kernel's factors; None if there is none or the kernel sources changed since it was taken."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("#") or ":" not in line:
            continue
        k, v = line.split(":", 1)
        vals[k.strip()] = v.strip()
    if vals.get("kernel_sources_sha256") != kernel_sources_hash():
        return None
    try:
        f = float(vals[f"fetch_kib[{kernel}]"]) * 1024 * float(vals["fetch_scale"])
        w = float(vals[f"write_kib[{kernel}]"]) * 1024 * float(vals["write_scale"])
    except KeyError:
        return None
    return f + w


def make_mesh(name):
    from meshgen import configs
    if name == "cfg3":
        return configs.cfg3(keep_node_lat=True), "ellipsoid-inclusion octree L8/9 (one GPU's share of a paper-scale run)"
    if name == "cfg2":
        return configs.cfg2(), "sphere-band octree L3/7 with every cell pattern"
    if name == "cfg4":
        return configs.cfg4(), "sphere-band octree L4/8"
    raise SystemExit(f"unknown config {name}")


def time_mode(sim, torch, stream, steps, warmup, instrumented=True):
    """Wall time per step over `steps` steps, from events around the whole region only; then,
    unless `instrumented` is false, the same number of steps again with HIP events that the
    library records around each launch on the same stream (the per-launch events add a few
    microseconds between launches, so the step time comes from the first region): the average
    duration of each kernel class and the wall time per step of that second region."""
    with torch.cuda.stream(stream):
        sim.step(warmup)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        sim.step(steps)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        if not instrumented:
            return ms, {}, None
        sim.gpu.profile(True)
        a.record(stream)
        sim.step(steps)
        b.record(stream)
        torch.cuda.synchronize()
        ms_inst = a.elapsed_time(b) / steps
    prof = sim.gpu.profile_read()
    sim.gpu.profile(False)
    kernels = {k: dict(ms_total=v[0], launches=v[1], ms_avg=(v[0] / v[1] if v[1] else 0.0)) for k, v in prof.items()}
    return ms, kernels, ms_inst


def cpu_baseline(seconds=12.0, single_seconds=8.0):
    """The oracle (as it stands) on a bounded sample of the same recipe at levels 5/6: its step
    loop with the host's BLAS threads, and again limited to one core."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from meshgen import configs
    from oracle.solver import Oracle
    m = configs.inclusion_mesh(seed=0, lcoarse=5, lfine=6)
    configs._run_params(m, fm=4.0, n_steps=200)
    o = Oracle(m, workers=min(16, os.cpu_count() or 1))
    dt = 0.5 * o.critical_dt()

    def loop(limit):
        u, um1 = o.initial_state(dt)
        t0 = time.perf_counter()
        n = 0
        while n < 3 or time.perf_counter() - t0 < limit:
            unew, _ = o.step(u, um1, n, dt)
            um1, u = u, unew
            n += 1
        return n, time.perf_counter() - t0

    n, el = loop(seconds)
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    with threadpool_limits(1):
        n1, el1 = loop(single_seconds)
    return dict(value=m.n_dof * n / el, unit="DOF-steps/s", cores=int(threads), kind="oracle",
                sample=f"oracle step loop, same recipe at octree levels 5/6 ({m.n_dof} dofs, {m.n_cells} cells), "
                       f"{n} steps in {el:.1f} s",
                single_core=dict(value=m.n_dof * n1 / el1, unit="DOF-steps/s", cores=1,
                                 sample=f"the same loop with one BLAS thread, {n1} steps in {el1:.1f} s"))


def serving(torch, args):
    """The request stream served twice (memory budget, then the free HBM)."""
    from concurrent.futures import ThreadPoolExecutor
    from meshgen import configs
    from paper_2103_09100_amd.serve import Request, Server, latency_stats, link_cells
    from paper_2103_09100_amd.solver import Simulation, device_patterns

    specs = configs.serving_requests(seed=5, n=args.serve)
    t0 = time.time()

    def make(i):
        sp = specs[i]
        r = Request(i, configs.request_mesh(sp["seed"], sp["target_dof"], sp["n_steps"]), sp["n_steps"],
                    sp["arrival"])
        r.mesh.node_lat = None
        return link_cells(r)

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        reqs = list(ex.map(make, range(len(specs))))
    total = sum(r.mesh.n_dof * r.n_steps for r in reqs)
    log(f"[serve] {len(reqs)} requests built and linked in {time.time() - t0:.0f} s: "
        f"{sum(r.mesh.n_dof for r in reqs) / 1e6:.1f} M dofs, {total:.3e} dof-steps, "
        f"arrivals over {reqs[-1].arrival:.1f} s")
    device_patterns(reqs[0].mesh.nu)
    st, st2 = torch.cuda.Stream(), torch.cuda.Stream()
    # owner-tile shapes tuned per size bucket before the clock starts (first request of each bucket)
    from paper_2103_09100_amd.autotune import SERVING_CANDIDATES, ShapeCache
    shapes = ShapeCache(prod=args.serve_prod, candidates=SERVING_CANDIDATES, stream=st.cuda_stream)
    t0 = time.time()
    for r in reqs:
        shapes.shape(r.mesh)
    log(f"[serve] tile shapes tuned for {len(shapes.shapes)} size buckets in {time.time() - t0:.0f} s: "
        + ", ".join(f"4^{b}: {shapes.shapes[b][0]}" for b in sorted(shapes.shapes)))
    free = torch.cuda.mem_get_info()[0]
    out = {}
    for label, budget in (("budget", int(args.serve_budget_gb * 1e9)), ("full_hbm", int(0.9 * free))):
        for r in reqs:
            r.reset()
        srv = Server(budget_bytes=budget, quantum=args.serve_quantum, prod=args.serve_prod,
                     stream=st.cuda_stream, setup_stream=st2.cuda_stream, shapes=shapes,
                     graph_steps=args.serve_graph_steps)
        t1 = time.time()
        srv.run(reqs)
        stats = latency_stats(reqs)
        stats.update(budget_bytes=budget, wall_s=time.time() - t1,
                     queue_p50_s=float(np.percentile([r.admitted - r.arrival for r in reqs], 50)),
                     queue_p99_s=float(np.percentile([r.admitted - r.arrival for r in reqs], 99)))
        out[label] = stats
        log(f"[serve] {label} ({budget / 1e9:.1f} GB): p50 {stats['p50_s']:.3f} s, p99 {stats['p99_s']:.3f} s, "
            f"{stats['dof_steps_per_s']:.3e} dof-steps/s over {stats['span_s']:.1f} s")
    # a seeded subset, each run alone, against its served result (last run)
    pick = np.random.default_rng(5).choice(len(reqs), size=min(4, len(reqs)), replace=False)
    worst = 0.0
    for i in pick:
        r = reqs[i]
        tn, bt, btm = shapes.shape(r.mesh)
        sim = Simulation(r.mesh, prod=args.serve_prod, stream=st.cuda_stream, tile_nodes=tn, block_threads=bt,
                         block_threads_mixed=btm)
        sim.step(r.n_steps)
        alone = sim.u()
        sim.close()
        worst = max(worst, float(np.abs(r.result - alone).max() / max(np.abs(alone).max(), 1e-300)))
    out["tile_shapes"] = {f"4^{b}": dict(chosen=list(shapes.shapes[b]),
                                         ms_per_step={str(list(c)): round(ms, 4) for c, ms in shapes.tables[b]})
                          for b in sorted(shapes.shapes)}
    out.update(requests=len(reqs), product=args.serve_prod, state="fp64", quantum=args.serve_quantum,
               graph_steps=args.serve_graph_steps,
               dof_steps=float(total), alone_vs_served_max_rel=worst, alone_checked=[int(i) for i in pick],
               workload="Poisson stream (20/s) of seeded inclusion octrees, 1e4-5e6 dofs log-uniform, "
                        "200-3000 steps, built before the clock")
    log(f"[serve] alone vs served, requests {list(map(int, pick))}: max rel {worst:.2e}")
    return out


def oracle_snapshots(mesh, steps, every):
    """The FP64 oracle's stored snapshots of this mesh (tests/golden), or None when the file
    does not cover this run (another mesh, step count or snapshot spacing)."""
    path = os.path.join(ROOT, "tests", "golden", "cfg4_oracle_snapshots.txt")
    if not os.path.exists(path):
        return None
    sys.path.insert(0, os.path.dirname(path))
    from make_oracle_snapshots import read
    ref = read(path)
    if ref["mesh_fingerprint"] != mesh.fingerprint() or ref["steps"] != steps or ref["every"] != every:
        return None
    return ref


def golden_error(ref, snaps):
    """e_max over the stored sample nodes and max nodes, over the largest stored |u|_inf."""
    sample = ref["sample_nodes"]
    num = 0.0
    for r in ref["snaps"]:
        u = snaps[r["step"]].reshape(-1, 3)
        num = max(num, float(np.abs(u[sample] - r["u"]).max()), float(np.abs(u[r["imax"]] - r["umax"]).max()))
    return num / max(r["norm"] for r in ref["snaps"])


def precision_sweep(torch, args):
    """Products FP64/FP32/FP16/BF16 x state FP64/compensated FP32/FP32 on the cfg4 mesh.
    Per combination: DOF-steps/s over a timed run; the max relative displacement error over
    the sampled steps of a --sweep-steps run against the FP64/FP64 path (itself pinned to the
    oracle by the tests; the oracle does not run at this size here); and the drift of the
    discrete energy H_{n+1/2} over the free-vibration phase after the load has ended (the
    undamped scheme keeps it constant), evaluated on the host in FP64 with the library's
    FP64 operator and lumped mass."""
    from meshgen import configs
    from paper_2103_09100_amd.solver import Simulation
    mesh = configs.cfg4(n_steps=args.sweep_steps)
    log(f"[sweep] cfg4 mesh: {mesh.n_cells} cells, {mesh.n_dof} dofs")
    stream = torch.cuda.Stream()
    n_total, every = args.sweep_steps, 100
    evaluator = Simulation(mesh, prod="fp64", state="fp64", stream=stream.cuda_stream)
    M = evaluator.gpu.read(3, stream.cuda_stream)[0]
    dt = evaluator.dt
    # the Ricker pulse is below 1e-12 P0 once (t - t1) / (t1 / 5) >= 8, i.e. for t >= 2.6 t1
    assert mesh.load["kind"] == "ricker"
    t_end = int(np.ceil(2.6 * mesh.load["t1"] / dt))
    if t_end >= n_total - 2 * every:
        raise SystemExit(f"the load lasts until step {t_end}: no free-vibration phase in {n_total} steps")
    h_at = sorted(set(list(range(t_end + every - t_end % every, n_total + 1, 2 * every)) + [n_total]))

    def energy(u, un):  # H_{n+1/2} from u_{n+1} = u, u_n = un
        evaluator.write(un, un, 0)
        f = evaluator.internal_force()
        d = u - un
        return 0.5 * (d @ (M * d)) / dt ** 2 + 0.5 * (u @ f)

    golden = oracle_snapshots(mesh, n_total, every)
    ref_snaps, rows = {}, []
    combos = [(p, st) for p in ("fp64", "fp32", "fp16", "bf16") for st in ("fp64", "kahan32", "fp32")]
    for prod, state in combos:
        sim = Simulation(mesh, prod=prod, state=state, stream=stream.cuda_stream)
        ms, _, _ = time_mode(sim, torch, stream, args.sweep_time_steps, 5, instrumented=False)
        sim.close()
        sim = Simulation(mesh, prod=prod, state=state, stream=stream.cuda_stream)
        snaps, H = {}, []
        done = 0
        while done < n_total:
            sim.step(every)
            done += every
            snaps[done] = sim.u()
            if done in h_at:
                u, n = sim.gpu.read(0, stream.cuda_stream)
                un, _ = sim.gpu.read(1, stream.cuda_stream)
                H.append(energy(u, un))
        sim.close()
        if (prod, state) == ("fp64", "fp64"):
            ref_snaps = snaps
        num = max(float(np.abs(snaps[k] - ref_snaps[k]).max()) for k in ref_snaps)
        den = max(float(np.abs(ref_snaps[k]).max()) for k in ref_snaps)
        H = np.array(H)
        drift = float(np.abs(H - H[0]).max() / abs(H[0])) if len(H) > 1 else float("nan")
        row = dict(product=prod, state=state, ms_per_step=ms, dof_steps_per_s=mesh.n_dof / (ms * 1e-3),
                   e_max_vs_fp64=num / den, energy_drift=drift, energy_samples=len(H))
        if golden is not None:
            row["e_max_vs_oracle_sampled"] = golden_error(golden, snaps)
        if prod in ("fp16", "bf16"):
            row["products_note"] = ("regular 8-node cells: Walsh operands and coefficients rounded to 16 bits, "
                                    "FP32 arithmetic; hanging-node cells: 16-bit matrix instructions with FP32 "
                                    "accumulation")
        rows.append(row)
        log(f"[sweep] {prod} products, {state} state: {ms:.3f} ms/step ({row['dof_steps_per_s']:.3e} DOF-steps/s), "
            f"e_max vs FP64 {row['e_max_vs_fp64']:.3e}, vs oracle (sampled) "
            f"{row.get('e_max_vs_oracle_sampled', float('nan')):.3e}, energy drift {drift:.3e} ({len(H)} samples)")
    evaluator.close()
    return dict(workload=f"cfg4 sphere-band octree L4/8, {mesh.n_dof} dofs, {mesh.n_cells} cells",
                steps=n_total, snapshot_every=every, load_ends_at_step=t_end, energy_steps=h_at, rows=rows)


def copy_bandwidth(torch, stream, n_bytes=1 << 30, reps=10):
    """HBM bandwidth of a plain copy on this GPU (read n_bytes, write n_bytes), the faster of
    the runtime's device copy and an elementwise kernel (y = 1 * x): the practical ceiling
    that the roofline fraction is also quoted against."""
    x = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    best = 0.0
    for op in (lambda: y.copy_(x), lambda: torch.mul(x, 1.0, out=y)):
        with torch.cuda.stream(stream):
            for _ in range(3):
                op()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                op()
            b.record(stream)
        torch.cuda.synchronize()
        best = max(best, 2 * n_bytes / (a.elapsed_time(b) / reps * 1e-3) / 1e9)
    del x, y
    torch.cuda.empty_cache()
    return best


def small_mesh_latency(torch, steps=1000, graph_steps=50, prods=("fp64", "fp32")):
    """Per-step time of the 2187-dof cube (launch-bound): steps launched one by one vs
    replayed from a graph of `graph_steps` steps; the two final states are compared."""
    from meshgen import configs
    from paper_2103_09100_amd.solver import Simulation
    stream = torch.cuda.Stream()
    m = configs.cfg1()
    out = {"workload": "cfg1: unit cube 8x8x8 cells, 2187 dofs, tiled assembly", "steps": steps,
           "graph_steps": graph_steps}
    for prod in prods:
        row = {}
        for label, g in (("direct", 0), ("graph", graph_steps)):
            sim = Simulation(m, prod=prod, assembly="tiled", stream=stream.cuda_stream, graph_steps=g)
            sim.step(2 * graph_steps)  # warm-up (captures the graph)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(steps)
            torch.cuda.synchronize()
            row[label + "_us_per_step"] = (time.perf_counter() - t0) / steps * 1e6
            row[label + "_u"] = sim.u()
            sim.close()
        row["rel_diff"] = float(np.abs(row.pop("graph_u") - row["direct_u"]).max() / np.abs(row["direct_u"]).max())
        row.pop("direct_u")
        out[prod] = row
        log(f"[bench] cfg1 {prod}: {row['direct_us_per_step']:.1f} us/step launched, "
            f"{row['graph_us_per_step']:.1f} us/step from graphs, diff {row['rel_diff']:.1e}")
    return out


def eigen_workload(torch, levels=(1, 2), k=100):
    """Sec. 5.1: the lowest k circular frequencies of the sliding cube (edge 8, E = 1000,
    nu = 0.3, rho = 1) by sbfem_eigen_lowest on the element-by-element operator; wall time of
    the call and the error against the analytic 3D frequencies (P and S waves with the
    paper's multiplicity rule)."""
    from meshgen import configs
    from paper_2103_09100_amd.solver import Simulation
    L, E, NU, RHO = 8.0, 1000.0, 0.3, 1.0
    vp = np.sqrt(E * (1 - NU) / (RHO * (1 + NU) * (1 - 2 * NU)))
    vs = np.sqrt(E / (2 * RHO * (1 + NU)))
    exact = []
    for i in range(12):
        for j in range(12):
            for l in range(12):
                if i == j == l == 0:
                    continue
                kk = np.pi * np.sqrt(i * i + j * j + l * l) / L
                zeros = (i == 0) + (j == 0) + (l == 0)
                exact += [vp * kk] + [vs * kk] * {2: 0, 1: 1, 0: 2}[zeros]
    exact = np.sort(exact)[:k]
    out = {"workload": f"Sec. 5.1 sliding cube, lowest {k} frequencies, FP64", "levels": []}
    for level in levels:
        m = configs.sliding_cube(level, L=L, E=E, rho=RHO, nu=NU)
        sim = Simulation(m, prod="fp64", state="fp64", assembly="tiled")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        w, r, it = sim.gpu.eigen_lowest(k, max_iter=400, tol=1e-9)
        dt = time.perf_counter() - t0
        sim.close()
        err = float(np.sqrt(((w - exact) ** 2).sum() / (exact ** 2).sum()))
        row = {"level": level, "n_dof": m.n_dof, "seconds": dt, "iterations": it, "max_residual": float(r.max()),
               "omega_1": float(w[0]), "omega_k": float(w[-1]), "rel_error_vs_analytic": err}
        out["levels"].append(row)
        log(f"[eigen] cube level {level} ({m.n_dof} dofs): {k} frequencies in {dt:.2f} s, {it} iterations, "
            f"residual {r.max():.1e}, error vs analytic {err:.4f}")
    return out


def cache_resident_mesh(torch, steps=500):
    """The 2e6-dof all-pattern mesh (it fits the 256 MB last-level cache): time per step and
    DOF-steps/s of the FP32 and FP64 paths, with their final states compared."""
    from meshgen import configs
    from paper_2103_09100_amd.solver import Simulation
    stream = torch.cuda.Stream()
    m = configs.cfg2()
    out = {"workload": f"cfg2: sphere-band octree L3/7 with every cell pattern, {m.n_dof} dofs, {m.n_cells} cells",
           "steps": steps}
    finals = {}
    for prod in ("fp32", "fp64"):
        sim = Simulation(m, prod=prod, assembly="tiled", stream=stream.cuda_stream)
        ms, _, _ = time_mode(sim, torch, stream, steps, 10, instrumented=False)
        finals[prod] = sim.u()
        out[prod] = {"ms_per_step": ms, "dof_steps_per_s": m.n_dof / (ms * 1e-3)}
        sim.close()
        log(f"[bench] cfg2 {prod}: {ms * 1e3:.1f} us/step, {m.n_dof / (ms * 1e-3):.3e} DOF-steps/s")
    out["rel_err_fp32_vs_fp64"] = float(np.abs(finals["fp32"] - finals["fp64"]).max() /
                                        max(np.abs(finals["fp64"]).max(), 1e-300))
    return out


def accuracy_run(torch, mesh, steps, every=250):
    """FP32 products against FP64 products (both FP64 state) on one mesh over `steps` steps:
    e_max = max over the sampled steps of |u32 - u64|_inf / max over the same steps of
    |u64|_inf (the error measure of the mixed path's target)."""
    from paper_2103_09100_amd.solver import Simulation
    stream = torch.cuda.Stream()
    sims = {p: Simulation(mesh, prod=p, assembly="tiled", stream=stream.cuda_stream) for p in ("fp32", "fp64")}
    num, den, done, samples = 0.0, 0.0, 0, []
    while done < steps:
        k = min(every, steps - done)
        for sim in sims.values():
            sim.step(k)
        done += k
        u32, u64 = sims["fp32"].u(), sims["fp64"].u()
        d, r = float(np.abs(u32 - u64).max()), float(np.abs(u64).max())
        num, den = max(num, d), max(den, r)
        samples.append({"step": done, "diff_inf": d, "ref_inf": r})
        log(f"[accuracy] step {done}: |u32 - u64| {d:.3e}, |u64| {r:.3e}")
    for sim in sims.values():
        sim.close()
    return {"steps": steps, "every": every, "e_max": num / den if den else 0.0, "samples": samples}


def run_modes(torch, mesh, plan, stream, label="bench"):
    """Create, time and read back each (prod:assembly, steps, warm-up) of the plan in turn."""
    from paper_2103_09100_amd.solver import Simulation
    results, finals = {}, {}
    for mode, n_steps, n_warm in plan:
        prod, assembly = mode.split(":")
        t1 = time.time()
        sim = Simulation(mesh, prod=prod, assembly=assembly, stream=stream.cuda_stream)
        info = sim.gpu.info()
        log(f"[{label}] {mode}: created in {time.time() - t1:.0f} s, dt={sim.dt:.4e}, "
            f"{info['n_colours']} colours, {info['device_bytes'] / 1e9:.1f} GB, layout {sim.gpu.layout()}")
        ms, prof, ms_inst = time_mode(sim, torch, stream, n_steps, n_warm)
        finals[mode] = sim.u()
        results[mode] = dict(ms_per_step=ms, value=mesh.n_dof / (ms * 1e-3), kernels=prof, steps=n_steps,
                             layout=sim.gpu.layout(), ms_per_step_instrumented=ms_inst)
        log(f"[{label}] {mode}: {ms:.3f} ms/step, {results[mode]['value']:.3e} DOF-steps/s, "
            + ", ".join(f"{k} {v['ms_avg']:.3f} ms x{v['launches']}" for k, v in prof.items()))
        sim.close()
        del sim
        torch.cuda.empty_cache()
    return results, finals


def pattern_rich(torch, stream, copy_gbs, steps, warmup):
    """The 2.07e7-dof sphere-band mesh (1.3 % hanging-node cells, every pattern): throughput
    and roofline of the FP32 and FP64 paths."""
    from meshgen import configs
    mesh = configs.cfg4()
    log(f"[cfg4] mesh: {mesh.n_cells} cells, {mesh.n_dof} dofs, "
        f"{int((mesh.cell_slots != 0).sum())} hanging-node cells")
    res, finals = run_modes(torch, mesh, [("fp32:tiled", steps, warmup), ("fp64:tiled", steps, warmup)], stream,
                            label="cfg4")
    out = {"workload": f"cfg4: sphere-band octree L4/8, {mesh.n_dof} dofs, {mesh.n_cells} cells", "steps": steps,
           "n_dof": mesh.n_dof}
    for mode, r in res.items():
        prod = mode.split(":")[0]
        out[prod] = {"ms_per_step": r["ms_per_step"], "value": r["value"],
                     "kernels_ms_avg": {c: d["ms_avg"] for c, d in r["kernels"].items()},
                     "roofline": roofline_block(r, copy_gbs, prod, config="cfg4")}
    out["speedup_fp32_vs_fp64"] = res["fp32:tiled"]["value"] / res["fp64:tiled"]["value"]
    ref = finals["fp64:tiled"]
    out["rel_err_fp32_vs_fp64"] = float(np.abs(finals["fp32:tiled"] - ref).max() / np.abs(ref).max())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="cfg3")
    ap.add_argument("--modes", default="fp32:tiled,fp64:tiled")
    ap.add_argument("--compare", default="fp32:atomic,fp32:colour",
                    help="assembly variants timed beside the headline over --compare-steps steps")
    ap.add_argument("--compare-steps", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--serve", type=int, default=256, help="requests in the serving stream (0: skip)")
    ap.add_argument("--small", type=int, default=1000, help="steps of the small-mesh latency check (0: skip)")
    ap.add_argument("--mid", type=int, default=500, help="steps of the cache-resident 2e6-dof mesh (0: skip)")
    ap.add_argument("--eigen-level", type=int, default=2,
                    help="finest refinement of the Sec. 5.1 eigenfrequency cube (-1: skip)")
    ap.add_argument("--pattern-rich-steps", type=int, default=200,
                    help="steps of the 2e7-dof all-pattern mesh, with its own roofline (0: skip)")
    ap.add_argument("--accuracy-steps", type=int, default=0,
                    help="only compare FP32 with FP64 products on the bench mesh over this many steps")
    ap.add_argument("--graph-steps", type=int, default=50, help="steps per captured graph")
    ap.add_argument("--serve-only", action="store_true", help="only the serving stream")
    ap.add_argument("--serve-budget-gb", type=float, default=4.0)
    ap.add_argument("--serve-quantum", type=int, default=50, help="steps per batched call")
    ap.add_argument("--serve-prod", default="fp32")
    ap.add_argument("--serve-graph-steps", type=int, default=0,
                    help="replay the batched steps of the serving loop from cached HIP graphs of this many steps")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (scale for the HBM byte counters)")
    ap.add_argument("--sweep", action="store_true",
                    help="precision sweep on the cfg4 mesh (products x state storage) instead of the benchmark")
    ap.add_argument("--sweep-steps", type=int, default=2000)
    ap.add_argument("--sweep-time-steps", type=int, default=200)
    ap.add_argument("--summarise", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT"),
                    help="write the HBM counter summary of two rocprofv3 --pmc runs and exit")
    ap.add_argument("--summarise-trace", nargs=2, metavar=("TRACE_DIR", "OUT"),
                    help="write the kernel statistics of a rocprofv3 --kernel-trace --stats run and exit")
    ap.add_argument("--summary-header", action="append", default=[],
                    help="comment line for --summarise / --summarise-trace (workload, commands)")
    args = ap.parse_args()
    if args.summarise:
        summarise_counters(*args.summarise, header=args.summary_header)
        return
    if args.summarise_trace:
        summarise_trace(*args.summarise_trace, header=args.summary_header)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU path "
              f"(one process per GPU with a halo exchange) is designed but not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2103_09100_amd.solver import Simulation

    if args.sweep:
        sw = precision_sweep(torch, args)
        print(json.dumps({"metric": "precision sweep: DOF-steps/s, max relative displacement error vs FP64, "
                                    "energy drift", "n_gpus": 1, "data": "synthetic", "sweep": sw}), flush=True)
        return

    if args.serve_only:
        sv = serving(torch, args)
        print(json.dumps({"metric": "p99 solve latency (serving stream)", "value": sv["budget"]["p99_s"],
                          "unit": "s", "n_gpus": 1, "higher_is_better": False, "vs_baseline": None,
                          "dtype": args.serve_prod, "data": "synthetic",
                          "config": {"workload": sv["workload"]}, "serving": sv}), flush=True)
        return

    t0 = time.time()
    mesh, desc = make_mesh(args.config)
    log(f"[bench] mesh {args.config}: {mesh.n_cells} cells, {mesh.n_nodes} nodes, {mesh.n_dof} dofs "
        f"({time.time() - t0:.0f} s)")
    if args.accuracy_steps > 0:
        acc = accuracy_run(torch, mesh, args.accuracy_steps)
        print(json.dumps({"metric": "max relative displacement difference, FP32 vs FP64 products (FP64 state)",
                          "value": acc["e_max"], "unit": "relative", "n_gpus": 1, "higher_is_better": False,
                          "data": "synthetic", "config": {"workload": f"{args.config}: {desc}"},
                          "accuracy": acc}), flush=True)
        return
    ab = dict(step=algorithmic_bytes(mesh))
    log(f"[bench] algorithmic bytes/step {ab['step'] / 1e9:.3f} GB ({ab['step'] / mesh.n_dof:.1f} B/dof)")

    stream = torch.cuda.Stream()
    if args.copy_probe:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        log("[bench] copy probe: 3 x (read 1 GiB, write 1 GiB) elementwise kernel")
        del x, y
    copy_gbs = copy_bandwidth(torch, stream)
    log(f"[bench] plain copy on this GPU: {copy_gbs:.0f} GB/s")
    plan = [(m, args.steps, args.warmup) for m in args.modes.split(",") if m]
    plan += [(m, args.compare_steps, 2) for m in args.compare.split(",") if m]
    results, finals = run_modes(torch, mesh, plan, stream)

    head = args.modes.split(",")[0]
    fp64 = next((m for m in args.modes.split(",") if m.startswith("fp64:")), None)
    r = results[head]
    roof = roofline_block(r, copy_gbs, head.split(":")[0], config=args.config)
    if roof["alg_bytes_per_step"] != ab["step"]:
        log(f"[bench] warning: per-pass algorithmic bytes {roof['alg_bytes_per_step']} != step bytes {ab['step']}")
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {desc}", "n_dof": mesh.n_dof, "n_cells": mesh.n_cells,
                   "product": head.split(":")[0], "state": "fp64", "assembly": head.split(":")[1],
                   "steps_per_call": args.steps},
        "roofline": roof,
        "modes": {k: dict(ms_per_step=v["ms_per_step"], value=v["value"], steps=v["steps"],
                          ms_per_step_instrumented=v["ms_per_step_instrumented"],
                          kernels_ms_avg={c: d["ms_avg"] for c, d in v["kernels"].items()})
                  for k, v in results.items()},
    }
    if fp64:
        out["fp64_plain"] = results[fp64]["value"]
        out["speedup_vs_fp64"] = r["value"] / results[fp64]["value"]
        ref = finals[fp64]
        out["rel_err_vs_fp64"] = float(np.abs(finals[head] - ref).max() / np.abs(ref).max())
    if args.pattern_rich_steps > 0:
        out["pattern_rich_mesh"] = pattern_rich(torch, stream, copy_gbs, args.pattern_rich_steps, 20)
    if args.small > 0:
        out["small_mesh_step_us"] = small_mesh_latency(torch, args.small, args.graph_steps)
    if args.mid > 0:
        out["cache_resident_mesh"] = cache_resident_mesh(torch, args.mid)
    if args.eigen_level >= 0:
        out["eigen_workload"] = eigen_workload(torch, levels=tuple(range(max(0, args.eigen_level - 1),
                                                                         args.eigen_level + 1)))
    if args.serve > 0:
        out["serving"] = serving(torch, args)
        out["p99_latency_s"] = out["serving"]["budget"]["p99_s"]
    if not args.no_cpu:
        log("[bench] oracle baseline on the host")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
