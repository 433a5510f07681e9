"""Throughput of the solid-LBM step on one MI355X.

A bench step is one lattice-Boltzmann time step of the whole plate: pull
streaming with the boundary rules, moments, density-gradient source term,
equilibrium, collision, displacement update and the non-finite guard, all in
the fused kernel.  The default workload is the 2048 x 2048 plate with a
centred hole of radius 256 (curved traction-free wall, lambda/mu = 2,
tau_bar = 0.6, fp32 populations, fp64 displacement).  Its line also carries
the fp64-plain step on the same plate, a 4096^2 plate, a 2048^2 plate with a
moving curved Dirichlet wall, the served trace (p50/p99 latency) and the
three-dimensional step on two 256^3 boxes (the pulled slab and the porous
solid) as sub-records.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-extras]
    python bench.py --workload batch64     # 64 uneven plates, batched vs one at a time
    python bench.py --workload serve       # served requests: continuous batching vs one at a time
    python bench.py --workload cube256     # the three-dimensional (D3Q19) step on a 256^3 slab
    python bench.py --workload cavities256 # the 3-D step on a 256^3 porous solid (64 pressurised cavities)

Prints one JSON line.  `value` is material-site updates per second (MLUPS)
with the state already in device memory when the timed region starts; the
roofline object relates the fused kernel's algorithmic bytes to the 8 TB/s
HBM peak (bound "mall" when the working set fits the 256 MB Infinity Cache,
which then serves most of it), and reports the measured DRAM-side traffic and
rate beside it; cpu_baseline times the plain CPU reference on a bounded
sample of the same plate.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def workload(name):
    from slbm_workloads import configs
    table = {
        "crack1024x512": (lambda: configs.edge_crack_plate(), "fp32"),
        # as specified (lambda/mu = 2, tau_bar = 0.6): its traction-free walls
        # grow a surface mode and the state overflows after ~150 steps; the
        # same geometry at lambda = mu does the same work for longer
        "hole2048": (lambda: configs.hole_plate(), "fp32"),
        "hole2048-lm1": (lambda: configs.hole_plate(lam=0.05, tau=0.55), "fp32"),
        "square128": (lambda: configs.square_clamped_pulled(), "fp64"),
        "square4096": (lambda: configs.square_clamped_pulled(4096, steps=2000), "fp32"),
        # curved Dirichlet walls, one moving (ramped): periodic, no free wall, stable
        "movinghole2048": (lambda: configs.moving_hole_plate(), "fp32"),
    }
    if name not in table:
        raise SystemExit(f"unknown workload {name}; choose from {sorted(table)}, batch64, serve, cube<N> or cavities<N>")
    f, prec = table[name]
    return f(), prec


def box3_workload(name):
    """("cube" | "cavities", n) for the 3-D workloads cube<n> and cavities<n>
    (n >= 64 for cavities), else None."""
    for kind in ("cube", "cavities"):
        tail = name[len(kind):]
        if name.startswith(kind) and tail.isdigit() and int(tail) > 0 and (kind == "cube" or int(tail) >= 64):
            return kind, int(tail)
    return None


def bytes_per_site(prec):
    # populations read once and written once, displacement (2 x fp64) read and written once
    return 9 * 2 * (4 if prec == "fp32" else 8) + 2 * 2 * 8


def shape_key(rows, strip, group, lists):
    """Name of a launch shape in the counter summaries: rows x strip, the XCD
    group, and whether the two-step kernel ran with per-tile cut-link lists."""
    return f"{rows}x{strip}" + (f"-g{group}" if group else "") + ("-lists" if lists else "")


def measured_traffic(plate, prec, tuned, group=0, lists=False):
    """HBM bytes per launch of the step kernel from the committed counter
    summary (profiles/traffic_<workload>_<precision>.json), or None when there
    is none for this workload and launch shape or the kernel changed since."""
    from paper_2208_04088_amd.build import kernel_fingerprint
    path = os.path.join(ROOT, "profiles", f"traffic_{plate.name}_{prec}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_fingerprint") != kernel_fingerprint():
        return None
    shape = d.get("shapes", {}).get(shape_key(tuned[0], tuned[1], group, lists))
    return shape["traffic_bytes_per_launch"] if shape else None


def cpu_baseline(plate, budget_s=15.0, one_core_s=8.0):
    """The plain CPU reference (fp64) on a bounded number of steps of the
    same plate, timed with every host thread it is allowed and with one."""
    import oracle
    from oracle import Oracle
    cores = oracle.set_threads(0)
    o = Oracle(plate)
    o.step(1)

    def rate(seconds):
        # steps in growing batches until the time budget is spent
        t0 = time.perf_counter()
        n = 0
        while True:
            el = time.perf_counter() - t0
            if el >= seconds:
                break
            k = 1 if n == 0 else max(1, min(int((seconds - el) / (el / n)) + 1, 2 * n))
            o.step(k)
            n += k
        dt = time.perf_counter() - t0
        return plate.n_material * n / dt / 1e6, n, dt

    v, n, dt = rate(budget_s)
    oracle.set_threads(1)
    v1, n1, dt1 = rate(one_core_s)
    oracle.set_threads(cores)
    return {"value": round(v, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{n} steps of {plate.name} ({plate.n_material} material sites), fp64, "
                      f"{dt:.1f} s on {cores} threads; then {n1} steps on 1 thread, {dt1:.1f} s",
            "value_one_core": round(v1, 3), **host_cpu()}


def host_cpu():
    """The host CPU model and the hardware threads this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count()
    return {"cpu_model": model, "host_threads_available": n}


def copy_ceiling(slbm, torch, dev, stream):
    """GB/s of the plain copy kernel over a 2 GiB buffer, timed like the step."""
    src_t = torch.empty(1 << 29, dtype=torch.float32, device=dev)
    dst_t = torch.empty_like(src_t)
    nbytes = src_t.numel() * 4
    for _ in range(3):
        slbm.copy(dst_t.data_ptr(), src_t.data_ptr(), nbytes, 0, stream.cuda_stream)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(10):
        slbm.copy(dst_t.data_ptr(), src_t.data_ptr(), nbytes, 0, stream.cuda_stream)
    c1.record(stream)
    torch.cuda.synchronize()
    return round(2 * nbytes * 10 / (c0.elapsed_time(c1) / 1e3) / 1e9, 1)


def bytes_per_site3(prec):
    # D3Q19 populations read once and written once, displacement (3 x fp64) read and written once
    return 19 * 2 * (4 if prec == "fp32" else 8) + 3 * 2 * 8


def link_record_bytes3(prec):
    # one cut link's record as the kernels read it: 12 reals and two 32-bit words
    return 56 if prec == "fp32" else 104


def bytes_per_step3(box, prec):
    """Algorithmic HBM bytes of one 3-D step: every material site's
    populations and displacement read and written once; with cut links also
    each site's flags (4 B) and each link record once."""
    if box.mask is None:
        return box.n_sites * bytes_per_site3(prec)
    return box.n_material * bytes_per_site3(prec) + 4 * box.n_sites + len(box.links) * link_record_bytes3(prec)


def has_ext_links3(box):
    """Whether the box has Neumann cut links whose data are extrapolated along
    the link (neumann_order 1, not thin): those take a launch of their own."""
    from slbm_workloads.box3d import NEUMANN
    if box.mask is None or not len(box.links) or box.neumann_order != 1:
        return False
    return any(box.groups[g].kind == NEUMANN for g in set(box.links["group"].tolist()))


def measured_traffic3(box, prec):
    """Calibrated counter bytes per step of the two 3-D kernels
    (profiles/traffic_<box>_<precision>.json), or None when there is none or
    the kernels changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{box.name}_{prec}.json")
    if not os.path.exists(path):
        return None
    from paper_2208_04088_amd.build import kernel_fingerprint
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_fingerprint") != kernel_fingerprint("step3_kernel.h"):
        return None
    shapes = d.get("shapes", {})
    kernels = ("k3_links_ext",) if has_ext_links3(box) else ()
    kernels += ("k3_density", "k3_step")
    parts = [shapes.get(k) for k in kernels]
    return None if None in parts else sum(p["traffic_bytes_per_launch"] for p in parts)


def cpu_baseline3(box, budget_s=15.0, sample=None):
    """The CPU reference (numpy, fp64) on a bounded sample: a 64^3 box of the
    same configuration (or `sample`), stepped for about `budget_s` seconds."""
    import numpy as np
    from oracle.slbm3d import Oracle3D
    from slbm_workloads import box3d as B
    if sample is None:
        n = min(64, box.nx)
        sample = B.Box3(n, min(64, box.ny), min(64, box.nz), lam=box.lam, mu=box.mu, tau=box.tau, rho=box.rho,
                        force=box.force, x_walls=box.x_walls, name=f"{box.name}-sample{n}")
    o = Oracle3D(sample)
    o.step(1)
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < budget_s:
        o.step(1)
        k += 1
    dt = time.perf_counter() - t0
    # numpy's elementwise loops and einsum (no BLAS path) run on one thread
    return {"value": round(sample.n_material * k / dt / 1e6, 3), "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{k} steps of a {sample.nx}x{sample.ny}x{sample.nz} box of the same configuration "
                      f"({sample.n_material} material sites), numpy fp64 on one thread, {dt:.1f} s", **host_cpu()}


STEPS3_SUB, WARMUP3_SUB = 200, 20     # the 3-D sub-records of the default line


def box3_of(kind, n, steps):
    """The n^3 box of a 3-D workload and, for the cavities, the smaller box
    the CPU baseline samples."""
    from slbm_workloads import box3d as B
    if kind == "cavities":
        box = B.cavities_box3(n, per_axis=max(1, n // 64), steps=steps)
        sample = B.cavities_box3(64, per_axis=1, radius=0.3 * n / max(1, n // 64), seed=1)
        return box, sample
    return B.cube_pulled(n, steps=steps), None


def time_box3(torch, stream, box, prec, steps, warm):
    """Times `steps` steps of `box` after `warm` untimed ones; returns the
    record (value, config, roofline) without the copy ceiling."""
    import numpy as np
    from paper_2208_04088_amd import slbm3
    s = slbm3.Solver3(box, prec, device=0, stream=stream.cuda_stream)
    s.step(warm)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    ev0.record(stream)
    s.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    t_step = ev0.elapsed_time(ev1) / 1e3 / steps
    try:
        s.sync()                          # the divergence flag (the timing does not depend on it)
        diverged = False
    except slbm3.S.SlbmError:
        diverged = True
    assert diverged or np.isfinite(s.displacement()).all()
    sites = box.n_material
    bps = bytes_per_site3(prec)
    step_bytes = bytes_per_step3(box, prec)
    achieved = step_bytes / t_step / 1e9
    result = {
        "metric": "MLUPS (site updates per second) of the D3Q19 solid-LBM step",
        "value": round(sites / t_step / 1e6, 1), "unit": "MLUPS", "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": round(t_step * 1e3, 6), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": box.name, "nx": box.nx, "ny": box.ny, "nz": box.nz, "sites": box.n_sites,
                   "material_sites": sites,
                   "precision": "fp32 populations and arithmetic, fp64 displacement" if prec == "fp32" else "fp64",
                   "lambda_over_mu": box.lam / box.mu, "tau": box.tau,
                   "bench_step": "one D3Q19 time step of the whole box (density pass and step kernel; "
                                 "with cut links the step also forms the next step's rule values)",
                   "diverged": diverged, "wall_s": round(wall, 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic3(box, prec),
                     "kernel": ("k3_links_ext + " if has_ext_links3(box) else "") + "k3_density + k3_step",
                     "bytes_per_site": bps, "bytes_per_step": step_bytes,
                     "launches_per_step": 3 if has_ext_links3(box) else 2,
                     "avg_step_us": round(t_step * 1e6, 3),
                     "note": "achieved counts the step's algorithmic bytes over the time of all its launches; "
                             "the density pass re-reads the pulled populations (traffic: measured bytes per step)"},
    }
    s.close()
    return result


def run_3d(args, torch, dev, stream, n, kind="cube"):
    """The three-dimensional (D3Q19) step on an n^3 box: kind "cube", a slab
    with face x = -1/2 clamped and face x = n - 1/2 pulled by a step
    traction, periodic in y and z; kind "cavities", a porous solid periodic on
    every axis with (n/64)^3 pressurised spherical cavities (cut links of
    every q and normal).  fp32 populations, fp64 displacement, from rest.  One
    bench step is one time step of the whole box (two launches: density pass,
    step); the rate counts material sites."""
    from paper_2208_04088_amd import slbm
    steps = args.steps if args.steps_given else 1000
    box, sample = box3_of(kind, n, steps)
    result = time_box3(torch, stream, box, args.precision or "fp32", steps, min(args.warmup, 100))
    result["roofline"]["copy_kernel_gbs"] = copy_ceiling(slbm, torch, dev, stream)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline3(box, sample=sample)
    print(json.dumps(result), flush=True)


def run_batch(args, slbm, torch, dev, stream):
    """64 independent plates of uneven size and geometry (seed 0), every one
    advanced `steps` steps: once as one batch (one launch per step, or two,
    for all plates, steps replayed from captured graphs, the launch shape
    picked by slbm_batch_autotune during warm-up), once one plate at a time
    with plain launches in each plate's autotuned shape.  Same plates, same
    arithmetic: the displacements of the plates that stay finite must agree
    bit for bit.  A plate whose state overflows (lambda/mu > 1 grows a mode
    at traction-free walls) is retired by the batch and stopped, at the next
    check, one at a time; throughput counts the plates that completed."""
    import numpy as np
    from slbm_workloads import configs
    steps = args.steps if args.steps_given else 5000
    plates = configs.batch_plates(seed=0, count=64, steps=steps)
    warm = 512
    check = 1024                          # one-at-a-time divergence check interval (steps)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    # batched: warm-up steps pick the launch shape (or the one given), then the timed steps
    b = slbm.Batch(200 << 30, device=0, stream=stream.cuda_stream)
    slots = [b.add(p, warm + steps, "fp32") for p in plates]
    if args.seg:
        b.set_launch(args.seg, args.strip or 62)
        b.set_xcd_group(args.xcd_group)
        b.step(warm)
    else:
        b.autotune(warm)
        taken = max(b.solver(sl).time()[0] for sl in slots)   # plates still running took every trial step
        b.step(warm - taken)
    shape = b.launch()
    # the cooperative batched kernel runs when every plate carries tile lists
    batch_lists = shape[1] == 58 and all(b.solver(sl).boundary_lists()[0] == shape[0] for sl in slots)
    b.sync()
    e0, e1 = ev(), ev()
    w0 = time.perf_counter()
    e0.record(stream)
    b.step(steps)
    e1.record(stream)
    b.sync()
    torch.cuda.synchronize()
    wall_b = time.perf_counter() - w0
    t_batch = e0.elapsed_time(e1) / 1e3
    u_batch, ok_batch = [], []
    for sl in slots:
        sv = b.solver(sl)
        try:
            sv.sync()
            ok_batch.append(True)
        except slbm.SlbmError as e:
            if e.code != -4:
                raise
            ok_batch.append(False)
        u_batch.append(sv.displacement())
    b.close()

    # one plate at a time: the same warm-up and step counts, plain launches
    t_seq, ok_seq, equal = 0.0, [], 0
    for p, ub, okb in zip(plates, u_batch, ok_batch):
        s = slbm.Solver(p, "fp32", device=0, stream=stream.cuda_stream)
        s.step(warm)
        torch.cuda.synchronize()
        s.autotune()
        e0, e1 = ev(), ev()
        e0.record(stream)
        done, ok = 0, True
        while done < steps:
            k = min(check, steps - done)
            s.step(k)
            done += k
            try:
                s.sync()
            except slbm.SlbmError as e:
                if e.code != -4:
                    raise
                ok = False
                break
        e1.record(stream)
        torch.cuda.synchronize()
        t_seq += e0.elapsed_time(e1) / 1e3
        ok_seq.append(ok)
        if ok and okb:
            equal += bool(np.array_equal(s.displacement(), ub))
        s.close()
    done_sites = sum(p.n_material for p, ok in zip(plates, ok_batch) if ok)
    mlups = done_sites * steps / t_batch / 1e6
    achieved = done_sites * bytes_per_site("fp32") * steps / t_batch / 1e9
    result = {
        "metric": "MLUPS (material-site updates per second) of the fused D2Q9 solid-LBM step",
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": round(t_batch / steps * 1e3, 6), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": "batch64-seed0", "plates": len(plates),
            "material_sites": sum(p.n_material for p in plates), "completed_material_sites": done_sites,
            "precision": "fp32 populations and arithmetic, fp64 displacement",
            "bench_step": "one lattice-Boltzmann time step of all 64 plates (one batched launch per one or "
                          "two steps); throughput counts the plates that stay finite",
            "batched_launch_shape": list(shape),
            "sequential_mlups": round(done_sites * steps / t_seq / 1e6, 1),
            "speedup_vs_sequential": round(t_seq / t_batch, 3),
            "plates_completed": [sum(ok_batch), sum(ok_seq)],
            "plates_diverged": [len(plates) - sum(ok_batch), len(plates) - sum(ok_seq)],
            "completed_plates_bitwise_equal_to_sequential": equal,
            "wall_s": round(wall_b, 4),
        },
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            # the plate mix of a batched launch changes as plates finish or are
            # retired: a profiled run's average bytes per launch (in the batch's
            # profile) does not describe the timed region's launches
            "traffic": None,
            "traffic_note": "per-launch DRAM bytes depend on which plates are still running; the batch's profile "
                            "gives the average over a profiled run",
            "kernel": "k_step2_batch" if shape[1] == 58 else "k_step_batch",
            "tile_lists": batch_lists,
            "bytes_per_site": bytes_per_site("fp32"),
            "steps_per_launch": 2 if shape[1] == 58 else 1,
            "avg_launch_us": round(t_batch / steps * 1e6 * (2 if shape[1] == 58 else 1), 3),
            "copy_kernel_gbs": copy_ceiling(slbm, torch, dev, stream),
        },
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(plates[0])
    print(json.dumps(result), flush=True)


def serve_record(args, slbm, torch, stream, both_orders=False):
    """The first `--requests` requests of the served trace (seed 1, Poisson
    arrivals at `--rate` per second, 50 by default, plates 256^2-4096^2,
    1e3-2e4 steps; the rate only stretches the arrival times) under a 200 GB
    budget: continuous batching (paper_2208_04088_amd.serve.Server, rounds
    of about 20 ms of device work, two rounds in flight) against the same
    requests one plate at a time (least work first; with both_orders also
    oldest first).  Latency runs from a request's arrival to its
    displacement being back on the host; percentiles and throughput are over
    the requests that completed, and requests whose state overflowed
    (lambda/mu > 1) are counted apart."""
    from paper_2208_04088_amd import serve
    from slbm_workloads import configs
    t = time.perf_counter()
    trace = configs.served_trace(seed=1, count=args.requests, rate=args.rate)
    t_build = time.perf_counter() - t
    # two steps per launch; rows per tile and XCD map as given (--seg, --xcd-group), else 10 rows, bands
    launch = (args.seg, args.strip or 58) if args.seg else (10, 58)
    srv = serve.Server(200 << 30, chunk=64, stream=stream.cuda_stream, launch=launch,
                       max_resident_sites=2_000_000, policy="swf", xcd_group=args.xcd_group, round_ms=20.0,
                       timing_stream=stream)
    res = srv.run(trace)
    srv.close()
    torch.cuda.synchronize()
    st = serve.summary(res)
    seq_swf = serve.summary(serve.run_one_at_a_time(trace, stream=stream.cuda_stream, policy="swf",
                                                    launch=launch, xcd_group=args.xcd_group))
    out = {
        "workload": f"served-trace-seed1-first{args.requests}" + ("" if args.rate == 50 else f"-rate{args.rate:g}"),
        "requests": args.requests, "arrival_rate_per_s": args.rate, "hbm_budget_gb": 200,
        "precision": "fp32 populations and arithmetic, fp64 displacement",
        "policy": "least work first, at most 2M material sites resident (more when one plate is larger)",
        "launch_shape": list(launch), "xcd_group": args.xcd_group,
        "p50_latency_s": st.get("p50_latency_s"), "p99_latency_s": st.get("p99_latency_s"),
        "aggregate_mlups": st.get("aggregate_mlups"),
        "completed": st["requests"], "diverged": st["diverged"],
        "gpu_busy_fraction": (round(srv.gpu_busy_s / srv.gpu_span_s, 4) if srv.gpu_span_s else None),
        "rounds": srv.rounds,
        "served": st, "one_at_a_time_least_work_first": seq_swf,
        "speedup_vs_one_at_a_time": round(seq_swf["makespan_s"] / st["makespan_s"], 3),
        "peak_resident_plates": srv.peak_resident, "peak_device_gb": round(srv.peak_bytes / 1e9, 2),
        "trace_build_s": round(t_build, 1),
    }
    if both_orders:
        seq = serve.summary(serve.run_one_at_a_time(trace, stream=stream.cuda_stream, launch=launch,
                                                    xcd_group=args.xcd_group))
        out["one_at_a_time"] = seq
        out["speedup_vs_one_at_a_time_oldest_first"] = round(seq["makespan_s"] / st["makespan_s"], 3)
    return out, trace


def run_serve(args, slbm, torch, dev, stream):
    """The served trace as its own line (see serve_record)."""
    rec, trace = serve_record(args, slbm, torch, stream, both_orders=True)
    st = rec["served"]
    st.setdefault("aggregate_mlups", 0.0)
    result = {
        "metric": "MLUPS (material-site updates per second) of the fused D2Q9 solid-LBM step",
        "value": st["aggregate_mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": int(sum(r.steps for r in trace)),
        "warmup": 0, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": dict(rec, bench_step="serve every request of the trace (each plate its own step count)"),
        "roofline": {
            "bound": "hbm", "achieved": round(st["aggregate_mlups"] * bytes_per_site("fp32") / 1e3, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(st["aggregate_mlups"] * bytes_per_site("fp32") / 1e3 / HBM_PEAK_GBS, 4),
            "traffic": None, "kernel": "k_step2_batch", "steps_per_launch": 2,
            "bytes_per_site": bytes_per_site("fp32"),
        },
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(trace[0].plate)
    print(json.dumps(result), flush=True)


MALL_BYTES = 256 << 20          # the Infinity Cache (MALL) in front of HBM


def working_set_bytes(plate, prec):
    """Device bytes one step touches: both population buffers, U and the
    per-site flags, in the library's padded layout (64 columns of left
    padding, rows rounded to 64, one row of padding above and below)."""
    ld = (64 + plate.nx + 1 + 63) // 64 * 64
    plane = ld * (plate.ny + 2)
    es = 4 if prec == "fp32" else 8
    return plane * (2 * 9 * es + 2 * 8 + 1)


def time_plate(args, slbm, torch, stream, plate, prec, steps, warmup, shape=None):
    """One plate: warm-up steps, the launch shape (autotuned on this plate, or
    `shape` = (rows, strip, xcd group)), then `steps` steps timed with events
    on the library's stream.  Returns the line's fields without cpu_baseline."""
    s = slbm.Solver(plate, prec, device=0, stream=stream.cuda_stream)

    def diverged_sync():
        # a plate that overflowed (SLBM_E_DIVERGED) keeps stepping at the same
        # cost; the line reports the flag
        try:
            s.sync()
            return False
        except slbm.SlbmError as e:
            if e.code != -4:
                raise
            return True

    if shape is not None:
        s.set_launch(shape[0], shape[1])
        s.set_xcd_group(shape[2])
        s.step(warmup)
        diverged_warm = diverged_sync()
    else:
        s.step(warmup)
        diverged_warm = diverged_sync()
        s.autotune()                  # rows per tile, strip width and XCD map, measured on this plate
    rows, strip, group = s.launch()
    strip = strip or 62
    lists = s.boundary_lists()
    torch.cuda.synchronize()

    # timed region: K steps queued back to back on one stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    ev0.record(stream)
    s.step(steps)
    ev1.record(stream)
    diverged = diverged_sync() or diverged_warm
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    region_ms = ev0.elapsed_time(ev1)

    # per-launch kernel time: events around single launches (a launch takes
    # two steps with strip width 58)
    spl = 2 if strip == 58 else 1
    n_probe = min(200, max(20, steps // 50))
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_probe)]
    for a, b in evs:
        a.record(stream)
        s.step(spl)
        b.record(stream)
    torch.cuda.synchronize()
    launch_ms = sorted(a.elapsed_time(b) for a, b in evs)
    launch_med_ms = launch_ms[len(launch_ms) // 2]
    # the probe launches step on past the timed region: report the state at the end
    diverged_end = diverged_sync()
    steps_end = s.time()[0]
    if not diverged_end:
        import numpy as np
        assert np.isfinite(s.displacement()).all()
    s.close()

    sites = plate.n_material
    t_step = region_ms / 1e3 / steps
    bps = bytes_per_site(prec)
    achieved = sites * bps / t_step / 1e9
    avg_launch_us = t_step * spl * 1e6
    ws = working_set_bytes(plate, prec)
    traffic = measured_traffic(plate, prec, (rows, strip), group, lists=strip == 58 and lists[0] == rows)
    roof = {
        # a working set inside the Infinity Cache is served from it, not from HBM
        "bound": "hbm" if ws > MALL_BYTES else "mall",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "achieved_dram_gbs": None if traffic is None else round(traffic / avg_launch_us / 1e3, 1),
        "kernel": "k_step2" if spl == 2 else "k_step",
        "bytes_per_site": bps,
        "steps_per_launch": spl,
        "avg_launch_us": round(avg_launch_us, 3),
        "single_launch_median_us": round(launch_med_ms * 1e3, 3),
        "rows_per_tile": rows,
        "strip_width": strip,
        "xcd_group": group,
        "working_set_bytes": ws,
    }
    if spl == 2:
        # the boundary rules evaluated tile by tile from per-tile cut-link lists
        roof["tile_lists"] = {"rows": lists[0], "records": lists[1], "max_per_tile": lists[2]}
        roof["note"] = (
            "achieved counts bytes_per_site per site update (the one-step minimum); this kernel takes two "
            "steps per launch and reads and writes the state once per launch, so it needs half that from HBM; "
            "traffic is the measured bytes per launch and achieved_dram_gbs the rate it moves them at")
    return {
        "value": round(sites / t_step / 1e6, 1),
        "ms_per_step": round(t_step * 1e3, 6),
        "dtype": "f32" if prec == "fp32" else "f64",
        "config": {
            "workload": plate.name, "nx": plate.nx, "ny": plate.ny, "material_sites": sites,
            "precision": "fp32 populations and arithmetic, fp64 displacement" if prec == "fp32" else "fp64",
            "lambda_over_mu": plate.lam / plate.mu, "tau": plate.tau, "neumann_order": plate.neumann_order,
            "bench_step": "one lattice-Boltzmann time step of the whole plate",
            "wall_s": round(wall, 4),
            "diverged": diverged,
            "diverged_after_probes": diverged_end, "steps_after_probes": steps_end,
        },
        "roofline": roof,
    }


def sub_record(r, steps, warmup):
    """A timed plate as a sub-record of the line."""
    out = {"metric": "MLUPS", "value": r["value"], "unit": "MLUPS", "steps": steps, "warmup": warmup,
           "ms_per_step": r["ms_per_step"], "dtype": r["dtype"]}
    out.update({"config": r["config"], "roofline": r["roofline"]})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="hole2048")
    ap.add_argument("--rate", type=float, default=50.0, help="arrival rate of the served trace (requests/s)")
    ap.add_argument("--precision", default=None)
    ap.add_argument("--seg", type=int, default=0, help="rows per tile (0: autotuned)")
    ap.add_argument("--strip", type=int, default=0,
                    help="strip width 62 or 64, or 58 for two steps per launch (0: autotuned)")
    ap.add_argument("--xcd-group", type=int, default=0,
                    help="with --seg, and for the served workload: workgroups to XCDs, 0 contiguous bands, "
                         "g interleaved groups of g")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="the hole plate alone, without the fp64, 4096^2, moving-wall, served and 3-D sub-records")
    ap.add_argument("--requests", type=int, default=256, help="served workload: requests of the trace")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design, not a build", file=sys.stderr)
        sys.exit(2)

    args.steps_given = args.steps is not None
    default_line = args.workload == "hole2048" and not args.no_extras and args.precision in (None, "fp32") \
        and not args.seg
    if args.steps is None:
        args.steps = 20 if args.workload == "hole2048" else 10000
    if args.warmup is None:
        args.warmup = 5 if args.workload == "hole2048" else 500
    special = args.workload in ("batch64", "serve") or box3_workload(args.workload) is not None
    if not special:
        workload(args.workload)          # exits with the list of workloads for an unknown name
    if args.precision not in (None, "fp32", "fp64"):
        raise SystemExit(f"unknown precision {args.precision}; choose fp32 or fp64")

    import torch
    from paper_2208_04088_amd import slbm

    torch.cuda.init()
    dev = torch.device("cuda:0")
    # a stream of torch's (default priority) that the library queues on, so
    # that torch's events time the library's kernels
    stream = torch.cuda.Stream(device=dev)
    assert stream.cuda_stream != 0
    if args.workload == "batch64":
        run_batch(args, slbm, torch, dev, stream)
        return
    if args.workload == "serve":
        run_serve(args, slbm, torch, dev, stream)
        return
    if box3_workload(args.workload) is not None:
        run_3d(args, torch, dev, stream, *reversed(box3_workload(args.workload)))
        return

    plate, prec = workload(args.workload)
    prec = args.precision or prec
    shape = (args.seg, args.strip or 62, args.xcd_group) if args.seg else None
    r = time_plate(args, slbm, torch, stream, plate, prec, args.steps, args.warmup, shape)
    result = {
        "metric": "MLUPS (material-site updates per second) of the fused D2Q9 solid-LBM step",
        "value": r["value"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": r["dtype"],
        "data": "synthetic",
        "config": r["config"],
        "roofline": r["roofline"],
    }
    # streaming reference: a plain copy of a 2 GiB buffer, timed the same way
    result["roofline"]["copy_kernel_gbs"] = copy_ceiling(slbm, torch, dev, stream)
    if default_line:
        # the metric's other halves on the same line: the fp64-plain step on
        # the same plate, a 4096^2 plate (1.5 GB, far above the cache), the
        # moving-wall plate and the served trace with its latency percentiles
        r64 = time_plate(args, slbm, torch, stream, plate, "fp64", args.steps, args.warmup)
        result["fp64"] = sub_record(r64, args.steps, args.warmup)
        big, _ = workload("square4096")
        steps_big = max(args.steps, 20)
        rbig = time_plate(args, slbm, torch, stream, big, "fp32", steps_big, args.warmup)
        result["square4096"] = sub_record(rbig, steps_big, args.warmup)
        # curved Dirichlet walls, one of them moving (eq:bbnoncon with j* != 0)
        mov, _ = workload("movinghole2048")
        rmov = time_plate(args, slbm, torch, stream, mov, "fp32", args.steps, args.warmup)
        result["movinghole2048"] = sub_record(rmov, args.steps, args.warmup)
        result["served"], _ = serve_record(args, slbm, torch, stream)
        # the three-dimensional step: the pulled slab and the porous solid
        # with pressurised cavities (cut links of every q and normal), 256^3
        for kind in ("cube", "cavities"):
            box, _ = box3_of(kind, 256, STEPS3_SUB)
            r3 = time_box3(torch, stream, box, "fp32", STEPS3_SUB, WARMUP3_SUB)
            result[f"{kind}256"] = sub_record(r3, STEPS3_SUB, WARMUP3_SUB)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(plate)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
