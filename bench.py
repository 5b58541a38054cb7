#!/usr/bin/env python3
"""Throughput of the modal DG shallow-water SSP-RK3 loop on one GPU.

    python bench.py [--steps K] [--warmup W] [--dtype f64|f32]

Workload: r = 3 (16 modes per variable, 4 x 4 Gauss-Legendre nodes),
180 x 90 latitude-longitude elements, h = 1e4 m plus a seeded band-limited
spherical-harmonic perturbation (l <= 16, 100 m) and a non-divergent
band-limited wind (20 m/s), SSP-RK3 at Courant number 0.1.  A step is one
SSP-RK3 step (three fused stage kernels).  The state is resident in GPU
memory before the timed region.

Prints one JSON line: DOF-updates/s (3 E N unknowns times stages per second),
the roofline of the stage kernel (algorithmic bytes per launch over its
average launch duration, measured with events on the launch stream), and
the FP64 oracle timed on the host on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_LON, N_LAT, ORDER, L_MAX, SEED, CFL = 180, 90, 3, 16, 2, 0.1
HBM_PEAK_GBS = 8000.0
METRIC = "DG RHS DOF-updates/s + % HBM roofline; learned r=1 vs plain r=4 at equal err"
COUNTERS = os.path.join(ROOT, "profiles", "k_dg_stage_r3_180x90.md")
# the sources of the stage kernel: counters recorded for another version of
# them are not reported
KERNEL_SRC = [os.path.join(ROOT, "paper_2303_11767_amd", "csrc", f)
              for f in ("dgsw_stage.hpp", "dgsw_kernels.hip", "dgsw_device.hpp")]
LEARNED_MODEL = os.path.join(ROOT, "paper_2303_11767_amd", "models", "learned_r1_360x180.npz")


def kernel_sha():
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(dtype, kernel, path=COUNTERS):
    """HBM bytes per stage launch from committed rocprofv3 counter runs,
    or None when they are missing or the kernel source changed since."""
    try:
        with open(path) as f:
            for line in f:
                if line.startswith("{") and '"kernel_sha"' in line:
                    rec = json.loads(line)
                    if (rec.get("dtype") == dtype and rec.get("kernel") == kernel
                            and rec.get("kernel_sha") == kernel_sha()):
                        return rec["hbm_bytes_per_launch"]
    except OSError:
        pass
    return None


def hbm_probe(nbytes=1 << 30, repeats=10):
    """Achievable device bandwidth: a device-to-device copy of `nbytes` (read
    plus write counted), the median of `repeats` copies."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.copy_(a)
    ts = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    t = sorted(ts)[len(ts) // 2]
    del a, b
    return {"kind": "device-to-device copy (torch copy_)", "bytes_copied": nbytes,
            "GBs": 2.0 * nbytes / t / 1e9, "us": t * 1e6}


def _oracle_steps(seconds):
    """SSP-RK3 steps of the benchmark workload by the FP64 oracle, as it
    stands, on one host thread, until about `seconds` of work: (steps,
    elapsed seconds, DOFs)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from dg_inputs import band_limited_state
    from oracle import SphereDG
    q, info = band_limited_state(N_LON, N_LAT, ORDER, L_MAX, SEED)
    with threadpool_limits(limits=1):
        m = SphereDG(N_LON, N_LAT, ORDER)
        dt = m.cfl_time_step(info.cmax, CFL)
        steps = 0
        t0 = time.perf_counter()
        while True:
            q = m.ssp_rk3_step(q, dt)
            steps += 1
            el = time.perf_counter() - t0
            if el >= seconds:
                break
    assert np.all(np.isfinite(q))
    return steps, el, 3 * m.E * m.N


def host_cpu():
    """Model name and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def cpu_baseline(seconds, max_procs=16):
    """The FP64 oracle timed on the host: one thread, and one single-threaded
    oracle process per available core (capped at `max_procs`) each stepping
    its own copy of the workload (aggregate rate, weak scaling).  The
    all-core figure is the reported baseline, the one-thread figure rides
    along."""
    import multiprocessing as mp
    model, ncpu = host_cpu()
    steps, el, dofs = _oracle_steps(seconds)
    single = dofs * 3 * steps / el
    procs = max(1, min(ncpu, max_procs))
    ctx = mp.get_context("spawn")
    with ctx.Pool(procs) as pool:
        res = pool.map(_oracle_steps, [seconds] * procs)
    agg = sum(d * 3 * s / e for s, e, d in res)
    return {"value": agg, "unit": "DOF-updates/s", "cores": procs, "kind": "oracle",
            "sample": f"SSP-RK3 steps of the 180x90 r=3 workload in FP64 NumPy: {procs} single-threaded "
                      f"oracle processes, one per core, each ~{seconds:.0f} s "
                      f"({sum(r[0] for r in res)} steps in all); host CPU {model}, {ncpu} cores available",
            "single_thread": {"value": single, "cores": 1,
                              "sample": f"{steps} steps on 1 host thread, {el:.1f} s"},
            "host_cpu": model}


def run(args):
    import numpy as np
    import torch

    import paper_2303_11767_amd as dg
    from dg_inputs import band_limited_state

    torch.cuda.set_device(0)
    q_h, info = band_limited_state(N_LON, N_LAT, ORDER, L_MAX, SEED)
    href = 1.0e4 if args.dtype == "f32" else 0.0
    mesh = dg.Mesh(N_LON, N_LAT, ORDER, dtype=args.dtype, h_ref=href)
    tdt = mesh.dtype
    q = torch.from_numpy(q_h).to(device="cuda", dtype=tdt).contiguous()
    work = mesh.empty_work()
    dt = dg.cfl_time_step(mesh, info.cmax, CFL)
    dofs = 3 * mesh.E * mesh.N
    state_bytes = dofs * q.element_size()
    stream = torch.cuda.current_stream()

    # warmup, then the timed region: exactly K steps, replayed from a HIP graph
    # of `chunk` captured steps (the library's graph path; the same kernels
    # and arguments as the eager launches)
    chunk = math.gcd(args.steps, 100)
    graph = mesh.graph(q, work, dt, nsteps=chunk)
    mesh.rk_step(q, work, dt, nsteps=args.warmup)
    graph.launch(stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # the timed region (exactly K steps between two synchronisations),
    # repeated; the median repeat is reported
    reps, walls = [], []
    for _ in range(max(1, args.repeats)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(args.steps // chunk):
            graph.launch(stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        reps.append(ev0.elapsed_time(ev1) * 1e-3)
    order = sorted(range(len(reps)), key=lambda k: reps[k])
    med = order[len(order) // 2]
    elapsed = max(reps[med], 1e-12)
    wall = walls[med]
    graph.close()
    mass = mesh.mass(q)
    if not all(np.isfinite(mass)):
        raise RuntimeError("state became non-finite")
    # the same K steps launched eagerly, for reference
    ev0.record(stream)
    mesh.rk_step(q, work, dt, nsteps=args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    eager_s = ev0.elapsed_time(ev1) * 1e-3

    # dg_rhs alone (dq/dt = M^-1 h(q), no stage combination): blocks of 100
    # calls between events, the median of the repeats; 2 state transfers each
    rhs_out = torch.empty_like(q)
    mesh.rhs(q, rhs_out, stream=stream)
    rhs_t = []
    for _ in range(max(1, args.repeats)):
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(100):
            mesh.rhs(q, rhs_out, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        rhs_t.append(ev0.elapsed_time(ev1) * 1e-3 / 100)
    rhs_s = sorted(rhs_t)[len(rhs_t) // 2]
    del rhs_out

    # the stage kernel alone: events around every launch of full 3-stage
    # cycles on the launch stream (for reference)
    w0, w1 = work[: q.numel()].view_as(q), work[q.numel():].view_as(q)
    cycles = args.kernel_cycles
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(3 * cycles)]
    torch.cuda.synchronize()
    for c in range(cycles):
        a, b = evs[3 * c]
        a.record(stream); mesh.rk_stage(q, None, w0, 0.0, 1.0, dt); b.record(stream)
        a, b = evs[3 * c + 1]
        a.record(stream); mesh.rk_stage(w0, q, w1, 0.75, 0.25, dt); b.record(stream)
        a, b = evs[3 * c + 2]
        a.record(stream); mesh.rk_stage(w1, q, q, 1.0 / 3.0, 2.0 / 3.0, dt); b.record(stream)
    torch.cuda.synchronize()
    per_launch = np.array([a.elapsed_time(b) for a, b in evs]) * 1e-3
    launch_s = float(per_launch.mean())
    alg_bytes = 8.0 * state_bytes / 3.0        # mean over the three stages
    # the stage kernel's mean duration over the timed region: 3 K launches back
    # to back from the graph, between two events on the launch stream (no host
    # launch cost between them); events around each single launch, which add
    # their own overhead, are reported beside it
    stage_s = elapsed / (3 * args.steps)
    achieved = alg_bytes / stage_s / 1e9
    kernel_name = "k_dg_stage_h2" if mesh.kernel == "half" else "k_dg_stage"
    traffic = measured_traffic(args.dtype, kernel_name)

    out = {
        "metric": METRIC,
        "value": dofs * 3 * args.steps / elapsed,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "plain DG SWE, r=3, 180x90 lat-lon elements, SSP-RK3, CFL 0.1, "
                               "band-limited l<=16 seed 2",
                   "n_lon": N_LON, "n_lat": N_LAT, "order": ORDER, "dofs": dofs,
                   "dt_s": dt, "h_ref": href, "state_bytes": state_bytes},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel_name, "alg_bytes_per_launch": alg_bytes,
                     "launch_us": stage_s * 1e6, "launch_us_events": launch_s * 1e6,
                     "stage_us": [float(per_launch[k::3].mean() * 1e6) for k in range(3)]},
        "wall_s_timed": wall,
        "repeats_ms_per_step": [r / args.steps * 1e3 for r in reps],
        "dof_steps_per_s": dofs * args.steps / elapsed,
        "timed_with": f"HIP graph of {chunk} steps replayed {args.steps // chunk} times; "
                      f"median of {len(reps)} repeats of the {args.steps}-step region",
        "value_eager_launches": dofs * 3 * args.steps / eager_s,
        "rhs_alone": {"us_per_call": rhs_s * 1e6, "dof_per_s": dofs / rhs_s,
                      "alg_GBs": 2.0 * state_bytes / rhs_s / 1e9,
                      "timed_with": "100 back-to-back dg_rhs calls between events, median of the repeats"},
    }
    return out


BIG = (1440, 720, 3, 32, 5)       # n_lon, n_lat, order, l_max, seed
BIG_COUNTERS = os.path.join(ROOT, "profiles", "k_dg_stage_r3_1440x720.md")


def big_fields():
    """Input of the large-mesh section (host work, run in a worker process
    while the GPU sections run)."""
    from dg_inputs import band_limited_state
    n_lon, n_lat, order, lmax, seed = BIG
    return band_limited_state(n_lon, n_lat, order, lmax, seed)


def big_section(fields, probe, steps=50, repeats=5):
    """The 1440 x 720 r = 3 FP64 mesh (398 MB state, beyond the 256 MB
    Infinity Cache, so the stage kernel streams from HBM): SSP-RK3 steps
    timed as the benchmark (median of `repeats`), the stage kernel's
    algorithmic bandwidth against the 8 TB/s peak and against the measured
    copy bandwidth, and its counter-measured HBM traffic."""
    import numpy as np
    import torch

    import paper_2303_11767_amd as dg
    n_lon, n_lat, order, lmax, seed = BIG
    q_h, info = fields
    mesh = dg.Mesh(n_lon, n_lat, order, dtype="f64")
    q = torch.from_numpy(q_h).to("cuda")
    work = mesh.empty_work()
    dt = dg.cfl_time_step(mesh, info.cmax, CFL)
    stream = torch.cuda.current_stream()
    mesh.rk_step(q, work, dt, nsteps=3)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        e0.record(stream)
        mesh.rk_step(q, work, dt, nsteps=steps)
        e1.record(stream)
        torch.cuda.synchronize()
        reps.append(e0.elapsed_time(e1) * 1e-3 / steps)
    step_s = sorted(reps)[len(reps) // 2]
    stage_s = step_s / 3.0              # three back-to-back stage launches per step
    if not all(np.isfinite(mesh.mass(q))):
        raise RuntimeError("large-mesh run became non-finite")
    dofs = 3 * mesh.E * mesh.N
    state_bytes = dofs * 8
    alg = 8.0 * state_bytes / 3.0
    achieved = alg / stage_s / 1e9
    kernel_name = "k_dg_stage_h2" if mesh.kernel == "half" else "k_dg_stage"
    traffic = measured_traffic("f64", kernel_name, BIG_COUNTERS)
    out = {"workload": f"plain DG SWE, r={order}, {n_lon}x{n_lat} lat-lon elements, FP64, SSP-RK3, "
                       f"CFL 0.1, band-limited l<={lmax} seed {seed}",
           "dofs": dofs, "state_bytes": state_bytes, "steps": steps,
           "ms_per_step": step_s * 1e3, "repeats_ms_per_step": [r * 1e3 for r in reps],
           "dof_updates_per_s": dofs * 3 / step_s,
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel_name,
                        "alg_bytes_per_launch": alg, "launch_us": stage_s * 1e6,
                        "frac_of_copy_probe": achieved / probe["GBs"]}}
    del q, work
    torch.cuda.empty_cache()
    return out


def ensemble_section(steps=10):
    """64 members of uneven order (r in 2..4) and resolution (90x45 to
    360x180), FP32: the batched launches (autotuned schedule, graph replay)
    against one plain launch sequence per member, same GPU, same steps."""
    import torch

    import paper_2303_11767_amd as dg
    from dg_inputs import band_limited_state, ensemble_members
    mem = ensemble_members(64, seed=4)
    ens = dg.Ensemble(mem, dtype="f32", h_ref=1e4)
    q = ens.empty_state()
    work = ens.empty_work()
    dts = []
    for k, (m, v) in enumerate(zip(ens.members, ens.views(q))):
        qh, info = band_limited_state(m.n_lon, m.n_lat, m.order, 16, mem[k]["seed"])
        v.copy_(torch.from_numpy(qh).to(v.dtype))
        dts.append(dg.cfl_time_step(m, info.cmax, 0.1))
    ens.set_dt(dts)
    dofs = sum(m.state_size() for m in ens.members)
    schedule = ens.autotune(q, work)

    def timed(fn):
        fn(2)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn(steps)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) * 1e-3 / steps

    t_ens = timed(lambda n: ens.rk_step(q, work, nsteps=n))
    g = ens.graph(q, work, nsteps=steps)
    t_graph = timed(lambda n: g.launch())
    g.close()
    orders = sorted({m.order for m in ens.members})
    layouts = {o: ens.kernel(o) for o in orders}
    # the single fused launch over all orders (line layout only)
    ens.set_schedule(schedule[0], 0, False)
    for o in orders:
        ens.set_kernel(o, "line")
    ens.set_schedule(schedule[0], schedule[1], True)
    t_fused = timed(lambda n: ens.rk_step(q, work, nsteps=n))
    ens.set_schedule(schedule[0], 0, False)
    for o in orders:
        ens.set_kernel(o, layouts[o])
    ens.set_schedule(*schedule)
    views = ens.views(q)
    works = [m.empty_work() for m in ens.members]

    def plain(n):
        for _ in range(n):
            for k, m in enumerate(ens.members):
                m.rk_step(views[k], works[k], dts[k], nsteps=1)

    t_plain = timed(plain)
    state_bytes = dofs * 4
    t_best = min(t_ens, t_graph)
    alg = 8.0 * state_bytes                     # SSP-RK3: 8 state transfers per step
    return {"members": 64, "dofs": dofs, "dtype": "f32", "state_bytes": state_bytes,
            "roofline": {"bound": "hbm", "achieved": alg / t_best / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": alg / t_best / 1e9 / HBM_PEAK_GBS,
                         "alg_bytes_per_step": alg, "kernels": "k_ens_stage* (batched schedule)"},
            "batched_over_plain": t_plain / t_best,
            "schedule": {"waves_per_group": schedule[0], "groups": schedule[1],
                         "fused": schedule[2], "layouts": {str(o): layouts[o] for o in orders}},
            "ms_per_step": {"batched": t_ens * 1e3, "batched_graph": t_graph * 1e3,
                            "fused_single_launch": t_fused * 1e3, "plain_per_member": t_plain * 1e3},
            "dof_updates_per_s": {"batched": 3 * dofs / t_ens, "plain_per_member": 3 * dofs / t_plain},
            "alg_GBs_batched": 8 * state_bytes / t_ens / 1e9}


LEARNED_SEEDS = tuple(range(200, 220))      # held-out seeds of the learned-correction evaluation
LEARNED_HORIZON_S = 30.0


def learned_fields(seed):
    """Initial order-4 polynomial of one held-out seed (host work, run in a
    worker process while the GPU sections run)."""
    from paper_2303_11767_amd import train_learned as tl
    from dg_inputs import band_limited_state
    return band_limited_state(tl.N_LON, tl.N_LAT, 4, tl.L_MAX, seed)


def learned_section(model_path, fields, seeds=LEARNED_SEEDS, t_eval=LEARNED_HORIZON_S):
    """The learned r = 1 form against plain r = 1 .. 4, evaluated against
    the plain r = 5 solver (FP64, held-out seeds), with wall-clock; the
    equal-error comparison names the lowest plain order that reaches the
    learned error."""
    import argparse as _ap
    import contextlib
    from paper_2303_11767_amd import train_learned as tl
    model, meta = tl.load_model(model_path)
    with contextlib.redirect_stdout(sys.stderr):      # stdout carries only the JSON line
        rep = tl.evaluate(_ap.Namespace(kappa=meta.get("kappa", 1.0)), model, seeds, t_eval,
                          fields=fields)
    rep["model"] = os.path.relpath(model_path, ROOT)
    return rep


def mesh_section(n_lon, n_lat, order, dtype, lmax, seed, steps, repeats=5, graph=False):
    """SSP-RK3 throughput of one plain mesh: `steps` steps between events
    (replayed from a HIP graph of those steps when `graph`), median of
    `repeats`; the stage kernel's algorithmic bandwidth (8/3 of the state per
    launch) at the mean stage duration."""
    import numpy as np
    import torch

    import paper_2303_11767_amd as dg
    from dg_inputs import band_limited_state
    q_h, info = band_limited_state(n_lon, n_lat, order, lmax, seed)
    mesh = dg.Mesh(n_lon, n_lat, order, dtype=dtype, h_ref=1.0e4 if dtype == "f32" else 0.0)
    q = torch.from_numpy(q_h).to(device="cuda", dtype=mesh.dtype).contiguous()
    work = mesh.empty_work()
    dt = dg.cfl_time_step(mesh, info.cmax, CFL)
    stream = torch.cuda.current_stream()
    mesh.rk_step(q, work, dt, nsteps=10)
    g = mesh.graph(q, work, dt, nsteps=steps) if graph else None
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        e0.record(stream)
        if g is not None:
            g.launch(stream)
        else:
            mesh.rk_step(q, work, dt, nsteps=steps)
        e1.record(stream)
        torch.cuda.synchronize()
        reps.append(e0.elapsed_time(e1) * 1e-3 / steps)
    if g is not None:
        g.close()
    if not all(np.isfinite(mesh.mass(q))):
        raise RuntimeError(f"{n_lon}x{n_lat} r={order} run became non-finite")
    step_s = sorted(reps)[len(reps) // 2]
    dofs = 3 * mesh.E * mesh.N
    alg = 8.0 * dofs * q.element_size() / 3.0
    out = {"workload": f"plain DG SWE, r={order}, {n_lon}x{n_lat} lat-lon elements, {dtype.upper()}, SSP-RK3, "
                       f"CFL 0.1, band-limited l<={lmax} seed {seed}",
           "dofs": dofs, "steps": steps, "kernel": mesh.kernel, "ms_per_step": step_s * 1e3,
           "repeats_ms_per_step": [r * 1e3 for r in reps], "dof_updates_per_s": dofs * 3 / step_s,
           "timed_with": ("HIP graph of the steps" if graph else "eager launches") + f", median of {repeats}",
           "roofline": {"bound": "hbm", "achieved": alg / (step_s / 3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": alg / (step_s / 3) / 1e9 / HBM_PEAK_GBS, "alg_bytes_per_launch": alg,
                        "launch_us": step_s / 3 * 1e6}}
    del q, work
    torch.cuda.empty_cache()
    return out


def contraction_ab(n_elem=64800, reps=50):
    """The r = 5 FP32 volume contraction in its sum-factorised VALU form and
    its dense MFMA form (see probe_contraction), as a dict."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2303_11767_amd", "libdgsw_probe.so"))
    lib.dgp_contraction_time.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_double)]
    lib.dgp_contraction_check.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    out = {"probe": "volume contraction r=5 FP32 over the 360x180 elements", "n_elem": n_elem, "reps": reps}
    for name, variant in (("valu_sum_factorised", 0), ("mfma_dense", 1)):
        ms = ctypes.c_double()
        rc = lib.dgp_contraction_time(variant, n_elem, reps, ctypes.byref(ms))
        if rc != 0:
            raise RuntimeError(f"contraction probe {name}: error {rc}")
        out[name] = {"us_per_launch": ms.value * 1e3, "ns_per_element": ms.value * 1e6 / n_elem}
    rel = ctypes.c_double()
    if lib.dgp_contraction_check(4096, ctypes.byref(rel)) != 0:
        raise RuntimeError("contraction probe check failed")
    out["max_rel_difference"] = rel.value
    out["mfma_over_valu_time"] = out["mfma_dense"]["us_per_launch"] / out["valu_sum_factorised"]["us_per_launch"]
    return out


def latency_floor(n_lon=N_LON, n_lat=N_LAT, reps=300):
    """The floor under one stage of the benchmark mesh (libdgsw_probe.so),
    per launch with the FP64 r = 3 half layout's grid, back to back on one
    stream and as the nodes of one graph: a kernel that does nothing, one
    that moves the stage's own bytes (q and q^n in, the new state out) and
    one that adds the neighbour reads of the stage."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2303_11767_amd", "libdgsw_probe.so"))
    lib.dgp_floor_time.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_double)]
    out = {"mesh": f"{n_lon}x{n_lat} r=3 FP64", "launches": reps, "unit": "us per launch"}
    for mode, graph in (("eager", 0), ("graph", 1)):
        out[mode] = {}
        for name, variant in (("empty", 0), ("own_bytes", 1), ("own_and_neighbour_bytes", 2)):
            us = ctypes.c_double()
            rc = lib.dgp_floor_time(variant, n_lon, n_lat, graph, reps, ctypes.byref(us))
            if rc != 0:
                raise RuntimeError(f"floor probe {mode} {name}: error {rc}")
            out[mode][name] = us.value
    return out


# the configurations the oracle is timed on: name, n_lon, n_lat, order, l_max, seed
ORACLE_CONFIGS = (("C1", 32, 16, 1, 6, 1), ("C2", 180, 90, 3, 16, 2), ("C3", 360, 180, 5, 32, 3),
                  ("C5", 360, 180, 1, 32, 200))


def oracle_timings():
    """The FP64 oracle, as it stands, on one host thread: one right-hand side
    and one SSP-RK3 step per configuration (seconds and DOF-updates/s), each
    timed after one untimed call of the same kind."""
    from threadpoolctl import threadpool_limits
    from dg_inputs import band_limited_state
    from oracle import SphereDG
    out = {}
    with threadpool_limits(limits=1):
        for name, nl, nt, r, lmax, seed in ORACLE_CONFIGS:
            q, info = band_limited_state(nl, nt, r, lmax, seed)
            m = SphereDG(nl, nt, r)
            dofs = 3 * m.E * m.N
            m.rhs(q)
            t0 = time.perf_counter()
            m.rhs(q)
            t_rhs = time.perf_counter() - t0
            dt = m.cfl_time_step(info.cmax, CFL)
            m.ssp_rk3_step(q, dt)
            t0 = time.perf_counter()
            m.ssp_rk3_step(q, dt)
            t_step = time.perf_counter() - t0
            out[name] = {"mesh": f"{nl}x{nt} r={r}", "dofs": dofs, "rhs_s": t_rhs, "step_s": t_step,
                         "rhs_dof_per_s": dofs / t_rhs, "step_dof_updates_per_s": 3 * dofs / t_step}
    return out


def planar_section(dtype="f64"):
    """The geostrophic-adjustment run of section 4.2 as timed in section 5.1:
    50 x 50 elements on the 1e7 m f-plane, r = 3, classical RK4, dt = 100 s,
    T = 36000 s (360 steps), Gaussian bump at rest.  The paper's time for the
    same run (its Table of G4GT computational times, p = 3: 430.21 s on a
    12-core Xeon E5-2690 v3) is context, not a target: other hardware, other
    code, and its flux evaluation may differ."""
    import numpy as np
    import torch

    import paper_2303_11767_amd as dg
    from dg_inputs import gaussian_bump_plane
    L = 1.0e7
    mesh = dg.Plane(50, 50, 3, L, L, dtype=dtype, f=1.0e-4, gravity=9.81,
                    h_ref=1000.0 if dtype == "f32" else 0.0)
    q0 = torch.from_numpy(gaussian_bump_plane(50, 50, 3, L, L)).to("cuda", mesh.dtype)
    q = q0.clone()
    work = mesh.empty_work(dg.DG_RK4)
    mesh.rk_step(q, work, 100.0, scheme=dg.DG_RK4, nsteps=20)     # warm-up
    q.copy_(q0)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    mesh.rk_step(q, work, 100.0, scheme=dg.DG_RK4, nsteps=360)
    b.record()
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) * 1e-3
    mass = mesh.mass(q)
    if not np.all(np.isfinite(mass)):
        raise RuntimeError("planar run became non-finite")
    dofs = 3 * mesh.E * mesh.N
    return {"workload": "geostrophic adjustment, 50x50 f-plane, r=3, RK4, dt=100 s, 360 steps",
            "dtype": dtype, "seconds": sec, "dof_updates_per_s": dofs * 4 * 360 / sec,
            "us_per_stage": sec / (4 * 360) * 1e6,
            "paper_context": {"seconds": 430.21, "hardware": "Intel Xeon E5-2690 v3, 12 cores "
                              "(G4GT, Table of computational times, p = 3)"}}


def advection_section():
    """Section 4.1's convergence run on the GPU at the paper's finest mesh:
    160 x 160 elements, r = 3, FP64, classical RK4 to T = 1; time, per-stage
    bandwidth (13 state transfers per RK4 step) and the L2 error against the
    exact solution beside the paper's printed 5.030e-10."""
    import numpy as np
    import torch

    import paper_2303_11767_amd as dg
    from dg_inputs import sine_square
    k, p = 160, 3
    adv = dg.Advection(k, k, p)
    q0 = torch.from_numpy(sine_square(k, p)).cuda()
    q = q0.clone()
    work = adv.empty_work()
    n = int(np.ceil(1.0 / (0.1 * (1.0 / k) / ((2 * p + 1) * 2.0))))
    adv.rk_step(q, work, 1.0 / n, nsteps=10)
    q.copy_(q0)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    adv.rk_step(q, work, 1.0 / n, nsteps=n)
    b.record()
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) * 1e-3
    state = q.numel() * q.element_size()
    # after one period the exact solution is the initial field again; the
    # error is measured against its projection (the paper's is against the
    # exact field, which adds the projection error in quadrature)
    err = float(torch.sqrt(((q - q0) ** 2).sum() * (1.0 / k) ** 2 / 4.0).item())
    return {"workload": "linear advection, 160x160 periodic unit square, r=3, RK4 to T=1",
            "steps": n, "seconds": sec, "us_per_stage": sec / (4 * n) * 1e6,
            "alg_GBs": 13 * state * n / sec / 1e9, "l2_error_vs_projection": err,
            "paper_l2_error": 5.030e-10}


def _plane_rk4_seconds(mesh, q, steps):
    """Seconds per classical RK4 step over `steps` steps of dt = 100 s."""
    import torch

    import paper_2303_11767_amd as dg
    work = mesh.empty_work(dg.DG_RK4)
    mesh.rk_step(q, work, 100.0, scheme=dg.DG_RK4, nsteps=3)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    mesh.rk_step(q, work, 100.0, scheme=dg.DG_RK4, nsteps=steps)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) * 1e-3 / steps


def scaling_section():
    """The two scaling studies of section 5.2 with the section 4.2 f-plane
    (r = 3, FP64, classical RK4, dt = 100 s, Gaussian bump):
    horizontal, K x K elements for K = 20 .. 640 (the paper doubles K up to
    640); vertical, 300 x 300 elements with nz identical layers advanced by
    one launch per stage (dg_set_levels).  The paper reports these as
    figures only; the numbers here are throughput per layer."""
    import torch

    import paper_2303_11767_amd as dg
    from dg_inputs import gaussian_bump_plane
    L = 1.0e7
    horiz = []
    for k in (20, 40, 80, 160, 320, 640):
        mesh = dg.Plane(k, k, 3, L, L, f=1.0e-4, gravity=9.81)
        q = torch.from_numpy(gaussian_bump_plane(k, k, 3, L, L)).to("cuda")
        steps = max(10, min(400, int(4e9 / (q.numel() * 8 * 13))))
        s = _plane_rk4_seconds(mesh, q, steps)
        horiz.append({"elements": f"{k}x{k}", "ms_per_step": s * 1e3,
                      "dof_updates_per_s": 3 * mesh.E * mesh.N * 4 / s})
    vert = []
    k = 300
    q1 = torch.from_numpy(gaussian_bump_plane(k, k, 3, L, L)).to("cuda")
    for nz in (1, 2, 4, 8, 16, 32, 64):
        mesh = dg.Plane(k, k, 3, L, L, f=1.0e-4, gravity=9.81)
        mesh.levels = nz
        q = q1.unsqueeze(0).repeat(nz, 1, 1, 1).contiguous()
        steps = max(5, min(100, int(4e9 / (q.numel() * 8 * 13))))
        s = _plane_rk4_seconds(mesh, q, steps)
        vert.append({"levels": nz, "ms_per_step": s * 1e3, "ms_per_step_per_level": s * 1e3 / nz,
                     "dof_updates_per_s": 3 * mesh.E * mesh.N * nz * 4 / s})
        del q
    return {"workload": "f-plane r=3 FP64 RK4 (section 4.2 bump), section 5.2 scaling studies",
            "horizontal": horiz, "vertical_300x300": vert}


def profile_probe(args):
    """Short run for rocprofv3 counter passes: a few 3-stage cycles of the
    stage kernel, then device-to-device copies of a known size (the
    calibration of the counters)."""
    import torch

    import paper_2303_11767_amd as dg
    from dg_inputs import band_limited_state
    n_lon, n_lat, order, lmax, seed = N_LON, N_LAT, ORDER, L_MAX, SEED
    if args.probe_mesh:          # another mesh for counter runs: NLONxNLATxR (l <= 32, seed 5)
        n_lon, n_lat, order = (int(v) for v in args.probe_mesh.split("x"))
        lmax, seed = 32, 5
    q_h, info = band_limited_state(n_lon, n_lat, order, lmax, seed)
    href = 1.0e4 if args.dtype == "f32" else 0.0
    mesh = dg.Mesh(n_lon, n_lat, order, dtype=args.dtype, h_ref=href)
    q = torch.from_numpy(q_h).to(device="cuda", dtype=mesh.dtype).contiguous()
    work = mesh.empty_work()
    dt = dg.cfl_time_step(mesh, info.cmax, CFL)
    mesh.rk_step(q, work, dt, nsteps=args.warmup)
    mesh.rk_step(q, work, dt, nsteps=args.steps)
    torch.cuda.synchronize()
    nbytes = 256 << 20
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "done", "mesh": [n_lon, n_lat, order], "kernel": mesh.kernel,
                      "state_bytes": q.numel() * q.element_size(), "copy_bytes": nbytes,
                      "stage_launches": 3 * args.steps}), flush=True)


def profile_probe_learned(args):
    """Short run for rocprofv3 passes over the learned stage: `steps`
    SSP-RK3 steps of the learned r = 1 form on 360 x 180 elements (FP64,
    stored model), then `steps` training steps of the network on 8192 random
    standardised rows (the training GEMMs), then the calibration copies."""
    import numpy as np
    import torch

    import paper_2303_11767_amd as dg
    from paper_2303_11767_amd import learned
    from paper_2303_11767_amd import train_learned as tl
    from dg_inputs import band_limited_state
    model, meta = tl.load_model(LEARNED_MODEL)
    m1 = dg.Mesh(tl.N_LON, tl.N_LAT, 1, dtype="f64")
    net = learned.LearnedRHS(m1, model["params"], model["feat_mean"], model["feat_istd"],
                             model["out_mean"], model["out_std"], kappa=meta.get("kappa", 1.0))
    qh, info = band_limited_state(tl.N_LON, tl.N_LAT, 1, tl.L_MAX, 200)
    q = torch.from_numpy(qh).cuda()
    dt = dg.cfl_time_step(m1, info.cmax, CFL)
    work = m1.empty_work()
    net.rk_step(q, work, dt, nsteps=args.steps)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    rows = 8192
    X = torch.from_numpy(rng.standard_normal((rows, 108)).astype(np.float32)).cuda()
    T = torch.from_numpy(rng.standard_normal((rows, 12)).astype(np.float32)).cuda()
    P = learned.param_count()
    params = model["params"].clone()
    mom, var = torch.zeros(P, device="cuda"), torch.zeros(P, device="cuda")
    for step in range(1, args.steps + 1):
        learned.mlp_train_step(params, X, T, tl.MASK, mom, var, step, 1e-4)
    torch.cuda.synchronize()
    nbytes = 256 << 20
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"probe": "done", "learned_stages": 3 * args.steps, "train_steps": args.steps,
                      "rows": int(m1.E), "copy_bytes": nbytes}), flush=True)


def profile_probe_ensemble(args):
    """Short run for rocprofv3 passes over the ensemble kernels: the 64-member
    FP32 ensemble of the benchmark with every member at rest (the kernels run
    the same instructions on any state), autotuned, then `steps` SSP-RK3
    steps, then the calibration copies."""
    import torch

    import paper_2303_11767_amd as dg
    from dg_inputs import ensemble_members, lake_at_rest_state
    mem = ensemble_members(64, seed=4)
    ens = dg.Ensemble(mem, dtype="f32", h_ref=1e4)
    q = ens.empty_state()
    for m, v in zip(ens.members, ens.views(q)):
        v.copy_(torch.from_numpy(lake_at_rest_state(m.n_lon, m.n_lat, m.order)).to(v.dtype))
    ens.set_dt([1.0] * ens.n)
    work = ens.empty_work()
    schedule = ens.autotune(q, work)
    ens.rk_step(q, work, nsteps=args.steps)
    torch.cuda.synchronize()
    nbytes = 256 << 20
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    orders = sorted({m.order for m in ens.members})
    print(json.dumps({"probe": "done", "schedule": schedule, "layouts": {o: ens.kernel(o) for o in orders},
                      "state_bytes": ens.size * 4, "steps": args.steps, "copy_bytes": nbytes}), flush=True)


def probe_contraction():
    """The r = 5 FP32 volume contraction alone, in the sum-factorised VALU form
    the stage kernels use and the dense MFMA form (libdgsw_probe.so; nodal
    values synthesised in registers, so no memory traffic): time per launch
    of each and the largest difference between their results."""
    print(json.dumps(contraction_ab()), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--kernel-cycles", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--repeats", type=int, default=5,
                    help="repeats of the timed region (the median is reported)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the ensemble and learned-correction sections")
    ap.add_argument("--profile-probe", action="store_true",
                    help="short run for rocprofv3 counter passes (prints no bench line)")
    ap.add_argument("--probe-mesh", default=None, metavar="NLONxNLATxR",
                    help="mesh of the profile probe (default: the benchmark mesh)")
    ap.add_argument("--probe-contraction", action="store_true",
                    help="time the r = 5 FP32 volume contraction in its VALU and MFMA forms "
                         "(prints no bench line)")
    ap.add_argument("--probe-ensemble", action="store_true",
                    help="short run of the 64-member ensemble for rocprofv3 passes (prints no bench line)")
    ap.add_argument("--probe-learned", action="store_true",
                    help="short run of the learned stage and the network's training step "
                         "for rocprofv3 passes (prints no bench line)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the DG loop runs on a single device "
              "(sharding across GPUs is not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.profile_probe:
        profile_probe(args)
        return
    if args.probe_learned:
        profile_probe_learned(args)
        return
    if args.probe_contraction:
        probe_contraction()
        return
    if args.probe_ensemble:
        profile_probe_ensemble(args)
        return
    pool = futs = None
    if not args.no_extras:
        # host-side inputs of the large sections, synthesised in worker
        # processes (forked before this process touches the GPU) while the
        # GPU sections run
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor
        pool = ProcessPoolExecutor(max_workers=6, mp_context=mp.get_context("fork"))
        futs = {"big": pool.submit(big_fields), "oracle": pool.submit(oracle_timings)}
        if os.path.exists(LEARNED_MODEL):
            futs.update({s: pool.submit(learned_fields, s) for s in LEARNED_SEEDS})
    out = run(args)
    if not args.no_extras:
        # the same workload and loop in the other precision the configuration names
        other = argparse.Namespace(**vars(args))
        other.dtype = "f32" if args.dtype == "f64" else "f64"
        o = run(other)
        out["other_precision"] = {k: o[k] for k in ("dtype", "value", "unit", "ms_per_step", "roofline")}
        probe = hbm_probe()
        out["hbm_copy_probe"] = probe
        out["roofline"]["frac_of_copy_probe"] = out["roofline"]["achieved"] / probe["GBs"]
        out["latency_floor"] = latency_floor()
        out["ensemble"] = ensemble_section()
        out["planar"] = planar_section()
        out["advection"] = advection_section()
        out["scaling_studies"] = scaling_section()
        out["large_mesh"] = big_section(futs.pop("big").result(), probe)
        out["small_mesh_c1"] = mesh_section(32, 16, 1, "f64", 6, 1, steps=100, graph=True)
        out["order5_c3"] = mesh_section(360, 180, 5, "f32", 32, 3, steps=50)
        out["order5_c3"]["contraction_valu_vs_mfma"] = contraction_ab()
        if os.path.exists(LEARNED_MODEL):
            out["learned"] = learned_section(LEARNED_MODEL, lambda seed: futs[seed].result())
    # the per-configuration oracle timings ran in a worker beside the GPU
    # sections; they end before the all-core baseline starts
    oracle_cfg = futs.pop("oracle").result() if futs is not None else None
    if pool is not None:
        pool.shutdown()
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline(args.cpu_seconds)
    if out["cpu_baseline"] is not None and oracle_cfg is not None:
        out["cpu_baseline"]["oracle_per_config"] = oracle_cfg
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
