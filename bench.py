"""Benchmark of the TDSLDA time step on one MI355X.

Default workload: 32^3 periodic lattice, 8192 two-component qpwfs (the
lowest-|k| BCS states, Delta0 = 0.3, mu = 0.5, g = 2, beta = 0.37) with a
ramped Gaussian external well, FP64, dt = 0.002.  A "step" is one
Adams-Bashforth-Milne step of all qpwfs (two Hamiltonian applications, two
density rebuilds).  Inputs are generated on the host, uploaded, and the
series-expansion start-up plus the warm-up steps run before the timed region.

Prints one JSON line: qpwf-steps/s of the whole job, the roofline of the
dominant kernel (the plane kernel of the ABM phases, timed with HIP events
inside the library on its stream), and the CPU oracle timed on a bounded
sample of the same workload.
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12           # MI355X HBM3E, bytes/s
METRIC = "qpwf-steps/sec + % HBM roofline, FP32/batched vs FP64 at stated density error"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name, M=None):
    import workloads as wl
    if name == "cfg2":
        return wl.config2(M=M)
    if name == "cfg2_fp32":
        w = wl.config2(M=M)
        w.functional.precision = wl.FP32
        w.name = w.name.replace("fp64", "fp32")
        return w
    if name == "cfg1":
        return wl.config1(M=M)
    if name == "cfg3":
        return wl.config3(M=M)                      # 48^3 vortex, FP32 bulk + FP64 sums
    if name == "cfg4":
        return wl.config4(M=M)                      # 64^3, C = 4, bf16x3 MFMA xy-kinetic term
    if name == "cfg4_fp32":
        w = wl.config4(M=M, precision=wl.FP32)      # same, FP32 register FFTs
        w.name = w.name + "_stockham"
        return w
    raise ValueError(name)


_POOL = None


def start_pool():
    """Host threads for the seeded inputs (numpy releases the GIL in its array loops)."""
    global _POOL
    from concurrent.futures import ThreadPoolExecutor
    n = min(16, len(os.sched_getaffinity(0)))
    if n > 1:
        _POOL = ThreadPoolExecutor(max_workers=n)


def upload(ctx, w, piece=None):
    per_qpwf = w.functional.ncomp * w.lattice.n * 16
    if piece is None:
        piece = max(1, min(512, (64 << 20) // per_qpwf))
    ranges = [(j0, min(piece, w.M - j0)) for j0 in range(0, w.M, piece)]
    if _POOL is None:
        for j0, k in ranges:
            ctx.set_qpwf(j0, np.ascontiguousarray(w.qpwfs(j0, k)))
        return
    # generate ahead on the pool, upload in order; at most 2x workers pieces in flight
    futs = {}
    nxt = 0
    depth = 2 * _POOL._max_workers
    for i, (j0, k) in enumerate(ranges):
        while nxt < len(ranges) and nxt < i + depth:
            jj, kk = ranges[nxt]
            futs[nxt] = _POOL.submit(lambda a, b: np.ascontiguousarray(w.qpwfs(a, b)), jj, kk)
            nxt += 1
        ctx.set_qpwf(j0, futs.pop(i).result())


def run_gpu(w, steps, warmup, tuning=None, profile=True, autotune=False):
    import torch
    import paper_2009_00745_amd as lise
    stream = torch.cuda.current_stream().cuda_stream
    ctx = lise.Context(w.lattice, w.M, w.functional, stream=stream)
    if tuning:
        ctx.set_tuning(**tuning)
    t0 = time.time()
    upload(ctx, w)
    log(f"{w.name}: uploaded {w.M} qpwfs in {time.time() - t0:.1f}s, device memory {ctx.memory() / 2**30:.1f} GiB")
    ctx.startup(w.dt)
    chosen = None
    if autotune:
        t0 = time.time()
        chosen = ctx.autotune(w.dt, 3)
        log(f"{w.name}: autotune picked {chosen} in {time.time() - t0:.1f}s")
    if warmup:
        ctx.step(w.dt, warmup)
    torch.cuda.synchronize()
    log(f"{w.name}: start-up + {warmup} warm-up steps done")
    if profile:
        ctx.profile(1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.step(w.dt, steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    prof = {}
    prof_steps = steps
    if profile:
        classes = ((0, "plane"), (1, "zaxis"), (2, "fields"))
        for cls, name in classes:
            prof[name] = ctx.profile_read(cls)
        if prof["plane"][0] == 0:
            # graph replays carry no per-launch events: a few eager steps give the kernel times
            prof_steps = 4
            ctx.step(w.dt, prof_steps)
            for cls, name in classes:
                prof[name] = ctx.profile_read(cls)
        ctx.profile(0)
    prof["steps"] = prof_steps
    log(f"{w.name}: {steps} steps in {t2 - t1:.3f}s")
    prof["tuning"] = chosen
    return ctx, t2 - t1, prof


def reduced_error(name, steps, M):
    """Density error of the float32 forms against float64 on a reduced instance of a
    workload whose float64 state does not fit at full size: the same lattice and
    recipe with fewer qpwfs, compared after the same number of ABM steps."""
    import torch
    import workloads as wl
    make = {"cfg3": wl.config3, "cfg4": wl.config4}[name]
    forms = {"cfg3": [("fp32", wl.FP32)],
             "cfg4": [("fp32_register_fft", wl.FP32), ("fp32_mfma_bf16x3", wl.FP32_MFMA)]}[name]

    def run(prec):
        w = make(M=M, precision=prec)
        ctx, _, _ = run_gpu(w, steps, 0, None, profile=False)
        n, k = ctx.densities()
        st = ctx.time()[1]
        ctx.close()
        torch.cuda.empty_cache()
        return n, k, st

    n64, k64, s64 = run(wl.FP64)
    out = {"M": M, "after_steps": int(s64), "reference": "fp64 on the GPU (parity-tested against the oracle)"}
    for label, prec in forms:
        n, k, st = run(prec)
        out[label] = {"n": float(np.linalg.norm(n - n64) / np.linalg.norm(n64)),
                      "kappa": float(np.linalg.norm(k - k64) / np.linalg.norm(k64))} if st == s64 else None
    return out


def run_batched(nsys, steps, warmup, graph=1):
    """Independent FP32 systems (16^3/20^3/24^3, 512-3072 qpwfs each) advanced together,
    each on its own forked stream (with its own four-step graph replays when graph = 1)."""
    import torch
    import workloads as wl
    import paper_2009_00745_amd as lise
    systems = wl.config5_systems(seed=0, nsys=nsys)
    stream = torch.cuda.current_stream().cuda_stream
    ctxs = []
    t0 = time.time()
    for w in systems:
        c = lise.Context(w.lattice, w.M, w.functional, stream=stream)
        # the systems already overlap one another on their own streams: each
        # keeps its z kernel on its stream (64 systems: 2.09e6 vs 1.99e6 with
        # the per-system z stream; 16 systems: equal)
        c.set_tuning(graph=int(bool(graph)), no_overlap=1)
        upload(c, w)
        ctxs.append(c)
    log(f"batched: {nsys} systems uploaded in {time.time() - t0:.1f}s")
    b = lise.Batch(ctxs, stream=stream)
    dt = systems[0].dt
    b.step(dt, 4 * max(1, warmup))       # start-up, graph capture, warm-up replays
    torch.cuda.synchronize()
    nst = 4 * max(1, steps // 4)
    t1 = time.perf_counter()
    b.step(dt, nst)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    qsteps = sum(w.M for w in systems) * nst
    sizes = {}
    for w in systems:
        sizes.setdefault(w.lattice.nx, [0, 0])
        sizes[w.lattice.nx][0] += 1
        sizes[w.lattice.nx][1] += w.M
    b_alg = sum(w.M * 16 * 2 * w.lattice.n * 8 for w in systems) * nst / el
    b.close()
    for c in ctxs:
        c.close()
    return {"value": qsteps / el, "unit": "qpwf-steps/s", "systems": nsys, "steps": nst,
            "ms_per_step": 1e3 * el / nst, "qpwf_total": sum(w.M for w in systems),
            "lattices": {f"{k}^3": {"systems": v[0], "qpwfs": v[1]} for k, v in sorted(sizes.items())},
            "step_hbm_frac": b_alg / HBM_PEAK}


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "kp_fast_fp64_32c_traffic.md")
KERNEL_SOURCES = ("paper_2009_00745_amd/csrc/lise_device.hpp", "paper_2009_00745_amd/csrc/lise_fast.hpp")


def measured_traffic():
    """Per-qpwf HBM traffic of the ABM plane kernels from the committed PMC summary, or None
    when the kernel sources changed since the counters were taken."""
    import hashlib
    try:
        line = [ln for ln in open(TRAFFIC_PROFILE) if ln.startswith("TRAFFIC_JSON ")][0]
    except (OSError, IndexError):
        return None
    rec = json.loads(line[len("TRAFFIC_JSON "):])
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return rec if h.hexdigest()[:16] == rec["source_hash"] else None


def copy_bandwidth(nbytes=2 << 30, reps=3):
    """Read + write bandwidth of a plain device-to-device copy (torch), best of reps."""
    import torch
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    best = None
    for _ in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3
        best = t if best is None else min(best, t)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / best


def cpu_baseline(w_name, M_sample, steps):
    """The oracle, unchanged, on M_sample qpwfs of the same workload."""
    import oracle
    w = make_workload(w_name, M=M_sample)
    psi = w.qpwfs()
    ev = oracle.Evolver(w.lattice, w.functional, psi)
    ev.startup(w.dt)
    t0 = time.perf_counter()
    for _ in range(steps):
        ev.abm_step()
    dt = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": M_sample * steps / dt, "unit": "qpwf-steps/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{w.name}: {M_sample} of the workload's qpwfs on the same lattice, "
                      f"{steps} ABM steps after the start-up ({dt:.1f}s); oracle cost is linear "
                      f"in qpwfs; densities summed over the sample only; CPU {cpu}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--M", type=int, default=None)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--jgroup", type=int, default=0)
    ap.add_argument("--no-overlap", action="store_true", help="z kernel on the same stream as the plane kernel")
    ap.add_argument("--graph", action="store_true", help="replay four-step HIP graphs (kept by the autotuner)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=32)
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-phase", action="store_true",
                    help="skip the variant with the trivial phase removed (Eq. sp_en)")
    ap.add_argument("--batched", type=int, default=16,
                    help="number of independent systems in the batched variant (0 = skip; 64 = full workload)")
    ap.add_argument("--reduced-error", type=int, default=0, metavar="M",
                    help="cfg3/cfg4: also measure the float32 density error against float64 on the same "
                         "workload with M qpwfs (4096 for cfg3, 1024 for cfg4 fit in float64)")
    ap.add_argument("--reduced-steps", type=int, default=100)
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the path is built and measured on a single MI355X; "
              "multi-GPU sharding over qpwfs is a design note, not a run (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    # the batched leg runs one stream per system; HIP maps streams onto this many
    # hardware queues (default 4), read when HIP initialises
    if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4) < 16:
        os.environ["GPU_MAX_HW_QUEUES"] = "16"
    start_pool()
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    import paper_2009_00745_amd as lise
    lise.load_library()

    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calibrate_copy} MiB done")
        del src, dst

    w = make_workload(args.workload, M=args.M)
    tuning = {}
    fixed_shape = bool(args.chunk or args.jgroup or args.no_overlap)
    if fixed_shape or args.graph:
        tuning = {"chunk_qpwf": args.chunk, "jgroup": args.jgroup, "no_overlap": int(args.no_overlap),
                  "graph": int(args.graph)}
    C, N = w.functional.ncomp, w.lattice.n
    esz = 16 if w.functional.precision == 0 else 8
    autotune = not args.no_autotune and not fixed_shape
    leg_tuning = dict(tuning) or None              # what the other legs start from
    ctx, elapsed, prof = run_gpu(w, args.steps, args.warmup, tuning, autotune=autotune)
    chosen = prof.pop("tuning")
    prof_steps = prof.pop("steps")
    value = w.M * args.steps / elapsed
    ms_step = 1e3 * elapsed / args.steps
    b_alg = 16 * C * N * esz                      # compulsory state bytes per qpwf-step
    n_plane, ms_plane = prof["plane"]
    # the plane kernel moves the ABM state: phase 1 reads 6 and writes 1 state array,
    # phase 2 reads 7 and writes 2, per qpwf (the split of the 16-array step minimum)
    alg_bytes_total = prof_steps * w.M * b_alg
    avg_launch_s = ms_plane / n_plane / 1e3
    achieved = (alg_bytes_total / n_plane) / avg_launch_s
    traffic = None
    rec = measured_traffic() if (w.lattice.nx, w.lattice.ny, w.lattice.nz, C, esz) == (32, 32, 32, 2, 16) else None
    if rec:
        qpwf_per_launch = prof_steps * w.M * 2 / n_plane
        traffic = 0.5 * (rec["abm1_bytes_per_qpwf"] + rec["abm2_bytes_per_qpwf"]) * qpwf_per_launch
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": achieved / HBM_PEAK, "traffic": traffic,
                "measured_copy_GBps": copy_bandwidth() / 1e9,
                "kernel": "plane kernel, ABM phases (kp_fast on 8..64 sides)", "launches": n_plane,
                "avg_launch_ms": ms_plane / n_plane,
                "alg_bytes_per_launch": alg_bytes_total / n_plane}
    if prof_steps != args.steps:
        roofline["kernel_times_from"] = (f"{prof_steps} eager steps after the timed graph replays "
                                         "(replays carry no per-launch events)")
    state_bytes = 7 * w.M * C * N * esz           # the seven state copies
    if state_bytes < 256e6:
        roofline["note"] = (f"the state ({state_bytes / 1e6:.0f} MB) fits in the 256 MB Infinity Cache: "
                            "the HBM fraction is not meaningful for this workload")
    breakdown = {k: {"launches": n, "ms_per_step": ms / prof_steps} for k, (n, ms) in prof.items()}
    if chosen:
        tuning = {"autotuned": chosen}
    t_now, s_now = ctx.time()
    n64, k64 = ctx.densities()
    obs = ctx.observables()
    ctx.close()
    del ctx
    torch.cuda.empty_cache()

    variants = {}
    if not args.no_fp32 and args.workload == "cfg2":
        w32 = make_workload("cfg2_fp32", M=args.M)
        ctx32, el32, prof32 = run_gpu(w32, args.steps, args.warmup, leg_tuning,
                                      autotune=autotune)
        chosen32 = prof32.pop("tuning")
        ps32 = prof32.pop("steps")
        n32, k32 = ctx32.densities()
        t32, s32 = ctx32.time()
        ctx32.close()
        same = s32 == s_now    # densities are compared after equal step counts only
        variants["fp32_same_workload"] = {
            "value": w32.M * args.steps / el32, "unit": "qpwf-steps/s",
            "ms_per_step": 1e3 * el32 / args.steps,
            "kernel_ms_per_step": {k: ms / ps32 for k, (n, ms) in prof32.items()},
            "speedup_vs_fp64": (w32.M * args.steps / el32) / value,
            "density_rel_l2_vs_fp64": {
                "n": float(np.linalg.norm(n32 - n64) / np.linalg.norm(n64)),
                "kappa": float(np.linalg.norm(k32 - k64) / np.linalg.norm(k64))} if same else None,
            "after_steps": int(s32),
            "tuning": chosen32,
            "step_hbm_frac": (w32.M * args.steps / el32) * 16 * C * N * 8 / HBM_PEAK}

    if not args.no_phase and args.workload == "cfg2":
        wp = make_workload("cfg2", M=args.M)
        wp.functional.remove_phase = 1
        ctxp, elp, profp = run_gpu(wp, args.steps, args.warmup, leg_tuning,
                                   autotune=autotune)
        chosenp = profp.pop("tuning")
        psp = profp.pop("steps")
        n_p, k_p = ctxp.densities()
        tp, sp = ctxp.time()
        ctxp.close()
        same = sp == s_now
        valp = wp.M * args.steps / elp
        variants["phase_removed_fp64"] = {
            "value": valp, "unit": "qpwf-steps/s", "ms_per_step": 1e3 * elp / args.steps,
            "kernel_ms_per_step": {k: ms / psp for k, (n, ms) in profp.items()},
            "cost_vs_plain": value / valp,
            "density_rel_l2_vs_plain": {
                "n": float(np.linalg.norm(n_p - n64) / np.linalg.norm(n64)),
                "kappa": float(np.linalg.norm(k_p - k64) / np.linalg.norm(k64))} if same else None,
            "after_steps": int(sp), "tuning": chosenp,
            "note": "eta by Parseval on the register-FFT path: the pass re-reads x once, 22 state arrays per step instead of 20"}

    if args.reduced_error and args.workload in ("cfg3", "cfg4", "cfg4_fp32"):
        variants["reduced_error"] = reduced_error(args.workload[:4], args.reduced_steps, args.reduced_error)

    if args.batched and args.workload == "cfg2":
        variants["batched_fp32"] = run_batched(args.batched, args.steps, args.warmup)

    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle on a sample")
        cpu = cpu_baseline(args.workload, args.cpu_sample, args.cpu_steps)

    out = {
        "metric": METRIC, "value": value, "unit": "qpwf-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if w.functional.precision == 0 else "f32", "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.lattice.nx}^3 lattice, {w.M} {'two' if C == 2 else 'four'}-component qpwfs, "
                               f"dt={w.dt}, {w.notes}",
                   "lattice": [w.lattice.nx, w.lattice.ny, w.lattice.nz], "n_qpwf": w.M,
                   "ncomp": C, "dt": w.dt, "tuning": tuning or "default"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "step_hbm_frac": value * b_alg / HBM_PEAK,
        "b_alg_per_qpwf_step": b_alg,
        "kernel_ms_per_step": breakdown,
        "observables": {"t": t_now, "N": obs["N"], "E": obs["E"], "norm_drift_max": obs["norm_drift_max"]},
        "variants": variants,
        "host": platform.node(),
    }
    print(json.dumps(out), flush=True)
    if _POOL is not None:
        _POOL.shutdown(wait=False)


if __name__ == "__main__":
    main()
