"""Benchmark of the TDSLDA time step on one MI355X.

Default workload: 32^3 periodic lattice, 8192 two-component qpwfs (the
lowest-|k| BCS states, Delta0 = 0.3, mu = 0.5, g = 2, beta = 0.37) with a
ramped Gaussian external well, FP64, dt = 0.002.  A "step" is one
Adams-Bashforth-Milne step of all qpwfs (two Hamiltonian applications, two
density rebuilds).  Inputs are generated on the host, uploaded, and the
series-expansion start-up plus the warm-up steps run before the timed region.

Prints one JSON line: qpwf-steps/s of the whole job, the roofline of the
dominant kernel (the plane kernel of ABM phase 1, timed with HIP events inside
the library on its stream) beside the whole step's fraction, norm and energy
drift, the CPU oracle timed on a bounded sample of the same workload, and the
other forms at their own workloads: float32 on the same workload, phase
removal, the 48^3 float32 vortex workload (16384 qpwfs) and the 64-system
batch, each float32 form with its density error against float64.
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


PROF_CLASSES = ((0, "plane_abm1"), (4, "plane_abm2"), (1, "zaxis"), (2, "fields"))


def run_gpu(w, steps, warmup, tuning=None, profile=True, autotune=False):
    """Upload, start up, optionally autotune, warm up, then time `steps` ABM steps.
    Returns the context, the elapsed seconds, per-class kernel times and the
    observables at the start of the timed region."""
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
        # start again from the uploaded state, so that every leg runs the same steps
        # whatever number of trial steps its autotuner took
        upload(ctx, w)
        ctx.set_time(0.0)
        ctx.startup(w.dt)
    if warmup:
        ctx.step(w.dt, warmup)
    torch.cuda.synchronize()
    obs0 = ctx.observables()
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
        for cls, name in PROF_CLASSES:
            prof[name] = ctx.profile_read(cls)
        if prof["plane_abm1"][0] == 0:
            # graph replays carry no per-launch events: a few eager steps give the kernel times
            prof_steps = 4
            ctx.step(w.dt, prof_steps)
            for cls, name in PROF_CLASSES:
                prof[name] = ctx.profile_read(cls)
        ctx.profile(0)
    prof["steps"] = prof_steps
    log(f"{w.name}: {steps} steps in {t2 - t1:.3f}s")
    prof["tuning"] = chosen
    prof["obs0"] = obs0
    return ctx, t2 - t1, prof


def drift(obs0, obs1, steps):
    """Energy change over the timed steps, relative to |E|, and the norm drift since the
    qpwfs were set (the library's per-qpwf maximum)."""
    dE = (obs1["E"] - obs0["E"]) / abs(obs0["E"])
    return {"E_start": obs0["E"], "E_end": obs1["E"], "E_rel_change": dE, "E_rel_change_per_step": dE / steps,
            "norm_drift_max": obs1["norm_drift_max"], "norm_drift_mean": obs1["norm_drift_mean"],
            "N_rel_change": (obs1["N"] - obs0["N"]) / obs0["N"]}


def in_kernel_z(prof):
    """True when the ABM phases ran without z-axis launches: the plane kernel with the
    z-term inside (kp_fast_zd) or the single-pass kernel."""
    return prof["zaxis"][0] == 0 and prof["plane_abm1"][0] > 0


def phase_roofline(prof, prof_steps, M, b_alg, rec=None):
    """Per-kernel bandwidth of the step.  The dominant kernel is the plane kernel of ABM
    phase 1; each ABM phase is charged half of the step's algorithmic bytes B_alg per
    qpwf (the unit the step fraction uses), and its design traffic (state arrays it
    moves from HBM, including the z-term scratch where the z-axis kernel runs) is given
    beside it."""
    out = {}
    arr = b_alg / 16.0                     # one state array of one qpwf
    if in_kernel_z(prof):
        design = {"plane_abm1": 9, "plane_abm2": 5, "zaxis": 0}
    else:
        design = {"plane_abm1": 10, "plane_abm2": 6, "zaxis": 4}   # arrays per qpwf-step
    for name in ("plane_abm1", "plane_abm2", "zaxis"):
        n, ms = prof[name]
        if n == 0:
            continue
        per_launch_q = prof_steps * M / n * (2 if name == "zaxis" else 1)
        avg_s = ms / n / 1e3
        d = {"launches": n, "avg_launch_ms": ms / n, "qpwfs_per_launch": per_launch_q,
             "design_arrays_per_qpwf": design[name] / (2 if name == "zaxis" else 1),
             "design_GBps": design[name] / (2 if name == "zaxis" else 1) * arr * per_launch_q / avg_s / 1e9}
        if name != "zaxis":
            d["alg_bytes_per_launch"] = 0.5 * b_alg * per_launch_q
            d["alg_GBps"] = d["alg_bytes_per_launch"] / avg_s / 1e9
            d["frac"] = d["alg_GBps"] * 1e9 / HBM_PEAK
        if rec:
            key = {"plane_abm1": "abm1_bytes_per_qpwf", "plane_abm2": "abm2_bytes_per_qpwf",
                   "zaxis": "kz_bytes_per_qpwf"}[name]
            d["pmc_traffic_per_launch"] = rec[key] * per_launch_q
        out[name] = d
    return out


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


def run_cfg3(steps, warmup, err_M, err_steps):
    """48^3 float32 vortex workload at full size (16384 qpwfs, 203 GB of state) timed,
    plus its float32 density error against float64 on a reduced instance."""
    import torch
    w = make_workload("cfg3")
    ctx, el, prof = run_gpu(w, steps, warmup, None, autotune=True)
    ps = prof.pop("steps")
    chosen = prof.pop("tuning")
    obs0 = prof.pop("obs0")
    obs1 = ctx.observables()
    mem = ctx.memory()
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    C, N, esz = w.functional.ncomp, w.lattice.n, 8
    b_alg = 16 * C * N * esz
    value = w.M * steps / el
    rec = measured_traffic("cfg3")
    out = {"workload": f"{w.name}: 48^3 lattice, {w.M} two-component qpwfs, LDA vortex line, float32 state "
                       "with float64 density/energy sums, dt=0.002",
           "value": value, "unit": "qpwf-steps/s", "ms_per_step": 1e3 * el / steps, "steps": steps,
           "dtype": "f32", "device_memory_GiB": mem / 2**30,
           "step_hbm_frac": value * b_alg / HBM_PEAK, "b_alg_per_qpwf_step": b_alg,
           "kernels": phase_roofline(prof, ps, w.M, b_alg, rec),
           "kernel_ms_per_step": {k: ms / ps for k, (n, ms) in prof.items()},
           "tuning": chosen,
           "drift": drift(obs0, obs1, steps)}
    if err_M:
        out["density_error_vs_fp64"] = reduced_error("cfg3", err_steps, err_M)
    return out


def run_batched(nsys, steps, warmup, err_group=16, with_error=True):
    """The 64-system workload (16^3/20^3/24^3, 512-3072 float32 qpwfs each): systems of
    one lattice side share one z-axis and one plane-kernel launch per ABM phase, and
    four steps replay as one captured graph.  Afterwards the same systems run in
    float64 (err_group at a time, the float64 state of all 64 would crowd the device)
    for the same number of steps, and the float32 densities are compared with them."""
    import torch
    import workloads as wl
    import paper_2009_00745_amd as lise
    systems = wl.config5_systems(seed=0, nsys=nsys)
    stream = torch.cuda.current_stream().cuda_stream
    ctxs = []
    t0 = time.time()
    for w in systems:
        c = lise.Context(w.lattice, w.M, w.functional, stream=stream)
        c.set_tuning(no_overlap=1)     # one z-scratch per context (the batch has its own)
        upload(c, w)
        ctxs.append(c)
    log(f"batched: {nsys} systems uploaded in {time.time() - t0:.1f}s")
    b = lise.Batch(ctxs, stream=stream)
    dt = systems[0].dt
    wsteps = 4 * max(1, (warmup + 3) // 4)
    b.step(dt, wsteps)                 # start-up, tables, graph capture, warm-up replays
    torch.cuda.synchronize()
    groups = b.info()
    obs0 = [c.observables() for c in ctxs]
    nst = 4 * max(1, steps // 4)
    t1 = time.perf_counter()
    b.step(dt, nst)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    obs1 = [c.observables() for c in ctxs]
    # kernel times from eager steps with events (graph replays carry none)
    b.profile(1)
    b.step(dt, 4)
    kt = {name: b.profile_read(cls) for cls, name in ((0, "plane_abm1"), (3, "plane_abm2"), (1, "zaxis"),
                                                       (2, "fields"))}
    b.profile(0)
    total_steps = ctxs[0].time()[1]
    dens32 = [c.densities() for c in ctxs]
    b.close()
    for c in ctxs:
        c.close()
    del ctxs
    torch.cuda.empty_cache()
    qsteps = sum(w.M for w in systems) * nst
    sizes = {}
    for w in systems:
        sizes.setdefault(w.lattice.nx, [0, 0])
        sizes[w.lattice.nx][0] += 1
        sizes[w.lattice.nx][1] += w.M
    b_alg_step = sum(w.M * 16 * 2 * w.lattice.n * 8 for w in systems)
    # float64 reference of every system, err_group systems at a time, same step count
    errs = []
    t0 = time.time()
    for g0 in range(0, nsys if with_error else 0, err_group):
        sub = []
        for w in systems[g0:g0 + err_group]:
            w.functional.precision = wl.FP64
            c = lise.Context(w.lattice, w.M, w.functional, stream=stream)
            c.set_tuning(no_overlap=1)
            upload(c, w)
            sub.append(c)
        bb = lise.Batch(sub, stream=stream)
        bb.step(dt, total_steps - 3)
        for k, c in enumerate(sub):
            n64, k64 = c.densities()
            n32, k32 = dens32[g0 + k]
            errs.append((float(np.linalg.norm(n32 - n64) / np.linalg.norm(n64)),
                         float(np.linalg.norm(k32 - k64) / np.linalg.norm(k64))))
        bb.close()
        for c in sub:
            c.close()
        torch.cuda.empty_cache()
    log(f"batched: float64 reference of {nsys} systems in {time.time() - t0:.1f}s")
    ms_plane = kt["plane_abm1"][1] / 4
    dE = [abs(o1["E"] - o0["E"]) / abs(o0["E"]) for o0, o1 in zip(obs0, obs1)]
    rec = measured_traffic("cfg5")
    traffic = None
    if rec:
        # per lattice group: HBM bytes per qpwf of one ABM step over all its kernels
        # (plane and z kernels, or the single-pass kernel and its density pass)
        per = 0.0
        for w in systems:
            per += w.M * rec.get(f"step_bytes_per_qpwf_{w.lattice.nx}", float("nan"))
        traffic = {"bytes_per_step": per, "vs_alg_bytes": per / b_alg_step,
                   "GBps_over_step": per * nst / el / 1e9}
    return {"workload": f"cfg5: {nsys} independent float32 systems (lattice 16^3/20^3/24^3, 512-3072 "
                        "two-component qpwfs each, Delta0 in [0.1, 0.6]), dt=0.002",
            "value": qsteps / el, "unit": "qpwf-steps/s", "systems": nsys, "steps": nst,
            "ms_per_step": 1e3 * el / nst, "qpwf_total": sum(w.M for w in systems), "dtype": "f32",
            "groups": groups[0], "systems_alone": groups[1], "graph": "one captured graph per 4 ABM steps",
            "lattices": {f"{k}^3": {"systems": v[0], "qpwfs": v[1]} for k, v in sorted(sizes.items())},
            "step_hbm_frac": b_alg_step * nst / el / HBM_PEAK,
            "kernel_ms_per_step": {k: ms / 4 for k, (n, ms) in kt.items()},
            "launches_per_step": {k: n / 4 for k, (n, ms) in kt.items()},
            "plane_abm1_alg_frac": 0.5 * b_alg_step / (ms_plane / 1e3) / HBM_PEAK if ms_plane > 0 else None,
            "density_error_vs_fp64": {"after_steps": int(total_steps), "systems": len(errs),
                                      "n_max": max(e[0] for e in errs), "kappa_max": max(e[1] for e in errs),
                                      "reference": "the same systems stepped in float64 on the GPU"} if errs else None,
            "pmc_traffic": traffic,
            "drift": {"E_rel_change_max": max(dE), "norm_drift_max": max(o["norm_drift_max"] for o in obs1)}}


PROFILES = os.path.join(ROOT, "profiles")
# PMC traffic summaries: workload key -> file, each with one TRAFFIC_JSON line
TRAFFIC_FILES = {"cfg2": "kp_fast_zd_fp64_32c_traffic.md", "cfg2_fp32": "kp_fast_fp32_32c_traffic.md",
                 "cfg3": "kp_fast_fp32_48c_traffic.md", "cfg4": "kp_mfma_64c4_traffic.md",
                 "cfg4_fp32": "kp_fast_fp32_64c4_traffic.md", "cfg5": "kp_fast_batch_cfg5_traffic.md"}
KERNEL_SOURCES = ("paper_2009_00745_amd/csrc/lise_device.hpp", "paper_2009_00745_amd/csrc/lise_fast.hpp",
                  "paper_2009_00745_amd/csrc/lise_cube.hpp", "paper_2009_00745_amd/csrc/lise_mfma.hpp")


def source_hash():
    """Hash of the kernel sources without their comments and blank space, so that a
    change to the documentation alone keeps the traffic records valid."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(" ".join(line.split()) for line in text.splitlines() if line.strip())
        h.update(code.encode())
    return h.hexdigest()[:16]


def measured_traffic(key="cfg2"):
    """Per-qpwf HBM traffic of the ABM kernels from the committed PMC summary of the
    workload, or None when there is none or the kernel sources changed since the
    counters were taken."""
    if key not in TRAFFIC_FILES:
        return None
    try:
        line = [ln for ln in open(os.path.join(PROFILES, TRAFFIC_FILES[key])) if ln.startswith("TRAFFIC_JSON ")][0]
    except (OSError, IndexError):
        return None
    rec = json.loads(line[len("TRAFFIC_JSON "):])
    return rec if rec["source_hash"] == source_hash() else None


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
    ap.add_argument("--z-lanes", type=int, default=0, help="lanes per z-column of the z kernel (1, 2, 4; 0 = default)")
    ap.add_argument("--z-dense", type=int, default=0,
                    help="z-term inside the plane kernel in the ABM phases (1 on, -1 off; 0 = default)")
    ap.add_argument("--single-pass", type=int, default=0,
                    help="1 = the single-pass ABM kernel wherever it fits, -1 = never, 0 = library default")
    ap.add_argument("--graph", action="store_true", help="replay four-step HIP graphs (kept by the autotuner)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=32)
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-phase", action="store_true",
                    help="skip the variant with the trivial phase removed (Eq. sp_en)")
    ap.add_argument("--batched", type=int, default=64,
                    help="number of independent systems in the batched form (0 = skip; 64 = the full workload)")
    ap.add_argument("--batch-no-error", action="store_true",
                    help="skip the float64 reference run of the batched systems (profiling runs)")
    ap.add_argument("--cfg3", type=int, default=1,
                    help="1 = also time the 48^3 float32 vortex workload (16384 qpwfs); 0 = skip")
    ap.add_argument("--cfg3-error-M", type=int, default=2048,
                    help="qpwfs of the reduced 48^3 instance on which float32 is compared with float64")
    ap.add_argument("--reduced-error", type=int, default=0, metavar="M",
                    help="cfg3/cfg4 as the main workload: also measure the float32 density error against "
                         "float64 on the same workload with M qpwfs")
    ap.add_argument("--reduced-steps", type=int, default=100)
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the path is built and measured on a single MI355X; "
              "multi-GPU sharding over qpwfs is a design note, not a run (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

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
    fixed_shape = bool(args.chunk or args.jgroup or args.no_overlap or args.z_lanes or args.single_pass or
                       args.z_dense)
    if fixed_shape or args.graph:
        tuning = {"chunk_qpwf": args.chunk, "jgroup": args.jgroup, "no_overlap": int(args.no_overlap),
                  "graph": int(args.graph), "z_lanes": args.z_lanes, "single_pass": args.single_pass,
                  "z_dense": args.z_dense}
    C, N = w.functional.ncomp, w.lattice.n
    esz = 16 if w.functional.precision == 0 else 8
    autotune = not args.no_autotune and not fixed_shape
    leg_tuning = dict(tuning) or None              # what the other legs start from
    ctx, elapsed, prof = run_gpu(w, args.steps, args.warmup, tuning, autotune=autotune)
    chosen = prof.pop("tuning")
    prof_steps = prof.pop("steps")
    obs0 = prof.pop("obs0")
    value = w.M * args.steps / elapsed
    ms_step = 1e3 * elapsed / args.steps
    b_alg = 16 * C * N * esz                      # compulsory state bytes per qpwf-step
    step_frac = value * b_alg / HBM_PEAK
    key = args.workload if args.workload in TRAFFIC_FILES else None
    rec = measured_traffic(key) if key else None
    kernels = phase_roofline(prof, prof_steps, w.M, b_alg, rec)
    dom = kernels["plane_abm1"]
    roofline = {"bound": "hbm", "achieved": dom["alg_GBps"], "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": dom["frac"],
                "traffic": dom.get("pmc_traffic_per_launch"),
                "kernel": ("plane kernel of ABM phase 1 with the z-term inside (kp_fast_zd, mode KP_ABM1)"
                           if in_kernel_z(prof) else "plane kernel of ABM phase 1 (kp_fast, mode KP_ABM1)"),
                "launches": dom["launches"], "avg_launch_ms": dom["avg_launch_ms"],
                "alg_bytes_per_launch": dom["alg_bytes_per_launch"],
                "alg_unit": "B_alg / 2 per qpwf of the launch (half of the step's 16 state arrays)",
                "step_frac": step_frac,
                "phases": kernels,
                "measured_copy_GBps": copy_bandwidth() / 1e9}
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
    drift_main = drift(obs0, obs, args.steps)
    if w.functional.ext_A != 0.0:
        drift_main["note"] = ("the external well is ramped on over the first 100 steps of the run: E changes "
                              "by the work of the time-dependent field, not by integration error alone")
        # after the timed region: the same state stepped on past the end of the ramp, then E
        # over 20 steps of a static Hamiltonian, where its change is integration error alone
        past = int(np.ceil(w.functional.ext_t_on / w.dt)) + 1 - int(round(t_now / w.dt))
        if past > 0:
            ctx.step(w.dt, past)
        oa = ctx.observables()
        ctx.step(w.dt, 20)
        ob = ctx.observables()
        drift_main["after_ramp"] = dict(drift(oa, ob, 20), steps=20, t_start=float(oa["t"]))
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
        o32 = prof32.pop("obs0")
        n32, k32 = ctx32.densities()
        t32, s32 = ctx32.time()
        o32b = ctx32.observables()
        ctx32.close()
        same = abs(t32 - t_now) < 1e-9 * max(1.0, abs(t_now))   # compared at equal times only
        val32 = w32.M * args.steps / el32
        b32 = 16 * C * N * 8
        variants["fp32_same_workload"] = {
            "value": val32, "unit": "qpwf-steps/s",
            "ms_per_step": 1e3 * el32 / args.steps,
            "kernel_ms_per_step": {k: ms / ps32 for k, (n, ms) in prof32.items()},
            "kernels": phase_roofline(prof32, ps32, w32.M, b32, measured_traffic("cfg2_fp32")),
            "speedup_vs_fp64": val32 / value,
            "density_rel_l2_vs_fp64": {
                "n": float(np.linalg.norm(n32 - n64) / np.linalg.norm(n64)),
                "kappa": float(np.linalg.norm(k32 - k64) / np.linalg.norm(k64))} if same else None,
            "after_steps": int(round(t32 / w32.dt)),
            "tuning": chosen32,
            "drift": drift(o32, o32b, args.steps),
            "step_hbm_frac": val32 * b32 / HBM_PEAK}

    if not args.no_phase and args.workload == "cfg2":
        wp = make_workload("cfg2", M=args.M)
        wp.functional.remove_phase = 1
        ctxp, elp, profp = run_gpu(wp, args.steps, args.warmup, leg_tuning,
                                   autotune=autotune)
        chosenp = profp.pop("tuning")
        psp = profp.pop("steps")
        profp.pop("obs0")
        n_p, k_p = ctxp.densities()
        tp, sp = ctxp.time()
        ctxp.close()
        same = abs(tp - t_now) < 1e-9 * max(1.0, abs(t_now))
        valp = wp.M * args.steps / elp
        variants["phase_removed_fp64"] = {
            "value": valp, "unit": "qpwf-steps/s", "ms_per_step": 1e3 * elp / args.steps,
            "kernel_ms_per_step": {k: ms / psp for k, (n, ms) in profp.items()},
            "cost_vs_plain": value / valp,
            "density_rel_l2_vs_plain": {
                "n": float(np.linalg.norm(n_p - n64) / np.linalg.norm(n64)),
                "kappa": float(np.linalg.norm(k_p - k64) / np.linalg.norm(k64))} if same else None,
            "after_steps": int(round(tp / wp.dt)), "tuning": chosenp,
            "note": "eta by Parseval on the register-FFT path: the pass re-reads x once, 22 state arrays per step instead of 20"}

    if args.reduced_error and args.workload in ("cfg3", "cfg4", "cfg4_fp32"):
        variants["reduced_error"] = reduced_error(args.workload[:4], args.reduced_steps, args.reduced_error)

    if args.cfg3 and args.workload == "cfg2":
        variants["cfg3_fp32_48c_m16384"] = run_cfg3(args.steps // 2, args.warmup, args.cfg3_error_M,
                                                    args.reduced_steps)

    if args.batched and args.workload == "cfg2":
        variants["batched_fp32"] = run_batched(args.batched, args.steps, args.warmup,
                                               with_error=not args.batch_no_error)

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
        "step_hbm_frac": step_frac,
        "b_alg_per_qpwf_step": b_alg,
        "kernel_ms_per_step": breakdown,
        "observables": {"t": t_now, "N": obs["N"], "E": obs["E"], "norm_drift_max": obs["norm_drift_max"]},
        "drift": drift_main,
        "variants": variants,
        "host": platform.node(),
    }
    print(json.dumps(out), flush=True)
    if _POOL is not None:
        _POOL.shutdown(wait=False)


if __name__ == "__main__":
    main()
