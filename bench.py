#!/usr/bin/env python
"""Throughput of the two-fluid finite-volume step on one MI355X.

Workload (default): the 8192 x 8192 roofline case -- 2000 seeded air bubbles
(radius U[16, 48] cells) in water hit by a planar 1 GPa shock, transmissive
walls, CFL 0.4 -- advanced in fast FP64 (FP64 with Newton-refined hardware
divisions and square roots, within 1e-12 of the FP64 contract), FP64 (the
contract bit for bit), FP32-bulk/FP64-accumulate and pure FP32.  A step is one
pass of the whole hot path: CFL time step from the device-side maximum, both
split sweeps (MUSCL-Hancock + HLLC + non-conservative z1 term), the pointwise
stage and the next step's CFL maximum.  Inputs are resident in HBM before the
timed region starts.

Prints ONE JSON line.  The fast FP64 mode is the headline `value` and its
state-update kernel the `roofline` (HBM bound: one read and one write of the
state per step against 8 TB/s, the library's copy kernel beside it as the
achievable ceiling); the other modes are reported under "modes", the serving
benchmark under "serving", and the paper's regular cavity array in water,
inert and reacting nitromethane under "liquids".
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
# One wave64 VALU instruction per SIMD every 4 cycles: 256 CU x 4 SIMD x 16
# lanes x 2.4 GHz lane-instructions/s (a diagnostic of how busy the issue
# slots are; the published 78.6 TFLOP/s FP64 counts a fused multiply-add as two)
VALU_ISSUE_PEAK = 256 * 4 * 16 * 2.4e9 / 1e12
BYTES_PER_CELL = {"fp64": 96, "fp64_fast": 96, "fp32_fp64acc": 96, "fp32": 48}   # 1 read + 1 write of 6 planes
DTYPE = {"fp64": "f64", "fp64_fast": "f64", "fp32_fp64acc": "f32/f64", "fp32": "f32"}
METRIC = "cell-updates/s/GPU FP32 vs FP64 (+% HBM roofline); batched p50/p99 latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the kernel sources with comments and whitespace removed (a
    comment edit does not invalidate a counter summary of the same code)."""
    h = hashlib.sha256()
    for f in ("meso_device.h", "meso_kernels.hip", "meso_kernels_fast.hip",
              "meso_kernels_fast64.hip", "meso_kernels_fp32.hip",
              "meso_kernels_react.hip", "meso_kernels_react_fast.hip", "meso_internal.h",
              "meso_api.hip"):
        text = open(os.path.join(ROOT, "paper_1905_05727_amd", "csrc", f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("".join(text.split()).encode())
    # the build flags of the kernels (contraction, scheduler) are part of what was measured
    h.update(open(os.path.join(ROOT, "paper_1905_05727_amd", "build.py"), "rb").read())
    return h.hexdigest()[:16]


def counters_from_profiles(mode: str):
    """Mean counters per launch of the step kernel from the committed rocprofv3
    summary of the roofline field, if it was taken on the current kernel source
    and build flags."""
    p = os.path.join(ROOT, "profiles", "step_kernel_roofline_8192_counters.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("modes", {}).get(mode)


def traffic_from_profiles(mode: str):
    """HBM bytes per launch (FETCH_SIZE and WRITE_SIZE scaled by a plain copy)."""
    m = counters_from_profiles(mode)
    return None if m is None else m.get("hbm_bytes_per_launch")


# Diagnostics of Sec. 4 timed on the state a mode leaves: transverse averages,
# domain integrals (both from one pass over the columns) and the mass-weighted
# log-binned PDFs of pressure and density (400 bins, as in the paper's figures).
DIAGNOSTICS = (("y_averages", lambda o: o.y_averages()),
               ("integrals", lambda o: o.integrals()),
               ("pdf_p", lambda o: o.log_histogram(9, 4.0, 0.0125, 400, 1.0)),       # p
               ("pdf_rho", lambda o: o.log_histogram(6, -1.0, 0.01, 400, 1.0)))      # rho


def time_diagnostics(obj, reps: int):
    """Wall-clock ms per call of each diagnostic (every call returns its result
    to the host, so it includes the launch, the synchronisation and the copy)."""
    out = {}
    for name, f in DIAGNOSTICS:
        f(obj)
        t = time.perf_counter()
        for _ in range(reps):
            f(obj)
        out[name] = 1e3 * (time.perf_counter() - t) / reps
    return out


def run_mode(sc, prec, steps, warmup, diagnostics=False, active=None):
    import torch
    from paper_1905_05727_amd import meso
    s = meso.Solver.from_scenario(sc, precision=prec)
    info = s.launch_info()
    s.run_steps(warmup)
    s.sync()
    s.enable_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.run_steps(steps)
    s.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, launches = s.kernel_time()
    t_sim, nstep, _ = s.time()
    out = {"s": t1 - t0, "kernel_ms_avg": kms / max(launches, 1), "launches": launches,
           "t_sim": t_sim, "step": nstep, "launch": info}
    out["fields"] = {k: s.read_field(k) for k in ("rho", "p")}
    if diagnostics:
        out["diagnostics_ms"] = time_diagnostics(s, 5)
    if active and active[0] > nstep:
        # a later window of the same run, where the shock has crossed more of
        # the field and more faces carry flow (the timed window above is the
        # near-rest start of the run)
        s.run_steps(active[0] - nstep)
        s.sync()
        s.enable_timing(True)
        s.run_steps(active[1])
        s.sync()
        kms2, l2 = s.kernel_time()
        out["active"] = {"from_step": active[0], "steps": active[1],
                         "kernel_ms_avg": kms2 / max(l2, 1)}
    s.close()
    torch.cuda.empty_cache()
    return out


def time_recording(sc, prec, steps, warmup):
    """Cost of the fused diagnostics: the same steps of the workload timed
    without recording, recording the transverse averages (Sec. 4.2, an x-t row
    per step), and recording the averages, the domain integrals (Eq. (10)) and
    a 400-bin mass-weighted pressure PDF (Sec. 4.5) together -- state kernel
    time by HIP events and wall time per step, which with recording includes
    the small kernels that finish each row."""
    import torch
    from paper_1905_05727_amd import meso
    out = {}
    nbins = 400
    with meso.Solver.from_scenario(sc, precision=prec) as s:
        m_ref = float(s.integrals()[1])
        s.run_steps(warmup)
        s.sync()
        avg = torch.empty((steps, 3, sc.nx), dtype=torch.float64, device="cuda")
        itg = torch.empty((steps, s.nplanes + 1), dtype=torch.float64, device="cuda")
        pdf = torch.empty((steps, nbins), dtype=torch.float64, device="cuda")
        for key in ("plain", "recording", "recording_all"):
            if key != "plain":
                s.record_averages(avg.data_ptr(), steps)
            if key == "recording_all":
                s.record_integrals(itg.data_ptr(), steps)
                s.record_histogram("p", 4.0, 0.015, nbins, m_ref, pdf.data_ptr(), steps)
            s.enable_timing(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.run_steps(steps)
            s.sync()
            t1 = time.perf_counter()
            kms, launches = s.kernel_time()
            out[key] = {"step_kernel_ms": kms / max(launches, 1),
                        "wall_ms_per_step": 1e3 * (t1 - t0) / steps}
            s.record_averages(0, 0)
            s.record_integrals(0, 0)
            s.record_histogram("p", 4.0, 0.015, nbins, m_ref, 0, 0)
        assert bool(torch.isfinite(avg).all()) and bool(torch.isfinite(itg).all())
        assert bool(torch.isfinite(pdf).all()) and float(pdf.sum()) > 0.0
        del avg, itg, pdf
    for key, k in (("extra_ms_per_step", "recording"), ("extra_ms_per_step_all", "recording_all")):
        out[key] = out[k]["wall_ms_per_step"] - out["plain"]["wall_ms_per_step"]
    torch.cuda.empty_cache()
    return out


def copy_bandwidth(gib: float = 2.0, reps: int = 5):
    """Achievable HBM ceiling: the library's plain HIP copy kernel
    (mf_stream_copy) moving `gib` GiB (one read + one write per byte, like the
    step's algorithmic traffic) in each of its variants and three grid sizes,
    the best of which is the ceiling; torch's copy_ of the same buffers beside
    it.  The same copy is the reference against which rocprofv3's FETCH_SIZE
    and WRITE_SIZE are scaled."""
    import torch
    from paper_1905_05727_amd import meso
    n = int(gib * 2 ** 30) // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    nbytes = n * 8
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(f):
        f()
        torch.cuda.synchronize()
        e0.record(st)
        for _ in range(reps):
            f()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    kernels = {}
    for variant, name in ((0, "x1"), (1, "x4"), (2, "x1_nt"), (3, "x4_nt")):
        for wg in (0, 4096, 16384):
            ms = timed(lambda: meso.stream_copy(a.data_ptr(), b.data_ptr(), nbytes, variant, wg,
                                                st.cuda_stream))
            kernels[f"{name}_wg{wg or 'auto'}"] = 2 * nbytes / (ms * 1e-3) / 1e9
    assert torch.equal(a, b), "stream copy result differs from its source"
    ms_torch = timed(lambda: b.copy_(a))
    best = max(kernels, key=kernels.get)
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_per_launch": 2 * nbytes, "GBs": kernels[best], "best": best,
            "kernels_GBs": kernels, "torch_copy_GBs": 2 * nbytes / (ms_torch * 1e-3) / 1e9}


def serving_bench(nreq: int, nsteps: int, precision: str = "fp32_fp64acc"):
    """Serving workload: `nreq` independent shock-bubble solves of sizes
    {128^2, 256^2, 512^2}, `nsteps` steps each.  Sequential capacity first
    (solves back to back, one at a time, per-solve launches), then Poisson
    arrivals at 0.8x and 2x that capacity through the batched server and
    through the sequential baseline, and a burst of all requests at once (on a
    fresh server, then on the warm one).  At 2x and in the warm burst, a
    second sequential baseline: a one-slot server (one solve at a time with
    its own launches, but no allocation per request)."""
    from paper_1905_05727_amd import scenario, serve
    t = time.perf_counter()
    reqs = scenario.serving_workload(nreq, steps=nsteps)
    log(f"serving: {nreq} requests generated ({time.perf_counter() - t:.1f} s)")
    work = float(sum(r.nx * r.ny for r in reqs)) * nsteps
    serve.solve_alone(reqs[0], 5, precision)          # warm up allocator and code objects
    t = time.perf_counter()
    for sc in reqs:
        serve.solve_alone(sc, nsteps, precision)
    t_seq = time.perf_counter() - t
    cap = nreq / t_seq
    log(f"serving: sequential back-to-back {t_seq:.2f} s -> capacity {cap:.1f} req/s, "
        f"{work / t_seq / 1e9:.2f} G cell-updates/s")
    out = {"requests": nreq, "steps": nsteps, "precision": precision,
           "sizes": sorted({r.nx for r in reqs}), "cell_updates": work,
           "sequential_capacity_req_per_s": cap,
           "sequential_back_to_back_cell_updates_per_s": work / t_seq, "rates": {}}
    budget = 16 << 30
    # A second sequential baseline without per-request allocation: the same
    # server machinery with one slot (one solve at a time, its own launches,
    # pooled pinned buffers), warmed up on a few requests first.
    one = serve.Server(budget, max_slots=1, precision=precision, max_inflight=8)
    serve.serve(one, reqs[:8], np.zeros(8), nsteps)
    # One server for every run, as a serving process keeps it: the first burst
    # finds its pinned host pools empty and allocates them (reported as the
    # cold start); the later runs reuse them.
    with serve.Server(budget, max_slots=64, precision=precision, max_inflight=8) as srv:
        for key, mult in (("burst_cold_start", None), ("0.8x", 0.8), ("2.0x", 2.0),
                          ("burst", None)):
            # None: a burst -- every request arrives at t = 0 (capacity of each path)
            arr = np.zeros(nreq) if mult is None else scenario.poisson_arrivals(nreq, mult * cap)
            ticks0 = srv.stats()["ticks"]
            b = serve.serve(srv, reqs, arr, nsteps)
            entry = {
                "arrival_rate_req_per_s": None if mult is None else mult * cap,
                "batched": {"p50_ms": 1e3 * b["p50_s"], "p99_ms": 1e3 * b["p99_s"],
                            "cell_updates_per_s": b["cell_updates_per_s"],
                            "makespan_s": b["makespan_s"],
                            "peak_hbm_bytes": b["stats"]["peak_bytes"], "hbm_budget": budget,
                            "ticks": b["stats"]["ticks"] - ticks0}}
            msg = (f"serving {key}: batched p50 {1e3 * b['p50_s']:.1f} ms p99 "
                   f"{1e3 * b['p99_s']:.1f} ms {b['cell_updates_per_s'] / 1e9:.2f} G/s")
            if key != "burst_cold_start":
                sq = serve.serve_sequential(reqs, arr, nsteps, precision)
                entry["sequential"] = {"p50_ms": 1e3 * sq["p50_s"], "p99_ms": 1e3 * sq["p99_s"],
                                       "cell_updates_per_s": sq["cell_updates_per_s"],
                                       "makespan_s": sq["makespan_s"]}
                msg += (f" | sequential p50 {1e3 * sq['p50_s']:.1f} ms p99 "
                        f"{1e3 * sq['p99_s']:.1f} ms {sq['cell_updates_per_s'] / 1e9:.2f} G/s")
                if key in ("2.0x", "burst"):
                    o1 = serve.serve(one, reqs, arr, nsteps)
                    entry["sequential_one_slot_server"] = {
                        "p50_ms": 1e3 * o1["p50_s"], "p99_ms": 1e3 * o1["p99_s"],
                        "cell_updates_per_s": o1["cell_updates_per_s"],
                        "makespan_s": o1["makespan_s"]}
                    msg += (f" | one-slot server p50 {1e3 * o1['p50_s']:.1f} ms p99 "
                            f"{1e3 * o1['p99_s']:.1f} ms {o1['cell_updates_per_s'] / 1e9:.2f} G/s")
            out["rates"][key] = entry
            log(msg)
    one.close()
    return out


def oracle_of(sc, rows=None):
    """The FP64 oracle on the scenario's initial state (its first `rows` rows
    if given)."""
    import oracle
    ny = sc.ny if rows is None else rows
    bc = [{"transmissive": oracle.TRANSMISSIVE, "periodic": oracle.PERIODIC}[b] for b in sc.bc]
    prob = oracle.Problem(sc.nx, ny, sc.dx, sc.dy, gamma1=sc.gamma1, pinf1=sc.pinf1,
                          gamma2=sc.gamma2, pinf2=sc.pinf2, cfl=sc.cfl, zeps=sc.zeps,
                          bc_xlo=bc[0], bc_xhi=bc[1], bc_ylo=bc[2], bc_yhi=bc[3],
                          eos2=sc.eos2, cc=sc.cc, reactive=int(sc.reactive), rx=sc.rx)
    o = oracle.Oracle(prob)
    o.set_primitive(sc.prim[:, :ny, :])
    return o


def oracle_diagnostics(sc, rows):
    """The oracle's diagnostics on the first `rows` rows of the initial state,
    per call, scaled to the full grid (they are linear in the cell count)."""
    import oracle
    o = oracle_of(sc, rows)
    ms = time_diagnostics(o, 1)
    scale = sc.ny / rows
    return {"ms": {k: v * scale for k, v in ms.items()}, "cores": oracle.num_threads(),
            "sample": f"{sc.nx}x{rows} crop of the initial state, scaled x{scale:g}"}


def cpu_one_core(sc, rows: int, nsteps: int):
    """The oracle on one thread: `nsteps` steps of the first `rows` rows of the
    workload (the cell-update rate does not depend on the row count)."""
    import oracle
    o = oracle_of(sc, rows)
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        o.run(nsteps)
        dt = time.perf_counter() - t0
    finally:
        oracle.set_threads(0)
    return {"value": sc.nx * rows * nsteps / dt, "unit": "cell-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{nsteps} step(s) of a {sc.nx}x{rows} crop of the workload, 1 thread "
                      f"({dt:.1f} s)"}


def cpu_baseline(sc, nsteps):
    import oracle
    o = oracle_of(sc)
    t0 = time.perf_counter()
    o.run(nsteps)
    dt = time.perf_counter() - t0
    return {"value": sc.nx * sc.ny * nsteps / dt, "unit": "cell-updates/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"first {nsteps} steps of the full {sc.nx}x{sc.ny} workload, FP64 "
                      f"oracle ({dt:.1f} s)"}


# The paper's regular cavity array (Sec. 2.4: d_c = 100 cells, porosity 8 %,
# spacing 313 cells, 24000 cells long, periodic in y) with each liquid of the
# build: water (stiffened gas), inert nitromethane (Cochran-Chan, shocked to
# 7.81 GPa) and reacting nitromethane (7th conserved plane, Arrhenius stage).
LIQUIDS = (("water", {}),
           ("nitromethane", {"liquid": "nm", "p_shock": 7.81e9}),
           ("nitromethane_reactive", {"liquid": "nm", "p_shock": 7.81e9, "reactive": True}))


def valu_per_cell_from_profiles(liquid: str, mode: str):
    """Measured VALU instructions per cell-step of the regular-array kernels
    from the committed rocprofv3 counter summary, if it was taken on the
    current kernel source and build flags."""
    p = os.path.join(ROOT, "profiles", "step_kernel_regular_array_counters.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("valu_per_cell", {}).get(f"{liquid}/{mode}")


def liquids_bench(modes, steps, warmup, cpu_steps):
    """Cell-updates/s of the regular cavity array for each liquid and mode,
    with the HBM fraction (algorithmic bytes), the VALU-issue fraction (counted
    instructions) and the FP64 oracle on the host cores beside it."""
    from paper_1905_05727_amd import scenario
    out = {}
    for name, kw in LIQUIDS:
        sc = scenario.regular_array(**kw)
        N = sc.nx * sc.ny
        planes = 7 if sc.reactive else 6
        row = {"grid": [sc.nx, sc.ny], "cavities": sc.meta["ncavities"], "modes": {}}
        for m in modes:
            r = run_mode(sc, m, steps, warmup)
            kms = r["kernel_ms_avg"]
            nbytes = 2 * planes * (4 if m == "fp32" else 8) * N
            d = {"value": N * steps / r["s"], "kernel_ms": kms,
                 "hbm_algorithmic_GBs": nbytes / (kms * 1e-3) / 1e9}
            d["hbm_frac"] = d["hbm_algorithmic_GBs"] / HBM_PEAK_GBS
            v = valu_per_cell_from_profiles(name, m)
            if v is not None:
                d["valu_per_cell"] = v
                d["valu_issue_frac"] = v * N / (kms * 1e-3) / (VALU_ISSUE_PEAK * 1e12)
            row["modes"][m] = d
            log(f"  {name} {m}: {d['value'] / 1e9:.2f} G cell-updates/s, kernel {kms:.3f} ms")
        if cpu_steps:
            row["cpu_baseline"] = cpu_baseline(sc, cpu_steps)
            log(f"  {name} oracle: {row['cpu_baseline']['value'] / 1e6:.1f} M cell-updates/s")
        out[name] = row
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=8192, help="grid size (n x n)")
    ap.add_argument("--modes", default="fp64_fast,fp64,fp32_fp64acc,fp32")
    ap.add_argument("--headline", default="fp64_fast",
                    help="mode whose rate is the line's value (an FP64 mode: fp64_fast, fp64)")
    ap.add_argument("--active-from", type=int, default=600,
                    help="step from which a second window of each run is timed")
    ap.add_argument("--active-steps", type=int, default=20,
                    help="steps of that window (0: skip it)")
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--serving-steps", type=int, default=500)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--liquid-steps", type=int, default=200,
                    help="timed steps of each regular-array run (0: skip that section)")
    ap.add_argument("--liquids-only", action="store_true",
                    help="only the regular-array section (for profiling its kernels)")
    ap.add_argument("--serving-only", action="store_true",
                    help="only the serving section (for profiling the batched kernels)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this solver runs one domain on one GPU; multi-GPU runs are not "
              "supported (the domain decomposition over several GPUs is a design, not code). "
              "Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1905_05727_amd import scenario
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)

    modes = [m for m in args.modes.split(",") if m]
    if args.liquids_only:
        print(json.dumps({"liquids": liquids_bench(modes, args.liquid_steps, args.warmup, 0)}),
              flush=True)
        return
    if args.serving_only:
        print(json.dumps({"serving": serving_bench(args.serving_requests, args.serving_steps)}),
              flush=True)
        return

    t = time.perf_counter()
    sc = scenario.roofline_8192(n=args.n)
    log(f"scenario {sc.name} {sc.nx}x{sc.ny}: {sc.meta['nbubbles']} bubbles, porosity "
        f"{sc.meta['porosity']:.3f} ({time.perf_counter() - t:.1f} s)")
    N = sc.nx * sc.ny
    active = (args.active_from, args.active_steps) if args.active_steps > 0 else None
    res = {}
    for m in modes:
        log(f"mode {m}: warmup {args.warmup}, timing {args.steps} steps")
        res[m] = run_mode(sc, m, args.steps, args.warmup, diagnostics=(m == "fp64"),
                          active=active)
        r = res[m]
        log(f"  {N * args.steps / r['s'] / 1e9:.2f} G cell-updates/s, kernel "
            f"{r['kernel_ms_avg']:.3f} ms/launch, t_sim {r['t_sim']:.3e}"
            + (f"; steps {r['active']['from_step']}+: kernel "
               f"{r['active']['kernel_ms_avg']:.3f} ms" if "active" in r else ""))

    cp = copy_bandwidth()
    log(f"copy kernel: {cp['GBs']:.0f} GB/s ({cp['best']}; torch copy_ "
        f"{cp['torch_copy_GBs']:.0f} GB/s; {cp['bytes_per_launch'] / 2 ** 30:.1f} GiB moved "
        f"per launch)")

    mode_out = {}
    ref = res.get("fp64")
    for m, r in res.items():
        cups = N * args.steps / r["s"]
        ach = BYTES_PER_CELL[m] * N / (r["kernel_ms_avg"] * 1e-3) / 1e9
        d = {"value": cups, "ms_per_step": 1e3 * r["s"] / args.steps,
             "kernel_ms": r["kernel_ms_avg"], "hbm_algorithmic_GBs": ach,
             "hbm_frac": ach / HBM_PEAK_GBS, "copy_ceiling_frac": ach / cp["GBs"],
             "dtype": DTYPE[m]}
        if "active" in r:
            a_ms = r["active"]["kernel_ms_avg"]
            d["active_window"] = {
                "from_step": r["active"]["from_step"], "steps": r["active"]["steps"],
                "kernel_ms": a_ms,
                "hbm_frac": BYTES_PER_CELL[m] * N / (a_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        tb = traffic_from_profiles(m)
        if tb is not None:      # counted HBM bytes of the same kernel / its time here
            d["hbm_measured_GBs"] = tb / (r["kernel_ms_avg"] * 1e-3) / 1e9
            d["hbm_measured_frac"] = d["hbm_measured_GBs"] / HBM_PEAK_GBS
        cm = counters_from_profiles(m)
        if cm is not None and "SQ_INSTS_VALU" in cm:
            # counted VALU instructions (one per wave, 64 lanes) of the same kernel / its
            # time here, against one wave64 instruction per SIMD every 4 cycles
            d["valu_per_cell"] = cm["SQ_INSTS_VALU"] * 64 / N
            d["valu_issue_frac"] = (cm["SQ_INSTS_VALU"] * 64 / (r["kernel_ms_avg"] * 1e-3)
                                    / (VALU_ISSUE_PEAK * 1e12))
        if ref is not None and m != "fp64":
            for k in ("rho", "p"):
                d[f"rel_l1_{k}_vs_fp64"] = float(np.abs(r["fields"][k] - ref["fields"][k]).sum()
                                                 / np.abs(ref["fields"][k]).sum())
        mode_out[m] = d

    head = args.headline if args.headline in res else modes[0]
    h = mode_out[head]
    r = res[head]
    line = {
        "metric": METRIC,
        "value": h["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": h["dtype"],
        "data": "synthetic",
        "config": {"workload": f"roofline case {sc.nx}x{sc.ny}: {sc.meta['nbubbles']} air "
                               f"bubbles R~U[16,48] cells in water (centre spacing >= 2.5 "
                               f"mean diameters), 1 GPa planar shock, CFL 0.4, "
                               f"seed {sc.meta['seed']}",
                   "cells": N, "precision": head, "parallelism": "single GPU",
                   "launch": r["launch"]},
        "roofline": {"bound": "hbm", "achieved": h["hbm_algorithmic_GBs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": h["hbm_frac"],
                     "traffic": traffic_from_profiles(head),
                     "kernel": f"step_kernel ({head}, fused x/y sweep)",
                     "bytes_per_cell": BYTES_PER_CELL[head], "cells_per_launch": N,
                     "kernel_ms": h["kernel_ms"],
                     "copy_ceiling_GBs": cp["GBs"], "copy_ceiling_frac": h["copy_ceiling_frac"],
                     "valu_issue": {"instr_per_cell": h.get("valu_per_cell"),
                                    "frac": h.get("valu_issue_frac")}},
        "modes": mode_out,
        "copy_kernel": cp,
    }
    if not args.no_serving:
        line["serving"] = serving_bench(args.serving_requests, args.serving_steps)
    if args.liquid_steps:
        log(f"regular cavity array: {args.liquid_steps} steps per liquid and mode")
        line["liquids"] = liquids_bench(modes, args.liquid_steps, args.warmup,
                                        0 if args.no_cpu_baseline else 4)
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle, {args.cpu_steps} steps")
        line["cpu_baseline"] = cpu_baseline(sc, args.cpu_steps)
        line["cpu_baseline_one_core"] = cpu_one_core(sc, min(sc.ny, 512), 1)
    if "fp64" in res:
        # each diagnostic reads the whole FP64 state once (6 planes x 8 B per cell)
        nbytes = 48 * N
        g = res["fp64"]["diagnostics_ms"]
        fused = {m: time_recording(sc, m, 20, args.warmup) for m in (head, "fp32_fp64acc")
                 if m in res}
        for m, f in fused.items():
            log(f"fused averages {m}: step kernel {f['plain']['step_kernel_ms']:.3f} -> "
                f"{f['recording']['step_kernel_ms']:.3f} ms, wall +{f['extra_ms_per_step']:.3f} "
                f"ms per step (separate pass {g['y_averages']:.3f} ms); with integrals and "
                f"pressure PDF {f['recording_all']['step_kernel_ms']:.3f} ms, wall "
                f"+{f['extra_ms_per_step_all']:.3f} ms (separate passes "
                f"{g['y_averages'] + g['integrals'] + g['pdf_p']:.3f} ms)")
        line["diagnostics"] = {
            "fused_averages": fused,
            "state": "FP64 roofline field after the timed steps", "bytes_read": nbytes,
            "gpu_ms": g, "gpu_GBs": {k: nbytes / (v * 1e-3) / 1e9 for k, v in g.items()},
            "gpu_hbm_frac": {k: nbytes / (v * 1e-3) / 1e9 / HBM_PEAK_GBS for k, v in g.items()},
            "oracle": (None if args.no_cpu_baseline
                       else oracle_diagnostics(sc, min(sc.ny, 1024)))}
        log("diagnostics (ms): " + ", ".join(f"{k} {v:.2f}" for k, v in g.items()))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
