"""Benchmark of the PRS domain-wall hot path on one MI355X.

One benchmark step is one whole run of the 2D matter-era workload: a
8192^2 periodic lattice, W0 = 10, m = 2, deta = 0.25, eta 1 -> 4096
(16380 leapfrog steps), seeded uniform initial field, wall diagnostics fused
every 64 steps plus the final state, and the scaling-exponent fit over the
last decade.  The metric is lattice-site updates per second (sites x steps /
wall time), with the inputs already in HBM when the timed region starts.

Prints one JSON line (see the "roofline" and "cpu_baseline" objects for how
the kernel and the oracle were measured).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
# MI355X vector-ALU issue rate without packed FP32 (the kernels are built
# without it): 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
# Algorithmic HBM bytes of one pass per site (FP32): phi and phi_dot read
# once and written once, whatever the number of steps the pass fuses
BYTES_PER_SITE_PASS = 16
# The same 16 bytes per site-update is the traffic of a single-step pass: the
# figure the site-update rate is compared with as "effective" bandwidth
BYTES_PER_UPDATE = 16
# HBM bytes of one launch of a pass kernel, by (lattice, vec, rows, ty, steps
# per pass): rocprofv3 FETCH_SIZE + WRITE_SIZE (KiB per dispatch) scaled by
# what the same counters read for a plain copy of known size (factors 2.00 and
# 1.00), from the profile named in each entry, taken on kernel sources whose
# digest (kernel_digest()) is recorded with it.  When the sources differ now
# the counters no longer describe the kernel and the bench reports null.
TRAFFIC_PER_LAUNCH = {
    ("2d8192", 4, 71, 1, 8): {"bytes": 1132171638, "profile": "profiles/k_tb2d_2d8192.md",
                              "sources": "b7b7a7ed00d3f01c"},
    ("2d8192", 2, 64, 1, 8): {"bytes": 1158439244, "profile": "profiles/k_tb2d_2d8192.md",
                              "sources": "b7b7a7ed00d3f01c"},
    ("3d1024", 2, 32, 16, 4): {"bytes": 23574425145, "profile": "profiles/k_tb3l_3d1024.md",
                               "sources": "b7b7a7ed00d3f01c"},
}

WORKLOAD = {
    "name": "2D PRS 8192^2, matter era m=2, W0=10, deta=0.25, eta 1->4096 (16380 steps), "
            "diagnostics every 64 steps + final, exponent fit over the last decade",
    "key": "2d8192", "shape": (8192, 8192), "m": 2.0, "W0": 10.0, "deta": 0.25, "eta_end": 4096.0,
    "diag_every": 64, "seed": 1,
}
WORKLOAD_3D = {
    "name": "3D PRS 1024^3, radiation era m=1, W0=10, deta=0.2, eta 1->512 (2555 steps), "
            "diagnostics every 50 steps + final, exponent fit over the last decade",
    "key": "3d1024", "shape": (1024, 1024, 1024), "m": 1.0, "W0": 10.0, "deta": 0.2, "eta_end": 512.0,
    "diag_every": 50, "seed": 1,
}


def kernel_digest():
    """Digest of the kernel sources (device code and its launch templates)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("prs_device.h", "prs_kernels.hip", "prs_ensemble.hip", "prs_internal.h"):
        with open(os.path.join(ROOT, "paper_1710_10420_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def n_steps(w):
    return int(round((w["eta_end"] - 1.0) / w["deta"]))


def one_run(sim, prs, w, S, stream_handle):
    """Reset to the seeded initial field and run the whole evolution."""
    cur_phi = prs.prs_get_state(sim.ctx)[0]
    prs.prs_fill_uniform(cur_phi, sim.phi_a.numel(), w["seed"], stream_handle)
    sim.dphi.zero_()
    prs.prs_set_state(sim.ctx, None, None, 0)
    recs = sim.step_n(S)
    recs.append(sim.wall_stats())
    mu, nu = prs.prs_fit_scaling(recs, w["eta_end"] / 10.0)
    return recs, mu, nu


def cpu_baseline(w, budget_s=12.0):
    """The FP64 oracle on the host cores over a bounded prefix of the same
    run (the first steps from the same seeded field): once on every core the
    process may use and once on a single thread (the paper's CPU baseline is
    sequential code)."""
    from oracle import oracle as O
    from paper_1710_10420_amd.inputs import uniform_field

    shape = w["shape"]
    op = O.params(shape, deta=w["deta"], m=w["m"], W0=w["W0"])
    phi = uniform_field(shape, w["seed"]).astype(np.float64).reshape(-1)
    pi = np.zeros_like(phi)
    sites = phi.size
    out = {}
    cores = len(os.sched_getaffinity(0))
    for label, threads in (("all_cores", cores), ("single_thread", 1)):
        O.set_threads(threads)
        t0 = time.perf_counter()
        O.run(op, phi, pi, 1)                       # calibration step
        per = time.perf_counter() - t0
        steps = max(1, min(64, int(budget_s / max(per, 1e-6))))
        t0 = time.perf_counter()
        O.run(op, phi, pi, steps, diag_every=w["diag_every"])
        dt = time.perf_counter() - t0
        out[label] = {"value": sites * steps / dt, "cores": threads, "steps": steps, "seconds": dt}
    O.set_threads(cores)
    a = out["all_cores"]
    return {"value": a["value"], "unit": "site-updates/s", "cores": a["cores"], "kind": "oracle",
            "sample": "FP64 oracle, first %d of %d steps of the same %s run (diagnostics every %d included), "
                      "%.1f s on %d threads" % (a["steps"], n_steps(w), "x".join(map(str, shape)),
                                                 w["diag_every"], a["seconds"], a["cores"]),
            "single_thread": dict(out["single_thread"], unit="site-updates/s",
                                  sample="first %d steps on one thread" % out["single_thread"]["steps"])}


def copy_ceiling(prs, torch, nbytes=1 << 30, reps=10):
    """Bandwidth of the library's plain copy kernel (prs_copy) between two
    1 GiB buffers: bytes read plus bytes written per second, the best of
    `reps` timed copies."""
    stream = torch.cuda.current_stream()
    sh = prs._stream_handle(stream)
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    prs.prs_copy(dst.data_ptr(), src.data_ptr(), nbytes, sh)
    best = 1e30
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        prs.prs_copy(dst.data_ptr(), src.data_ptr(), nbytes, sh)
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    ok = bool(torch.equal(src[:1024], dst[:1024]))
    del src, dst
    torch.cuda.empty_cache()
    return {"kernel": "k_copy16 (prs_copy)", "bytes_per_copy": 2 * nbytes, "best_us": best * 1e6,
            "gbs": 2 * nbytes / best / 1e9, "frac_of_peak": 2 * nbytes / best / 1e9 / HBM_PEAK_GBS,
            "checked": ok}


def isa_counts():
    path = os.path.join(ROOT, "paper_1710_10420_amd", "isa_counts.json")
    try:
        with open(path) as f:
            return json.load(f)
    except OSError:
        return None


def pass_valu_lane_ops(shape, tiling, T, counts):
    """Vector-ALU lane operations of one launch of the T-step pass over the
    lattice, from the march loop's instruction count in this build: a wave
    issues the loop's VALU instructions per iteration for every level that
    has a row (2D) or plane (3D) at that iteration (level k starts 2(k-1)
    iterations late; a tile of r rows or planes runs r + 2T - 2 iterations),
    64 lanes each.  (None, None) when the counts are missing."""
    vec, rows, ty = tiling
    if counts is None:
        return None, None
    H = -(-T // vec)
    W = (64 - 2 * H) * vec
    tiles_x = -(-shape[0] // W)
    M = shape[-1]
    if len(shape) == 2:
        own_rows = 1
        c = counts.get("k_tb2d<%d,%d,0,1,f>" % (vec, T))
        tiles_q = 1
    elif ty in (8, 16, 32, 64):
        # LDS-staged pass: workgroups of NW waves with R rows each, of which
        # the middle NW R - 2T rows are stored; every wave computes its R rows
        NW = 16 if ty >= 32 else 8
        R = ty // 16 if ty >= 32 else ty // 4
        own_rows = R
        c = counts.get("k_tb3l<%d,%d,%d,%d,0,1,0,f>" % (vec, T, R, NW))
        tiles_q = -(-shape[1] // (NW * R - 2 * T)) * NW
    else:
        own_rows = 8 if ty == 4 else 4             # rows along y a wave owns
        c = counts.get("k_tb3d<%d,%d,%d,0,1,f>" % (vec, T, own_rows))
        tiles_q = -(-shape[1] // own_rows)
    if not c or c["vmem_store"] < 2 * own_rows:
        return None, None
    iters_in_loop = c["vmem_store"] / (2.0 * own_rows)   # level T stores phi and phi_dot of the wave's rows
    per_iter = c["valu"] / iters_in_loop
    level_iters = 0
    for s0 in range(0, M, rows):
        n = min(rows, M - s0) + 2 * T - 2
        level_iters += sum(n - 2 * (k - 1) for k in range(1, T + 1))
    lane_ops = per_iter / T * level_iters * tiles_x * tiles_q * 64
    stored_rows = own_rows
    if len(shape) == 3 and ty in (8, 16, 32, 64):
        stored_rows = (NW * R - 2 * T) / float(NW)
    return lane_ops, {"valu_per_iteration": per_iter,
                      "valu_per_owned_site_update": per_iter / (vec * stored_rows * T),
                      "loop_instructions": c}


def forward_leg(prs, torch, w, runs, warmup, tiling=None, steps_per_pass=None, extra=True):
    """Whole runs of a forward workload: tuned (or given) tiling and steps per
    pass, `warmup` untimed runs, then `runs` timed runs bracketed by stream
    events, with launch timing on, so that the average duration of the pass
    kernel is measured live over the timed region."""
    S = n_steps(w)
    stream = torch.cuda.current_stream()
    sh = prs._stream_handle(stream)
    gp = prs.make_params(w["shape"], deta=w["deta"], m=w["m"], W0=w["W0"], diag_every=w["diag_every"])
    sites = prs.sites(gp)
    sim = prs.Sim(gp, seed=w["seed"])
    if tiling:
        sim.set_tiling(*tiling)
        sim.set_time_blocking(steps_per_pass or 1)
    else:
        prs.prs_autotune(sim.ctx, None, 0)    # tiling and steps per pass, before the timed region
    log(w["key"], "tiling", sim.tiling(), "steps/pass", sim.time_blocking(), "steps/run", S)
    for i in range(warmup):
        log(w["key"], "warmup run", i)
        one_run(sim, prs, w, S, sh)
    torch.cuda.synchronize()
    prs.prs_set_launch_timing(sim.ctx, True)
    prs.prs_get_launch_timing(sim.ctx, reset=True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    results = []
    for i in range(runs):
        results.append(one_run(sim, prs, w, S, sh))
        log(w["key"], "timed run", i, "done")
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    k_ms, k_launches = prs.prs_get_launch_timing(sim.ctx, reset=True)
    prs.prs_set_launch_timing(sim.ctx, False)

    updates = float(sites) * S * runs
    T = sim.time_blocking()
    til = tuple(sim.tiling())
    multi, single = prs.prs_plan_passes(sim.ctx, S, True)
    avg_launch_s = k_ms / 1e3 / k_launches if k_launches else None
    per_launch_bytes = BYTES_PER_SITE_PASS * sites           # algorithmic bytes of one pass
    achieved = per_launch_bytes / avg_launch_s / 1e9 if avg_launch_s else None
    digest = kernel_digest()
    tr = TRAFFIC_PER_LAUNCH.get((w["key"],) + til + (T,))
    traffic = tr["bytes"] if tr and tr["sources"] == digest else None
    lane_ops, isa = pass_valu_lane_ops(w["shape"], til, T, isa_counts()) if T > 1 else (None, None)
    if T == 1:
        kernel = "k_step (one fused leapfrog step per pass)"
    elif len(w["shape"]) == 3 and til[2] in (8, 16, 32, 64):
        kernel = ("k_tb3l<vec=%d,T=%d,waves=%d> (%d fused leapfrog steps per pass, row halos through LDS)"
                  % (til[0], T, 16 if til[2] >= 32 else 8, T))
    else:
        kernel = "k_tb%dd<vec=%d,T=%d> (%d fused leapfrog steps per pass)" % (len(w["shape"]), til[0], T, T)
    recs, mu, nu = results[-1]
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved else None,
            "traffic": traffic,
            "kernel": kernel,
            "algorithmic_bytes_per_launch": per_launch_bytes,
            "algorithmic_bytes_per_site_per_pass": BYTES_PER_SITE_PASS,
            "site_updates_per_launch": sites * T,
            "avg_launch_us": avg_launch_s * 1e6 if avg_launch_s else None,
            "timed_launches": k_launches,
            "launch_timing": "HIP events on the library's stream around each run of consecutive pass-kernel "
                             "launches inside the timed region (prs_set_launch_timing)",
            # the site-update rate of the pass as the bandwidth a single-step
            # pass (16 B per site-update) would need, over the HBM peak
            "effective_single_step_gbs": (BYTES_PER_UPDATE * sites * T / avg_launch_s / 1e9
                                          if avg_launch_s else None),
            "effective_single_step_frac": (BYTES_PER_UPDATE * sites * T / avg_launch_s / 1e9 / HBM_PEAK_GBS
                                           if avg_launch_s else None),
            "passes_per_run": {"multi_step": multi, "single_step": single}}
    if traffic:
        roof["dram_gbs"] = traffic / avg_launch_s / 1e9
        roof["dram_frac"] = roof["dram_gbs"] / HBM_PEAK_GBS
        roof["traffic_over_algorithmic"] = traffic / per_launch_bytes
        roof["traffic_source"] = tr["profile"] + " (kernel sources " + tr["sources"] + ")"
    else:
        roof["traffic_source"] = ("no counters for this tiling and these kernel sources (%s)" % digest)
    if lane_ops and avg_launch_s:
        roof["valu_lane_ops_per_launch"] = lane_ops
        roof["valu_frac"] = lane_ops / avg_launch_s / VALU_PEAK_LANE_OPS
        roof["valu_peak_lane_ops_per_s"] = VALU_PEAK_LANE_OPS
        roof["valu_per_owned_site_update"] = isa["valu_per_owned_site_update"]
        roof["valu_source"] = "march-loop instruction counts of this build (isa_counts.json)"
    out = {"value": updates / wall, "wall_s": wall, "ms_per_run": wall / runs * 1e3,
           "event_ms_per_run": ev_ms / runs, "sites": sites, "steps_per_run": S,
           "records_per_run": len(recs), "tiling": list(til), "steps_per_pass": T,
           "roofline": roof,
           "result": {"mu": mu, "nu": nu, "final_links": recs[-1]["links"],
                      "final_area_density": recs[-1]["area_density"]}}
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


ADJOINT = [
    dict(name="2D 2048^2", shape=(2048, 2048), deta=0.25),
    dict(name="3D 256^3", shape=(256, 256, 256), deta=0.2),
]
ADJ_STEPS, ADJ_K = 1024, 64


def adjoint_leg(prs, torch, reps=3):
    """Checkpointed adjoint of 1024 steps (m = 1, W0 = 10), loss = sum V/V0
    of the final field: forward-with-checkpoints and reverse sweep timed
    separately with stream events."""
    out = {"workload": "adjoint, 1024 steps from seed 7, m=1, W0=10, checkpoints every 64, "
                       "loss = sum V(phi)/V0; grad w.r.t. phi0 and W0",
           "single_step_bytes_per_site_update": {"forward": 16, "backward": 36}}
    stream = torch.cuda.current_stream()
    for cfg in ADJOINT:
        p = prs.make_params(cfg["shape"], deta=cfg["deta"], m=1.0, W0=10.0)
        sites = prs.sites(p)
        nb = prs.prs_adjoint_workspace_bytes(p, ADJ_STEPS, ADJ_K)
        work = torch.empty(nb, dtype=torch.uint8, device="cuda")
        gphi = torch.empty(sites, dtype=torch.float32, device="cuda")
        sim = prs.Sim(p, seed=7)
        prs.prs_autotune(sim.ctx, None, 0)
        prs.prs_autotune(sim.ctx, None, prs.PRS_TUNE_ADJOINT)
        phi0 = sim.phi_a.clone()
        fwd, bwd = [], []
        for r in range(reps + 1):
            sim.set_state(phi0, torch.zeros_like(phi0), 0)
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record(stream)
            loss = prs.prs_adjoint_forward(sim.ctx, ADJ_STEPS, ADJ_K, work.data_ptr(), nb)
            e1.record(stream)
            gw = prs.prs_adjoint_backward(sim.ctx, work.data_ptr(), nb, gphi.data_ptr(), None)
            e2.record(stream)
            torch.cuda.synchronize()
            if r > 0:
                fwd.append(e0.elapsed_time(e1))
                bwd.append(e1.elapsed_time(e2))
        tf, tb = min(fwd), min(bwd)
        su = float(sites) * ADJ_STEPS
        out[cfg["name"]] = {
            "forward_ms": tf, "backward_ms": tb, "backward_over_forward": tb / tf,
            "total_over_forward": (tf + tb) / tf,
            "forward_site_updates_per_s": su / (tf / 1e3),
            "adjoint_site_updates_per_s": su / (tb / 1e3),
            "forward_effective_single_step_frac": su * 16 / (tf / 1e3) / (HBM_PEAK_GBS * 1e9),
            "backward_effective_single_step_frac": su * 36 / (tb / 1e3) / (HBM_PEAK_GBS * 1e9),
            "loss": loss, "grad_W0": gw, "tiling": list(sim.tiling()),
            "steps_per_pass": sim.time_blocking(),
            "adjoint_tiling": list(prs.prs_get_adjoint_tiling(sim.ctx)),
            "adjoint_steps_per_pass": prs.prs_get_adjoint_time_blocking(sim.ctx),
            "recompute_tiling_and_steps": list(prs.prs_get_recompute_tiling(sim.ctx)),
        }
        log("adjoint", cfg["name"], "fwd %.2f ms bwd %.2f ms" % (tf, tb))
        sim.close()
        del work, gphi, sim, phi0
        torch.cuda.empty_cache()
    return out


def batch_leg(prs, torch, reps=2):
    """The seeded ensemble: 48 2D realisations (512^2/1024^2/2048^2) and 16 3D
    (128^3/256^3), m in {0.5,1,2}, W0 in {5,10}, each to eta = N/2.  Each
    realisation runs its tuned single-run pass sequence (tiling and steps per
    pass) on one of four concurrent streams.  The one-launch persistent mode
    (the ensemble kernel replayed from a hipGraph, with the tilings and steps
    per pass the tuner picks among those it runs) is timed beside it.  In
    both modes the marching-tile lengths are then refined by timing the
    whole ensemble (prs_batch_autotune)."""
    from paper_1710_10420_amd.inputs import ensemble_draw
    items = ensemble_draw(2017)
    specs = [dict(shape=(it["N"],) * it["ndim"], deta=it["deta"], m=it["m"], W0=it["W0"],
                  nsteps=it["steps"], diag_every=64 if it["ndim"] == 2 else 50, seed=it["seed"])
             for it in items]
    b = prs.Batch(specs)
    su = float(sum(int(np.prod(sp["shape"])) * sp["nsteps"] for sp in specs))

    def timed(mode, flags):
        tuned = {}
        for r, sp in enumerate(specs):            # one tuning per distinct lattice
            key = sp["shape"]
            if key not in tuned:
                p = prs.make_params(sp["shape"], deta=sp["deta"], m=sp["m"], W0=sp["W0"])
                t = prs.Sim(p, seed=1)
                prs.prs_autotune(t.ctx, None, flags)
                tuned[key] = (t.tiling(), t.time_blocking())
                t.close()
            til, T = tuned[key]
            b.set_time_blocking(r, 1)
            b.set_tiling(r, *til)
            b.set_time_blocking(r, T)
        b.set_mode(mode)
        b.autotune()                              # marching tiles refined on the whole ensemble
        kept = {}
        for r, sp in enumerate(specs):
            kept.setdefault(sp["shape"], b.tiling(r))
        b.run()                                   # builds and instantiates the graph
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            recs = b.run()
            times.append(time.perf_counter() - t0)
        return min(times), recs, kept

    t_p, _, tuned_p = timed(prs.PRS_BATCH_PERSISTENT_GRAPH, prs.PRS_TUNE_BATCH)
    t, recs, tuned = timed(prs.PRS_BATCH_STREAMS, 0)
    out = {"workload": "ensemble of 64 realisations (master seed 2017): 48 2D from "
                       "{512^2,1024^2,2048^2}, 16 3D from {128^3,256^3}, m in {0.5,1,2}, "
                       "W0 in {5,10}, each to eta = N/2, diagnostics every 64 (2D) / 50 (3D)",
           "realisations": len(specs), "site_updates": su, "ms_per_run": t * 1e3,
           "site_updates_per_s": su / t,
           "effective_single_step_frac": su * 16 / t / (HBM_PEAK_GBS * 1e9),
           "records": sum(len(r) for r in recs), "mode": "4 concurrent streams",
           "tilings": {"x".join(map(str, k)): {"tiling": list(v[0]), "steps_per_pass": v[1]}
                       for k, v in tuned.items()},
           "persistent_kernel": {"ms_per_run": t_p * 1e3, "site_updates_per_s": su / t_p,
                                 "over_streams": t_p / t,
                                 "mode": "one persistent launch replayed from a hipGraph",
                                 "tilings": {"x".join(map(str, k)): {"tiling": list(v[0]), "steps_per_pass": v[1]}
                                             for k, v in tuned_p.items()}}}
    log("batch %.1f ms (persistent kernel %.1f ms)" % (t * 1e3, t_p * 1e3))
    b.close()
    return out


def table1_leg(prs):
    """Table I of the paper in kind: five seeds of 2048^2 and 128^3 in single
    and double precision, exponents fitted for ln(eta) > 2.58 (mean and
    one-sigma error over the five runs)."""
    from paper_1710_10420_amd import validation
    t0 = time.perf_counter()
    table = validation.scaling_table(prs)
    out = {"workload": "5 seeds x {2048^2, 128^3} x {single, double}, m=1, W0=10, to eta = N/2, "
                       "fit for ln(eta) > 2.58",
           "seconds": time.perf_counter() - t0}
    for name, row in table.items():
        out[name] = {label: {"mu": r["mu"], "nu": r["nu"]} for label, r in row.items()}
    log("table1 %.1f s" % out["seconds"])
    return out


SLABS = {
    "3d": dict(shape=(1024, 1024, 128), deta=0.2, m=1.0, W0=10.0, T=3, tiling=(2, 64, 2), passes=20,
               name="1024x1024x128 z-slab (1/8 of 1024^3) with 3 halo planes per face, three-step passes, "
                    "tiling (2, 64, 2), 20 passes"),
    "2d": dict(shape=(8192, 1024), deta=0.25, m=2.0, W0=10.0, T=8, tiling=(2, 64, 1), passes=40,
               name="8192x1024 y-slab (1/8 of 8192^2) with 8 halo rows per face, eight-step passes, "
                    "tiling (2, 64, 1), 40 passes"),
}
XGMI_LINK_GBS = 153.0          # one MI355X xGMI link, per direction (published)


def slab_leg(prs, torch, cfg, reps=2):
    """The per-device kernel of a lattice sharded along its last axis over
    eight devices (1024^3 along z, 8192^2 along y): a slab stored with T halo
    planes or rows below and above, advanced by T-step slab passes (the halos
    are those a neighbour would send; here they stay as initialised).
    Reports the slab's site-update rate and what one halo exchange per pass
    would cost on one xGMI link."""
    shape = cfg["shape"]
    T = cfg["T"]
    p = prs.make_params(shape, deta=cfg["deta"], m=cfg["m"], W0=cfg["W0"])
    face = 1
    for n in shape[:-1]:
        face *= n
    n_ext = face * (shape[-1] + 2 * T)
    f = [torch.empty(n_ext, dtype=torch.float32, device="cuda") for _ in range(4)]
    stream = torch.cuda.current_stream()
    s = prs._stream_handle(stream)
    prs.prs_fill_uniform(f[0].data_ptr(), n_ext, 1, s)
    f[2].zero_()
    f[1].copy_(f[0])
    f[3].zero_()
    times = []
    for r in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        a, b, pa, pb = f
        for k in range(cfg["passes"]):
            prs.prs_slab_pass(p, k * T, T, cfg["tiling"], a.data_ptr(), b.data_ptr(), pa.data_ptr(),
                              pb.data_ptr(), s)
            a, b, pa, pb = b, a, pb, pa
        e1.record(stream)
        torch.cuda.synchronize()
        if r > 0:
            times.append(e0.elapsed_time(e1))
    ms = min(times)
    su = float(face * shape[-1]) * T * cfg["passes"]
    halo_bytes = 2 * 2 * T * face * 4          # phi and phi_dot, T planes or rows, both faces
    out = {"workload": cfg["name"],
           "ms_per_pass": ms / cfg["passes"], "site_updates_per_s": su / (ms / 1e3),
           "halo_bytes_per_pass": halo_bytes,
           "halo_exchange_ms_one_link": halo_bytes / (XGMI_LINK_GBS * 1e9) * 1e3}
    log("slab %dD %.3f ms per pass" % (len(shape), ms / cfg["passes"]))
    del f
    torch.cuda.empty_cache()
    return out


F64_STEPS = 2048


def f64_leg(prs, torch, w, reps=2):
    """The same 8192^2 lattice in float64 (the paper runs both precisions):
    the first 2048 steps of the run with its fused records, autotuned tiling
    and steps per pass; algorithmic bytes 32 per site-update."""
    p = prs.make_params(w["shape"], deta=w["deta"], m=w["m"], W0=w["W0"], diag_every=w["diag_every"],
                        precision=prs.PRS_F64)
    sim = prs.Sim(p, seed=w["seed"])
    prs.prs_autotune(sim.ctx, None, 0)
    phi0 = sim.state()[0].clone()
    stream = torch.cuda.current_stream()
    times = []
    for r in range(reps + 1):
        sim.set_state(phi0, torch.zeros_like(phi0), 0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step_n(F64_STEPS)
        e1.record(stream)
        torch.cuda.synchronize()
        if r > 0:
            times.append(e0.elapsed_time(e1) / 1e3)
    t = min(times)
    su = float(prs.sites(p)) * F64_STEPS
    out = {"workload": "8192^2 in float64, first %d steps of the run (records every 64)" % F64_STEPS,
           "site_updates_per_s": su / t, "ms": t * 1e3, "bytes_per_site_update": 32,
           "effective_single_step_frac": su * 32 / t / (HBM_PEAK_GBS * 1e9),
           "tiling": list(sim.tiling()), "steps_per_pass": sim.time_blocking()}
    log("f64 %.1f ms for %d steps" % (t * 1e3, F64_STEPS))
    sim.close()
    del phi0
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip every leg after the headline and the copy")
    ap.add_argument("--tiling", default=None, help="vec,rows,ty for the main run (default: autotuned)")
    ap.add_argument("--steps-per-pass", type=int, default=2, help="with --tiling")
    ap.add_argument("--leg", choices=("c2", "c3"), default="c2",
                    help="c3: only the 1024^3 forward leg (with --tiling, --steps, --warmup) and the copy "
                         "kernel, as one JSON line, for profiling that leg's pass kernel")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the PRS path is built and timed on a single "
              "MI355X (no multi-GPU path); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1710_10420_amd import prs

    w = WORKLOAD
    torch.cuda.set_device(0)
    tiling = [int(v) for v in args.tiling.split(",")] if args.tiling else None
    if args.leg == "c3":
        c3 = forward_leg(prs, torch, WORKLOAD_3D, args.steps, args.warmup, tiling, args.steps_per_pass)
        c3["copy_ceiling"] = copy_ceiling(prs, torch)
        c3["workload"] = WORKLOAD_3D["name"]
        print(json.dumps(c3), flush=True)
        return
    c2 = forward_leg(prs, torch, w, args.steps, args.warmup, tiling, args.steps_per_pass)
    roof = c2["roofline"]
    copy = copy_ceiling(prs, torch)
    if roof["achieved"]:
        roof["copy_ceiling_gbs"] = copy["gbs"]
        roof["frac_of_copy_ceiling"] = roof["achieved"] / copy["gbs"]
    out = {
        "metric": "site-updates/s (PRS forward step, fused wall diagnostics)",
        "value": c2["value"],
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": c2["ms_per_run"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: seeded uniform(-1,1) initial field (SplitMix64), phi_dot = 0",
        "config": {"workload": w["name"], "sites": c2["sites"], "steps_per_run": c2["steps_per_run"],
                   "records_per_run": c2["records_per_run"], "tiling": c2["tiling"],
                   "steps_per_pass": c2["steps_per_pass"]},
        "roofline": roof,
        "result": c2["result"],
        "copy_ceiling": copy,
    }
    if not args.no_extra:
        c3 = forward_leg(prs, torch, WORKLOAD_3D, 1, 1)
        if c3["roofline"]["achieved"]:
            c3["roofline"]["frac_of_copy_ceiling"] = c3["roofline"]["achieved"] / copy["gbs"]
        c3["workload"] = WORKLOAD_3D["name"]
        out["c3"] = c3
        out["adjoint"] = adjoint_leg(prs, torch)
        out["batch"] = batch_leg(prs, torch)
        out["f64"] = f64_leg(prs, torch, w)
        out["table1"] = table1_leg(prs)
        out["slab"] = slab_leg(prs, torch, SLABS["3d"])
        out["slab_2d"] = slab_leg(prs, torch, SLABS["2d"])
    if not args.no_cpu:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
