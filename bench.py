#!/usr/bin/env python3
"""Benchmark of the grid-Poisson SDF reconstruction on one MI355X.

Workload (one "step" = the whole forward hot path on one synthetic cloud):
flapping ellipsoid (semi-axes 0.30, 0.12, 0.08) under a travelling-wave shear,
300,000 oriented points per time step, 256^3 grid on the unit cube, Poisson
solve warm-started from the previous step to FP64 relative residual 1e-6,
surface + signed distance on every grid node, then SDF and normals sampled at
65,536 query points.  Inputs for every step are resident in HBM before the
timed region.  Metric: reconstructions per second.  Steps run through the
pipelined entry point (a step's distance walk and sampling overlap the next
step's splat and solve); the same loop without pipelining is reported too.

Also reported on the same JSON line:
  roofline      the dominant kernel's algorithmic bytes (or nodes) per launch
                over its average launch duration, timed with HIP events on its
                stream during the timed region;
  cpu_baseline  the FP64 oracle on a bounded sample of one step (all steps but
                the distance run in full; the distance on a node sample,
                scaled to the grid);
  oracle_error  GPU vs oracle on the last timed step;
  adjoint       the reverse pass (adjoint solve included) at the same size;
  serving       a replayed Poisson-arrival request stream, continuous batching
                vs one request at a time;
  secondary     the 128^3 torus (1e6 queries) and the 16-coefficient gradient
                (forward + backward against 32 finite-difference forwards),
                each with its error against the oracle (with cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VALU_TFLOPS = 157.3       # MI355X FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (packed) x 2 (FMA) x 2.4 GHz
FP32_UNPACKED_TFLOPS = 78.6    # the same without packed FP32 (the library is built with packed FP32 off)

# FP32 operations of one test of the distance walk, counted from its formulas
# (every FP32 VALU operation, min / max / abs included, as they issue at the
# same rate; comparisons, selects and the stack bookkeeping not counted).  A
# lane's kTZ nodes share x and y, so part of each test is done once per lane
# and part once per node: (shared, per node).  Node-triangle test (tri_d2):
# shared p - a in x and y and the x, y parts of ab.ap and ac.ap (2 + 3 + 3);
# per node the z parts (1 + 2 + 2), the offsets d3..d6 (4), the three region
# determinants (3 x 3), the barycentric weights (2), the closest-point offset
# ap - v ab - w ac (12) and its squared length (5).  Axis-aligned box: shared
# the clamped x and y distances and their squares (11), per node the z
# distance and the sum (7).  Oriented box: shared the offsets and the three
# in-plane projections (17), per node three clamped distances and the sum (18).
WALK_OPS = {"tri": (8.0, 37.0), "aabb": (11.0, 7.0), "obb": (17.0, 18.0)}


def walk_flops(counts, ktz):
    """Algorithmic FP32 operations of the walk from its counted tests."""
    per_node = {k: sh / ktz + pn for k, (sh, pn) in WALK_OPS.items()}
    return (counts["tri_tests"] * per_node["tri"] + counts["aabb_tests"] * per_node["aabb"]
            + counts["obb_tests"] * per_node["obb"])


def angle_between(a, b):
    """Angle between rows of two normal fields: normalised in float64 and taken
    as atan2(|a x b|, a . b) (arccos of a float32 unit vector's dot product
    reads ~4e-4 rad for a norm off by 1e-7)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    a = a / np.maximum(np.linalg.norm(a, axis=1, keepdims=True), 1e-300)
    b = b / np.maximum(np.linalg.norm(b, axis=1, keepdims=True), 1e-300)
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), np.sum(a * b, axis=1))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_run(args):
    import torch

    from paper_2609_20964_amd import _lib, synth
    from paper_2609_20964_amd.recon import Recon

    n, npts, nq = args.n, args.points, args.queries
    fl = synth.Flapping(n_points=npts)
    total = args.warmup + args.steps + args.adjoint_steps + 1
    log(f"generating {total} steps of {npts} points")
    clouds = []
    for t in range(total):
        x, nrm = fl.step(t)
        clouds.append((torch.from_numpy(x).cuda(), torch.from_numpy(nrm).cuda()))
        if t % 100 == 99:
            log(f"  {t + 1} clouds")
    q = torch.from_numpy(synth.uniform_queries(nq, 4001)).cuda()
    r = Recon(n, npts)
    kinds = list(_lib.PROF_KINDS)
    # the cold step: the first step on a new handle (cold solve, cold walk), outputs complete
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    r.step(*clouds[0], q, rel_tol=args.tol, warm_start=False)
    r.wait()
    torch.cuda.synchronize()
    cold_ms = (time.perf_counter() - c0) * 1e3
    log(f"cold step 0: {cold_ms:.2f} ms")
    # warm-up, then the last three warm-up clouds again as plain steps (no
    # overlap, so each kind's event-timed duration is its own) with every
    # kernel kind profiled, to find the dominant one
    for t in range(args.warmup):
        st, _, _ = r.step(*clouds[t], q, rel_tol=args.tol, warm_start=t > 0)
        log(f"warmup {t}: iters {st['iters']} rel_res {st['rel_res']:.2e} ms {[round(v, 2) for v in st['ms'][:5]]}")
    r.wait()
    torch.cuda.synchronize()
    _lib.profile_reset()
    _lib.profile_enable(kinds)
    prof_steps = list(range(max(args.warmup - 3, 0), args.warmup)) or [0]
    n_prof = len(prof_steps)
    for t in prof_steps:
        r.forward(*clouds[t], rel_tol=args.tol, warm_start=args.warmup > 0)
        r.sample(q)
    torch.cuda.synchronize()
    per_kind = {k: _lib.profile_read(k) for k in kinds}
    walk_plain = _lib.profile_walk_counts()
    dominant = max(per_kind, key=lambda k: per_kind[k]["ms"])
    log("plain-step kernel time by kind (ms):", {k: round(v["ms"], 3) for k, v in per_kind.items()})
    _lib.profile_enable([])
    _lib.profile_reset()
    _lib.profile_enable([dominant])

    # timed: pipelined steps (each step's distance walk and sampling overlap the
    # next step's splat and solve), all outputs complete at the final synchronise
    stats = []
    stamps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        t = args.warmup + k
        st, phi, nq_out = r.step(*clouds[t], q, rel_tol=args.tol, warm_start=True)
        stats.append(st)
        stamps.append(time.perf_counter())   # host time at each return (the pipeline's pace)
    r.wait()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _lib.profile_enable([])
    prof = _lib.profile_read(dominant)
    walk_timed = _lib.profile_walk_counts()
    elapsed = t1 - t0

    # the same loop without pipelining (forward, then sample), for reference
    plain_steps = min(args.steps, 10)
    plain_stats = []
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    for k in range(plain_steps):
        t = args.warmup + args.steps - plain_steps + k
        plain_stats.append(r.forward(*clouds[t], rel_tol=args.tol, warm_start=True))
        r.sample(q)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - p0) / plain_steps * 1e3

    # two more (untimed) steps with every kind profiled: the solver's kernels as a group
    _lib.profile_reset()
    _lib.profile_enable(kinds)
    solve_ms = []
    for k in range(2):
        t = args.warmup + args.steps - 2 + k
        st2 = r.forward(*clouds[t], rel_tol=args.tol, warm_start=True)
        solve_ms.append(st2["ms"][1])
    torch.cuda.synchronize()
    _lib.profile_enable([])
    solver_kinds = {k: _lib.profile_read(k) for k in SOLVER_KINDS}
    _lib.profile_reset()
    last_t = args.warmup + args.steps - 1
    fields = r.fields()
    gpu_last = {"chi": fields["chi"].cpu().numpy(), "phi": fields["phi"].cpu().numpy(),
                "iso_c": st2["iso_c"], "phi_q": phi.cpu().numpy(), "t": last_t}
    # every 25th timed step again as a plain forward (warm-started from the step
    # before it), its field and SDF kept for the oracle comparison
    samples = []
    for k in range(24, args.steps, 25):
        t = args.warmup + k
        r.forward(*clouds[t - 1], rel_tol=args.tol, warm_start=True)
        stk = r.forward(*clouds[t], rel_tol=args.tol, warm_start=True)
        fk = r.fields()
        samples.append({"t": t, "chi": fk["chi"].cpu().numpy(), "phi": fk["phi"].cpu().numpy(),
                        "iso_c": stk["iso_c"], "cloud": tuple(c.cpu().numpy() for c in clouds[t])})

    # reverse pass at the same size: L = mean phi(q)^2 (one untimed warm-up call first)
    adj_ms = []
    for k in range(args.adjoint_steps + 1 if args.adjoint_steps else 0):
        t = args.warmup + args.steps + k
        r.forward(*clouds[t], rel_tol=args.tol, warm_start=True)
        phi, _ = r.sample(q, normals=False)
        torch.cuda.synchronize()
        a0 = time.perf_counter()
        r.backward(q, (2.0 / nq) * phi, rel_tol=args.tol)
        torch.cuda.synchronize()
        if k > 0:
            adj_ms.append((time.perf_counter() - a0) * 1e3)
    exact = exact_run(args, r, clouds, q, kinds) if args.exact_steps else None
    r.close()
    return {"elapsed": elapsed, "stats": stats, "prof": prof, "dominant": dominant, "per_kind": per_kind,
            "exact": exact, "cold_ms": cold_ms, "samples": samples, "stamps": np.asarray(stamps) - t0,
            "gpu_last": gpu_last, "clouds_last": tuple(c.cpu().numpy() for c in clouds[last_t]),
            "q": q.cpu().numpy(), "adj_ms": adj_ms, "solver_kinds": solver_kinds, "solve_ms": solve_ms,
            "plain_ms": plain_ms, "plain_steps": plain_steps, "plain_stats": plain_stats, "n_prof": n_prof,
            "walk_timed": walk_timed, "walk_plain": walk_plain, "walk_ktz": 4 if n ** 3 >= 1 << 23 else 1,
            "tol": args.tol}


def exact_run(args, r, clouds, q, kinds):
    """The Galerkin system with exact quadrature (27-point stiffness,
    consistent right-hand side) on the same handle and clouds: plain steps
    (forward, then sampling), timed, then two more with the solver's kernels
    profiled.  The first step switches the system and is not timed."""
    import torch

    from paper_2609_20964_amd import _lib

    ns = args.exact_steps
    base = max(args.warmup + args.steps - ns - 3, 0)
    cl = lambda t: clouds[t % len(clouds)]
    r.forward(*cl(base), rel_tol=args.tol, warm_start=True, quadrature="exact")
    r.sample(q)
    torch.cuda.synchronize()
    st = []
    t0 = time.perf_counter()
    for k in range(ns):
        st.append(r.forward(*cl(base + 1 + k), rel_tol=args.tol, warm_start=True, quadrature="exact"))
        r.sample(q)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / ns * 1e3
    _lib.profile_reset()
    _lib.profile_enable(kinds)
    solve_ms = []
    for k in range(2):
        solve_ms.append(r.forward(*cl(base + 1 + k), rel_tol=args.tol, warm_start=True,
                                  quadrature="exact")["ms"][1])
    torch.cuda.synchronize()
    _lib.profile_enable([])
    out = {"ms_per_step_plain": ms, "steps": ns, "stats": st, "solve_ms": solve_ms,
           "solver_kinds": {k: _lib.profile_read(k) for k in SOLVER_KINDS}, "splat": _lib.profile_read("splat")}
    _lib.profile_reset()
    return out


def exact_summary(res, copy_gbs):
    e = res["exact"]
    st = e["stats"]
    return {"ms_per_step_plain": e["ms_per_step_plain"], "recons_per_s_plain": 1e3 / e["ms_per_step_plain"],
            "vertex_ms_per_step_plain": res["plain_ms"], "steps": e["steps"],
            "iters_mean": float(np.mean([s["iters"] for s in st])),
            "rel_res_max": float(max(s["rel_res"] for s in st)),
            "phase_ms_plain": {k: float(np.mean([s["ms"][i] for s in st]))
                               for i, k in enumerate(["splat", "solve", "iso", "surface", "sdf"])},
            "splat_kernel_ms": e["splat"]["ms"] / 2,
            "solver_roofline": solver_hbm({"solver_kinds": e["solver_kinds"], "solve_ms": e["solve_ms"]}, copy_gbs,
                                          counters=False),
            "kernels": "k_splat_chunks<kSplatExact>, k_stencil27<OpPMatvec> (sweep), k_stencil27<OpResid64> "
                       "(resid64), k_stencil27<OpJacobi27a/b> + k_vc_pre (smooth)",
            "workload": "the headline clouds and grid, exact-quadrature system, plain steps, rel res "
                        f"{res['tol']:g}"}


# algorithmic cost model of each timed kind: units are bytes, except the distance walk (nodes)
KIND_BOUND = {"splat": "hbm", "sweep": "hbm", "smooth": "hbm", "resid64": "hbm", "transfer": "hbm",
              "cgupdate": "hbm", "mc": "hbm", "sample": "hbm", "sdf": "alu"}
# kernel names as rocprofv3 lists them
KIND_KERNEL = {"sweep": "k_stencil4<OpPMatvec>", "smooth": "k_vc_pre", "resid64": "k_stencil4<OpResid64>",
               "sdf": "k_sdf", "splat": "k_splat_chunks", "mc": "k_mc_count/k_mc_emit",
               "transfer": "k_vc_post", "cgupdate": "k_cg_update", "sample": "k_sample"}


SOLVER_KINDS = ("sweep", "smooth", "resid64", "transfer", "cgupdate")


# the kernel of each solver kind whose counter row prices the kind's bytes
SOLVER_PMC_ROW = {"sweep": "k_stencil4<OpPMatvec<false> >", "smooth": "k_vc_pre", "transfer": "k_vc_post<true>",
                  "resid64": "k_stencil4<OpResid64<float> >", "cgupdate": "k_cg_update<false>"}


def solver_counter_ratios(path=None):
    """Counter bytes over algorithmic bytes per solver kind, from the committed
    rocprofv3 summary of the finest-level kernels (calibrated FETCH_SIZE +
    WRITE_SIZE), if it was taken on the current solver source; else {}."""
    path = path or os.path.join(ROOT, "profiles", "pmc_solver_flapping256.txt")
    if not os.path.exists(path):
        return {}
    rows, sha = {}, None
    for line in open(path):
        if line.startswith("# source_sha "):
            sha = line.split()[2]
        elif line.startswith("  ") and len(line) > 46:
            nums = line[46:].split("#")[0].split()
            if len(nums) == 5:
                rows[line[2:46].strip()] = float(nums[2]) / float(nums[3])
    if sha != source_sha("paper_2609_20964_amd/csrc/solver.hip"):
        return {}
    return {k: rows[name] for k, name in SOLVER_PMC_ROW.items() if name in rows}


def solver_hbm(res, copy_gbs=None, counters=True):
    """HBM roofline of the Poisson solve taken as a whole: algorithmic bytes of
    its bandwidth-bound kernels over (a) their own event-timed duration and
    (b) the whole solve phase (reductions, coarse solve and host waits
    included); both also against a measured device copy, and the kernels'
    bytes as the counters measured them (each kind priced by its finest-level
    kernel's counter/algorithmic ratio) over their duration."""
    kinds = res["solver_kinds"]
    units = sum(v["units"] for v in kinds.values())
    ms = sum(v["ms"] for v in kinds.values())
    if ms <= 0:
        return None
    phase_ms = sum(res["solve_ms"])
    per = {k: {"GB_s": v["units"] / (v["ms"] * 1e6) if v["ms"] > 0 else None, "launches": v["launches"],
               "ms": v["ms"] / len(res["solve_ms"])} for k, v in kinds.items()}
    out = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "kernels_GB_s": units / (ms * 1e6), "kernels_frac": units / (ms * 1e6) / HBM_PEAK_GBS,
           "phase_GB_s": units / (phase_ms * 1e6), "phase_frac": units / (phase_ms * 1e6) / HBM_PEAK_GBS,
           "bytes_per_solve": units / len(res["solve_ms"]), "phase_ms": phase_ms / len(res["solve_ms"]),
           "per_kind": per}
    if copy_gbs:
        out.update({"copy_GB_s": copy_gbs, "kernels_frac_of_copy": out["kernels_GB_s"] / copy_gbs,
                    "phase_frac_of_copy": out["phase_GB_s"] / copy_gbs})
    ratios = solver_counter_ratios() if counters else {}   # the rows are of the 7-point system's kernels
    if ratios and all(k in ratios for k in kinds):
        counted = sum(v["units"] * ratios[k] for k, v in kinds.items())
        out.update({"counter_GB_s": counted / (ms * 1e6), "counter_frac": counted / (ms * 1e6) / HBM_PEAK_GBS})
    return out


def roofline(res):
    p = res["prof"]
    kind = res["dominant"]
    if p["launches"] == 0:
        return None
    avg_s = p["ms"] / p["launches"] / 1e3
    per_launch = p["units"] / p["launches"]
    pmc = load_pmc(kind)
    traffic = pmc.get("traffic_bytes_per_launch")
    if KIND_BOUND[kind] == "hbm":
        achieved = per_launch / avg_s / 1e9
        out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": achieved / HBM_PEAK_GBS, "traffic": traffic}
    else:
        # distance walk: FP32 operations of the tests it counted on the device
        # during these launches, over the event-timed launch duration
        counts, ktz = res["walk_timed"], res["walk_ktz"]
        flops = walk_flops(counts, ktz) / p["launches"]
        achieved = flops / avg_s / 1e12
        nodes = max(counts["nodes"], 1)
        out = {"bound": "alu", "achieved": achieved, "peak": FP32_VALU_TFLOPS, "unit": "TFLOP/s",
               "frac": achieved / FP32_VALU_TFLOPS, "traffic": traffic,
               "peak_unpacked": FP32_UNPACKED_TFLOPS, "frac_unpacked": achieved / FP32_UNPACKED_TFLOPS,
               "flops_per_launch": flops, "flops_per_node": flops / per_launch, "nodes_per_s": per_launch / avg_s,
               "tests_per_node": {"triangle": counts["tri_tests"] / nodes, "aabb": counts["aabb_tests"] / nodes,
                                  "obb": counts["obb_tests"] / nodes},
               "valu_lane_util": pmc.get("valu_lane_util")}
    out.update({"kernel": KIND_KERNEL[kind], "launches": p["launches"], "avg_launch_us": avg_s * 1e6,
                "units_per_launch": per_launch})
    # the same kernel in the plain (not overlapped) profiled steps: in the timed
    # pipelined steps it shares the device with the next step's solve
    a = res["per_kind"].get(kind)
    if a and a["launches"] > 0 and a["ms"] > 0:
        avg_a = a["ms"] / a["launches"] / 1e3
        alone = {"launches": a["launches"], "avg_launch_us": avg_a * 1e6}
        if out["bound"] == "alu":
            fl = walk_flops(res["walk_plain"], res["walk_ktz"]) / a["launches"]
            alone.update({"achieved": fl / avg_a / 1e12, "frac": fl / avg_a / 1e12 / FP32_VALU_TFLOPS,
                          "frac_unpacked": fl / avg_a / 1e12 / FP32_UNPACKED_TFLOPS,
                          "traffic": pmc.get("traffic_bytes_per_launch_alone")})
        else:
            alone["frac"] = out["frac"] * avg_s / avg_a
        out["alone"] = alone
    return out


def source_sha(rel):
    """First 16 hex digits of the SHA-256 of a source file of the library."""
    import hashlib
    return hashlib.sha256(open(os.path.join(ROOT, rel), "rb").read()).hexdigest()[:16]


# the file each profiled kernel kind is compiled from
KIND_SOURCE = {"sdf": "paper_2609_20964_amd/csrc/surface.hip", "mc": "paper_2609_20964_amd/csrc/surface.hip",
               "sample": "paper_2609_20964_amd/csrc/surface.hip", "splat": "paper_2609_20964_amd/csrc/splat.hip"}


def load_pmc(kind):
    """Per-launch figures from the committed rocprofv3 counter summary for this
    kernel and workload (`key value` lines), if one exists and was taken on the
    current source of the kernel (its `source_sha` line); counters of an older
    build are not reported."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kind}_flapping256.txt")
    vals = {}
    if os.path.exists(path):
        for line in open(path):
            parts = line.split()
            if len(parts) == 2 and parts[0] in ("traffic_bytes_per_launch", "traffic_bytes_per_launch_alone",
                                                 "valu_lane_util", "source_sha"):
                vals[parts[0]] = parts[1] if parts[0] == "source_sha" else float(parts[1])
    src = KIND_SOURCE.get(kind, "paper_2609_20964_amd/csrc/solver.hip")
    if vals.get("source_sha") != source_sha(src):
        return {}
    return vals


def sample_errors(res, n, sample_nodes):
    """GPU against the oracle on every 25th timed step (re-run as plain
    forwards): field, iso-value and SDF on `sample_nodes` random nodes."""
    from oracle import discretize as D
    from oracle import pipeline as P

    from concurrent.futures import ThreadPoolExecutor

    grid = D.Grid.unit(n)
    rng = np.random.default_rng(4003)
    picks = [rng.choice(n ** 3, sample_nodes, replace=False) for _ in res["samples"]]

    def one(k):
        s, nodes = res["samples"][k], picks[k]
        x, nrm = s["cloud"]
        ref = P.Recon(grid, x, nrm)
        e = {"step": int(s["t"]),
             "chi_rel_l2": float(np.linalg.norm(s["chi"] - ref.chi) / np.linalg.norm(ref.chi)),
             "iso_c_rel": float(abs(s["iso_c"] - ref.c) / np.abs(ref.chi).max()),
             "phi_max_abs_over_h": float(np.abs(s["phi"].reshape(-1)[nodes].astype(np.float64) -
                                                ref.phi_nodes(nodes)).max() * n),
             "nodes_compared": int(sample_nodes)}
        log(f"oracle at step {e['step']}: field {e['chi_rel_l2']:.2e}, SDF {e['phi_max_abs_over_h']:.2e} h")
        return e

    # the oracle's heavy parts (numpy, scipy.fft, its C distance) release the GIL: four samples at a time
    with ThreadPoolExecutor(max_workers=4) as ex:
        return list(ex.map(one, range(len(res["samples"]))))


def oracle_timing(cmp, reps=3):
    """The oracle on the 32^3 sphere and the 128^3 torus at one thread and at
    all cores (BLAS / OpenMP pools and scipy.fft workers), median of `reps`:
    forward in full, distance on 1,500 random nodes scaled to the grid."""
    from threadpoolctl import threadpool_limits
    import scipy.fft

    from oracle import discretize as D
    from oracle import pipeline as P

    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"cores_all": cores, "cpu_model": cpu_model()}
    for name, n, key in (("sphere_32", 32, "sphere"), ("torus_128", 128, "torus")):
        c = cmp[key]
        rng = np.random.default_rng(4004)
        nodes = rng.choice(n ** 3, 1500, replace=False)
        row = {}
        for label, th in (("one_thread", 1), ("all_cores", cores)):
            times = []
            log(f"oracle timing {name}, {th} thread(s)")
            for _ in range(reps):
                with threadpool_limits(th), scipy.fft.set_workers(th):
                    t0 = time.perf_counter()
                    ref = P.Recon(D.Grid.unit(n), c["x"], c["nrm"])
                    t1 = time.perf_counter()
                    ref.phi_nodes(nodes)
                    t2 = time.perf_counter()
                times.append((t1 - t0) + (t2 - t1) / len(nodes) * n ** 3)
            row[label] = {"recons_per_s": 1.0 / float(np.median(times)), "seconds_median": float(np.median(times)),
                          "threads": th}
        out[name] = row
    out["sample"] = ("oracle forward in full; brute-force distance on 1,500 random nodes scaled to the grid; "
                     f"median of {reps}")
    return out


def eikonal(phi, h, band=3.0):
    """|grad phi| (Eq. 32) by central differences at the interior nodes within
    `band` cells of the surface: median, percentiles and the share within 5%
    of 1 (an SDF of a mesh has |grad phi| = 1 away from its medial axis)."""
    p = np.asarray(phi, np.float64)
    c = p[1:-1, 1:-1, 1:-1]
    gx = (p[1:-1, 1:-1, 2:] - p[1:-1, 1:-1, :-2]) / (2 * h)
    gy = (p[1:-1, 2:, 1:-1] - p[1:-1, :-2, 1:-1]) / (2 * h)
    gz = (p[2:, 1:-1, 1:-1] - p[:-2, 1:-1, 1:-1]) / (2 * h)
    g = np.sqrt(gx * gx + gy * gy + gz * gz)[np.abs(c) < band * h]
    return {"nodes": int(g.size), "median": float(np.median(g)), "p01": float(np.percentile(g, 1)),
            "p99": float(np.percentile(g, 99)), "within_5pct": float(np.mean(np.abs(g - 1.0) < 0.05)),
            "band_cells": band}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(res, n, sample_nodes):
    """The FP64 oracle on the last timed step: every stage in full except the
    brute-force distance, which runs on `sample_nodes` grid nodes and is scaled
    to all n^3 nodes.  Also returns the GPU-vs-oracle error on that step."""
    from oracle import discretize as D
    from oracle import pipeline as P

    x, nrm = res["clouds_last"]
    grid = D.Grid.unit(n)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    log("cpu baseline: the oracle on the last timed step")
    t0 = time.perf_counter()
    ref = P.Recon(grid, x, nrm)
    t1 = time.perf_counter()
    rng = np.random.default_rng(4002)
    nodes = rng.choice(n ** 3, sample_nodes, replace=False)
    phi_ref = ref.phi_nodes(nodes)
    t2 = time.perf_counter()
    per_node = (t2 - t1) / sample_nodes
    t_full = (t1 - t0) + per_node * n ** 3
    g = res["gpu_last"]
    chi_ref = ref.chi
    err = {
        "chi_rel_l2": float(np.linalg.norm(g["chi"] - chi_ref) / np.linalg.norm(chi_ref)),
        "iso_c_rel": float(abs(g["iso_c"] - ref.c) / np.abs(chi_ref).max()),
        "phi_max_abs_over_h": float(np.abs(g["phi"].reshape(-1)[nodes].astype(np.float64) - phi_ref).max() * n),
        "nodes_compared": int(sample_nodes),
        "step": int(g["t"]),
    }
    base = {"value": 1.0 / t_full, "unit": "recons/s", "cores": threads, "kind": "oracle",
            "sample": (f"one {n}^3 step (t={g['t']}, {len(x)} points): splat, divergence, DCT solve, "
                       f"iso-value and Marching Cubes in full ({t1 - t0:.1f} s); brute-force distance on "
                       f"{sample_nodes} random nodes ({t2 - t1:.1f} s) scaled to {n ** 3} nodes"),
            "seconds_measured": t2 - t0}
    return base, err


def secondary_run():
    """The smaller workloads: the 32^3 sphere (4,096 points and queries, rel.
    res 1e-8), the noisy 128^3 torus (200,000 points, 1,000,000 queries, rel.
    res 1e-6, cold solve) and the differentiable 128^3 superellipsoid (100,000
    points, 65,536 targets): forward + backward, chained to the 16 shape
    coefficients, against the 32 forward evaluations a central
    finite-difference gradient needs."""
    import torch

    from paper_2609_20964_amd import synth
    from paper_2609_20964_amd.recon import Recon

    out = {}
    reps = 5
    x, nrm = synth.sphere()
    q = torch.from_numpy(synth.uniform_queries(4096, 102)).cuda()
    xd, nd = torch.from_numpy(x).cuda(), torch.from_numpy(nrm).cuda()
    r = Recon(32, len(x))
    r.forward(xd, nd, rel_tol=1e-8)
    r.sample(q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r.forward(xd, nd, rel_tol=1e-8)
        pq, nq = r.sample(q)
    torch.cuda.synchronize()
    t_s = (time.perf_counter() - t0) / reps
    cmp = {"sphere": {"x": x, "nrm": nrm, "phi": r.fields()["phi"].cpu().numpy(), "q": q.cpu().numpy(),
                      "phi_q": pq.cpu().numpy(), "n_q": nq.cpu().numpy()}}
    r.close()
    out["sphere_32"] = {"recons_per_s": 1.0 / t_s, "ms_per_recon": t_s * 1e3,
                        "workload": "sphere r 0.3, 4096 points, 32^3, rel res 1e-8, SDF and normals at 4096 queries"}

    x, nrm = synth.torus(200_000)
    q = torch.from_numpy(synth.uniform_queries(1_000_000, 204)).cuda()
    xd, nd = torch.from_numpy(x).cuda(), torch.from_numpy(nrm).cuda()
    r = Recon(128, len(x))
    r.forward(xd, nd, rel_tol=1e-6)
    r.sample(q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r.forward(xd, nd, rel_tol=1e-6)
        r.sample(q)
    torch.cuda.synchronize()
    t_rec = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        r.sample(q)
    torch.cuda.synchronize()
    t_q = (time.perf_counter() - t0) / reps
    # kept for the oracle comparison of the cpu_baseline leg
    rng = np.random.default_rng(205)
    nodes = rng.choice(128 ** 3, 400, replace=False)
    pq, nq = r.sample(q[:200])
    f = r.fields()
    cmp["torus"] = {"x": x, "nrm": nrm, "chi": f["chi"].cpu().numpy(), "nodes": nodes,
                     "phi_nodes": f["phi"].reshape(-1)[torch.from_numpy(nodes).cuda()].cpu().numpy(),
                     "q": q[:200].cpu().numpy(), "phi_q": pq.cpu().numpy(), "n_q": nq.cpu().numpy()}
    r.close()
    out["torus_128"] = {"recons_per_s": 1.0 / t_rec, "ms_per_recon": t_rec * 1e3,
                        "queries_per_s": q.shape[0] / t_q, "workload": "torus R 0.3 r 0.1, 200000 noisy points, "
                        "128^3, cold solve to rel res 1e-6, SDF and normals at 1e6 queries"}

    case = synth.diff_case()
    ct = torch.tensor(case.shape.coeffs, dtype=torch.float64, requires_grad=True)
    xt, nt = synth.star_points_torch(case.shape, case.dirs, ct)
    xs, ns = xt.detach().numpy().astype(np.float32), nt.detach().numpy().astype(np.float32)
    xd, nd = torch.from_numpy(xs).cuda(), torch.from_numpy(ns).cuda()
    tq = torch.from_numpy(case.targets).cuda()
    T = tq.shape[0]
    r = Recon(128, len(xs))

    def fwd():
        r.forward(xd, nd, rel_tol=1e-6)
        phi, _ = r.sample(tq, normals=False)
        return phi

    phi = fwd()
    gx, gn, _ = r.backward(tq, (2.0 / T) * phi, rel_tol=1e-6)
    # dL/dc: the point gradients chained through the shape generator (torch autograd, FP64, CPU)
    (dldc,) = torch.autograd.grad((xt * gx.cpu().double()).sum() + (nt * gn.cpu().double()).sum(), ct,
                                  retain_graph=True)
    cmp["superellipsoid"] = {"x": xs, "nrm": ns, "targets": case.targets, "g_xyz": gx.cpu().numpy(),
                             "g_nrm": gn.cpu().numpy(), "dldc": dldc.numpy(), "xt": xt, "nt": nt, "ct": ct}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        phi = fwd()
        r.backward(tq, (2.0 / T) * phi, rel_tol=1e-6)
    torch.cuda.synchronize()
    t_ad = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(32):
        fwd()
    torch.cuda.synchronize()
    t_fd = time.perf_counter() - t0
    r.close()
    out["superellipsoid_128_gradient"] = {"forward_backward_ms": t_ad * 1e3, "fd_32_forwards_ms": t_fd * 1e3,
                                          "fd_over_adjoint": t_fd / t_ad,
                                          "workload": "16-coefficient superellipsoid, 100000 points, 128^3, "
                                          "loss mean phi^2 at 65536 targets, rel res 1e-6"}
    return out, cmp


def cost_vs_grid(densities=(50, 100, 200, 400), reps=5):
    """The paper's cost study (Sec. 3.4): the fish-like cloud (200,000 points)
    on grids over its bounding box at several densities d; per grid the plain
    forward + sampling of 65,536 queries (median of `reps` after one warm-up,
    warm-started), the handle's resident bytes, and the log-log slopes of time
    and memory against the number of cells."""
    import torch

    from paper_2609_20964_amd import synth
    from paper_2609_20964_amd.recon import Recon, grid_from_cloud

    x, nrm = synth.fish(200_000)
    xd, nd = torch.from_numpy(x).cuda(), torch.from_numpy(nrm).cuda()
    rows = []
    for d in densities:
        n, lo, h = grid_from_cloud(xd, d)
        q = torch.from_numpy((np.asarray(lo) + synth.uniform_queries(65_536, 4201) * np.asarray(n) * h)
                             .astype(np.float32)).cuda()
        r = Recon(n, len(x), lo=lo, h=h)
        r.forward(xd, nd, rel_tol=1e-6)
        r.sample(q)
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = r.forward(xd, nd, rel_tol=1e-6, warm_start=True)
            r.sample(q)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        cells = int(np.prod(n))
        rows.append({"density": d, "grid": list(n), "cells": cells, "ms": float(np.median(times) * 1e3),
                     "bytes_resident": int(st["bytes_resident"])})
        r.close()
    lc = np.log([rw["cells"] for rw in rows])
    slope_t = float(np.polyfit(lc, np.log([rw["ms"] for rw in rows]), 1)[0])
    slope_m = float(np.polyfit(lc, np.log([rw["bytes_resident"] for rw in rows]), 1)[0])
    big = rows[-2:]   # the two largest grids, where fixed costs no longer dominate
    slope_t_big = float(np.log(big[1]["ms"] / big[0]["ms"]) / np.log(big[1]["cells"] / big[0]["cells"]))
    return {"rows": rows, "time_slope": slope_t, "time_slope_two_largest": slope_t_big, "memory_slope": slope_m,
            "workload": "fish-like body, 200,000 points, grids over its bounding box (pad 3 cells), rel res 1e-6, "
                        "forward + SDF/normals at 65,536 queries, median of 5"}


def normals_run(n_points=200_000, radius=0.1, gamma_r=2.5, n_tol=2, reps=3):
    """Unoriented clouds (Sec. 2.1-2.2) at the defaults of Table 1: D-PCA
    normals and their orientation for the fish-like cloud (200,000 points,
    bounding box 0.8 x 0.28 x 0.36), timed per call (each call blocks and
    allocates its work buffers on the stream); quality against the body's
    analytic outward normals.  Keeps a seeded sample for the oracle."""
    import torch

    from paper_2609_20964_amd import synth
    from paper_2609_20964_amd.normals import dpca_normals, orient_normals

    x, n_true = synth.fish(n_points)
    xd = torch.from_numpy(x).cuda()
    nd = dpca_normals(xd, radius)
    orient_normals(xd, nd, gamma_r, n_tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        nd = dpca_normals(xd, radius)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        no, info, cnt = orient_normals(xd, nd, gamma_r, n_tol, counts=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    un, on = nd.cpu().numpy(), no.cpu().numpy()
    cosang = np.sum(on.astype(np.float64) * n_true, 1)
    line_ang = np.arccos(np.clip(np.abs(np.sum(un.astype(np.float64) * n_true, 1)), 0, 1))
    out = {"dpca_ms": (t1 - t0) / reps * 1e3, "orient_ms": (t2 - t1) / reps * 1e3,
           "points_per_s": n_points / ((t2 - t0) / reps), "outward_frac": float((cosang > 0).mean()),
           "dpca_angle_median_rad": float(np.median(line_ang)), "dpca_angle_p99_rad": float(np.percentile(line_ang, 99)),
           "orient_info": info,
           "workload": f"fish-like star body, {n_points} points, R = {radius}, gamma_r = {gamma_r}, N_tol = {n_tol} "
                       "(Table 1 defaults)"}
    rng = np.random.default_rng(4101)
    pick = np.sort(rng.choice(n_points, 200, replace=False))
    cmp = {"x": x, "pick": pick, "dpca": un[pick], "nrm_in": un, "counts": cnt.cpu().numpy()[pick],
           "oriented": on[pick], "info": info, "radius": radius, "gamma_r": gamma_r, "n_tol": n_tol}
    return out, cmp


def normals_oracle_error(cmp):
    """Part of the cpu_baseline leg: the oracle's D-PCA normal and ray counts
    at 200 seeded points of the fish cloud (full neighbourhoods and rays
    against the whole cloud)."""
    from scipy.spatial import cKDTree

    from oracle import normals as NO

    x = cmp["x"]
    t0 = time.perf_counter()
    tree = cKDTree(x.astype(np.float64))
    p = NO.ray_params(x, cmp["gamma_r"])
    worst, counts_equal, signs_equal = 0.0, 0, 0
    R2 = NO.r2_f32(cmp["radius"])
    for k, i in enumerate(cmp["pick"]):
        cand = np.asarray(tree.query_ball_point(x[i].astype(np.float64), cmp["radius"] * 1.00001), np.int64)
        nb = np.sort(cand[NO._d2_f32(x[i], x[cand]) <= R2])
        n_ref, _ = NO.dpca_point(x, i, nb, 1e-6 * cmp["radius"])
        g = cmp["dpca"][k].astype(np.float64)
        worst = max(worst, float(np.arctan2(np.linalg.norm(np.cross(g, n_ref)), abs(g @ n_ref))))
        c = []
        for sg in (np.float32(1), np.float32(-1)):
            y = NO.probes(x[i], (sg * cmp["nrm_in"][i]).astype(np.float32), p["M"], p["ds_f32"])
            c.extend(NO.crossings(NO.detect(tree, x, y, p["rd"], p["rd2_f32"])))
        counts_equal += int((np.asarray(c) == cmp["counts"][k]).all())
        s = NO.orient_signs(np.asarray([c]), cmp["n_tol"])[0]
        signs_equal += int((s * cmp["nrm_in"][i] == cmp["oriented"][k]).all())
    return {"dpca_max_angle_rad": worst, "ray_counts_equal": counts_equal, "signs_equal": signs_equal,
            "points_compared": len(cmp["pick"]), "spacing2_equal": bool(cmp["info"]["spacing2"] == float(p["d2max"])),
            "seconds": time.perf_counter() - t0}


def secondary_oracle_error(cmp):
    """Part of the cpu_baseline leg: the GPU results of the smaller workloads
    against the FP64 oracle (the sphere's SDF on every node and at every
    query; the torus field, SDF on 400 random nodes, SDF and normals at 200
    queries; the superellipsoid's point gradients, all 100,000 points, and
    its dL/dc through the same shape generator)."""
    from oracle import discretize as D
    from oracle import pipeline as P

    s = cmp["sphere"]
    g32 = D.Grid.unit(32)
    ref = P.Recon(g32, s["x"], s["nrm"])
    vq, nq = ref.sample(s["q"])
    ok = np.linalg.norm(nq, axis=1) > 0
    ang = angle_between(s["n_q"][ok], nq[ok])
    sphere = {"phi_grid_max_abs_over_h": float(np.abs(s["phi"].astype(np.float64) - ref.phi_grid()).max() * 32),
              "phi_queries_max_abs_over_h": float(np.abs(s["phi_q"] - vq).max() * 32),
              "normal_angle_max_rad": float(ang.max()), "nodes_compared": 32 ** 3, "queries_compared": len(s["q"])}
    log("oracle: sphere done, torus next")
    grid = D.Grid.unit(128)
    t = cmp["torus"]
    ref = P.Recon(grid, t["x"], t["nrm"])
    vq, nq = ref.sample(t["q"])
    ok = np.linalg.norm(nq, axis=1) > 0
    ang = angle_between(t["n_q"][ok], nq[ok])
    torus = {"chi_rel_l2": float(np.linalg.norm(t["chi"] - ref.chi) / np.linalg.norm(ref.chi)),
             "phi_nodes_max_abs_over_h": float(np.abs(t["phi_nodes"] - ref.phi_nodes(t["nodes"])).max() * 128),
             "phi_queries_max_abs_over_h": float(np.abs(t["phi_q"] - vq).max() * 128),
             "normal_angle_max_rad": float(ang.max()), "nodes_compared": len(t["nodes"]),
             "queries_compared": len(t["q"])}
    log("oracle: torus done, superellipsoid reverse pass next")
    e = cmp["superellipsoid"]
    ref = P.Recon(grid, e["x"], e["nrm"])
    phi, _ = ref.sample(e["targets"])
    gx, gn, _ = ref.backward(e["targets"], 2.0 * phi / len(phi))
    want = np.concatenate([gx, gn]).reshape(-1)
    got = np.concatenate([e["g_xyz"], e["g_nrm"]]).reshape(-1).astype(np.float64)
    import torch
    (dldc_ref,) = torch.autograd.grad((e["xt"] * torch.from_numpy(gx)).sum() + (e["nt"] * torch.from_numpy(gn)).sum(),
                                      e["ct"])
    dldc_ref = dldc_ref.numpy()
    sup = {"point_grad_rel_l2": float(np.linalg.norm(got - want) / np.linalg.norm(want)), "points": len(e["x"]),
           "dL_dc_rel_l2": float(np.linalg.norm(e["dldc"] - dldc_ref) / np.linalg.norm(dldc_ref)),
           "dL_dc_max_rel": float(np.abs(e["dldc"] - dldc_ref).max() / np.abs(dldc_ref).max())}
    return {"sphere_32": sphere, "torus_128": torus, "superellipsoid_128_gradient": sup}


def _request_inputs(args):
    """One request's cloud and queries (a process-pool task: the shapes'
    normals come from torch autograd on the CPU, about 75 ms per request)."""
    index, n_requests = args
    import torch

    from paper_2609_20964_amd import synth
    torch.set_num_threads(1)
    rq = synth.request_stream(n_requests)[index]
    x, nrm = rq.cloud()
    return x, nrm, rq.queries()


def generate_requests(n_requests):
    """The request stream's inputs, made by a pool of forked processes before
    this process touches the GPU."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    from paper_2609_20964_amd import synth

    reqs = synth.request_stream(n_requests)
    with ProcessPoolExecutor(max_workers=12, mp_context=mp.get_context("fork")) as ex:
        data = list(ex.map(_request_inputs, [(i, n_requests) for i in range(n_requests)], chunksize=8))
    return [(rq,) + d for rq, d in zip(reqs, data)]


def serving_run(generated, warmup, max_inflight, budget_gb):
    """The request stream replayed on two resident servers, continuous
    batching (max_inflight at once) and one request at a time: first the
    `warmup` leading requests untimed at saturation (the servers' handle pools
    fill, as a long-running server's would), then the rest at the stream's own
    Poisson arrival times (latency at the offered load) and with every request
    arriving at once (throughput at saturation)."""
    import torch

    from paper_2609_20964_amd.serving import Server

    reqs = [(rq, torch.from_numpy(x).cuda(), torch.from_numpy(nrm).cuda(), torch.from_numpy(q).cuda())
            for rq, x, nrm, q in generated]
    warm, reqs = reqs[:warmup], reqs[warmup:]
    out = {"offered_load": {}, "saturated": {}}
    cmp = None
    for mode, inflight in (("batched", max_inflight), ("plain", 1)):
        srv = Server(int(budget_gb * (1 << 30)), max_inflight=inflight)
        if warm:
            replay(srv, warm, 0.0)
        stats, done = replay(srv, reqs, 1.0, keep=True)
        out["offered_load"][mode] = dict(max_inflight=inflight, **stats)
        stats, _ = replay(srv, reqs, 0.0)
        out["saturated"][mode] = dict(max_inflight=inflight, **stats)
        srv.close()
        log(f"serving {mode} done")
        if mode == "batched":
            # kept for the oracle comparison of the cpu_baseline leg: a seeded
            # subset of the 64^3 requests and of the others, SDF and normals at
            # their first 200 queries
            rng = np.random.default_rng(506)
            small = [i for i, (rq, *_) in enumerate(reqs) if rq.n == 64]
            big = [i for i, (rq, *_) in enumerate(reqs) if rq.n != 64]
            n_big = max(2, int(round(0.05 * len(big)))) if big else 0
            pick = sorted(small + rng.choice(big, min(n_big, len(big)), replace=False).tolist())
            cmp = []
            for i in pick:
                rq, x, nrm, q = reqs[i]
                outs = done[i][0][1]
                cmp.append({"n": rq.n, "x": x.cpu().numpy(), "nrm": nrm.cpu().numpy(), "q": q[:200].cpu().numpy(),
                            "phi_q": outs["phi"][:200].cpu().numpy(), "n_q": outs["nrm"][:200].cpu().numpy()})
    out["workload"] = (f"{len(reqs)} measured requests after {len(warm)} warm-up ones, Poisson arrivals 50/s, "
                       "grids 64/128/256 (0.5/0.3/0.2), log-normal points (median 50k), 30% with gradient, "
                       "65,536 queries each, rel. res 1e-6; saturated = all measured requests at t=0")
    return out, cmp


def serving_oracle_error(cmp):
    """Part of the cpu_baseline leg: served results (batched, offered load)
    against the FP64 oracle: SDF and normals at the first 200 queries of every
    64^3 request and of a seeded 5% (at least 2) of the larger ones."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import discretize as D
    from oracle import pipeline as P

    def one(c):
        ref = P.Recon(D.Grid.unit(c["n"]), c["x"], c["nrm"])
        vq, nq = ref.sample(c["q"])
        ok = np.linalg.norm(nq, axis=1) > 0
        ang = angle_between(c["n_q"][ok], nq[ok])
        return float(np.abs(c["phi_q"] - vq).max() * c["n"]), float(ang.max()) if ang.size else 0.0

    with ThreadPoolExecutor(max_workers=4) as ex:
        errs = list(ex.map(one, cmp))
    sizes = [c["n"] for c in cmp]
    return {"phi_queries_max_abs_over_h": max(e[0] for e in errs), "normal_angle_max_rad": max(e[1] for e in errs),
            "requests_compared": {str(n): sizes.count(n) for n in sorted(set(sizes))}, "queries_per_request": 200}


def latency_by_grid(grids, lat_s):
    """p50 / p99 latency (ms) and count of the requests of each grid size."""
    grids, lat = np.asarray(grids), np.asarray(lat_s, np.float64) * 1e3
    out = {}
    for n in sorted(set(grids.tolist())):
        v = lat[grids == n]
        out[str(n)] = {"requests": int(v.size), "p50_ms": float(np.percentile(v, 50)),
                       "p99_ms": float(np.percentile(v, 99))}
    return out


def replay(srv, reqs, time_scale, keep=False):
    import threading

    import torch

    a0 = reqs[0][0].arrival_s
    arrival = [(rq.arrival_s - a0) * time_scale for rq, *_ in reqs]
    tickets = [None] * len(reqs)
    start = time.perf_counter()

    def client():
        for i, (rq, x, nrm, q) in enumerate(reqs):
            delay = arrival[i] - (time.perf_counter() - start)
            if delay > 0:
                time.sleep(delay)
            gphi = torch.full((q.shape[0],), 1.0 / q.shape[0], device="cuda") if rq.want_grad else None
            tickets[i] = (srv.submit(rq.n, x, nrm, q, gphi=gphi, rel_tol=1e-6), time.perf_counter() - start)

    th = threading.Thread(target=client)
    th.start()
    done = {}
    while len(done) < len(reqs):
        for i in range(len(reqs)):
            if i in done or tickets[i] is None:
                continue
            res = srv.poll(tickets[i][0])
            if res is not None:
                done[i] = (res, time.perf_counter() - start)
        time.sleep(0.0005)
    th.join()
    lat = np.array([done[i][1] - arrival[i] for i in range(len(reqs))])
    span = max(d[1] for d in done.values()) - arrival[0]
    ok = sum(1 for d in done.values() if d[0][0] in (0, -3))
    cells = sum(rq.n ** 3 for rq, *_ in reqs)
    stats = {"req_per_s": len(reqs) / span, "cells_per_s": cells / span,
             "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
             "by_grid": latency_by_grid([rq.n for rq, *_ in reqs], lat),
             "ok": ok, "requests": len(reqs),
             "max_rel_res": max(d[0][2]["stats"]["rel_res"] for d in done.values())}
    return stats, (done if keep else None)


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """Device-to-device copy rate (GB/s, read + write bytes) of the library's
    streaming copy kernel (wg_stream_copy), timed with events on the stream it
    runs on: the bandwidth a streaming kernel reaches on this device."""
    import torch

    from paper_2609_20964_amd import _lib

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    run = lambda: _lib.check(_lib.lib().wg_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes, s.cuda_stream))
    run()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        run()
    e1.record(s)
    e1.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def copy_probe():
    """Five 1 GiB streaming copies (wg_stream_copy): the calibration run of
    the rocprofv3 byte counters."""
    import torch

    from paper_2609_20964_amd import _lib

    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        _lib.check(_lib.lib().wg_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes,
                                             torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 5}), flush=True)


def short_kernel_name(name):
    for ns in ("wg::scan::(anonymous namespace)::", "wg::(anonymous namespace)::", "wg::"):
        name = name.replace(ns, "")
    if name.startswith("void "):
        name = name[5:]
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def pmc_summary(path, periods=()):
    """Mean counter value per dispatch, by kernel name (namespaces and
    argument lists dropped) and grid size.  A kernel that runs on several
    multigrid levels with the same grid size is split by its dispatch order
    (`periods`: NAME=P gives level i mod P of that kernel's dispatches of one
    grid size).  Dispatches below 5% of their group's median are launches that
    returned at once (an inner iteration enqueued after the one that stopped
    the solve): they are counted apart and left out of the means."""
    import csv
    from collections import defaultdict

    period = dict(p.split("=") for p in periods)
    rows_by = defaultdict(list)
    with open(path) as f:
        rows = csv.DictReader(f)
        if "Kernel_Name" not in (rows.fieldnames or []) or "Counter_Name" not in rows.fieldnames:
            raise SystemExit(f"unexpected columns in {path}: {rows.fieldnames}")
        for row in rows:
            name = short_kernel_name(row["Kernel_Name"])
            rows_by[(name, row.get("Grid_Size", ""))].append(row)
    for (name, grid), rs in sorted(rows_by.items(), key=lambda kv: -len(kv[1])):
        disp = sorted({int(r["Dispatch_Id"]) for r in rs})
        per = int(period.get(name, 1))
        for lvl in range(per):
            ids = set(disp[lvl::per])
            vals = defaultdict(dict)
            for r in rs:
                d = int(r["Dispatch_Id"])
                if d in ids:
                    vals[d][r["Counter_Name"]] = vals[d].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            first = sorted({c for v in vals.values() for c in v})
            key = first[0] if first else None
            med = sorted(v.get(key, 0.0) for v in vals.values())[len(vals) // 2] if vals else 0.0
            live = [v for v in vals.values() if v.get(key, 0.0) >= 0.05 * med]
            if not live:
                continue
            means = " ".join(f"{c}={sum(v.get(c, 0.0) for v in live) / len(live):.6g}" for c in first)
            tag = f" [grid {grid}]" + (f" [level {lvl} of {per}]" if per > 1 else "")
            print(f"{name}{tag} | dispatches={len(live)} (+{len(vals) - len(live)} returned at once) | {means}")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    # 6 warm-up steps + 494 timed ones: the configuration's 500 steps of the flapping wave (5 periods)
    ap.add_argument("--steps", type=int, default=494)
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--points", type=int, default=300_000)
    ap.add_argument("--queries", type=int, default=65_536)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--adjoint-steps", type=int, default=3)
    ap.add_argument("--exact-steps", type=int, default=5,
                    help="plain steps of the exact-quadrature system on the same clouds (0: skip)")
    ap.add_argument("--serving", type=int, default=1050,
                    help="requests in the serving replay, warm-up ones included (0: skip)")
    ap.add_argument("--serving-warmup", type=int, default=50, help="leading requests that only warm the servers")
    ap.add_argument("--serving-inflight", type=int, default=4, help="worker threads of the batched server")
    ap.add_argument("--cpu-sample-nodes", type=int, default=1500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the two 128^3 workloads")
    ap.add_argument("--no-normals", action="store_true", help="skip the normal estimation and orientation run")
    ap.add_argument("--no-cost-sweep", action="store_true", help="skip the cost-versus-grid-size sweep")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (calibrates rocprofv3 byte counters)")
    ap.add_argument("--pmc-period", metavar="NAME=P", action="append", default=[],
                    help="with --pmc-summary: split NAME's dispatches of one grid size into P levels by order")
    ap.add_argument("--pmc-summary", metavar="CSV",
                    help="only summarise a rocprofv3 counter_collection.csv: mean per dispatch by kernel")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary, args.pmc_period)
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library runs one reconstruction per device and has no "
              "multi-GPU path; run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    generated = None
    if args.serving > 0:
        log(f"generating {args.serving} serving requests")
        generated = generate_requests(args.serving)   # before this process touches the GPU
    res = gpu_run(args)
    copy_gbs = copy_bandwidth()
    steps = args.steps
    value = steps / res["elapsed"]
    st = res["stats"]
    line = {
        "metric": "grid recons/s at 256^3 (rel res 1e-6) + % HBM peak; batched p50/p99 vs plain",
        "value": value,
        "unit": "recons/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": res["elapsed"] / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 sweeps + f64 reductions/refinement",
        "data": "synthetic",
        "config": {"workload": f"flapping ellipsoid, {args.points} points, {args.n}^3 grid, warm-started, "
                               f"rel res {args.tol:g}, {args.queries} queries sampled per step",
                   "grid": args.n, "points": args.points, "queries": args.queries, "rel_tol": args.tol},
        "roofline": roofline(res),
        "solver_roofline": solver_hbm(res, copy_gbs),
        "solver": {"iters_mean": float(np.mean([s["iters"] for s in st])),
                   "refinements_mean": float(np.mean([s["refinements"] for s in st])),
                   "rel_res_max": float(max(s["rel_res"] for s in st)),
                   "n_tris_mean": float(np.mean([s["n_tris"] for s in st]))},
        "unpipelined": {"ms_per_step": res["plain_ms"], "recons_per_s": 1e3 / res["plain_ms"],
                        "steps": res["plain_steps"]},
        # phases of the steps run one after another (in pipelined steps they overlap)
        "phase_ms_plain": {k: float(np.mean([s["ms"][i] for s in res["plain_stats"]]))
                           for i, k in enumerate(["splat", "solve", "iso", "surface", "sdf"])},
        "kernel_ms_per_step_plain": {k: v["ms"] / res["n_prof"] for k, v in res["per_kind"].items()},
        "adjoint_ms_mean": float(np.mean(res["adj_ms"])) if res["adj_ms"] else None,
        "cold_step_ms": res["cold_ms"],
        "ms_per_step_by_100_steps": [float(v) for v in np.diff(np.concatenate([[0.0], res["stamps"][99::100]])) / 100 * 1e3],
        "eikonal": eikonal(res["gpu_last"]["phi"].reshape(args.n, args.n, args.n), 1.0 / args.n),
        "exact_quadrature": exact_summary(res, copy_gbs) if res["exact"] else None,
    }
    if not args.no_cpu_baseline:
        base, err = cpu_baseline(res, args.n, args.cpu_sample_nodes)
        log(f"oracle every 25th step: {len(res['samples'])} steps")
        line["cpu_baseline"] = base
        line["oracle_error"] = err
        line["oracle_error_every_25th_step"] = sample_errors(res, args.n, args.cpu_sample_nodes)
    if args.serving > 0:
        log("serving replay")
        line["serving"], scmp = serving_run(generated, min(args.serving_warmup, args.serving - 1),
                                            args.serving_inflight, 64.0)
        del generated
        if not args.no_cpu_baseline:
            line["serving"]["oracle_error"] = serving_oracle_error(scmp)
    if not args.no_cost_sweep:
        log("cost versus grid size")
        line["cost_vs_grid"] = cost_vs_grid()
    if not args.no_normals:
        log("normals run")
        line["normals"], ncmp = normals_run()
        if not args.no_cpu_baseline:
            line["normals"]["oracle_error"] = normals_oracle_error(ncmp)
    if not args.no_secondary:
        log("secondary workloads")
        line["secondary"], cmp = secondary_run()
        if not args.no_cpu_baseline:
            log("secondary workloads against the oracle")
            for k, v in secondary_oracle_error(cmp).items():
                line["secondary"][k]["oracle_error"] = v
            line["secondary"]["oracle_timing"] = oracle_timing(cmp)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
