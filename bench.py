"""Benchmark of the per-frame dynamic mesh-Gaussian update on one MI355X.

One step = one frame of the workload through the whole per-frame path:
  a1  frame index + vertex-buffer write of the fixed-topology mesh
  a2  Gaussian re-pose from their faces (mean, quaternion, covariance)
  a4  LBVH refit on the fixed template topology
  a5  closest-point queries of the collision particles (normals on demand)
  a6  rebuild of the varying-topology target's LBVH (the comparison path)
  a5' collision queries against the rebuilt target, and template projection
      (Eq. 2 of the paper): every template vertex onto the target.
Inputs are synthetic, seeded and device-resident before timing.  Warm-up steps
run eagerly; the K timed steps are captured once into a HIP graph and replayed
(so host launch overhead is not measured), bracketed by synchronisations.

Workload c1 times the small icosphere case the same way without the
comparison path (no varying-topology target), plus its 60 frames as one
persistent launch; track times temporal correspondence tracking (one step = one frame),
c3 times the batched form instead (one step = one persistent launch
over all scenes x frames, against the plain per-frame path on the same GPU),
and c4 the differentiable form (one step = one Adam step of the template
projection loss, forward + backward + update).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c1|c2|c3|c4|c5|track|sdf|contact]
Prints one JSON line.
"""

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Dense fp32 vector peak without packed instructions (the build turns them off):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops per FMA x 2.4 GHz.
FP32_VECTOR_NONPACKED_TFLOPS = 78.6
QUERY_COMPULSORY_BYTES = 40.0      # query point in, closest point, id and distance out
# c2 is the default line; c1 (the small icosphere case, no varying-topology target)
# and the others are optional lines.
WORKLOADS = {
    "c1": (1, "icosphere 2,562 V / 5,120 F, 30,720 Gaussians, 10,000 queries, 60 frames of sinusoidal "
              "vertex displacement"),
    "c2": (2, "UV-sphere template 20,002 V / 40,000 F, 100,000 Gaussians, 50,000 particles, "
              "200 frames, marching-tetrahedra targets ~46-53k F"),
    "c3": (3, "batched: 6 UV-sphere scenes of 5k/10k/20k/30k/40k/50k F, 20k-300k Gaussians, "
              "10k-100k queries, 64 frames each, one persistent launch"),
    "c4": (4, "differentiable template projection: 20,002 V / 40,000 F template, 100,000 Gaussians, "
              "100,000 target samples; one Adam step of P + Chamfer"),
    "c5": (5, "UV-sphere 250,002 V / 500,000 F, 1,000,000 Gaussians, 1,000,000 queries, 100 frames, "
              "1,000,000-face split rebuild targets"),
    "contact": (2, "sphere-mesh contact: 50,000 spheres (radius 1% of the template) falling at 240 steps/s onto "
                   "the deforming 40,000-face template; per step vertex copy, refit, integration, closest "
                   "points with normals, contact response"),
    "sdf": (2, "index signed-distance grid: the 40,000-face template's 64^3 grid (4 nearest template faces "
               "per node) updated per frame, the 50,000 particles sampled through it; 200 frames"),
    "track": (2, "temporal correspondence tracking (Eq. 1): the 20,002-vertex template carried through "
                 "200 marching-tetrahedra targets of ~46-53k faces, re-anchored every 50 frames"),
}
METRIC = "frames/s and closest-point queries/s, refit vs rebuild; achieved HBM GB/s"
# (timed steps, warm-up steps) per workload: each default run times about a second of GPU work
# Algorithmic float32 operations (an FMA counts two) of the closest-point traversal per counted unit:
# a node expansion bounds its two internal children (box distance 17 and
# normal-slab distance 12 each, plus the query's slab margin 6), a leaf bound
# test takes the triangle's bounds and their box distance (29), an exact test
# is the closest point on a triangle (80).
OPS_EXPANSION, OPS_LEAF_BOUND, OPS_EXACT = 64.0, 29.0, 80.0

DEFAULT_STEPS = {"c1": (60, 5), "c2": (200, 10), "c3": (10, 2), "c4": (200, 10), "c5": (20, 3), "track": (199, 0), "sdf": (200, 10), "contact": (200, 10)}


def _target_job(args):
    cfg, t = args
    from synth import make_config
    sc = make_config(cfg)
    return sc.target(t)


def make_targets(cfg, ts):
    """Varying-topology targets for frames ts, generated on host worker processes."""
    import multiprocessing as mp
    workers = max(1, min(16, len(ts), os.cpu_count() or 1))
    if workers == 1:
        return [_target_job((cfg, t)) for t in ts]
    # close and join (not the context manager's terminate): the workers exit on their own
    pool = mp.get_context("fork").Pool(workers)
    try:
        out = pool.map(_target_job, [(cfg, t) for t in ts])
    finally:
        pool.close()
        pool.join()
    return out


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


_CSRC = "paper_2606_00444_amd/csrc/"
KERNEL_SOURCES = {
    "gaussian_update": [_CSRC + f for f in ("gaussian.hip", "repose.hpp", "mgu_internal.hpp")],
    "refit": [_CSRC + f for f in ("lbvh.hip", "refit.hpp", "mgu_internal.hpp")],
    "frame_update": [_CSRC + f for f in ("lbvh.hip", "refit.hpp", "repose.hpp", "mgu_internal.hpp")],
    "collide": [_CSRC + f for f in ("query.hip", "traverse.hpp", "mgu_internal.hpp")],
    "batch": [_CSRC + f for f in ("batch.hip", "traverse.hpp", "refit.hpp", "repose.hpp", "mgu_internal.hpp")],
}


def measured_traffic(workload, kernel):
    """HBM bytes per launch of kernel in workload from the committed rocprofv3 counter
    summary (profiles/traffic.json, keyed by workload then kernel), if it was taken
    on the current source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(workload, {}).get(kernel)
    except (OSError, ValueError, AttributeError):
        return None
    if not rec or rec.get("source_hash") != source_hash(KERNEL_SOURCES.get(kernel, [])):
        return None
    return rec.get("bytes_per_launch")


def measured_counters(workload, kernel):
    """Per-dispatch counter figures (VALU busy, occupancy, ...) of kernel in workload
    from profiles/counters.json, if taken on the current source; else None."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(workload, {}).get(kernel)
    except (OSError, ValueError, AttributeError):
        return None
    if not rec or rec.get("source_hash") != source_hash(KERNEL_SOURCES.get(kernel, [])):
        return None
    return {k: v for k, v in rec.items() if k != "source_hash"}


def cpu_baseline(sc, frames_np, targets_np, n_sample, n_single, reps=5):
    """The float64 oracle on the phases of a step, frames 1..reps, as frames/s.

    Per frame: the re-pose of every Gaussian, the refit of the template tree and
    the rebuild of the frame's target (numpy, one thread), and the three query
    sets (plain-C brute force, OpenMP) on n_sample random queries per set with
    every host core, and on n_single with one thread, each scaled to the full set.
    A frame's all-core time is the numpy phases plus the all-core query time, its
    single-thread time the numpy phases plus the one-thread query time; the
    values are medians over the reps frames."""
    from oracle import gaussians as og, lbvh as ol, closest as oc, frame as ofr
    t_all = time.perf_counter()
    ref = ol.build(sc.verts0, sc.faces)          # the rest-pose tree, built once at initialisation
    rng = np.random.default_rng(0)
    cores = omp_threads()
    reps = max(1, min(reps, len(frames_np) - 1, len(targets_np) - 1))
    host = {k: [] for k in ("update", "refit", "rebuild")}
    qall = {k: [] for k in ("collide", "collide_target", "project")}
    q1 = {k: [] for k in qall}

    def queries(mv, mf, q, n, threads):
        idx = rng.choice(q.shape[1], min(n, q.shape[1]), replace=False)
        oc.set_threads(threads)
        t = time.perf_counter()
        oc.closest_point_mesh(mv, mf, q[:, idx])
        return (time.perf_counter() - t) * q.shape[1] / idx.size

    try:
        for f in range(1, reps + 1):
            V = frames_np[f]
            tv, tf = targets_np[f]
            t = time.perf_counter()
            live = ofr.vertex_buffer_update(frames_np, f)
            og.repose(live, sc.faces, sc.binding)
            host["update"].append(time.perf_counter() - t)
            t = time.perf_counter()
            ol.refit(ref["tree"], ol.leaf_boxes(V, sc.faces, ref["perm"]))
            host["refit"].append(time.perf_counter() - t)
            t = time.perf_counter()
            ol.build(tv, tf)
            host["rebuild"].append(time.perf_counter() - t)
            qs = {"collide": (V, sc.faces, sc.queries), "collide_target": (tv, tf, sc.queries),
                  "project": (tv, tf, sc.verts0)}
            for name, (mv, mf, q) in qs.items():
                qall[name].append(queries(mv, mf, q, n_sample, cores))
                q1[name].append(queries(mv, mf, q, n_single, 1))
    finally:
        oc.set_threads(cores)
    host_s = np.sum([host[k] for k in host], axis=0)
    all_core = host_s + np.sum([qall[k] for k in qall], axis=0)
    single = host_s + np.sum([q1[k] for k in q1], axis=0)
    med = lambda d: {k: round(float(np.median(v)), 4) for k, v in d.items()}
    return {
        "value": 1.0 / float(np.median(all_core)), "unit": "frames/s", "cores": cores, "kind": "oracle",
        "sample": (f"median of {reps} frames (1-{reps}): float64 numpy re-pose of all {sc.n_gauss} Gaussians, "
                   f"template refit and target rebuild (one thread); plain-C brute-force closest points on "
                   f"{n_sample} random queries per query set with {cores} OpenMP threads, scaled to the full "
                   f"sets ({sc.queries.shape[1]} particles twice, {sc.n_verts} template vertices)"),
        "single_thread": {"value": 1.0 / float(np.median(single)), "unit": "frames/s", "cores": 1,
                          "sample": f"the same frames and host phases; {n_single} random queries per set on one "
                                    f"thread, scaled"},
        "seconds_per_frame_median": dict(med(host), **{k + "_all_cores": v for k, v in med(qall).items()},
                                         **{k + "_one_thread": v for k, v in med(q1).items()}),
        "wall_s": round(time.perf_counter() - t_all, 2),
    }


def sample_frames(T, k=6):
    """k frames spread evenly over a sequence of T (both ends included)."""
    return sorted({round(i * (T - 1) / (k - 1)) for i in range(k)}) if T > 1 else [0]


def graph_ms(fn, reps, torch):
    """Average ms of fn over a HIP graph of `reps` back-to-back calls (HIP events on the launch stream)."""
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for r in range(reps):
            fn(r)
    g.replay()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    g.replay()
    z.record(s)
    torch.cuda.synchronize()
    return a.elapsed_time(z) / reps


def timed_region(run, steps, torch):
    """Events and wall clock around one call of run (K steps), synchronised on both sides."""
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    e0.record(s)
    run()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, time.perf_counter() - t


def omp_threads():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def run_contact(args):
    """Spheres falling onto the deforming template: one step = one frame of the contact simulation."""
    from synth import make_config
    t0 = time.perf_counter()
    sc = make_config(2)
    T = sc.n_frames
    frames_np = sc.frames(range(T))
    setup_s = time.perf_counter() - t0

    import torch
    import paper_2606_00444_amd as mg
    from paper_2606_00444_amd.contact import Spheres
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    mg.check_device()
    D = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    frames, F, V0 = D(frames_np), D(sc.faces), D(sc.verts0)
    NV, NF = sc.n_verts, sc.n_faces
    P = 50_000
    L = float(np.ptp(sc.verts0, axis=1).max())
    lo, hi = sc.verts0.min(1), sc.verts0.max(1)
    rng = np.random.default_rng(60644499)
    x0 = np.stack([rng.uniform(lo[0], hi[0], P), rng.uniform(lo[1], hi[1], P),
                   rng.uniform(hi[2], hi[2] + 0.5 * L, P)]).astype(np.float32)
    dt, r, e = 1.0 / 240.0, 0.01 * L, 0.3
    live = torch.empty(3, NV, device=dev)
    bvh = mg.lbvh_build(V0, F)
    S = Spheres(D(x0), torch.zeros(3, P, device=dev), r, restitution=e)

    def step(i):
        mg.vertex_buffer_update(frames, i % T, live)
        mg.lbvh_refit(bvh, live)
        S.step(bvh, live, dt)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    if args.eager:
        run = lambda: [step(i) for i in range(args.steps)]
    else:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for i in range(args.warmup, args.warmup + args.steps):
                step(i)
        run = g.replay
    ms_per_step, wall = timed_region(run, args.steps, torch)
    contacts = int(S.contact.sum().item())
    # per-phase durations in the final state
    xs = S.x.clone()
    vs = S.v.clone()
    rec = S.rec
    # the next step's query would start from the last step's faces (a copy here,
    # so that the timed launches do not feed each other)
    hint = rec["face"].clone()
    ph = {"refit": graph_ms(lambda _: mg.lbvh_refit(bvh, live), 50, torch),
          "closest": graph_ms(lambda _: mg.closest_point_query(bvh, live, xs, normal=True, out=rec, hint=hint), 20,
                              torch)}
    S.x.copy_(xs)
    S.v.copy_(vs)
    cnt = torch.zeros(4, dtype=torch.int64, device=dev)
    mg.closest_point_query(bvh, live, xs, normal=True, out=rec, counters=cnt, hint=hint)
    torch.cuda.synchronize()
    n_exp, n_lbox, n_lex, n_q = (int(x) for x in cnt.cpu())
    ops = OPS_EXPANSION * n_exp + OPS_LEAF_BOUND * n_lbox + OPS_EXACT * n_lex
    achieved = ops / (ph["closest"] * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": round(1000.0 / ms_per_step, 2), "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"contact: {WORKLOADS['contact'][1]}", "spheres": P, "radius": r, "dt": dt,
                   "restitution": e, "faces": NF, "timing": "eager" if args.eager else "hip-graph"},
        "contacts_last_step": contacts,
        "kernels_ms": {k: round(v, 5) for k, v in ph.items()},
        "queries_per_s": round(P * 1000.0 / ms_per_step, 1),
        "roofline": {"bound": "alu", "kernel": "traverse_batch_kernel (sphere centres onto the template)",
                     "achieved": round(achieved, 4), "peak": FP32_VECTOR_NONPACKED_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP32_VECTOR_NONPACKED_TFLOPS, 5), "traffic": None,
                     "alg_ops_per_launch": int(ops), "avg_launch_ms": round(ph["closest"], 5)},
        "wall_s": round(wall, 4), "setup_s": round(setup_s, 2),
    }
    if not args.no_cpu_baseline:
        from oracle import contact as oco
        idx = rng.choice(P, 4000, replace=False)
        tt = time.perf_counter()
        oco.step(x0[:, idx].astype(np.float64), np.zeros((3, idx.size)), frames_np[0], sc.faces, dt,
                 np.array([0.0, 0.0, -9.8]), r, e)
        sec = (time.perf_counter() - tt) * P / idx.size
        th = omp_threads()
        out["cpu_baseline"] = {"value": 1.0 / sec, "unit": "frames/s", "cores": th, "kind": "oracle",
                               "sample": f"one step of {idx.size} random spheres (brute-force plain-C closest "
                                         f"points, OpenMP {th} threads), scaled to all {P}"}
    print(json.dumps(out))


def run_sdf(args):
    """The index SDF as the collision structure: per frame copy, grid update, particle sampling."""
    from synth import make_config
    t0 = time.perf_counter()
    sc = make_config(2)
    T = sc.n_frames
    frames_np = sc.frames(range(T))
    setup_s = time.perf_counter() - t0

    import torch
    import paper_2606_00444_amd as mg
    from paper_2606_00444_amd.sdf import IndexSDF
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    mg.check_device()
    D = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    frames, F, V0, particles = D(frames_np), D(sc.faces), D(sc.verts0), D(sc.queries)
    NV, NF, Q = sc.n_verts, sc.n_faces, sc.queries.shape[1]
    res, k = 64, 4
    lo_, hi_ = sc.verts0.min(1), sc.verts0.max(1)
    pad = 0.15 * (hi_ - lo_)
    lo, hi = lo_ - pad, hi_ + pad
    h = float((hi - lo).max() / (res - 1))
    dims = tuple(int(np.ceil((hi[a] - lo[a]) / h)) + 1 for a in range(3))
    S = IndexSDF(V0, F, lo, h, dims, k=k)
    live = torch.empty(3, NV, device=dev)
    dist = torch.empty(Q, device=dev)

    def step(i):
        mg.vertex_buffer_update(frames, i % T, live)
        S.update(live)
        S.sample(particles, out=dist)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    if args.eager:
        run = lambda: [step(i) for i in range(args.steps)]
    else:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for i in range(args.steps):
                step(i)
        g.replay()
        torch.cuda.synchronize()
        run = g.replay
    ms_per_step, wall = timed_region(run, args.steps, torch)

    # per-phase durations at frame 100, and the BVH path the grid would replace
    mg.vertex_buffer_update(frames, 100, live)
    bvh = mg.lbvh_build(V0, F)
    mg.lbvh_refit(bvh, live)
    rec = mg.closest_point_query(bvh, live, particles)
    ph = {"sdf_update": graph_ms(lambda _: S.update(live), 50, torch),
          "sdf_sample": graph_ms(lambda _: S.sample(particles, out=dist), 50, torch),
          "bvh_refit": graph_ms(lambda _: mg.lbvh_refit(bvh, live), 50, torch),
          "bvh_closest": graph_ms(lambda _: mg.closest_point_query(bvh, live, particles, out=rec), 20, torch)}
    S.update(live)
    S.sample(particles, out=dist)
    torch.cuda.synchronize()
    sd = dist.cpu().numpy().astype(np.float64)
    ud = np.sqrt(rec["dist2"].cpu().numpy().astype(np.float64))
    ins = np.isfinite(sd)
    gap = np.abs(np.abs(sd[ins]) - ud[ins])
    n_nodes = S.n_nodes
    alg = 24.0 * n_nodes + 12.0 * NV          # per node k=4 face ids in, value and winner out; vertices
    achieved = alg / (ph["sdf_update"] * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": round(1000.0 / ms_per_step, 2), "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"sdf: {WORKLOADS['sdf'][1]}", "grid": list(dims), "nodes": n_nodes,
                   "faces_per_node": k, "particles": Q, "timing": "eager" if args.eager else "hip-graph"},
        "kernels_ms": {kk: round(v, 5) for kk, v in ph.items()},
        "sdf_vs_bvh_distance": {"mean_abs_gap": float(gap.mean()), "p99_abs_gap": float(np.percentile(gap, 99)),
                                "grid_spacing": h, "particles_inside_grid": int(ins.sum())},
        "roofline": {"bound": "hbm", "kernel": "sdf_update_kernel", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "alg_bytes_per_launch": int(alg), "avg_launch_ms": round(ph["sdf_update"], 5)},
        "wall_s": round(wall, 4), "setup_s": round(setup_s, 2),
    }
    if not args.no_cpu_baseline:
        from oracle import sdf as osdf
        fk = S.face_k.cpu().numpy().astype(np.int64)
        P = osdf.grid_points(tuple(lo), h, dims)
        rng = np.random.default_rng(0)
        idx = rng.choice(n_nodes, min(20000, n_nodes), replace=False)
        tt = time.perf_counter()
        osdf.sdf_from_faces(frames_np[1], sc.faces, P[:, idx], fk[:, idx])
        sec = (time.perf_counter() - tt) * n_nodes / idx.size
        out["cpu_baseline"] = {"value": 1.0 / sec, "unit": "frames/s", "cores": 1, "kind": "oracle",
                               "sample": f"frame 1: float64 numpy grid update of {idx.size} random nodes (single "
                                         f"thread), scaled to all {n_nodes} (sampling not included)"}
    print(json.dumps(out))


def run_track(args):
    """Temporal correspondence tracking: one step = one frame (rebuild, query, re-anchor every 50)."""
    from synth import make_config
    t0 = time.perf_counter()
    sc = make_config(2)
    T = min(sc.n_frames, args.steps + 1)
    targets_np = make_targets(2, list(range(T)))
    setup_s = time.perf_counter() - t0

    import torch
    import paper_2606_00444_amd as mg
    from paper_2606_00444_amd.tracking import Tracker
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    mg.check_device()
    D = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    targets = [(D(v), D(f)) for v, f in targets_np]
    V0 = D(sc.verts0)
    NV = sc.n_verts
    out = torch.empty(T, 3, NV, device=dev)
    mg.vertex_buffer_update(V0.reshape(1, 3, NV), 0, out[0])
    L = float(np.ptp(sc.verts0, axis=1).max())
    tr = Tracker(V0, max(f.shape[1] for _, f in targets_np), every=50, w_track=0.8, k=args.knn, eps=1e-6 * L)
    K = T - 1

    def run_all():
        for t in range(1, T):
            tr.step(out[t - 1], targets[t][0], targets[t][1], t, out[t])

    run_all()                                               # eager warm-up pass over every frame
    torch.cuda.synchronize()
    if args.eager:
        run = run_all
    else:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            run_all()
        g.replay()
        torch.cuda.synchronize()
        run = g.replay
    ms_per_step, wall = timed_region(run, K, torch)

    # per-phase durations on frame 1: the rebuild of its BVH and the query of the tracked points
    tv, tf = targets[1]
    bvh = mg.LBVH(tf.shape[1], mg.MG_PRIM_TRIANGLES, dev, buf=tr.buf, ws=tr.ws)
    mg.lbvh_build(tv, tf, bvh=bvh)
    from paper_2606_00444_amd.api import _query_out
    rec = _query_out(NV, dev, True, False, False, False)
    if args.knn > 1:
        kq = {"face": torch.empty(args.knn, NV, dtype=torch.int32, device=dev),
              "dist2": torch.empty(args.knn, NV, device=dev), "point": rec["point"]}
        project = lambda _: mg.knn_surface_query(bvh, tv, out[0], k=args.knn, eps=1e-6 * L, out=kq)
    else:
        project = lambda _: mg.closest_point_query(bvh, tv, out[0], out=rec)
    ph = {"rebuild": graph_ms(lambda _: mg.lbvh_build(tv, tf, bvh=bvh), 50, torch),
          "query": graph_ms(project, 50, torch)}
    cnt = torch.zeros(4, dtype=torch.int64, device=dev)
    if args.knn > 1:
        mg.knn_surface_query(bvh, tv, out[0], k=args.knn, eps=1e-6 * L, out=kq, counters=cnt)
    else:
        mg.closest_point_query(bvh, tv, out[0], out=rec, counters=cnt)
    torch.cuda.synchronize()
    n_exp, n_lbox, n_lex, n_q = (int(x) for x in cnt.cpu())
    ops = OPS_EXPANSION * n_exp + OPS_LEAF_BOUND * n_lbox + OPS_EXACT * n_lex
    if ph["query"] >= ph["rebuild"]:
        achieved = ops / (ph["query"] * 1e-3) / 1e12
        kname = "knn_lane_kernel" if args.knn > 1 else "traverse_batch_kernel"
        roofline = {"bound": "alu", "kernel": f"{kname} (tracked points onto the frame's mesh)",
                    "achieved": round(achieved, 4), "peak": FP32_VECTOR_NONPACKED_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(achieved / FP32_VECTOR_NONPACKED_TFLOPS, 5), "traffic": None,
                    "alg_ops_per_launch": int(ops), "avg_launch_ms": round(ph["query"], 5)}
    else:
        tf_mean = float(np.mean([f.shape[1] for _, f in targets_np]))
        alg = 200.0 * tf.shape[1] + 12.0 * tv.shape[1]
        achieved = alg / (ph["rebuild"] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": "rebuild (all build kernels)", "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": None, "alg_bytes_per_launch": int(alg), "avg_launch_ms": round(ph["rebuild"], 5),
                    "target_faces_mean": round(tf_mean)}
    out_json = {
        "metric": METRIC, "value": round(1000.0 / ms_per_step, 2), "unit": "frames/s", "n_gpus": 1,
        "steps": K, "warmup": 1, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"track: {WORKLOADS['track'][1]}", "frames": T, "template_vertices": NV,
                   "every": 50, "w_track": 0.8, "nearest_surface": "closest point" if args.knn <= 1 else
                   f"k-NN weighted, k = {args.knn}, w = 1/(d + 1e-6 L)", "timing": "eager" if args.eager else "hip-graph"},
        "kernels_ms": {k: round(v, 5) for k, v in ph.items()},
        "queries_per_s": round(NV * 1000.0 / ms_per_step, 1),
        "traversal": {"node_expansions_per_query": round(n_exp / n_q, 1),
                      "exact_leaf_tests_per_query": round(n_lex / n_q, 1)},
        "roofline": roofline,
        "wall_s": round(wall, 4), "setup_s": round(setup_s, 2),
    }
    if not args.no_cpu_baseline:
        out_json["cpu_baseline"] = cpu_baseline_track(sc, targets_np, args.cpu_sample or 4000)
    print(json.dumps(out_json))


def cpu_baseline_track(sc, targets_np, n_sample):
    """The float64 oracle's tracking step for frame 1 on a sample of template points, scaled to frames/s."""
    from oracle import tracking as otr
    rng = np.random.default_rng(0)
    idx = rng.choice(sc.n_verts, min(n_sample, sc.n_verts), replace=False)
    tv, tf = targets_np[1]
    t = time.perf_counter()
    otr.track_step(sc.verts0[:, idx].astype(np.float64), tv.astype(np.float64), tf)
    sec = (time.perf_counter() - t) * sc.n_verts / idx.size
    th = omp_threads()
    return {"value": 1.0 / sec, "unit": "frames/s", "cores": th, "kind": "oracle",
            "sample": (f"frame 1: brute-force plain-C closest points of {idx.size} random template vertices "
                       f"(OpenMP, {th} threads), scaled to all {sc.n_verts}"),
            "wall_s": round(time.perf_counter() - t, 2)}


def run_batched(args):
    """c3: all scenes x frames in one persistent launch vs the plain per-frame path."""
    from synth import make_config
    from synth.configs import C3_SCENES
    t0 = time.perf_counter()
    scs = [make_config(3, scene=i) for i in range(len(C3_SCENES))]
    frames_np = [sc.frames(range(sc.n_frames)) for sc in scs]
    setup_s = time.perf_counter() - t0

    import torch
    import paper_2606_00444_amd as mg
    from paper_2606_00444_amd import autotune
    from paper_2606_00444_amd.batch import BatchPlan
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    mg.check_device()
    D = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    scenes = [{"frames": D(fr), "faces": D(sc.faces), "gface": D(sc.binding["face"]), "bary": D(sc.binding["bary"]),
               "q_local": D(sc.binding["q_local"]), "log_scale": D(sc.binding["log_scale"]),
               "queries": D(sc.queries)} for sc, fr in zip(scs, frames_np)]
    plan = BatchPlan(scenes)
    tune = autotune.tune_batch(plan)
    for _ in range(args.warmup):
        plan.run()
    torch.cuda.synchronize()
    if plan.status() != 0:
        raise RuntimeError(f"batched run reported status {plan.status()}")
    if args.eager:
        run = lambda: [plan.run() for _ in range(args.steps)]
    else:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(args.steps):
                plan.run()
        g.replay()
        torch.cuda.synchronize()
        run = g.replay
    ms_per_step, wall = timed_region(run, args.steps, torch)
    if plan.status() != 0:
        raise RuntimeError(f"batched run reported status {plan.status()}")

    # the plain per-frame path on the same GPU with the same per-scene traversal:
    # per scene-frame a vertex-buffer write, the re-pose, the refit and the queries
    plain = []
    for sc, s, o in zip(scs, scenes, tune["per_scene"]):
        G, Q = sc.n_gauss, sc.queries.shape[1]
        plain.append({
            "live": torch.empty(3, sc.n_verts, device=dev), "bvh": mg.lbvh_build(s["frames"][0].contiguous(), s["faces"]),
            "g": {"mean": torch.empty(3, G, device=dev), "quat": torch.empty(4, G, device=dev),
                  "cov": torch.empty(6, G, device=dev)},
            "q": {"face": torch.empty(Q, dtype=torch.int32, device=dev), "point": torch.empty(3, Q, device=dev),
                  "bary": torch.empty(2, Q, device=dev), "dist2": torch.empty(Q, device=dev),
                  "normal": torch.empty(3, Q, device=dev)},
            "opts": {"kernel": "batch", "batch": o["batch"], "seed": o["seed"]}})

    def plain_all(_=0):
        # frames in order, so (like the batched form) a scene's queries in frame t > 0
        # start from their faces of frame t - 1, the output array they overwrite
        for s, p in zip(scenes, plain):
            for t in range(s["frames"].shape[0]):
                mg.vertex_buffer_update(s["frames"], t, p["live"])
                mg.mesh_gaussian_update(p["live"], s["faces"], s["gface"], s["bary"], s["q_local"], s["log_scale"],
                                        out=p["g"])
                mg.lbvh_refit(p["bvh"], p["live"])
                mg.closest_point_query(p["bvh"], p["live"], s["queries"], normal=True, out=p["q"],
                                       hint=p["q"]["face"] if t > 0 else None, **p["opts"])

    plain_all()
    torch.cuda.synchronize()
    plain_ms = graph_ms(plain_all, 1, torch)
    SF = sum(sc.n_frames for sc in scs)
    # algorithmic bytes of one launch: per scene-frame the frame's vertices, the Gaussians
    # (40 B in, 52 B out), the refit (face indices, vertices, 48 B of records per face) and
    # the queries (12 B in, 40 B out with normals)
    alg = sum(sc.n_frames * (12.0 * sc.n_verts + 92.0 * sc.n_gauss + 12.0 * sc.n_faces + 48.0 * sc.n_faces
                             + 52.0 * sc.queries.shape[1]) for sc in scs)
    achieved = alg / (ms_per_step * 1e-3) / 1e9
    n_q = sum(sc.n_frames * sc.queries.shape[1] for sc in scs)
    out = {
        "metric": METRIC, "value": round(SF / (ms_per_step * 1e-3), 2), "unit": "scene-frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"c3: {WORKLOADS['c3'][1]}", "scenes": len(scs), "scene_frames": SF,
                   "faces": [sc.n_faces for sc in scs], "gaussians": [sc.n_gauss for sc in scs],
                   "queries": [sc.queries.shape[1] for sc in scs], "timing": "eager" if args.eager else "hip-graph"},
        "plain_path": {"ms_per_pass": round(plain_ms, 4), "scene_frames_per_s": round(SF / (plain_ms * 1e-3), 1),
                       "launches_per_pass": 4 * SF},
        "batched_speedup": round(plain_ms / ms_per_step, 3),
        "queries_per_s": round(n_q / (ms_per_step * 1e-3), 1),
        "autotuned": {"per_scene": tune["per_scene"], "gauss_tile": tune["gauss_tile"],
                      "query_tile": tune["query_tile"]},
        "roofline": {"bound": "hbm", "kernel": "batch_persistent_kernel", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("c3", "batch"), "alg_bytes_per_launch": int(alg),
                     "avg_launch_ms": round(ms_per_step, 5)},
        "wall_s": round(wall, 4), "setup_s": round(setup_s, 2),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batched(scs, frames_np, 0 if args.cpu_sample is None else args.cpu_sample)
    print(json.dumps(out))


def cpu_baseline_batched(scs, frames_np, n_sample):
    """The float64 oracle on frame 1 of every scene, scaled to scene-frames/s (n_sample <= 0: all queries)."""
    from oracle import gaussians as og, lbvh as ol, closest as oc
    t_all = time.perf_counter()
    rng = np.random.default_rng(0)
    total = 0.0
    per_scene = n_sample // len(scs) if n_sample > 0 else 0
    for sc, fr in zip(scs, frames_np):
        V = fr[1]
        t = time.perf_counter()
        og.repose(V, sc.faces, sc.binding)
        ref = ol.build(sc.verts0, sc.faces)
        ol.refit(ref["tree"], ol.leaf_boxes(V, sc.faces, ref["perm"]))
        total += time.perf_counter() - t
        q = sc.queries
        n = q.shape[1] if per_scene <= 0 else min(per_scene, q.shape[1])
        idx = rng.choice(q.shape[1], n, replace=False)
        t = time.perf_counter()
        oc.closest_point_mesh(V, sc.faces, q[:, idx])
        total += (time.perf_counter() - t) * q.shape[1] / idx.size
    th = omp_threads()
    return {"value": len(scs) / total, "unit": "scene-frames/s", "cores": th, "kind": "oracle",
            "sample": (f"frame 1 of each of the {len(scs)} scenes: float64 numpy re-pose of all Gaussians and "
                       f"the tree refit (single thread), brute-force plain-C closest points on "
                       f"{'all' if per_scene <= 0 else per_scene} queries per scene (OpenMP, {th} threads)"
                       f"{'' if per_scene <= 0 else ', scaled to the full query counts'}"),
            "wall_s": round(time.perf_counter() - t_all, 2)}


def run_refine(args):
    """c4: Adam steps of the differentiable template projection, forward + backward + update."""
    from synth import make_config
    t0 = time.perf_counter()
    sc = make_config(4)
    Y_np = sc.extra["targets"]
    setup_s = time.perf_counter() - t0

    import torch
    import paper_2606_00444_amd as mg
    from paper_2606_00444_amd.refine import TemplateRefiner
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    mg.check_device()
    D = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    V0, F, Y = D(sc.verts0), D(sc.faces), D(Y_np)
    B = {k: D(v) for k, v in sc.binding.items()}
    K = args.steps
    r = TemplateRefiner(V0, F, B, Y, max_steps=max(K, args.warmup, 1))
    r.run(args.warmup)
    torch.cuda.synchronize()
    if args.eager:
        run = lambda: r.run(K)
    else:
        g = r.capture(K)
        g.replay()
        torch.cuda.synchronize()
        run = g.replay
    ms_per_step, wall = timed_region(run, K, torch)
    hist = r.losses().numpy()[:, 3]

    # per-kernel average durations at V1, the queries starting from V0's answers as
    # in the step (each phase alone in a graph of R launches; the hints are copies,
    # restored before each Chamfer launch, so that launches do not feed each other)
    r.reset()
    r.step()
    b = B
    hint_face = r.rec["face"].clone()
    nn_ab0, nn_ba0 = r.ch["nn_ab"].clone(), r.ch["nn_ba"].clone()
    mg.lbvh_refit(r.bvh, r.V)
    mg.mesh_gaussian_update(r.V, F, b["face"], b["bary"], b["q_local"], b["log_scale"], out={"mean": r.mu},
                            quat=False, cov=False)
    mg.lbvh_refit(r.bvh_mu, r.mu)
    torch.cuda.synchronize()

    def chamfer_warm():
        r.ch["nn_ab"].copy_(nn_ab0)
        r.ch["nn_ba"].copy_(nn_ba0)
        mg.chamfer(r.mu, r.bvh_mu, Y, r.bvh_y, out=dict(r.ch), warm=True, **r.nn_query)

    reps = 50
    ph = {
        "refit": graph_ms(lambda _: mg.lbvh_refit(r.bvh, r.V), reps, torch),
        "closest": graph_ms(lambda _: mg.closest_point_query(r.bvh, r.V, Y, out=r.rec, hint=hint_face, **r.query),
                            reps, torch),
        "repose_mean": graph_ms(lambda _: mg.mesh_gaussian_update(r.V, F, b["face"], b["bary"], b["q_local"],
                                                                  b["log_scale"], out={"mean": r.mu}, quat=False,
                                                                  cov=False), reps, torch),
        "refit_mu": graph_ms(lambda _: mg.lbvh_refit(r.bvh_mu, r.mu), reps, torch),
        "chamfer": graph_ms(lambda _: chamfer_warm(), reps, torch),
        "backward": graph_ms(lambda _: (mg.point_mesh_backward(r.V, F, Y, r.rec, 1.0 / r.ny, r.gV),
                                        mg.chamfer_backward(r.mu, Y, r.ch["nn_ab"], r.ch["nn_ba"], 1.0 / r.G,
                                                            1.0 / r.ny, r.gmu),
                                        mg.mesh_gaussian_update_backward(r.V, F, b["face"], b["bary"], b["q_local"],
                                                                         b["log_scale"], None, r.gmu,
                                                                         g_verts=r.gV)), reps, torch),
        "adam": graph_ms(lambda _: mg.adam_step(r.V, r.gV, r.m, r.v, 1, 0.0), reps, torch),
    }
    r.reset()
    cnt = torch.zeros(4, dtype=torch.int64, device=dev)
    mg.lbvh_refit(r.bvh, r.V)
    mg.closest_point_query(r.bvh, r.V, Y, out=r.rec, counters=cnt, hint=hint_face, **r.query)
    torch.cuda.synchronize()
    n_exp, n_lbox, n_lex, n_q = (int(x) for x in cnt.cpu())
    ops = OPS_EXPANSION * n_exp + OPS_LEAF_BOUND * n_lbox + OPS_EXACT * n_lex
    achieved = ops / (ph["closest"] * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": round(1000.0 / ms_per_step, 2), "unit": "Adam steps/s", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"c4: {WORKLOADS['c4'][1]}", "vertices": sc.n_verts, "faces": sc.n_faces,
                   "gaussians": sc.n_gauss, "targets": int(Y_np.shape[1]), "lr": r.lr,
                   "timing": "eager" if args.eager else "hip-graph"},
        "loss": {"first": float(hist[0]), "last": float(hist[-1])},
        "kernels_ms": {k: round(v, 5) for k, v in ph.items()},
        "traversal": {"node_expansions_per_query": round(n_exp / n_q, 1),
                      "leaf_bound_tests_per_query": round(n_lbox / n_q, 1),
                      "exact_leaf_tests_per_query": round(n_lex / n_q, 1)},
        "roofline": {"bound": "alu", "kernel": "traverse_batch_kernel (targets onto the template)",
                     "achieved": round(achieved, 4), "peak": FP32_VECTOR_NONPACKED_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP32_VECTOR_NONPACKED_TFLOPS, 5), "traffic": None,
                     "alg_ops_per_launch": int(ops), "avg_launch_ms": round(ph["closest"], 5)},
        "wall_s": round(wall, 4), "setup_s": round(setup_s, 2),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_refine(sc, Y_np)
    print(json.dumps(out))


def cpu_baseline_refine(sc, Y):
    """One whole float64 oracle step at V0 (loss, analytic gradient, Adam), as Adam steps/s."""
    from oracle import losses as olo, adam as oa
    V = sc.verts0.astype(np.float64)
    t = time.perf_counter()
    _, g, _ = olo.template_loss_grad(V, sc.faces, sc.binding, Y)
    oa.adam_step(V, g, np.zeros_like(V), np.zeros_like(V), 1, 1e-3)
    sec = time.perf_counter() - t
    th = omp_threads()
    return {"value": 1.0 / sec, "unit": "Adam steps/s", "cores": th, "kind": "oracle",
            "sample": (f"one whole step at V0, unsampled: brute-force plain-C closest points of all {Y.shape[1]} "
                       f"targets and both nearest-neighbour maps (OpenMP, {th} threads), float64 numpy re-pose, "
                       f"gradients and Adam (single thread)"),
            "wall_s": round(sec, 2)}


def kernel_roofline(workload, kernel, ms, alg_bytes, coll_ops, n_queries):
    """The roofline object of the step's dominant kernel (the phase of one kernel with
    the longest average launch).  HBM-bound kernels: algorithmic bytes per launch over
    the launch time against 8 TB/s.  The collision traversal is bound by VALU issue and
    latency (the tree stays in L2/MALL; a query's compulsory traffic is 40 B): its
    algorithmic fp32 operations (an FMA counts two) per launch over the launch time,
    against the non-packed fp32 peak, with the compulsory-byte fraction beside it."""
    if kernel == "collide":
        achieved = coll_ops / (ms * 1e-3) / 1e12
        comp = QUERY_COMPULSORY_BYTES * n_queries
        r = {"bound": "alu", "kernel": "traverse_batch_kernel (collision queries)", "achieved": round(achieved, 4),
             "peak": FP32_VECTOR_NONPACKED_TFLOPS, "unit": "TFLOP/s",
             "frac": round(achieved / FP32_VECTOR_NONPACKED_TFLOPS, 5),
             "traffic": measured_traffic(workload, kernel), "alg_flops_per_launch": int(coll_ops),
             "avg_launch_ms": round(ms, 5),
             "compulsory_bytes_per_launch": int(comp),
             "hbm_frac_of_compulsory_bytes": round(comp / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)}
    else:
        achieved = alg_bytes[kernel] / (ms * 1e-3) / 1e9
        r = {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(workload, kernel),
             "alg_bytes_per_launch": int(alg_bytes[kernel]), "avg_launch_ms": round(ms, 5)}
    c = measured_counters(workload, kernel)
    if c:
        r["counters"] = c
    return r


def run_c1(args):
    """c1: the icosphere's frames through copy, re-pose, refit and collision queries,
    one frame per step; beside it the same 60 frames as one persistent launch."""
    from synth import make_config
    t0 = time.perf_counter()
    sc = make_config(1)
    T = sc.n_frames
    frames_np = sc.frames(range(T))
    setup_s = time.perf_counter() - t0

    import torch
    import paper_2606_00444_amd as mg
    from paper_2606_00444_amd import autotune
    from paper_2606_00444_amd.batch import BatchPlan
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    mg.check_device()
    D = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    frames, F, V0, particles = D(frames_np), D(sc.faces), D(sc.verts0), D(sc.queries)
    b = {k: D(v) for k, v in sc.binding.items()}
    G, Q, NV, NF = sc.n_gauss, sc.queries.shape[1], sc.n_verts, sc.n_faces
    live = torch.empty(3, NV, device=dev)
    gout = {"mean": torch.empty(3, G, device=dev), "quat": torch.empty(4, G, device=dev),
            "cov": torch.empty(6, G, device=dev)}
    col = {"face": torch.full((Q,), -1, dtype=torch.int32, device=dev), "point": torch.empty(3, Q, device=dev),
           "bary": torch.empty(2, Q, device=dev), "dist2": torch.empty(Q, device=dev),
           "normal": torch.empty(3, Q, device=dev)}
    bvh = mg.lbvh_build(V0, F)
    order_p = mg.query_order(particles)
    mg.vertex_buffer_update(frames, 0, live)
    mg.lbvh_refit(bvh, live)
    o_col = autotune.options(autotune.tune_closest(bvh, live, particles, order=order_p, normal=True), order_p)
    none_hint = torch.full((Q,), -1, dtype=torch.int32, device=dev)

    def phase_update():
        mg.mesh_gaussian_update(live, F, b["face"], b["bary"], b["q_local"], b["log_scale"], out=gout)

    def phase_collide(hint=None):
        mg.closest_point_query(bvh, live, particles, normal=True, out=col, hint=col["face"] if hint is None else hint,
                               **o_col)

    def frame_update(k):
        mg.frame_update(frames, k, live, F, b["face"], b["bary"], b["q_local"], b["log_scale"], bvh, out=gout)

    def step(i):
        frame_update(i % T)
        phase_collide()

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    if args.eager:
        run = lambda: [step(i) for i in range(args.steps)]
    else:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for i in range(args.warmup, args.warmup + args.steps):
                step(i)
        g.replay()
        torch.cuda.synchronize()
        run = g.replay
    ms_per_step, wall = timed_region(run, args.steps, torch)

    reps = 100
    ph = {"vertex_copy": graph_ms(lambda r: mg.vertex_buffer_update(frames, r % T, live), reps, torch),
          "gaussian_update": graph_ms(lambda r: phase_update(), reps, torch),
          "refit": graph_ms(lambda r: mg.lbvh_refit(bvh, live), reps, torch)}
    ph["frame_update"] = graph_ms(lambda r: frame_update(r % T), reps, torch)
    hint = col["face"].clone()
    ph["collide"] = graph_ms(lambda r: phase_collide(hint=hint), reps, torch)
    cnt = torch.zeros(4, dtype=torch.int64, device=dev)
    mg.closest_point_query(bvh, live, particles, normal=True, out=col, counters=cnt, hint=hint, **o_col)
    torch.cuda.synchronize()
    n_exp, n_lbox, n_lex, _ = (int(x) for x in cnt.cpu())
    coll_ops = OPS_EXPANSION * n_exp + OPS_LEAF_BOUND * n_lbox + OPS_EXACT * n_lex
    alg_bytes = {
        "vertex_copy": 24.0 * NV,
        "gaussian_update": 92.0 * G + 12.0 * NF + 12.0 * NV,
        "refit": 12.0 * NV + 12.0 * NF + 48.0 * NF,
        # the minimum per frame of the refit path: vertices once, face indices once and
        # the 64 B of records per face, the Gaussians' 40 B in and 52 B out
        "frame_update": 12.0 * NV + 76.0 * NF + 92.0 * G,
        "collide": 52.0 * Q,
    }
    kernels = {}
    for k, ms in ph.items():
        gbs = alg_bytes[k] / (ms * 1e-3) / 1e9
        kernels[k] = {"ms": round(ms, 5), "alg_bytes": int(alg_bytes[k]), "GB_s": round(gbs, 1),
                      "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    single = {k: ph[k] for k in ("gaussian_update", "refit", "frame_update", "collide")}
    dom = max(single, key=single.get)

    # the same 60 frames as one persistent launch (re-pose, refit, queries per frame)
    scene = {"frames": frames, "faces": F, "gface": b["face"], "bary": b["bary"], "q_local": b["q_local"],
             "log_scale": b["log_scale"], "queries": particles}
    plan = BatchPlan([scene])
    autotune.tune_batch(plan)
    plan.run()
    torch.cuda.synchronize()
    if plan.status() != 0:
        raise RuntimeError(f"batched run reported status {plan.status()}")
    batch_ms = graph_ms(lambda r: plan.run(), 20, torch)
    b_alg = T * (12.0 * NV + 92.0 * G + 12.0 * NF + 48.0 * NF + 52.0 * Q)
    out = {
        "metric": METRIC, "value": round(1000.0 / ms_per_step, 2), "unit": "frames/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"c1: {WORKLOADS['c1'][1]}", "frames": T, "vertices": NV, "faces": NF,
                   "gaussians": G, "queries": Q, "timing": "eager" if args.eager else "hip-graph"},
        "frame_update": dict(kernels["frame_update"], what="vertex copy, Gaussian re-pose, refit in one launch"),
        "queries_per_s": round(Q * 1000.0 / ms_per_step, 1),
        "traversal": {"node_expansions_per_query": round(n_exp / Q, 1),
                      "leaf_bound_tests_per_query": round(n_lbox / Q, 1),
                      "exact_leaf_tests_per_query": round(n_lex / Q, 1)},
        "batched": {"what": f"all {T} frames in one persistent launch", "ms_per_launch": round(batch_ms, 5),
                    "frames_per_s": round(T / (batch_ms * 1e-3), 1), "alg_bytes": int(b_alg),
                    "hbm_frac": round(b_alg / (batch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "kernels": kernels,
        "roofline": kernel_roofline("c1", dom, ph[dom], alg_bytes, coll_ops, Q),
        "wall_s": round(wall, 4), "setup_s": round(setup_s, 2),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_c1(sc, frames_np)
    print(json.dumps(out))


def cpu_baseline_c1(sc, frames_np, reps=5):
    """The float64 oracle on frames 1..reps of c1 (re-pose, refit, every query), all
    host cores and one thread for the queries; medians over the frames."""
    from oracle import gaussians as og, lbvh as ol, closest as oc, frame as ofr
    t_all = time.perf_counter()
    ref = ol.build(sc.verts0, sc.faces)
    cores = omp_threads()
    tot = {"all": [], "one": []}
    try:
        for f in range(1, reps + 1):
            t = time.perf_counter()
            live = ofr.vertex_buffer_update(frames_np, f)
            og.repose(live, sc.faces, sc.binding)
            ol.refit(ref["tree"], ol.leaf_boxes(frames_np[f], sc.faces, ref["perm"]))
            host_s = time.perf_counter() - t
            for key, th in (("all", cores), ("one", 1)):
                oc.set_threads(th)
                t = time.perf_counter()
                oc.closest_point_mesh(frames_np[f], sc.faces, sc.queries)
                tot[key].append(host_s + time.perf_counter() - t)
    finally:
        oc.set_threads(cores)
    return {"value": 1.0 / float(np.median(tot["all"])), "unit": "frames/s", "cores": cores, "kind": "oracle",
            "sample": f"median of {reps} whole frames (1-{reps}): float64 numpy re-pose and refit (one thread), "
                      f"plain-C brute-force closest points of all {sc.queries.shape[1]} queries ({cores} threads)",
            "single_thread": {"value": 1.0 / float(np.median(tot["one"])), "unit": "frames/s", "cores": 1,
                              "sample": "the same frames with the queries on one thread"},
            "wall_s": round(time.perf_counter() - t_all, 2)}


def per_query_distribution(mg, torch, bvh, verts, queries, opts, hint, out, sample):
    """Node expansions and exact leaf tests per query over a seeded sample of the query
    set: each sampled query is traversed alone (same options, its own previous-frame hint),
    with its own counter row, and the percentiles of the counts are reported."""
    rng = np.random.default_rng(20260603)
    n = queries.shape[1]
    idx = np.sort(rng.choice(n, min(sample, n), replace=False))
    dev = queries.device
    qs = [queries[:, i:i + 1].contiguous() for i in idx]
    hs = [hint[i:i + 1].contiguous() for i in idx]
    one = {"face": torch.empty(1, dtype=torch.int32, device=dev), "point": torch.empty(3, 1, device=dev),
           "bary": torch.empty(2, 1, device=dev), "dist2": torch.empty(1, device=dev),
           "normal": torch.empty(3, 1, device=dev) if out.get("normal") is not None else None}
    cnt = torch.zeros(len(idx), 4, dtype=torch.int64, device=dev)
    for j in range(len(idx)):
        mg.closest_point_query(bvh, verts, qs[j], normal=one["normal"] is not None, out=one, counters=cnt[j],
                               hint=hs[j], **opts)
    c = cnt.cpu().numpy()
    pct = lambda x: {f"p{p}": float(np.percentile(x, p)) for p in (10, 50, 90, 99)} | {"max": int(x.max()),
                                                                                       "mean": float(x.mean())}
    return {"sample": int(len(idx)), "how": "each sampled query traversed alone with the step's options and its "
                                            "previous-frame hint (frame in the middle of the sampled ones)",
            "node_expansions": pct(c[:, 0]), "exact_leaf_tests": pct(c[:, 2])}


def copy_calibration(mb, reps):
    """A plain copy of known size (the vertex-buffer copy kernel): reads and writes mb MB per launch.
    Its FETCH_SIZE / WRITE_SIZE counters calibrate the counters of the other kernels."""
    import torch
    import paper_2606_00444_amd as mg
    dev = torch.device("cuda:0")
    n = (mb * 1000 * 1000) // 12                     # vertices of 12 B
    frames = torch.rand(2, 3, n, device=dev)
    live = torch.empty(3, n, device=dev)
    for r in range(reps):
        mg.vertex_buffer_update(frames, r % 2, live)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read_per_launch": 12 * n, "bytes_written_per_launch": 12 * n,
                                           "reps": reps}}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default per workload)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed warm-up steps (default per workload)")
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="queries the oracle baseline runs per query set (default: c2 all, c5 8000, c3 all)")
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of a HIP graph")
    ap.add_argument("--streams", type=int, choices=(1, 2, 3), default=3,
                    help="c2/c5: run the rebuild comparison path on a second stream (2), also the projection "
                         "onto the rebuilt target on a third (3), or everything serially (1)")
    ap.add_argument("--phase", choices=["copy", "update", "refit", "frame_update", "collide", "rebuild",
                                        "target_queries"],
                    help="profiling aid (c2/c5): run only this phase --reps times, eagerly, and exit")
    ap.add_argument("--reps", type=int, default=60)
    ap.add_argument("--knn", type=int, default=1, help="track: NearestSurface with the k nearest faces (1-8)")
    ap.add_argument("--copy-calibration", type=int, metavar="MB", default=0,
                    help="profiling aid: copy MB megabytes with the vertex-buffer copy kernel --reps times and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration, args.reps)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    steps, warmup = DEFAULT_STEPS[args.workload]
    args.steps = steps if args.steps is None else args.steps
    args.warmup = warmup if args.warmup is None else args.warmup
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c1":
        return run_c1(args)
    if args.workload == "c3":
        return run_batched(args)
    if args.workload == "c4":
        return run_refine(args)
    if args.workload == "track":
        return run_track(args)
    if args.workload == "sdf":
        return run_sdf(args)
    if args.workload == "contact":
        return run_contact(args)
    cfg, desc = WORKLOADS[args.workload]

    from synth import make_config
    t0 = time.perf_counter()
    sc = make_config(cfg)
    T = sc.n_frames
    # frames (and varying-topology targets) the run touches; a single-phase profiling run needs one
    n_used = 1 if args.phase else min(T, max(args.steps, args.warmup))
    frame_ids = list(range(n_used))
    frames_np = sc.frames(range(T))
    targets_np = make_targets(cfg, frame_ids)
    setup_s = time.perf_counter() - t0

    import torch
    import paper_2606_00444_amd as mg
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    mg.check_device()
    D = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)

    frames = D(frames_np)                                   # [T][3][V]
    F = D(sc.faces)
    b = {k: D(v) for k, v in sc.binding.items()}
    particles = D(sc.queries)
    V0 = D(sc.verts0)
    live = torch.empty(3, sc.n_verts, device=dev)
    G, Q, NV, NF = sc.n_gauss, sc.queries.shape[1], sc.n_verts, sc.n_faces
    gout = {"mean": torch.empty(3, G, device=dev), "quat": torch.empty(4, G, device=dev),
            "cov": torch.empty(6, G, device=dev)}

    def qout(n, normal):
        return {"face": torch.empty(n, dtype=torch.int32, device=dev), "point": torch.empty(3, n, device=dev),
                "bary": torch.empty(2, n, device=dev), "dist2": torch.empty(n, device=dev),
                "normal": torch.empty(3, n, device=dev) if normal else None}

    col = qout(Q, True)
    col["face"].fill_(-1)                                   # no previous frame yet: no hints
    col_t = qout(Q, True)
    proj = qout(NV, False)
    tgt_v = [D(v) for v, _ in targets_np]
    tgt_f = [D(f) for _, f in targets_np]
    max_tf = max(f.shape[1] for _, f in targets_np)
    tbuf = torch.empty(mg.lbvh_bytes(max_tf), dtype=torch.uint8, device=dev)
    tws = torch.empty(mg.lbvh_workspace_bytes(max_tf), dtype=torch.uint8, device=dev)
    tbvh = [mg.LBVH(f.shape[1], mg.MG_PRIM_TRIANGLES, dev, buf=tbuf, ws=tws) for _, f in targets_np]
    bvh = mg.lbvh_build(V0, F)                              # init: built once from the template (F_0)
    # init-time choices (untimed): Morton processing order of the fixed query sets,
    # and the traversal autotuned per query set on the first frame
    from paper_2606_00444_amd import autotune
    order_p = mg.query_order(particles)
    order_v0 = mg.query_order(V0)
    mg.vertex_buffer_update(frames, 0, live)
    mg.lbvh_refit(bvh, live)
    mg.lbvh_build(tgt_v[0], tgt_f[0], bvh=tbvh[0])
    tune = {
        "collide": autotune.tune_closest(bvh, live, particles, order=order_p, normal=True),
        "collide_target": autotune.tune_closest(tbvh[0], tgt_v[0], particles, order=order_p, normal=True),
        "project": autotune.tune_closest(tbvh[0], tgt_v[0], V0, order=order_v0),
    }
    o_col = autotune.options(tune["collide"], order_p)
    o_ct = autotune.options(tune["collide_target"], order_p)
    o_pr = autotune.options(tune["project"], order_v0)
    torch.cuda.synchronize()

    def phase_copy(k):
        mg.vertex_buffer_update(frames, k, live)

    def phase_update():
        mg.mesh_gaussian_update(live, F, b["face"], b["bary"], b["q_local"], b["log_scale"], out=gout)

    def phase_refit():
        mg.lbvh_refit(bvh, live)

    def phase_collide(counters=None, hint=None):
        # each particle starts from its face of the previous frame (the step's own
        # output array, which the call overwrites), unless a hint array is given
        mg.closest_point_query(bvh, live, particles, normal=True, out=col, counters=counters,
                               hint=col["face"] if hint is None else hint, **o_col)

    def phase_rebuild(j):
        mg.lbvh_build(tgt_v[j], tgt_f[j], bvh=tbvh[j])

    def phase_collide_target(j):
        mg.closest_point_query(tbvh[j], tgt_v[j], particles, normal=True, out=col_t, **o_ct)

    def phase_project(j):
        mg.closest_point_query(tbvh[j], tgt_v[j], V0, out=proj, **o_pr)

    def phase_target_queries(j):
        phase_collide_target(j)
        phase_project(j)

    # The refit path (template) and the rebuild comparison path (varying target) share
    # no data: with --streams 2 or 3 the rebuild path runs on a second HIP stream (default
    # priority), forked from and joined back into the launch stream every step, so each
    # path's kernels can use compute units the other leaves idle.  With --streams 3 the
    # two query sets against the rebuilt target (particles, template vertices) also run
    # side by side, the projection on a third stream forked after the rebuild.
    side = torch.cuda.Stream() if args.streams >= 2 else None
    side2 = torch.cuda.Stream() if args.streams == 3 else None
    def frame_update(k):
        """The frame update in one launch: copy frame k, re-pose the Gaussians, refit
        (mg_frame_update; bitwise the three separate calls, timed alone below)."""
        mg.frame_update(frames, k, live, F, b["face"], b["bary"], b["q_local"], b["log_scale"], bvh, out=gout)

    def step(i):
        # simulation runs at the reconstruction rate: step i at f_sim = f_recon -> frame i (mod T)
        k = mg.frame_index(i % T, 30, 1, 30, T)
        j = k % n_used
        if side is None:
            frame_update(k)
            phase_collide()
            phase_rebuild(j)
            phase_target_queries(j)
            return
        main = torch.cuda.current_stream()
        side.wait_stream(main)
        with torch.cuda.stream(side):
            phase_rebuild(j)
            if side2 is not None:
                side2.wait_stream(side)
                with torch.cuda.stream(side2):
                    phase_project(j)
                phase_collide_target(j)
            else:
                phase_target_queries(j)
        frame_update(k)
        phase_collide()
        main.wait_stream(side)
        if side2 is not None:
            main.wait_stream(side2)

    # A collision launch timed alone starts from the previous frame's answers, as
    # in the step (a copy, so that repeated launches do not feed each other).
    def prev_hints(f):
        phase_copy(max(f - 1, 0))
        phase_refit()
        phase_collide(hint=none_hint)
        h = col["face"].clone()
        phase_copy(f)
        phase_refit()
        return h

    none_hint = torch.full((Q,), -1, dtype=torch.int32, device=dev)

    if args.phase:
        # profiling aid: one phase alone, eagerly, so per-dispatch counters see only it
        frames_c = sample_frames(T)
        hints_c = [prev_hints(f) for f in frames_c] if args.phase == "collide" else None

        def collide_at(r):             # one collision launch per sampled frame, cyclically
            phase_copy(frames_c[r % len(frames_c)])
            phase_refit()
            phase_collide(hint=hints_c[r % len(frames_c)])

        phases = {"copy": lambda r: phase_copy(r % T), "update": lambda r: phase_update(),
                  "refit": lambda r: phase_refit(), "frame_update": lambda r: frame_update(r % T),
                  "collide": collide_at,
                  "rebuild": lambda r: phase_rebuild(r % n_used), "target_queries": lambda r: phase_target_queries(0)}
        phase_copy(0)
        phase_rebuild(0)
        for r in range(args.reps):
            phases[args.phase](r)
        torch.cuda.synchronize()
        print(json.dumps({"phase": args.phase, "reps": args.reps, "workload": args.workload,
                          "autotuned": {k: {"kernel": v["kernel"], "batch": v["batch"], "seed": v["seed"], "dynamic": v.get("dynamic", False),
                                            "order": v["order"]} for k, v in tune.items()}}))
        return
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    if args.eager:
        run = lambda: [step(i) for i in range(args.steps)]
    else:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for i in range(args.steps):
                step(i)
        g.replay()                                          # untimed replay (first replay uploads the graph)
        torch.cuda.synchronize()
        run = g.replay
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(stream)
    run()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    total_ms = e0.elapsed_time(e1)
    ms_per_step = total_ms / args.steps

    # per-phase and per-kernel average durations: each phase captured alone, R launches
    # back to back in one graph, timed with HIP events on the launch stream
    def timed(fn, reps):
        gg = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gg):
            for r in range(reps):
                fn(r)
        gg.replay()
        torch.cuda.synchronize()
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        gg.replay()
        z.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(z) / reps

    reps = max(20, min(200, args.steps))
    phase_copy(0)
    ph = {
        "vertex_copy": timed(lambda r: phase_copy(r % T), reps),
        "gaussian_update": timed(lambda r: phase_update(), reps),
        "refit": timed(lambda r: phase_refit(), reps),
        "rebuild": timed(lambda r: phase_rebuild(r % n_used), reps),
    }
    # the whole frame update (copy, re-pose, refit) as the step runs it
    ph["frame_update"] = timed(lambda r: frame_update(r % T), reps)
    # the collision query's cost follows the deformation: average it over frames
    # spread across the sequence (the same frames a --phase collide run cycles through)
    per_frame = []
    for f in sample_frames(T):
        h = prev_hints(f)
        per_frame.append(timed(lambda r: phase_collide(hint=h), max(10, reps // 6)))
    ph["collide"] = float(np.mean(per_frame))
    # the target BVHs share one buffer: time their queries on one freshly built target
    phase_rebuild(0)
    ph["target_queries"] = timed(lambda r: phase_target_queries(0), reps)
    # The paper's comparison on like terms: the same deformed template per frame, its
    # tree refit or rebuilt from scratch, and the same collision queries without
    # previous-frame hints on either tree.
    tmpl_rb = mg.LBVH(NF, mg.MG_PRIM_TRIANGLES, dev)
    like = {}
    for f in sample_frames(T):
        phase_copy(f)
        phase_refit()
        mg.lbvh_build(live, F, bvh=tmpl_rb)
        r_ms = timed(lambda r: phase_refit(), reps)
        b_ms = timed(lambda r: mg.lbvh_build(live, F, bvh=tmpl_rb), reps)
        qr = timed(lambda r: phase_collide(hint=none_hint), max(10, reps // 6))
        qb = timed(lambda r: mg.closest_point_query(tmpl_rb, live, particles, normal=True, out=col_t, **o_col),
                   max(10, reps // 6))
        for k, v in (("refit", r_ms), ("rebuild", b_ms), ("collide_refit_tree", qr), ("collide_rebuilt_tree", qb)):
            like.setdefault(k, []).append(v)
    like = {k: float(np.mean(v)) for k, v in like.items()}
    fu_ms = ph["vertex_copy"] + ph["gaussian_update"]
    refit_vs_rebuild = {
        "what": "same deformed template per frame (6 frames across the sequence): copy + re-pose, then the tree "
                "refit or rebuilt, then the collision queries without hints; kernel averages from HIP graphs",
        "refit_ms": round(like["refit"], 5), "rebuild_ms": round(like["rebuild"], 5),
        "collide_refit_tree_ms": round(like["collide_refit_tree"], 5),
        "collide_rebuilt_tree_ms": round(like["collide_rebuilt_tree"], 5),
        "refit_frame_ms": round(fu_ms + like["refit"] + like["collide_refit_tree"], 5),
        "rebuild_frame_ms": round(fu_ms + like["rebuild"] + like["collide_rebuilt_tree"], 5),
    }
    refit_vs_rebuild["tree_speedup"] = round(like["rebuild"] / like["refit"], 3)
    refit_vs_rebuild["frame_speedup"] = round(refit_vs_rebuild["rebuild_frame_ms"] / refit_vs_rebuild["refit_frame_ms"], 3)
    phase_copy(0)
    phase_refit()
    tf_mean = float(np.mean([f.shape[1] for _, f in targets_np]))
    tv_mean = float(np.mean([v.shape[1] for v, _ in targets_np]))
    alg_bytes = {
        "vertex_copy": 24.0 * NV,
        "gaussian_update": 92.0 * G + 12.0 * NF + 12.0 * NV,
        "refit": 12.0 * NV + 12.0 * NF + 48.0 * NF,
        # the minimum per frame of the refit path: vertices once, face indices once and
        # the 64 B of records per face, the Gaussians' 40 B in and 52 B out
        "frame_update": 12.0 * NV + 76.0 * NF + 92.0 * G,
        "collide": 52.0 * Q,
        "rebuild": 200.0 * tf_mean + 12.0 * tv_mean,
    }
    kernels = {}
    for k, ms in ph.items():
        e = {"ms": round(ms, 5)}
        if k in alg_bytes:
            gbs = alg_bytes[k] / (ms * 1e-3) / 1e9
            e.update({"alg_bytes": int(alg_bytes[k]), "GB_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)})
        kernels[k] = e
    refit_path_ms = ph["frame_update"] + ph["collide"]
    rebuild_path_ms = ph["rebuild"] + ph["target_queries"]
    # traversal statistics of one collision launch (outside the timed region)
    # traversal statistics over the same sampled frames (counters accumulate across launches)
    cnt = torch.zeros(4, dtype=torch.int64, device=dev)
    frames_c = sample_frames(T)
    for f in frames_c:
        h = prev_hints(f)
        phase_collide(cnt, hint=h)
    torch.cuda.synchronize()
    n_exp, n_lbox, n_lex, n_q = (int(x) for x in cnt.cpu())
    n_exp, n_lbox, n_lex = (x / len(frames_c) for x in (n_exp, n_lbox, n_lex))   # per launch
    n_q //= len(frames_c)
    trav = {"node_expansions_per_query": round(n_exp / n_q, 1), "leaf_bound_tests_per_query": round(n_lbox / n_q, 1),
            "exact_leaf_tests_per_query": round(n_lex / n_q, 1)}
    trav["per_query_distribution"] = per_query_distribution(
        mg, torch, bvh, live, particles, dict(o_col, order=None), prev_hints(frames_c[len(frames_c) // 2]),
        {k: v for k, v in col.items()}, 1000)
    phase_copy(0)
    phase_refit()
    coll_ops = OPS_EXPANSION * n_exp + OPS_LEAF_BOUND * n_lbox + OPS_EXACT * n_lex
    single = {k: ph[k] for k in ("gaussian_update", "refit", "frame_update", "collide")}   # one kernel each
    dom = max(single, key=single.get)
    roofline = kernel_roofline(args.workload, dom, ph[dom], alg_bytes, coll_ops, Q)
    q_per_frame = 2 * Q + NV
    fps = 1000.0 / ms_per_step
    out = {
        "metric": METRIC,
        "value": round(fps, 2), "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "frames": T, "vertices": NV, "faces": NF,
                   "gaussians": G, "particles": Q, "template_vertices_projected": NV,
                   "target_faces_mean": round(tf_mean), "timing": "eager" if args.eager else "hip-graph",
                   "streams": args.streams},
        "refit_path": {"ms_per_frame": round(refit_path_ms, 5), "frames_per_s": round(1000.0 / refit_path_ms, 1),
                       "what": "frame update + collision queries from the previous frame's faces"},
        "frame_update": dict(kernels["frame_update"], what="vertex copy, Gaussian re-pose, refit in one launch"),
        "rebuild_path": {"ms_per_frame": round(rebuild_path_ms, 5), "frames_per_s": round(1000.0 / rebuild_path_ms, 1),
                         "what": "varying-topology target: rebuild, collision queries and template projection "
                                 "onto it (no hints exist across topologies)"},
        "refit_vs_rebuild": refit_vs_rebuild,
        "queries_per_s": round(q_per_frame * fps, 1),
        "collide_queries_per_s": round(Q / (ph["collide"] * 1e-3), 1),
        "traversal": trav,
        "autotuned": {k: {"kernel": v["kernel"], "batch": v["batch"], "seed": v["seed"], "dynamic": v.get("dynamic", False), "order": v["order"],
                          "ms": round(v["ms"], 4)}
                      for k, v in tune.items()},
        "kernels": kernels,
        "roofline": roofline,
        "paper_context": {"fixed_topology_fps": 147.8, "varying_topology_fps": 31.8, "hardware": "not stated"},
        "wall_s": round(wall, 4), "setup_s": round(setup_s, 2),
    }
    if not args.no_cpu_baseline:
        # about 2 s per frame on 16 host cores at C2 (a quarter of each query set), and
        # 1,000 queries per set on one thread; C5 samples 4,000 and 250 queries per set
        # (its host phases alone take seconds per frame)
        n_all = args.cpu_sample or (12_500 if args.workload == "c2" else 4_000)
        out["cpu_baseline"] = cpu_baseline(sc, frames_np, make_targets(cfg, range(6)) if n_used < 6 else targets_np,
                                           n_all, max(50, n_all // (12 if args.workload == "c2" else 16)))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
