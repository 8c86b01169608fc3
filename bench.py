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

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c1|c5]
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
FP32_VECTOR_PEAK_TFLOPS = 157.3
WORKLOADS = {
    "c1": (1, "icosphere 2,562 V / 5,120 F, 30,720 Gaussians, 10,000 queries, 60 frames"),
    "c2": (2, "UV-sphere template 20,002 V / 40,000 F, 100,000 Gaussians, 50,000 particles, "
              "200 frames, marching-tetrahedra targets ~46-53k F"),
    "c5": (5, "UV-sphere 250,002 V / 500,000 F, 1,000,000 Gaussians, 1,000,000 queries, 100 frames, "
              "1,000,000-face split rebuild targets"),
}


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
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_target_job, [(cfg, t) for t in ts])


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {
    "gaussian_update": ["paper_2606_00444_amd/csrc/gaussian.hip", "paper_2606_00444_amd/csrc/mgu_internal.hpp"],
    "refit": ["paper_2606_00444_amd/csrc/lbvh.hip", "paper_2606_00444_amd/csrc/mgu_internal.hpp"],
    "collide": ["paper_2606_00444_amd/csrc/query.hip", "paper_2606_00444_amd/csrc/mgu_internal.hpp"],
}


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it still matches the source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_hash") != source_hash(KERNEL_SOURCES.get(kernel, [])):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(sc, frames_np, targets_np, n_sample):
    """The float64 oracle on a bounded sample of one frame, scaled to frames/s."""
    from oracle import gaussians as og, lbvh as ol, closest as oc, frame as ofr
    t_all = time.perf_counter()
    V = frames_np[1]
    tv, tf = targets_np[1]
    timings = {}
    t = time.perf_counter()
    live = ofr.vertex_buffer_update(frames_np, 1)
    og.repose(live, sc.faces, sc.binding)
    timings["update"] = time.perf_counter() - t
    ref = ol.build(sc.verts0, sc.faces)
    t = time.perf_counter()
    ol.refit(ref["tree"], ol.leaf_boxes(V, sc.faces, ref["perm"]))
    timings["refit"] = time.perf_counter() - t
    t = time.perf_counter()
    ol.build(tv, tf)
    timings["rebuild"] = time.perf_counter() - t
    rng = np.random.default_rng(0)
    qs = [(V, sc.faces, sc.queries), (tv, tf, sc.queries), (tv, tf, sc.verts0)]
    for name, (mv, mf, q) in zip(("collide", "collide_target", "project"), qs):
        idx = rng.choice(q.shape[1], min(n_sample, q.shape[1]), replace=False)
        t = time.perf_counter()
        oc.closest_point_mesh(mv, mf, q[:, idx])
        timings[name] = (time.perf_counter() - t) * q.shape[1] / idx.size
    per_frame = sum(timings.values())
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": 1.0 / per_frame, "unit": "frames/s", "cores": threads, "kind": "oracle",
        "sample": (f"one frame: float64 numpy re-pose of all {sc.n_gauss} Gaussians, refit and rebuild "
                   f"(single thread); brute-force plain-C closest points on {n_sample} random queries per "
                   f"query set (OpenMP, {threads} threads), scaled to the full query counts"),
        "seconds": {k: round(v, 4) for k, v in timings.items()},
        "wall_s": round(time.perf_counter() - t_all, 2),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=8000)
    ap.add_argument("--eager", action="store_true", help="time eager launches instead of a HIP graph")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    cfg, desc = WORKLOADS[args.workload]

    from synth import make_config
    t0 = time.perf_counter()
    sc = make_config(cfg)
    T = sc.n_frames
    n_used = min(T, max(args.steps, args.warmup))
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

    def phase_collide(counters=None):
        mg.closest_point_query(bvh, live, particles, normal=True, out=col, counters=counters, **o_col)

    def phase_rebuild(j):
        mg.lbvh_build(tgt_v[j], tgt_f[j], bvh=tbvh[j])

    def phase_target_queries(j):
        mg.closest_point_query(tbvh[j], tgt_v[j], particles, normal=True, out=col_t, **o_ct)
        mg.closest_point_query(tbvh[j], tgt_v[j], V0, out=proj, **o_pr)

    def step(i):
        # simulation runs at the reconstruction rate: step i at f_sim = f_recon -> frame i (mod T)
        k = mg.frame_index(i % T, 30, 1, 30, T)
        j = k % n_used
        phase_copy(k)
        phase_update()
        phase_refit()
        phase_collide()
        phase_rebuild(j)
        phase_target_queries(j)

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
        "collide": timed(lambda r: phase_collide(), reps),
        "rebuild": timed(lambda r: phase_rebuild(r % n_used), reps),
    }
    # the target BVHs share one buffer: time their queries on one freshly built target
    phase_rebuild(0)
    ph["target_queries"] = timed(lambda r: phase_target_queries(0), reps)
    tf_mean = float(np.mean([f.shape[1] for _, f in targets_np]))
    tv_mean = float(np.mean([v.shape[1] for v, _ in targets_np]))
    alg_bytes = {
        "vertex_copy": 24.0 * NV,
        "gaussian_update": 92.0 * G + 12.0 * NF + 12.0 * NV,
        "refit": 12.0 * NV + 12.0 * NF + 48.0 * NF,
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
    refit_path_ms = ph["vertex_copy"] + ph["gaussian_update"] + ph["refit"] + ph["collide"]
    rebuild_path_ms = ph["rebuild"] + ph["target_queries"]
    # traversal statistics of one collision launch (outside the timed region)
    cnt = torch.zeros(4, dtype=torch.int64, device=dev)
    phase_collide(cnt)
    torch.cuda.synchronize()
    n_exp, n_lbox, n_lex, n_q = (int(x) for x in cnt.cpu())
    trav = {"node_expansions_per_query": round(n_exp / n_q, 1), "leaf_bound_tests_per_query": round(n_lbox / n_q, 1),
            "exact_leaf_tests_per_query": round(n_lex / n_q, 1)}
    # algorithmic float32 operations per unit: expansion = two child box
    # distances (34), leaf bound = triangle bounds + box distance (29), exact test (80)
    coll_ops = 34.0 * n_exp + 29.0 * n_lbox + 80.0 * n_lex
    single = {k: ph[k] for k in ("gaussian_update", "refit", "collide")}   # one kernel per launch
    dom = max(single, key=single.get)
    if dom == "collide":
        achieved = coll_ops / (ph[dom] * 1e-3) / 1e12
        roofline = {"bound": "alu", "kernel": "traverse_batch_kernel (collision queries)", "achieved": round(achieved, 4),
                    "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 5),
                    "traffic": measured_traffic(dom), "alg_ops_per_launch": int(coll_ops),
                    "avg_launch_ms": round(ph[dom], 5), "hbm_frac_of_compulsory_bytes": kernels["collide"]["hbm_frac"]}
    else:
        achieved = alg_bytes[dom] / (ph[dom] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom),
                    "alg_bytes_per_launch": int(alg_bytes[dom]), "avg_launch_ms": round(ph[dom], 5)}
    q_per_frame = 2 * Q + NV
    fps = 1000.0 / ms_per_step
    out = {
        "metric": "frames/s and closest-point queries/s, refit vs rebuild; achieved HBM GB/s",
        "value": round(fps, 2), "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "frames": T, "vertices": NV, "faces": NF,
                   "gaussians": G, "particles": Q, "template_vertices_projected": NV,
                   "target_faces_mean": round(tf_mean), "timing": "eager" if args.eager else "hip-graph"},
        "refit_path": {"ms_per_frame": round(refit_path_ms, 5), "frames_per_s": round(1000.0 / refit_path_ms, 1)},
        "rebuild_path": {"ms_per_frame": round(rebuild_path_ms, 5), "frames_per_s": round(1000.0 / rebuild_path_ms, 1)},
        "queries_per_s": round(q_per_frame * fps, 1),
        "collide_queries_per_s": round(Q / (ph["collide"] * 1e-3), 1),
        "traversal": trav,
        "autotuned": {k: {"kernel": v["kernel"], "batch": v["batch"], "seed": v["seed"], "order": v["order"],
                          "ms": round(v["ms"], 4)}
                      for k, v in tune.items()},
        "kernels": kernels,
        "roofline": roofline,
        "paper_context": {"fixed_topology_fps": 147.8, "varying_topology_fps": 31.8, "hardware": "not stated"},
        "wall_s": round(wall, 4), "setup_s": round(setup_s, 2),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, frames_np, targets_np, args.cpu_sample)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
