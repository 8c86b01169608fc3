"""Autotuner for the closest-point / nearest-point traversal.

For a given BVH and query set it times every candidate traversal (one query per
lane, or one wave per batch of 1-16 queries with or without the greedy seed
descent, with batches dealt statically or taken from a work counter; in the
given query order or a supplied one such as Morton order), each
as a HIP graph of back-to-back launches bracketed by HIP events
on the launch stream, and keeps the fastest.  Choices are cached per device,
primitive kind, primitive count, query count and ordering in a JSON file
(MGU_AUTOTUNE_CACHE, default ~/.cache/mgu_autotune.json), so a workload is
tuned once.  Results never depend on the choice except among exact ties.
"""

import json
import os

import torch

from . import api

CANDIDATES = ([("lane", 0, False, False)] + [("batch", b, s, False) for b in (1, 2, 4, 8, 16) for s in (False, True)]
              + [("batch", b, True, True) for b in (2, 4, 8, 16)])


def _cache_path():
    return os.environ.get("MGU_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "mgu_autotune.json"))


def _load_cache():
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(cache):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def _graph_time(fn, reps):
    """Average milliseconds of fn over a HIP graph of `reps` launches."""
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    g.replay()
    z.record(s)
    torch.cuda.synchronize()
    return a.elapsed_time(z) / reps


def _key(kind, bvh, queries, ordered, extra=""):
    dev = torch.cuda.get_device_properties(queries.device)
    arch = getattr(dev, "gcnArchName", dev.name)
    return f"{arch}|{kind}|n={bvh.n}|q={queries.shape[1]}|ordered={int(ordered)}{extra}"


def _tune(key, run, orders, candidates, reps, use_cache):
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return cache[key]
    timings = {}
    for oname, order in orders.items():
        for kernel, batch, seed, dyn in candidates or CANDIDATES:
            timings[f"{kernel}/{batch}/{int(seed)}/{int(dyn)}/{oname}"] = _graph_time(
                lambda: run(kernel=kernel, batch=batch, seed=seed, dynamic=dyn, order=order), reps)
    best = min(timings, key=timings.get)
    k, b, s, d, o = best.split("/")
    res = {"kernel": k, "batch": int(b), "seed": bool(int(s)), "dynamic": bool(int(d)), "order": o,
           "ms": timings[best], "timings": timings}
    if use_cache:
        cache = _load_cache()
        cache[key] = res
        _store_cache(cache)
    return res


def tune_closest(bvh, verts, queries, *, order=None, normal=False, reps=5, use_cache=True, candidates=None,
                 waves=0):
    """Best traversal options for mg_closest_point_query on this BVH and query set.

    order: an optional processing order to consider besides the given one (e.g.
    query_order(queries)); the result's "order" is "given" or "order".  Returns
    {"kernel", "batch", "seed", "order", "ms", "timings"}; options(res, order)
    gives the keyword arguments for closest_point_query.  waves: the batch
    kernel's register allocation to time (0: by launch size, as the plain call).
    """
    orders = {"given": None} if order is None else {"given": None, "order": order}
    key = _key("closest", bvh, queries, order is not None, f"|normal={int(normal)}" + (f"|waves={waves}" if waves else ""))
    out = api.closest_point_query(bvh, verts, queries, normal=normal)
    run = lambda **kw: api.closest_point_query(bvh, verts, queries, normal=normal, out=out, waves=waves, **kw)
    return _tune(key, run, orders, candidates, reps, use_cache)


def tune_nearest(bvh, points, queries, *, order=None, reps=5, use_cache=True, candidates=None):
    """Best traversal options for mg_nearest_point_query (same contract as tune_closest)."""
    orders = {"given": None} if order is None else {"given": None, "order": order}
    key = _key("nearest", bvh, queries, order is not None)
    run = lambda **kw: api.nearest_point_query(bvh, points, queries, **kw)
    return _tune(key, run, orders, candidates, reps, use_cache)


def options(res, order=None):
    """Keyword arguments of a tuning result for the query calls (order: the candidate order tensor)."""
    kw = {"kernel": res["kernel"], "batch": res["batch"], "seed": res["seed"], "dynamic": res.get("dynamic", False)}
    if res.get("order") == "order":
        kw["order"] = order
    return kw


BATCH_CANDIDATES = [("batch", b, s, False) for b in (1, 2, 4, 8, 16) for s in (False, True)]
BATCH_TILES = [(g, q) for g in (1024, 2048, 4096) for q in (128, 256, 512, 1024)]


def tune_batch(plan, reps=3, use_cache=True):
    """Choose the batched launch's options and apply them to plan (a BatchPlan).

    Per scene: queries per wave and seed descent, by timing the plain
    closest-point traversal (the same device code, with the four-wave register
    allocation of the batched kernel) of the scene's queries on its frame 0.  Plan-wide: the Gaussian and query tile sizes, by timing whole
    runs of the plan.  Returns {"per_scene", "gauss_tile", "query_tile", "ms",
    "timings"} and leaves the plan configured with the best choice.
    """
    per_scene = []
    for sc in plan.scenes:
        V = sc["frames"][0].contiguous()
        bvh = api.lbvh_build(V, sc["faces"])
        r = tune_closest(bvh, V, sc["queries"], normal=True, reps=reps, use_cache=use_cache,
                         candidates=BATCH_CANDIDATES, waves=4)
        per_scene.append({"batch": r["batch"], "seed": r["seed"]})
    sizes = ",".join(f"{s['faces'].shape[1]}x{s['frames'].shape[0]}x{s['gface'].shape[0]}x{s['queries'].shape[1]}"
                     for s in plan.scenes)
    picks = ",".join(f"{p['batch']}{int(p['seed'])}" for p in per_scene)
    dev = torch.cuda.get_device_properties(plan.plan.device)
    key = f"{getattr(dev, 'gcnArchName', dev.name)}|batchplan|{sizes}|{picks}"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        res = cache[key]
    else:
        timings = {}
        for g, q in BATCH_TILES:
            plan.configure(gauss_tile=g, query_tile=q, per_scene=per_scene)
            timings[f"{g}/{q}"] = _graph_time(plan.run, reps)
        best = min(timings, key=timings.get)
        g, q = (int(x) for x in best.split("/"))
        res = {"per_scene": per_scene, "gauss_tile": g, "query_tile": q, "ms": timings[best], "timings": timings}
        if use_cache:
            cache = _load_cache()
            cache[key] = res
            _store_cache(cache)
    plan.configure(gauss_tile=res["gauss_tile"], query_tile=res["query_tile"], per_scene=res["per_scene"])
    return res
