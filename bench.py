"""Benchmark: forward + backward of the tile rasterizer over a batch of views per step.

Workload (default): 1,000,000 Gaussians in 32 clusters with degree-3 SH,
rendered at 1920x1080 (fx = fy = 1500) from 16 viewpoints on a radius-6
sphere; a step is the whole hot path for a batch of consecutive views (4 by
default, --views-per-step): projection, tile binning (depth order, counts
and scan, key emission, radix sort on the tile bits, tile ranges, dispatch
order), forward compositing, backward compositing and the projection
backward, each one call over all the step's cameras, as the paper's
rasterization call takes a batch of cameras (the projection backward sums
the views' gradients per Gaussian).  Every buffer of the step is allocated
before the timed loop (pipeline.ViewPipeline); a step only enqueues library
calls, and the intersection count stays on the device (the lists are built
in a buffer sized from an untimed pass over the same views, and every step's
count is checked after the loop), so the host never waits inside a step.
Inputs are resident in HBM before timing starts.

Prints one JSON line.  ms_per_step = wall-clock ms per step, ms_per_view =
per view; value = forward + backward Gaussian-pixel evaluations the timed
kernels execute, per second of wall time (counted exactly by an untimed pass
of the same views); the paper-equivalent rate (every pixel walking its
tile's whole 3-sigma list until it stops) is reported beside it, as are the
same views one per step (one camera per call), the per-step GPU times
(median, p10, p90), the host time of each stage and the step replayed as one
captured HIP graph.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms per fwd+bwd view and Gaussian-pixel evals/s @1M Gaussians 1080p; p99 serve latency"
PEAK_FP32_TFLOPS = 157.3      # MI355X vector FP32 (256 CU x 4 SIMD x 16 lanes x 2 FMA x 2 packed x 2.4 GHz)
PEAK_FP32_NONPACKED_TFLOPS = 78.6   # the same without packed FP32, which these kernels are built without
PEAK_HBM_GBS = 8000.0
# Algorithmic floating-point operations of the compositing formulas (an exp,
# a min and a reciprocal count as one each; compares count as none):
#   every evaluated entry: Delta (2), sigma (9), o exp(-sigma) (2), min (1)       = 14
#   forward, composited:   1 - alpha, T (1 - alpha), alpha T, colour += (6)      =  9
#   backward, composited:  1 - alpha, 1/(1-alpha), T_k, alpha T_k (4), dL/dc (3),
#                          dL/dalpha (15 + 3), S += (6), dL/do, dL/dsigma (2),
#                          dL/dmu' (8), dL/dconic (8)                             = 49
FLOPS_EVAL, FLOPS_FWD_COMP, FLOPS_BWD_COMP = 14, 9, 49

WORKLOADS = {
    "uniform10k_256": dict(
        desc="10k Gaussians, direct RGB colours, 256x256, fx=fy=256, one view from (0, 0, 4)",
        scene="scene_uniform10k_256", cams="cams_uniform10k_256", sh_degree=-1),
    "clusters1m_sh3_1080p": dict(
        desc="1M Gaussians, 32 clusters, SH degree 3, 1920x1080, fx=fy=1500, 16 views on a radius-6 sphere",
        scene="scene_clusters1m_sh3_1080p", cams="cams_clusters1m_sh3_1080p", sh_degree=3),
    "uniform100k_sh3_800": dict(
        desc="100k Gaussians, SH degree 3, 800x800, fx=fy=1100, one view on a radius-4 sphere",
        scene="scene_uniform100k_sh3_800", cams="cams_uniform100k_sh3_800", sh_degree=3),
    "box3m_sh3_1080p": dict(
        desc="3M Gaussians (2.4M in a 20x20x5 box + 0.6M on a radius-50 shell), SH degree 3, 1920x1080, "
             "fx=fy=1200, 4 views from inside the box",
        scene="scene_box3m_sh3_1080p", cams="cams_box3m_sh3_1080p", sh_degree=3),
}


def measured_traffic(summary="raster_bwd_clusters1m_sh3_1080p_traffic.md", sources=("raster_bwd.hip", "common.hpp"),
                     key="traffic_bytes_per_launch", views=None):
    """HBM bytes per launch of a kernel from its committed counter summary,
    or None when the kernel's sources have changed since the counters were
    taken (the summary records their sha256)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    t = re.search(rf"^{key}: ([0-9.]+)$", text, re.M)
    h = re.search(r"^source_sha256: ([0-9a-f]{64})$", text, re.M)
    if not (t and h):
        return None
    if views is not None:                     # the counters must be of a launch over as many views
        vv = re.search(r"^views_per_launch: ([0-9]+)$", text, re.M)
        if not vv or int(vv.group(1)) != views:
            return None
    sha = hashlib.sha256()
    for f in sources:
        sha.update(open(os.path.join(ROOT, "paper_2409_06765_amd", "csrc", f), "rb").read())
    return float(t.group(1)) if sha.hexdigest() == h.group(1) else None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16, help="timed steps (each of --views-per-step views)")
    ap.add_argument("--views-per-step", type=int, default=4,
                    help="views rendered and differentiated by one call of every stage (consecutive cameras)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clusters1m_sh3_1080p", choices=list(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-tiles", type=int, default=1800, help="tiles of view 0 the oracle rasterizes")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-graph", action="store_true", help="skip the captured-graph leg")
    ap.add_argument("--train-steps", type=int, default=200,
                    help="timed steps of the training leg (0 skips it; 1M workload only)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 256 MiB device copy (the reference for traffic counters)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-load", type=float, default=0.8, help="arrival rate as a fraction of the one-view capacity")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is a design note, "
              f"not an implemented path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2409_06765_amd import rasterize as R
    from paper_2409_06765_amd import scenes

    wl = WORKLOADS[args.workload]
    dev = "cuda:0"
    t0 = time.time()
    sc = getattr(scenes, wl["scene"])()
    cams = getattr(scenes, wl["cams"])()
    n_views = len(cams["W"])
    log(f"workload {args.workload}: N={sc['means'].shape[0]} views={n_views} generated in {time.time() - t0:.1f}s")
    d = {k: torch.from_numpy(v).to(dev) for k, v in sc.items() if isinstance(v, np.ndarray)}
    vms = torch.from_numpy(cams["viewmats"]).to(dev)
    Kss = torch.from_numpy(cams["Ks"]).to(dev)
    W, H = int(cams["W"][0]), int(cams["H"][0])
    npix = W * H
    N = int(sc["means"].shape[0])
    v_image_np, _ = scenes.upstream_grads(args.workload, npix, seed=0)
    v_image = torch.from_numpy(v_image_np).to(dev)
    p = R.make_params(sh_degree=wl["sh_degree"])               # the pipeline's defaults (culled binning)
    p_square = R.make_params(sh_degree=wl["sh_degree"], tile_cull=0)   # the paper's whole 3-sigma squares

    def counting_pass(v, pp):
        """Untimed: the same view through the allocating entry points with the
        forward's work counters (n_eval, five per pixel)."""
        vm, Ks = vms[v:v + 1], Kss[v:v + 1]
        proj = R.project(pp, d["means"], d["quats"], d["scales"], d["opacities"], d["sh"], vm, Ks, [W], [H])
        isect = R.intersect(pp, proj, [W], [H])
        fwd = R.rasterize_forward(pp, proj, d["opacities"], isect, [W], [H], None, n_eval=True)
        if isect.check():
            fwd = R.rasterize_forward(pp, proj, d["opacities"], isect, [W], [H], None, n_eval=True)
        ne = fwd["n_eval"].to(torch.int64)
        last = fwd["last_ids"].to(torch.int64)
        pix = torch.arange(npix, device=dev)
        tile = (pix // W // 16) * ((W + 15) // 16) + (pix % W) // 16
        start = isect["ranges"][tile, 0].to(torch.int64)
        e_bwd = torch.where(last >= 0, last - start + 1, torch.zeros_like(last)).sum()
        return dict(E_fwd=int(ne[:, 0].sum()), C=int(ne[:, 1].sum()), E_bwd=int(e_bwd), M=isect["M"],
                    E_fwd_exec=int(ne[:, 2].sum()), E_bwd_exec=int(ne[:, 3].sum()), E_fwd_issued=int(ne[:, 4].sum()))

    # Work counts of every view the timed loop runs (untimed).  Two
    # definitions: the paper's square 3-sigma tile lists, every pixel walking
    # its tile's list until it stops ("paper-equivalent"), and the work the
    # timed kernels really do: the culled lists, each pixel evaluating only
    # the entries of its 8x8 quad's list while it is live (forward), or up to
    # its last composited entry (backward).  A view's work does not depend on
    # the other views of its step (their tiles and lists are disjoint).
    V = max(1, min(int(args.views_per_step), n_views))
    while n_views % V:                       # a step's views are consecutive cameras of the workload
        V -= 1
    batches = [[(i * V + j) % n_views for j in range(V)] for i in range(args.steps)]
    views = [v for b in batches for v in b]
    counts = {}
    for v in sorted(set(views)):
        sq = counting_pass(v, p_square)
        cu = counting_pass(v, p)
        counts[v] = dict(E_fwd=sq["E_fwd"], E_bwd=sq["E_bwd"], C=sq["C"], M=sq["M"], M_culled=cu["M"],
                         E_fwd_lists=cu["E_fwd"], E_fwd_exec=cu["E_fwd_exec"], E_bwd_exec=cu["E_bwd_exec"],
                         E_fwd_issued=cu["E_fwd_issued"], C_culled=cu["C"])
        assert cu["C"] == sq["C"], "culled and square lists composite different entries"
    torch.cuda.synchronize()
    log(f"counts view {views[0]}: {counts[views[0]]}")

    # The timed step: V views in one call of every stage, every buffer allocated once, the step only
    # enqueues library calls.
    from paper_2409_06765_amd.pipeline import ViewPipeline
    warm_batches = [batches[i % len(batches)] for i in range(args.warmup)]
    M_batch = lambda b: sum(counts[v]["M_culled"] for v in b) if all(v in counts for v in b) else None
    cap = int(1.25 * max(M_batch(b) for b in batches)) + 1024
    nslots = args.warmup + args.steps
    pipe = ViewPipeline(p, d, [W] * V, [H] * V, cap, slots=nslots)
    v_image_b = v_image.repeat(V, 1) if V > 1 else v_image
    stream = torch.cuda.current_stream()
    stage_names = ["project_fwd", "intersect", "rasterize_fwd", "zero_grads", "rasterize_bwd", "project_bwd"]
    stages = [pipe.project, pipe.bin, pipe.rasterize_forward, pipe.zero_grads,
              lambda: pipe.rasterize_backward(v_image_b), pipe.project_backward]
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)] for _ in range(args.steps)]
    host = np.zeros((args.steps, len(stages)))

    def run(i, b, timed):
        pipe.set_cameras(vms[b[0]:b[0] + V], Kss[b[0]:b[0] + V], copy=False)
        ev = events[i] if timed else None
        if ev:
            ev[0].record(stream)
        for k, f in enumerate(stages):
            t0 = time.perf_counter()
            if k == 1:
                pipe.bin(slot=i + (args.warmup if timed else 0))
            else:
                f()
            if ev:
                host[i, k] = time.perf_counter() - t0
                ev[k + 1].record(stream)

    assert all(b[0] + V <= n_views and b == list(range(b[0], b[0] + V)) for b in batches + warm_batches), \
        "each step's views must be consecutive cameras"
    for i in range(args.warmup):
        run(i, warm_batches[i], False)
    torch.cuda.synchronize()
    if args.calibrate_copy:
        src = torch.ones(64 << 20, device=dev, dtype=torch.float32)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i, b in enumerate(batches):
        run(i, b, True)
    t_host = time.perf_counter() - t_start
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_start

    # every timed step's lists fitted the capacity (no host wait inside the loop; checked after)
    got = pipe.counts()
    assert max(got) <= cap, "intersection capacity exceeded in the timed loop"
    assert [got[args.warmup + i] for i in range(args.steps)] == [M_batch(b) for b in batches], \
        "timed steps built other lists than the counting pass"
    per_stage = np.array([[ev[k].elapsed_time(ev[k + 1]) for k in range(len(stages))] for ev in events])
    per_step = np.array([ev[0].elapsed_time(ev[-1]) for ev in events])
    stage_ms = {k: round(float(per_stage[:, i].mean()), 4) for i, k in enumerate(stage_names)}
    host_ms = {k: round(1e3 * float(host[:, i].mean()), 4) for i, k in enumerate(stage_names)}
    ms_per_step = 1e3 * t_wall / args.steps
    nv_timed = args.steps * V
    tot = lambda key: sum(counts[v][key] for v in views)
    E_fwd, E_bwd, C_tot = tot("E_fwd"), tot("E_bwd"), tot("C")
    E_fwd_x, E_bwd_x = tot("E_fwd_exec"), tot("E_bwd_exec")
    value = (E_fwd_x + E_bwd_x) / t_wall

    # dominant kernel: the backward compositing (bound by vector-instruction issue); one launch per step
    bwd_ms = stage_ms["rasterize_bwd"]
    bwd_flops_x = (FLOPS_EVAL * E_bwd_x + FLOPS_BWD_COMP * C_tot) / args.steps
    bwd_flops_p = (FLOPS_EVAL * E_bwd + FLOPS_BWD_COMP * C_tot) / args.steps
    achieved = bwd_flops_x / (bwd_ms * 1e-3) / 1e12
    achieved_p = bwd_flops_p / (bwd_ms * 1e-3) / 1e12
    fwd_tflops = (FLOPS_EVAL * E_fwd_x + FLOPS_FWD_COMP * C_tot) / args.steps / (stage_ms["rasterize_fwd"] * 1e-3) / 1e12
    roofline = {"kernel": "raster_bwd_rgb_kernel", "bound": "alu", "achieved": round(achieved, 3),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": None, "work": "executed (quad lists, live lanes)",
                "frac_of_nonpacked_peak": round(achieved / PEAK_FP32_NONPACKED_TFLOPS, 4),
                "achieved_paper_equivalent": round(achieved_p, 3),
                "frac_paper_equivalent": round(achieved_p / PEAK_FP32_TFLOPS, 4)}
    if args.workload == "clusters1m_sh3_1080p":
        t = measured_traffic(views=V)
        roofline["traffic"] = None if t is None else int(t)

    # device memory: the resident scene, and what the preallocated forward + backward state of one step takes
    memory = {"scene_bytes": int(sum(v.numel() * v.element_size() for v in d.values())),
              "per_step_state_bytes": int(_device_bytes(pipe)), "views_per_step": V,
              "device_bytes": int(torch.cuda.get_device_properties(0).total_memory)}
    log(f"memory: scene {memory['scene_bytes'] / 2**20:.0f} MiB, one {V}-view step's state "
        f"{memory['per_step_state_bytes'] / 2**20:.0f} MiB")
    del pipe
    torch.cuda.empty_cache()

    # the same views one per step (one camera per call of every stage), for comparison
    single = None
    if V > 1:
        cap1 = int(1.25 * max(counts[v]["M_culled"] for v in views)) + 1024
        p1 = ViewPipeline(p, d, [W], [H], cap1, slots=args.warmup + nv_timed)
        for i in range(args.warmup):
            p1.set_cameras(vms[i % n_views:i % n_views + 1], Kss[i % n_views:i % n_views + 1], copy=False)
            p1.step(v_image, slot=i)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i, v in enumerate(views):
            p1.set_cameras(vms[v:v + 1], Kss[v:v + 1], copy=False)
            p1.step(v_image, slot=args.warmup + i)
        torch.cuda.synchronize()
        t1 = time.perf_counter() - t1
        assert max(p1.counts()) <= cap1
        single = {"ms_per_view": round(1e3 * t1 / nv_timed, 4), "value": (E_fwd_x + E_bwd_x) / t1}
        log(f"one view per step: {single['ms_per_view']:.4f} ms/view")
        del p1
        torch.cuda.empty_cache()

    graph = None
    if not args.no_graph:
        from paper_2409_06765_amd.graph import CapturedStep
        cs = CapturedStep(p, d, [W] * V, [H] * V, v_image_b, (vms[0:V], Kss[0:V]), capacity=cap)
        for b in warm_batches:
            cs.replay(vms[b[0]:b[0] + V], Kss[b[0]:b[0] + V])
        seen = torch.zeros(len(batches), device=dev, dtype=torch.int64)
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for i, b in enumerate(batches):
            o = cs.replay(vms[b[0]:b[0] + V], Kss[b[0]:b[0] + V])
            seen[i:i + 1].copy_(o["isect"]["total_dev"][:1])
        torch.cuda.synchronize()
        tg = time.perf_counter() - tg
        assert int(seen.max()) <= cs.capacity, "a replay's lists exceeded the captured capacity"
        graph = {"ms_per_step": round(1e3 * tg / args.steps, 4), "ms_per_view": round(1e3 * tg / nv_timed, 4),
                 "value": (E_fwd_x + E_bwd_x) / tg, "capacity": cs.capacity}
        log(f"graph: {graph['ms_per_view']:.4f} ms/view (eager {1e3 * t_wall / nv_timed:.4f})")
        del cs

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Gaussian-pixel evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded generators, activated parameters)",
        "config": {"workload": f"{args.workload}: {wl['desc']}", "views_per_step": V, "views_timed": nv_timed,
                   "width": W, "height": H, "n_gaussians": int(sc["means"].shape[0])},
        "value_definition": "forward + backward evaluations the timed kernels execute (culled lists, each pixel's "
                            "quad list while live / up to its last composited entry) per second of wall time",
        "step_definition": f"{V} views through one call of every stage (projection, binning, forward and backward "
                           f"compositing, projection backward); the projection backward sums the views' gradients",
        "ms_per_view": round(1e3 * t_wall / nv_timed, 4),
        "ms_per_step_gpu": {"median": round(float(np.median(per_step)), 4),
                            "p10": round(float(np.percentile(per_step, 10)), 4),
                            "p90": round(float(np.percentile(per_step, 90)), 4)},
        "views_per_s": nv_timed / t_wall,
        "one_view_per_step": single,
        "stage_ms": stage_ms,
        "stage_ms_per_view": {k: round(v / V, 4) for k, v in stage_ms.items()},
        "stage_ms_median": {k: round(float(np.median(per_stage[:, i])), 4) for i, k in enumerate(stage_names)},
        "host_ms_per_stage": host_ms,
        "host_ms_per_step": round(1e3 * t_host / args.steps, 4),
        "evals": {"E_fwd_per_view": E_fwd / nv_timed, "E_bwd_per_view": E_bwd / nv_timed,
                  "composited_per_view": C_tot / nv_timed,
                  "E_fwd_exec_per_view": E_fwd_x / nv_timed, "E_bwd_exec_per_view": E_bwd_x / nv_timed,
                  "E_fwd_culled_lists_per_view": tot("E_fwd_lists") / nv_timed,
                  "E_fwd_issued_per_view": tot("E_fwd_issued") / nv_timed,
                  "E_fwd_issued_over_exec": round(tot("E_fwd_issued") / max(E_fwd_x, 1), 4),
                  "M_per_view": tot("M") / nv_timed, "M_culled_per_view": tot("M_culled") / nv_timed},
        "evals_paper_equivalent_per_s": (E_fwd + E_bwd) / t_wall,
        "raster_fwd_tflops_executed": round(fwd_tflops, 3),
        "roofline": roofline,
        "memory": memory,
    }
    if graph is not None:
        out["graph"] = graph
    if not args.no_serve and args.workload == "clusters1m_sh3_1080p":
        out["serving"] = serving(d, p, args)
    if args.train_steps > 0 and args.workload == "clusters1m_sh3_1080p":
        out["training"] = training(sc, cams, wl, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, cams, wl, args, counts, views[0])
    print(json.dumps(out), flush=True)


def _device_bytes(obj, skip=("scene", "cam")):
    """Bytes of the distinct device buffers an object holds (its attributes
    and the values of its dict attributes), leaving out ``skip``."""
    import torch
    seen, total = set(), 0
    for name, v in vars(obj).items():
        if name in skip:
            continue
        for t in (v.values() if isinstance(v, dict) else [v]):
            if isinstance(t, torch.Tensor) and t.is_cuda:
                st = t.untyped_storage()
                if st.data_ptr() not in seen:
                    seen.add(st.data_ptr())
                    total += st.nbytes()
    return total


def serving(d, p, args):
    """Render requests against the resident 1M-Gaussian scene: Poisson
    arrivals over {256^2, 512^2, 800^2, 1280x720, 1920x1080}, focal 1.2 W,
    poses on a radius-6 sphere.  The arrival rate is a fraction of the
    one-view-per-launch capacity measured on the same request mix; both
    policies replay the same trace."""
    import torch
    from paper_2409_06765_amd import scenes
    from paper_2409_06765_amd.serve import GpuBackend, Server, serve_one_at_a_time

    be = GpuBackend(d, p)
    probe = scenes.serving_trace(1.0, n_requests=60, seed=1)
    for r in probe:
        r.arrival = 0.0
    serve_one_at_a_time(be, probe)                           # warm up: every size (capacity, allocations)
    torch.cuda.synchronize()
    _, cap = serve_one_at_a_time(be, probe)
    Server(be, max_batch=16, mem_budget=24 << 30).run(probe)   # warm up the batched shapes too
    torch.cuda.synchronize()
    _, bcap = Server(be, max_batch=16, mem_budget=24 << 30).run(probe)
    log(f"serving: capacity {cap.views_per_s:.1f} views/s one at a time, {bcap.views_per_s:.1f} batched")
    pick = lambda st: {"views_per_s": round(st.views_per_s, 2), "p50_ms": round(st.p50_ms, 3),
                       "p99_ms": round(st.p99_ms, 3), "mean_batch": round(st.mean_batch, 2),
                       "done": st.n_done, "rejected": st.n_rejected}

    def at(load):
        """Both policies on one trace of Poisson arrivals at load x the one-view capacity."""
        rate = load * cap.views_per_s
        trace = scenes.serving_trace(rate, n_requests=args.serve_requests, seed=0)
        _, single = serve_one_at_a_time(be, trace)
        torch.cuda.synchronize()
        _, batched = Server(be, max_batch=16, mem_budget=24 << 30).run(trace)
        torch.cuda.synchronize()
        log(f"serving at {load}x ({rate:.0f} req/s): batched p50/p99 {batched.p50_ms:.2f}/{batched.p99_ms:.2f} ms, "
            f"mean batch {batched.mean_batch:.2f}; one view per launch {single.p50_ms:.2f}/{single.p99_ms:.2f} ms")
        return {"load": load, "arrival_rate_per_s": round(rate, 2), "batched": pick(batched),
                "one_view_per_launch": pick(single)}

    head = at(args.serve_load)
    sweep = [head if abs(x - args.serve_load) < 1e-9 else at(x) for x in (0.5, 0.8, 1.0, 1.5)]
    return {"requests": args.serve_requests, "arrival_rate_per_s": head["arrival_rate_per_s"],
            "one_view_capacity_views_per_s": round(cap.views_per_s, 2),
            "batched_capacity_views_per_s": round(bcap.views_per_s, 2),
            "batched": head["batched"], "one_view_per_launch": head["one_view_per_launch"],
            "sweep": sweep}


# Adam moves per element: param, exp_avg, exp_avg_sq read and written, the
# gradient read (28 bytes), plus the activated value written for the scales
# and opacities (4 bytes).
ADAM_BYTES_PER_ELEM, ACT_BYTES_PER_ELEM = 28, 4


def training(sc, cams, wl, args):
    """Synthetic fit of the 1M-Gaussian scene: targets are renders of the
    scene itself from the 16 views (untimed), the start is the scene with
    jittered centres and colours.  One view per step; ADC statistics every
    step and one refinement (plan, split / clone / prune, apply) at the last
    timed step, so its cost is amortised over the window; then the same
    window with the MCMC strategy.  The Adam launch is timed alone on the
    final parameter set for its roofline."""
    import torch
    from paper_2409_06765_amd import _lib as L
    from paper_2409_06765_amd.train import GaussianTrainer, TrainConfig

    dev = "cuda:0"
    raw = dict(means=sc["means"], quats=sc["quats"], log_scales=np.log(sc["scales"]),
               logits=np.log(sc["opacities"] / (1.0 - sc["opacities"])), sh=sc["sh"])
    V, H, W = len(cams["W"]), int(cams["H"][0]), int(cams["W"][0])
    gt = GaussianTrainer(raw, cams, torch.zeros((V, H, W, 3)), TrainConfig(strategy="none"),
                         sh_degree=wl["sh_degree"])
    targets = torch.stack([gt.render([v])[-1]["image"].reshape(H, W, 3) for v in range(V)])
    del gt
    g = np.random.default_rng(7)
    start = dict(raw)
    start["means"] = (raw["means"] + g.normal(0, 0.01, raw["means"].shape)).astype(np.float32)
    start["sh"] = raw["sh"].copy()
    start["sh"][:, 0, :] += g.normal(0, 0.1, start["sh"][:, 0, :].shape).astype(np.float32)
    warm, K = 10, args.train_steps
    out = {"workload": f"fit of {args.workload} to its own renders from {V} views, one view per step",
           "steps_timed": K, "warmup": warm}
    for strategy in ("adc", "mcmc"):
        # ADC: one refinement at the end of the warm-up (first launches of every kernel), none in the timed
        # window, then one more refinement timed on its own
        cfg = TrainConfig(strategy=strategy, refine_start=0, refine_every=warm, reset_every=10 ** 9,
                          lr_decay_steps=30_000)
        tr = GaussianTrainer(start, cams, targets, cfg, sh_degree=wl["sh_degree"])
        for _ in range(warm):
            tr.step()
        tr.cfg.refine_every = 10 ** 9
        torch.cuda.synchronize()
        N0 = tr.N
        losses = []
        host = 0.0
        t0 = time.perf_counter()
        for _ in range(K):
            th = time.perf_counter()
            losses.append(tr.step())
            host += time.perf_counter() - th
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ls = [float(x) for x in torch.cat(losses).cpu()]
        res = {"ms_per_step": round(1e3 * dt / K, 4), "steps_per_s": round(K / dt, 2),
               "host_ms_per_step": round(1e3 * host / K, 4), "n_gaussians": N0,
               "loss_first": round(ls[0], 6), "loss_last": round(ls[-1], 6)}
        if strategy == "adc":
            t0 = time.perf_counter()
            n_new = tr.densify()
            torch.cuda.synchronize()
            refine_ms = 1e3 * (time.perf_counter() - t0)
            res.update(refine_ms=round(refine_ms, 3), refine_n=[N0, n_new],
                       ms_per_step_refine_every_100=round(1e3 * dt / K + refine_ms / 100, 4))
        out[strategy] = res
        log(f"training {strategy}: {res}")
    # the Adam launch alone, on the last trainer's parameters and gradients
    names = ("means", "quats", "log_scales", "logits", "sh")
    gk = dict(means="v_means", quats="v_quats", log_scales="v_scales", logits="v_opacities", sh="v_sh")
    N = tr.N
    grads = {k: torch.zeros_like(tr.raw[k]) for k in names}
    groups = [dict(param=tr.raw[k], grad=grads[k], exp_avg=tr.m[k], exp_avg_sq=tr.v[k], lr=1e-4,
                   activated=tr.scales if k == "log_scales" else (tr.opacities if k == "logits" else None),
                   activation=L.GSR_ACT_EXP if k == "log_scales" else (L.GSR_ACT_SIGMOID if k == "logits" else 0),
                   row=48 if k == "sh" else 0, row_first=3 if k == "sh" else 0, lr_rest=1e-4) for k in names]
    s = torch.cuda.current_stream()
    for _ in range(3):
        L.gsr_adam_step(groups, 1000)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 20
    ev[0].record(s)
    for _ in range(reps):
        L.gsr_adam_step(groups, 1000, stream=s)
    ev[1].record(s)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    elems = sum(tr.raw[k].numel() for k in names)
    nbytes = ADAM_BYTES_PER_ELEM * elems + ACT_BYTES_PER_ELEM * (tr.raw["log_scales"].numel() + N)
    gbs = nbytes / (ms * 1e-3) / 1e9
    traffic_per_elem = measured_traffic("adam_clusters1m_sh3_traffic.md", ("train.hip", "common.hpp"),
                                        key="traffic_bytes_per_element")
    # reference: a plain device copy moving about as many bytes (half read, half written)
    src = torch.ones(nbytes // 8, device=dev, dtype=torch.float32)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev[0].record(s)
    for _ in range(reps):
        dst.copy_(src)
    ev[1].record(s)
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 4 / (ev[0].elapsed_time(ev[1]) / reps * 1e-3) / 1e9
    del src, dst
    out["adam"] = {"kernel": "adam_kernel", "bound": "hbm", "elements": elems, "bytes": nbytes, "ms": round(ms, 4),
                   "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                   "copy_reference_GBs": round(copy_gbs, 1),
                   "traffic": traffic_per_elem and int(round(traffic_per_elem * elems))}
    log(f"adam: {elems} elements in {ms:.4f} ms = {gbs:.0f} GB/s (device copy {copy_gbs:.0f} GB/s)")
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(sc, cams, wl, args, counts, v0):
    """The oracle (C, float32, gcc -O2) on view 0: full projection, binning
    and sort, then forward + backward compositing of tiles, on one thread (a
    sample of tiles, scaled by the evaluation counts) and on every host core
    this process may use (its loops over tiles on OpenMP threads, the whole
    frame).  The all-core figure is the reported value."""
    import oracle
    from oracle import Oracle, OracleParams
    from paper_2409_06765_amd import scenes

    o = Oracle(np.float32)
    P = OracleParams(sh_degree=wl["sh_degree"])
    one = {k: v[v0:v0 + 1] for k, v in cams.items()}
    W, H = int(one["W"][0]), int(one["H"][0])
    TX, TY = (W + 15) // 16, (H + 15) // 16
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    v_image, _ = scenes.upstream_grads(args.workload, W * H, seed=0)
    ys, xs = np.divmod(np.arange(W * H), W)
    tile_of_pix = (ys // 16) * TX + xs // 16
    E_view = counts[v0]["E_fwd"] + counts[v0]["E_bwd"]
    E_view_exec = counts[v0]["E_fwd_exec"] + counts[v0]["E_bwd_exec"]

    def run(threads, sample_tiles):
        oracle.set_threads(threads)
        try:
            t0 = time.perf_counter()
            proj = o.project(P, sc["means"], sc["quats"], sc["scales"], sc["opacities"], sc["sh"], one["viewmats"],
                             one["Ks"], one["W"], one["H"])
            t1 = time.perf_counter()
            isect = o.intersect(P, proj, one["W"], one["H"])
            t2 = time.perf_counter()
            lens = isect["ranges"][:, 1] - isect["ranges"][:, 0]
            busy = np.nonzero(lens > 0)[0]
            mask = np.zeros(TX * TY, np.uint8)
            if sample_tiles is None or sample_tiles >= busy.size:
                mask[busy] = 1
            else:
                mask[np.random.default_rng(0).choice(busy, size=sample_tiles, replace=False)] = 1
            ras = o.rasterize_fwd(P, proj, sc["opacities"], isect["ranges"], isect["ids"], one["W"], one["H"],
                                  tile_mask=mask)
            o.rasterize_bwd(P, proj, sc["opacities"], isect["ranges"], isect["ids"], one["W"], one["H"],
                            ras["final_T"], ras["last_ids"], v_image, tile_mask=mask)
            t3 = time.perf_counter()
        finally:
            oracle.set_threads(1)
        # evaluation counts of the tiles run (the same definitions as the GPU's square-list counts)
        pixmask = mask[tile_of_pix] == 1
        start = isect["ranges"][tile_of_pix, 0]
        last = ras["last_ids"]
        e_s = int(ras["n_eval"][pixmask].sum()) + int(np.where(last >= 0, last - start + 1, 0)[pixmask].sum())
        scale = E_view / max(e_s, 1)
        t_view = (t1 - t0) + (t2 - t1) + (t3 - t2) * scale
        desc = (f"projection of all {sc['means'].shape[0]} Gaussians ({1e3 * (t1 - t0):.0f} ms), binning + qsort "
                f"of M={isect['M']} ({1e3 * (t2 - t1):.0f} ms), forward+backward compositing of {int(mask.sum())} of "
                f"{TX * TY} tiles ({1e3 * (t3 - t2):.0f} ms, {e_s} evals)"
                + (f", scaled by evaluations x{scale:.2f}" if scale > 1.0001 else ""))
        return E_view_exec / t_view, 1e3 * t_view, desc, E_view / t_view

    v1, ms1, d1, sq1 = run(1, args.cpu_sample_tiles)
    vn, msn, dn, sqn = run(cores, None)
    log(f"cpu baseline: 1 thread {ms1:.0f} ms/view, {cores} threads {msn:.0f} ms/view")
    return {"value": vn, "unit": "Gaussian-pixel evals/s", "cores": cores, "kind": "oracle",
            "value_definition": "the evaluations the GPU path executes for view 0 (the definition of value) per "
                                "second of the oracle's time for that view; the oracle itself composites the "
                                "square lists: value_square_lists counts those",
            "value_square_lists": sqn,
            "ms_per_view_est": msn,
            "sample": f"view 0 on {cores} threads: {dn}; float32, gcc -O2 -fopenmp (compositing loops over tiles "
                      f"threaded, projection and binning on one thread)",
            "cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count(),
            "single_thread": {"value": v1, "value_square_lists": sq1, "cores": 1, "ms_per_view_est": ms1,
                              "sample": f"view 0: {d1}"}}


if __name__ == "__main__":
    main()
