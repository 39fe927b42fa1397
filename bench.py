"""Benchmark of the inverse-path-tracing hot path on one MI355X.

A step is one SGD iteration of the method over the full synthetic workload:
colour estimate (stream A) -> loss and adjoint image -> gradient estimate
(stream B: forward pass with vertex checkpoints + adjoint replay + block
reduction) -> projected Adam.  Inputs (scene, BVH, target images, parameters)
are resident on the device before the timed region.

Prints ONE JSON line.  value = gradient paths per second of the whole step
(B paths / step time); the breakdown gives colour paths/s and the
fwd+adjoint-only gradient paths/s.  The roofline entry is for the dominant
kernel, timed with HIP events inside the library on the stream it runs on;
algorithmic bytes come from the kernels' own work counters (BVH nodes x 64 B read
+ triangles x 48 B + checkpoint traffic).  cpu_baseline times the FP64 oracle
on a bounded pixel sample on this host's cores.
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

HBM_PEAK_GBS = 8000.0
# VALU peaks of MI355X (256 CUs x 4 SIMDs, 2.4 GHz): a SIMD retires one
# wave64 VALU instruction per 4 cycles (16 lanes per cycle), so the chip
# issues 256 x 4 x 2.4e9 / 4 = 6.14e11 wave instructions/s, i.e. 3.93e13
# lane instructions/s when all 64 lanes of every wave are active (fp32 FMA
# counted as one instruction; the 157.3 TFLOP/s vector figure counts an FMA
# as two flops and packed fp32 as two lanes)
VALU_WAVE_INST_PEAK = 256 * 4 * 2.4e9 / 4
VALU_LANE_INST_PEAK = VALU_WAVE_INST_PEAK * 64
TRI_B = 48
# BVH node bytes read per visit, by (children, bytes per node): 4-wide nodes
# with quantized boxes read their four float4 rows (64 B), with float boxes
# seven of their eight (112 B); binary nodes 64 B
NODE_READ_B = {(4, 64): 64, (4, 128): 112, (2, 64): 64}
# checkpoint traffic per path vertex: the gradient forward pass writes the hit
# record, a and c (3 x 16 B); the backward sweep reads a and c back (32 B) and
# writes the suffix radiance (16 B), in the forward pass when a guide collects
# training records, else at the start of the replay; the replay reads the hit
# record and the suffix radiance (32 B)
CK_WRITE_B = 48
CK_SWEEP_B = 48
CK_REPLAY_B = 32


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


# sources the path kernels and the tree they traverse are built from: the
# counters (VALU work, HBM traffic) are reported only while these still hash
# to the profiled version
KERNEL_SOURCES = ["paper_1903_07145_amd/csrc/" + f for f in
                  ("trace.hip", "ipt_math.h", "ipt_internal.h", "guide_dev.h", "disney.h", "api.hip",
                   "bvh_gpu.hip", "bvh_wide.cpp")] + \
                 ["paper_1903_07145_amd/build.py"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_counters(kernel, workload):
    """Per-launch hardware counters of `kernel` from the committed summaries
    under profiles/ (rocprofv3 --pmc runs of this script): VALU instructions
    and lane utilisation, and HBM bytes (FETCH_SIZE and WRITE_SIZE, each
    scaled by what the same counter reads for a plain copy of known size).
    Only lines whose kernel-source hash matches the current sources count;
    returns {} when there are none."""
    want = kernel_source_hash()
    out = {}
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return out
    for name in sorted(os.listdir(pdir)):
        if not name.endswith(".md"):
            continue
        for line in open(os.path.join(pdir, name)):
            if not line.startswith("counters:"):
                continue
            f = dict(kv.split("=", 1) for kv in line[len("counters:"):].split())
            if f.get("kernel") == kernel and f.get("workload") == workload and f.get("sources") == want:
                out.update({k: float(v) for k, v in f.items() if k not in ("kernel", "workload", "sources")})
    return out


def copy_reference(nbytes=256 << 20, launches=3):
    """A copy kernel of known size: each launch reads and writes `nbytes`.
    Also reports the achieved copy bandwidth (read + write bytes over the
    event-timed duration of 20 more launches): the practical HBM ceiling."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(launches):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * 20 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    print(json.dumps({"copy_reference_bytes": nbytes, "launches": launches, "copy_gbs": round(gbs, 1)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="apartment", choices=["cornell", "room", "apartment", "office_floor"])
    ap.add_argument("--target-spp", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--guide", action="store_true",
                    help="learned proposal: trained online during the warm-up, then each step samples it "
                         "(one-sample MIS with BRDF sampling, mix 0.5), writes training records and runs "
                         "--guide-steps training steps")
    ap.add_argument("--guide-steps", type=int, default=10)
    ap.add_argument("--guide-cells", type=int, default=0,
                    help="with --guide: sample the cached proposal (about this many cells per side, refilled "
                         "after each training call) instead of evaluating the network at every path vertex")
    ap.add_argument("--material", default="ggx", choices=["ggx", "disney"],
                    help="material model of every segment: Lambert + GGX (7 parameters, the workloads' own) or the "
                         "Disney model (13 parameters, seeded values; the same geometry, lights and views)")
    ap.add_argument("--copy-reference", action="store_true",
                    help="only run a plain device copy of 256 MiB three times (the kernel whose FETCH_SIZE and "
                         "WRITE_SIZE counters scale those of the path kernels to bytes) and exit")
    args = ap.parse_args()
    if args.copy_reference:
        copy_reference()
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only; runs on several GPUs are not implemented "
              "(paths would shard by pixel tiles with one gradient all-reduce per step).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1903_07145_amd import ipt, scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    t0 = time.time()
    sc = scenes.WORKLOADS[args.workload]()
    if args.material == "disney":
        sc = scenes.disney(sc, seed=11)
    cfg = sc["render"]
    log("scene %s: %d triangles, %d segments, %d emitters (%.1fs)" % (
        sc["name"], sc["tris"].shape[0], sc["num_segments"], len(sc["emitter_seg"]), time.time() - t0))
    t0 = time.time()
    g = ipt.Scene.from_dict(sc)
    info = g.info()
    log("scene build %.1fs (BVH %.0f ms, %d nodes, depth %d, SAH %.1f)" % (
        time.time() - t0, info["build_ms"], info["num_nodes"], info["bvh_depth"], info["sah_cost"]))
    dc = ipt.make_cameras(sc["cams"])
    V, W, H = dc["num_views"], dc["width"], dc["height"]
    npix = V * W * H
    spp, D, rr = cfg["spp"], cfg["max_depth"], cfg["rr_depth"]
    p_true = torch.as_tensor(sc["params"], device="cuda")
    # target images: the true parameters at target_spp (stream tag 0), in 16-spp passes
    tspp = args.target_spp or cfg["target_spp"]
    t0 = time.time()
    target = torch.zeros((npix, 3), dtype=torch.float32, device="cuda")
    npass = max(1, tspp // 16)
    for i in range(npass):
        o = ipt.render_opts(seed=1, stream_tag=0, iteration=i, spp=min(16, tspp), max_depth=D, rr_depth=rr, mis=2)
        target += g.render(dc, p_true, o)
    target /= npass
    torch.cuda.synchronize()
    log("target %d spp in %.1fs" % (npass * min(16, tspp), time.time() - t0))

    params = torch.as_tensor(scenes.init_theta(sc, cfg["init"], seed=7), device="cuda")
    scale = torch.as_tensor(sc["scale"], device="cuda")
    lo = torch.as_tensor(sc["lo"], device="cuda")
    hi = torch.as_tensor(sc["hi"], device="cuda")
    tr = torch.as_tensor(sc["trainable"], device="cuda")
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.zeros_like(params)
    lr = cfg["lr"]

    gd = None
    if args.guide:
        stride = max(1, (npix * spp * 3) // (1 << 20))   # about one million records per step
        gd = ipt.Guide(g, seed=7, batch=16384, ring_capacity=1 << 21, record_stride=stride)
    cached = 1 if (gd is not None and args.guide_cells > 0) else 0
    if cached:
        from paper_1903_07145_amd.optimize import cell_area_for
        gd.cache_build(cell_area_for(sc, args.guide_cells))   # allocates the cell table and rows

    def step(it):
        mix = 0.5 if (gd is not None and it >= 1) else 0.0
        co = ipt.render_opts(seed=11, stream_tag=1, iteration=it, spp=spp, max_depth=D, rr_depth=rr, mis=2,
                             guide=gd if mix > 0 else None, guide_mix=mix, guide_cached=cached)
        go = ipt.render_opts(seed=11, stream_tag=2, iteration=it, spp=spp, max_depth=D, rr_depth=rr, mis=2,
                             guide=gd, guide_mix=mix, guide_cached=cached)
        g.loss_grad(dc, params, target, co, go, 0, loss=loss, grad=grad)
        ipt.sgd_step(params, grad, m, v, it + 1, lr=lr, scale=scale, lo=lo, hi=hi, trainable=tr)
        if gd is not None and gd.records() >= 16384:
            gd.train(args.guide_steps, want_loss=False)
            if cached:
                gd.cache_build(gd.cell_area)

    # workspace sized once, outside the timed region
    g.workspace(dc, ipt.render_opts(spp=spp, max_depth=D, rr_depth=rr, guide=gd, guide_mix=0.5 if gd else 0.0,
                                    guide_cached=cached))
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    g.profile_reset()
    g.profile(True)
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.time()
    e0.record(st)
    for i in range(args.steps):
        step(args.warmup + i)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.time() - wall0
    g.profile(False)
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    prof = {ipt.KERNELS[k]: g.profile_read(k) for k in range(3)}
    paths_step = npix * spp
    value = paths_step / (ms_step * 1e-3)
    k_fwd, k_rep, k_col = prof["grad_forward"], prof["adjoint_replay"], prof["colour"]
    ms_grad = (k_fwd["total_ms"] + k_rep["total_ms"]) / args.steps
    ms_col = k_col["total_ms"] / args.steps
    log("step %.1f ms (wall %.1f ms): colour %.1f ms, grad fwd %.1f ms, replay %.1f ms" % (
        ms_step, 1e3 * wall / args.steps, ms_col, k_fwd["total_ms"] / args.steps, k_rep["total_ms"] / args.steps))

    node_b = NODE_READ_B[(info["node_width"], info["node_bytes"])]

    def kbytes(k, extra_per_vertex):
        return k["nodes"] * node_b + k["tris"] * TRI_B + k["vertices"] * extra_per_vertex

    per = {}
    sweep_fwd = CK_SWEEP_B if args.guide else 0
    for name, k, extra in (("colour", k_col, 0), ("grad_forward", k_fwd, CK_WRITE_B + sweep_fwd),
                           ("adjoint_replay", k_rep, CK_REPLAY_B + CK_SWEEP_B - sweep_fwd)):
        launches = max(1, k["launches"])
        avg_ms = k["total_ms"] / launches
        b = kbytes(k, extra) / launches
        per[name] = dict(avg_ms=avg_ms, bytes_per_launch=b, gbs=b / (avg_ms * 1e-3) / 1e9,
                         rays_per_launch=k["rays"] / launches,
                         nodes_per_ray=k["nodes"] / max(1, k["rays"]), tris_per_ray=k["tris"] / max(1, k["rays"]))
    dom = max(per, key=lambda n: per[n]["avg_ms"])
    d = per[dom]
    cnt = measured_counters(dom, sc["name"])
    traffic = cnt.get("hbm_bytes_per_launch")
    valu = None
    if "valu_insts_per_launch" in cnt:
        issue = cnt["valu_insts_per_launch"] / (d["avg_ms"] * 1e-3)
        lanes = cnt["lane_util"]
        valu = {"issued_wave_inst_per_s": round(issue, 1), "issue_peak": VALU_WAVE_INST_PEAK,
                "issue_frac": round(issue / VALU_WAVE_INST_PEAK, 4), "lane_util": round(lanes, 4),
                "valu_insts_per_launch": cnt["valu_insts_per_launch"],
                "source": "SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU, SQ_THREAD_CYCLES_VALU per launch (profiles/)"}
    hbm = {"algorithmic_gbs": round(d["gbs"], 1), "peak_gbs": HBM_PEAK_GBS,
           "frac": round(d["gbs"] / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": int(d["bytes_per_launch"]),
           "measured_gbs": round(traffic / (d["avg_ms"] * 1e-3) / 1e9, 1) if traffic else None}
    if valu is not None:
        # the counters show a VALU-issue-bound kernel: its roofline is the
        # VALU lane throughput, achieved = active lane instructions per second
        lane_rate = valu["issued_wave_inst_per_s"] * 64 * valu["lane_util"]
        roofline = {"bound": "alu", "achieved": round(lane_rate / 1e12, 3), "peak": round(VALU_LANE_INST_PEAK / 1e12, 3),
                    "unit": "Tlane-inst/s", "frac": round(lane_rate / VALU_LANE_INST_PEAK, 4), "traffic": traffic}
    else:
        roofline = {"bound": "hbm", "achieved": hbm["algorithmic_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": hbm["frac"], "traffic": traffic}
    roofline.update({"kernel": dom, "kernel_sources": kernel_source_hash(), "avg_launch_ms": round(d["avg_ms"], 3),
                     "valu": valu, "hbm": hbm,
                     "nodes_per_ray": round(d["nodes_per_ray"], 2), "tris_per_ray": round(d["tris_per_ray"], 2)})
    info2 = g.info()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(sc, cfg, params.cpu().numpy(), target.cpu().numpy(), args.cpu_seconds)

    out = {
        "metric": "grad paths/s (fwd+adjoint)",
        "value": round(value, 1),
        "unit": "grad paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %d triangles, %d segments, %d emitters, %d views %dx%d, %d spp, depth %d%s" % (
            sc["name"], sc["tris"].shape[0], sc["num_segments"], len(sc["emitter_seg"]), V, W, H, spp, D,
            ", RR from %d" % rr if rr >= 0 else ""),
            "step": "ipt_loss_grad (colour A + L2 loss/adjoint + gradient B fwd/replay/reduce) + ipt_sgd_step" +
                    (" + %d guide training steps; learned proposal mixed at 0.5" % args.guide_steps if gd else "") +
                    (" (cached: %d cells per side, refilled after training)" % gd.cache_build(gd.cell_area)
                     if cached else ""),
            "paths_per_step": {"colour": paths_step, "gradient": paths_step},
            "parallelism": "1 GPU"},
        "breakdown": {"colour_paths_per_s": round(paths_step / (ms_col * 1e-3), 1),
                      "grad_paths_per_s_fwd_adjoint": round(paths_step / (ms_grad * 1e-3), 1),
                      "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in val.items()}
                                  for k, val in per.items()},
                      "nonfinite_paths": info2["nonfinite_paths"], "stack_overflows": info2["stack_overflows"],
                      "final_loss": float(loss.item())},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(sc, cfg, params, target, budget_s):
    """The FP64 oracle on this host's cores: gradient paths/s of its
    forward+derivative pass (stream B) on a fixed pixel sample (every k-th
    pixel of every view at full spp), sized to about budget_s seconds."""
    from oracle import oracle

    t0 = time.time()
    o = oracle.Scene(sc["verts"], sc["tris"], sc["tri_seg"], sc["num_segments"], sc["emitter_seg"], sc["normals"],
                     material=sc.get("material", 0))
    log("oracle BVH %.1fs" % (time.time() - t0))
    V, W, H = sc["cams"]["cam_to_world"].shape[0], sc["cams"]["width"], sc["cams"]["height"]
    npix = V * W * H
    kw = dict(seed=11, stream_tag=2, iteration=0, spp=cfg["spp"], max_depth=cfg["max_depth"],
              rr_depth=cfg["rr_depth"], mis=2)
    rng = np.random.default_rng(0)
    # probe with a small sample, then size the timed sample to the budget
    stride = max(1, npix // 20000)
    pix = np.arange(0, npix, stride, dtype=np.int64)
    w = rng.normal(size=(pix.size, 3))
    t0 = time.time()
    o.run(sc["cams"], params, pixel_list=pix, w=w, want_grad=True, **kw)
    t_probe = max(time.time() - t0, 1e-3)
    n_target = int(pix.size * budget_s / t_probe)
    stride = max(1, npix // max(1, n_target))
    pix = np.arange(0, npix, stride, dtype=np.int64)
    w = rng.normal(size=(pix.size, 3))
    t0 = time.time()
    o.run(sc["cams"], params, pixel_list=pix, w=w, want_grad=True, **kw)
    dt = time.time() - t0
    paths = pix.size * cfg["spp"]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cpu_model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    log("oracle: %d gradient paths in %.1fs on %d threads" % (paths, dt, threads))
    # the same on one core, on a sixteenth of the sample
    pix1 = pix[::16]
    old = oracle.set_threads(1)
    t0 = time.time()
    o.run(sc["cams"], params, pixel_list=pix1, w=w[::16], want_grad=True, **kw)
    dt1 = time.time() - t0
    oracle.set_threads(old)
    log("oracle on one core: %d gradient paths in %.1fs" % (pix1.size * cfg["spp"], dt1))
    return {"value": round(paths / dt, 1), "unit": "grad paths/s", "cores": threads, "kind": "oracle",
            "sample": "every %d-th pixel of all %d views (%d pixels) at %d spp, forward+derivatives in FP64; "
                      "%.1f s; %s" % (stride, V, pix.size, cfg["spp"], dt, cpu_model),
            "single_core_value": round(pix1.size * cfg["spp"] / dt1, 1)}


if __name__ == "__main__":
    main()
