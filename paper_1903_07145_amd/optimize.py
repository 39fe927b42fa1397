"""Nested SGD of inverse path tracing (Sec. 3, Eq. 3-4): every iteration
renders an independent colour estimate (stream A), forms the L2 adjoint image
against the target, estimates the parameter gradient from an independent set
of paths (stream B) and takes a projected Adam step on the normalised
parameters.  With ``guide=True`` both estimates sample directions from the
learned proposal combined with BRDF sampling (one-sample MIS), the gradient
pass writes training records, and the proposal is trained online between
iterations (mixing weight 0 during the warm-up, ``guide_mix`` after).

Every step runs in the HIP library; this module only sequences the calls.

    python -m paper_1903_07145_amd.optimize --workload apartment --iters 200 --guide
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import ipt, scenes

TAG_TARGET, TAG_A, TAG_B = 0, 1, 2


def render_target(g, dc, p_true, spp_total, D, rr, seed=1, chunk=16, return_var=False):
    """Target images: the true parameters at spp_total samples (stream tag 0),
    rendered in passes of `chunk` samples; with return_var also the per-pixel
    variance of the target (across passes, divided by their number)."""
    npix = dc["num_views"] * dc["width"] * dc["height"]
    acc = torch.zeros((npix, 3), dtype=torch.float64, device="cuda")
    sq = torch.zeros((npix, 3), dtype=torch.float64, device="cuda")
    npass = max(1, spp_total // chunk)
    for i in range(npass):
        o = ipt.render_opts(seed=seed, stream_tag=TAG_TARGET, iteration=i, spp=min(chunk, spp_total),
                            max_depth=D, rr_depth=rr, mis=2)
        img = g.render(dc, p_true, o).double()
        acc += img
        sq += img * img
    mean = acc / npass
    target = mean.float().contiguous()
    if not return_var:
        return target
    var = (sq / npass - mean * mean).clamp_min(0.0) / max(1, npass - 1)
    return target, var.float()


def coverage(g, sc):
    """Pixels per segment hit by the pixel-centre camera rays of every view
    (ipt_trace_rays)."""
    cams = sc["cams"]
    W, H = int(cams["width"]), int(cams["height"])
    c2w = np.asarray(cams["cam_to_world"], np.float64)
    fov = np.asarray(cams["fov_y"], np.float64).reshape(-1)
    seg_of = torch.as_tensor(sc["tri_seg"], dtype=torch.int64, device="cuda")
    cov = torch.zeros(sc["num_segments"], dtype=torch.int64, device="cuda")
    ys, xs = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    for v in range(c2w.shape[0]):
        t = np.tan(0.5 * fov[v])
        d = np.stack([(2 * xs / W - 1) * t * W / H, (1 - 2 * ys / H) * t, -np.ones_like(xs)], -1).reshape(-1, 3)
        d = d @ c2w[v, :3, :3].T
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        o = np.ascontiguousarray(np.broadcast_to(c2w[v, :3, 3], d.shape))
        tri, _ = g.trace_rays(torch.as_tensor(o, dtype=torch.float32, device="cuda").contiguous(),
                              torch.as_tensor(d, dtype=torch.float32, device="cuda").contiguous())
        hit = tri >= 0
        cov += torch.bincount(seg_of[tri[hit].long()], minlength=sc["num_segments"])
    return cov.cpu().numpy()


def target_precision_fd(g, dc, sc, target_var, free, stride=16, spp=16, h=1e-3, seed=98):
    """The Cramer-Rao bound of the L2 fit with the full Gauss-Newton
    information H = J^T S^-1 J over the free set, J from central differences
    of renders at frozen sampling parameters (the same paths on both sides,
    so the difference is smooth) on every stride-th pixel, scaled by stride
    (a uniform pixel sample of the sum).  For free sets too large for the
    random projections of target_precision to estimate H: one render pair
    per parameter instead of several projections per parameter."""
    cfg = sc["render"]
    D, rr = cfg["max_depth"], cfg["rr_depth"]
    P = sc["params"].size
    idx = np.nonzero(free)[0]
    npix = dc["num_views"] * dc["width"] * dc["height"]
    pix = torch.arange(0, npix, stride, dtype=torch.int64, device="cuda")
    p = torch.as_tensor(sc["params"], device="cuda")
    scale = sc["scale"].astype(np.float64)
    lo, hi = sc["lo"].astype(np.float64), sc["hi"].astype(np.float64)
    sig = target_var.double().sqrt()
    sig = sig.clamp_min(1e-3 * float(sig.mean()) + 1e-12).index_select(0, pix).reshape(-1)
    o = ipt.render_opts(seed=seed, stream_tag=TAG_B, spp=spp, max_depth=D, rr_depth=rr, mis=2, pixel_list=pix)
    J = torch.empty((pix.numel() * 3, idx.size), dtype=torch.float32, device="cuda")
    for j, i in enumerate(idx):
        # a step in normalised units, kept inside the parameter's bounds
        th = float(p[i]) / scale[i]
        a, b = max(lo[i], th - h), min(hi[i], th + h)
        pp, pm = p.clone(), p.clone()
        pp[i] = b * scale[i]
        pm[i] = a * scale[i]
        ip = g.render(dc, pp, o, sampling_params=p).reshape(-1).double()
        im = g.render(dc, pm, o, sampling_params=p).reshape(-1).double()
        J[:, j] = ((ip - im) / (b - a) / sig).float()
    H = (J.T.double() @ J.double()) * stride
    H = H + 1e-9 * torch.trace(H) / idx.size * torch.eye(idx.size, dtype=H.dtype, device=H.device)
    cov = torch.linalg.pinv(H, hermitian=True)
    sigma = np.full(P, np.inf)
    sigma[idx] = np.sqrt(np.maximum(torch.diagonal(cov).cpu().numpy(), 0.0))
    return sigma


def target_precision(g, dc, sc, target_var, free=None, nproj=None, spp=16, seed=99, max_full=256):
    """How precisely the target images determine each parameter, in
    normalised units: the Cramer-Rao bound of the L2 fit under the target's
    per-pixel variance S.  H = J^T S^-1 J (Gauss-Newton information) comes
    from random projections of the adjoint: for Rademacher r and
    w = S^-1/2 r, E[(J^T w)(J^T w)^T] = H; two independent gradient estimates
    a, b per projection give the unbiased a b^T.  With at most max_full free
    parameters the bound is sqrt(diag(H_ff^-1)) over the free set (so a
    parameter whose effect other free parameters can mimic counts as poorly
    determined); above that, the per-parameter bound 1 / sqrt(H_ii)."""
    cfg = sc["render"]
    D, rr = cfg["max_depth"], cfg["rr_depth"]
    P = sc["params"].size
    free = np.ones(P, bool) if free is None else free
    idx = np.nonzero(free)[0]
    full = idx.size <= max_full
    nproj = nproj or (max(64, 8 * idx.size) if full else 16)
    p = torch.as_tensor(sc["params"], device="cuda")
    sig = target_var.double().sqrt()
    sig = sig.clamp_min(1e-3 * float(sig.mean()) + 1e-12)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    scale = torch.as_tensor(sc["scale"], dtype=torch.float64, device="cuda")
    fi = torch.as_tensor(idx, device="cuda")
    A, B = [], []
    for k in range(nproj):
        r = torch.randint(0, 2, sig.shape, generator=gen, device="cuda", dtype=torch.int64).double() * 2 - 1
        w = (r / sig).float().contiguous()
        ga = g.render_grad(dc, p, w, ipt.render_opts(seed=seed, stream_tag=TAG_B, iteration=2 * k, spp=spp,
                                                     max_depth=D, rr_depth=rr, mis=2)).double() * scale
        gb = g.render_grad(dc, p, w, ipt.render_opts(seed=seed, stream_tag=TAG_B, iteration=2 * k + 1, spp=spp,
                                                     max_depth=D, rr_depth=rr, mis=2)).double() * scale
        A.append(ga[fi])
        B.append(gb[fi])
    A = torch.stack(A)
    B = torch.stack(B)
    sigma = np.full(P, np.inf)
    if full:
        H = (A.T @ B + B.T @ A) / (2.0 * nproj)
        H = H + 1e-9 * torch.trace(H) / idx.size * torch.eye(idx.size, dtype=H.dtype, device=H.device)
        cov = torch.linalg.pinv(H, hermitian=True)
        sigma[idx] = np.sqrt(np.maximum(torch.diagonal(cov).cpu().numpy(), 0.0))
    else:
        h = (A * B).mean(0).cpu().numpy()
        sigma[idx] = 1.0 / np.sqrt(np.maximum(h, 1e-300))
    return sigma


def identifiable_masks(sc, cov, min_pixels=100, min_ks=0.05, min_emitter_pixels=16, sigma=None, max_sigma=2.5e-3):
    """Which trainable parameters the images determine.

    kd_e: the diffuse albedo of every non-emitting segment seen in at least
    min_pixels pixels, and the emission of every emitter seen directly in at
    least min_emitter_pixels pixels (an emitter's own reflectance is
    negligible next to its emission).
    This is the set the headline RMSE is taken over: the quantities the
    paper's evaluation reports (albedo and emission).
    all_id: kd_e plus specular reflectance of the seen segments, and their
    roughness where the true specular reflectance (mean RGB) is >= min_ks.
    With sigma (target_precision), a parameter also needs sigma <= max_sigma
    (a quarter of the 1e-2 RMSE target): the target must be able to pin it.
    Disney material (13 per segment): the base colour plays the albedo's
    part, and all_id takes every parameter of a seen segment (their
    identifiability is left to sigma)."""
    S = sc["num_segments"]
    P = sc["params"].size
    nm = params_per_segment(sc)
    tr = sc["trainable"].astype(bool)
    emit = set(int(x) for x in sc["emitter_seg"])
    kd_e = np.zeros(P, bool)
    all_id = np.zeros(P, bool)
    for s in range(S):
        if cov[s] < min_pixels or s in emit:
            continue
        kd_e[nm * s:nm * s + 3] = True
        if nm != 7:
            all_id[nm * s:nm * s + nm] = True
            continue
        all_id[7 * s:7 * s + 6] = True
        if sc["params"][7 * s + 3:7 * s + 6].mean() >= min_ks:
            all_id[7 * s + 6] = True
    for k, s in enumerate(sc["emitter_seg"]):
        if cov[s] >= min_emitter_pixels:
            kd_e[nm * S + 3 * k:nm * S + 3 * k + 3] = True
            all_id[nm * S + 3 * k:nm * S + 3 * k + 3] = True
    if sigma is not None:
        ok = sigma <= max_sigma
        kd_e &= ok
        all_id &= ok
    return kd_e & tr, all_id & tr


def unrecoverable_mask(sc, cov, min_pixels=100, min_emitter_pixels=16):
    """Parameters no view can recover: every parameter of a segment seen in
    fewer than min_pixels pixels, the reflectance of emitting segments, and the
    emission of emitters seen in fewer than min_emitter_pixels.  Left free they
    drift and bias the parameters they light (an unseen box's albedo sets the
    indirect light on a seen one), so the optimisation holds them at their true
    values."""
    S = sc["num_segments"]
    nm = params_per_segment(sc)
    fixed = np.zeros(sc["params"].size, bool)
    emit = set(int(x) for x in sc["emitter_seg"])
    for s in range(S):
        if cov[s] < min_pixels or s in emit:
            fixed[nm * s:nm * s + nm] = True
    for k, s in enumerate(sc["emitter_seg"]):
        if cov[s] < min_emitter_pixels:
            fixed[nm * S + 3 * k:nm * S + 3 * k + 3] = True
    return fixed


def param_rmse(params, p_true, scale, trainable):
    """RMSE of the normalised trainable parameters."""
    m = trainable.bool()
    d = (params[m] - p_true[m]) / scale[m]
    return float(torch.sqrt(torch.mean(d * d)))


def params_per_segment(sc):
    return 13 if sc.get("material", 0) == 1 else 7


def group_rmse(params, p_true, scale, trainable, S, nm=7):
    """RMSE per parameter group: diffuse, specular, roughness, emission
    (Lambert + GGX); base colour, the ten other parameters, emission
    (Disney, nm = 13)."""
    d = ((params - p_true) / scale).cpu().numpy()
    t = trainable.cpu().numpy().astype(bool)
    idx = np.arange(d.size)
    if nm == 7:
        groups = dict(kd=(idx < 7 * S) & (idx % 7 < 3), ks=(idx < 7 * S) & (idx % 7 >= 3) & (idx % 7 < 6),
                      alpha=(idx < 7 * S) & (idx % 7 == 6), e=idx >= 7 * S)
    else:
        groups = dict(base=(idx < nm * S) & (idx % nm < 3), other=(idx < nm * S) & (idx % nm >= 3), e=idx >= nm * S)
    return {k: float(np.sqrt(np.mean(d[m & t] ** 2))) for k, m in groups.items() if (m & t).any()}


def cell_area_for(sc, cells):
    """Cell area giving about `cells` cached-proposal cells per side over the
    scene's surface (triangles smaller than a cell get one cell each)."""
    v = np.asarray(sc["verts"], np.float64)
    t = np.asarray(sc["tris"], np.int64)
    area = 0.5 * np.linalg.norm(np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]]), axis=1).sum()
    return float(np.float32(area / cells))


def optimize(sc, iters=None, seed=7, guide=False, guide_mix=0.5, warmup=50, guide_steps=10, guide_lr=2e-3,
             guide_batch=16384, record_stride=None, target_rmse=1e-2, stop_at_target=False, target=None,
             g=None, log=None, spp=None, lr=None, lr_schedule="const", masks=None, lr_final=None, log_every=10,
             fixed=None, beta2=0.999, guide_cells=0, guide_every=1, p_init=None, mis=2, state=None,
             stop_after=None, want_state=False):
    """Runs the optimisation; returns a dict with the RMSE/loss history and timings.

    The time to target is taken on the RMSE over masks[0] (identifiable
    albedo and emission, see identifiable_masks); the RMSE over every
    trainable parameter and over masks[1] is recorded beside it.  Wall-clock
    time counts from the first iteration (scene build and target render
    excluded) and includes guide training in the guided arm.  guide_cells > 0:
    the path kernels sample the cached proposal (about that many cells per
    side, refilled after every training call) instead of evaluating the
    network at every vertex; guide_every: training (and refill) every that
    many iterations.

    The headline is the RMSE over every trainable parameter; the time to
    target is recorded for it (time_to_target_all) and for masks[0]
    (time_to_target).  state (a previous call's result["state"]) resumes a
    run: parameters, Adam moments, iteration, elapsed time, history and,
    with a guide, its weights and up to STATE_RECORDS of its training records
    (its own Adam moments restart).  stop_after ends this call after that many iterations, so a run
    longer than one process can be split; the learning-rate schedule spans
    all `iters`."""
    cfg = sc["render"]
    iters = iters or cfg["iters"]
    spp = spp or cfg["spp"]
    D, rr = cfg["max_depth"], cfg["rr_depth"]
    lr0 = lr or cfg["lr"]
    g = g or ipt.Scene.from_dict(sc)
    if masks is None or fixed is None:
        cov = coverage(g, sc)
        masks = masks if masks is not None else identifiable_masks(sc, cov)
        fixed = fixed if fixed is not None else unrecoverable_mask(sc, cov)
    m_head = torch.as_tensor(masks[0].astype(np.uint8), device="cuda")
    m_id = torch.as_tensor(masks[1].astype(np.uint8), device="cuda")
    dc = ipt.make_cameras(sc["cams"])
    npix = dc["num_views"] * dc["width"] * dc["height"]
    p_true = torch.as_tensor(sc["params"], device="cuda")
    if target is None:
        target = render_target(g, dc, p_true, cfg["target_spp"], D, rr)
    p0 = scenes.init_theta(sc, cfg["init"], seed=seed) if p_init is None else np.array(p_init, np.float32)
    p0[fixed] = sc["params"][fixed]
    params = torch.as_tensor(p0, device="cuda")
    scale = torch.as_tensor(sc["scale"], device="cuda")
    lo = torch.as_tensor(sc["lo"], device="cuda")
    hi = torch.as_tensor(sc["hi"], device="cuda")
    tr_all = torch.as_tensor(sc["trainable"], device="cuda")
    tr = torch.as_tensor((sc["trainable"].astype(bool) & ~fixed).astype(np.uint8), device="cuda")
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.zeros_like(params)
    gd = None
    if guide:
        # about one million training records per iteration
        stride = record_stride or max(1, (npix * spp * 3) // (1 << 20))
        gd = ipt.Guide(g, seed=seed, lr=guide_lr, batch=guide_batch, ring_capacity=1 << 21, record_stride=stride)
        if guide_cells:
            gd.cache_build(cell_area_for(sc, guide_cells))
    cached = 1 if (gd is not None and guide_cells) else 0
    g.workspace(dc, ipt.render_opts(spp=spp, max_depth=D, rr_depth=rr, guide=gd, guide_mix=guide_mix if gd else 0.0,
                                    guide_cached=cached))
    hist = dict(it=[], t=[], rmse=[], rmse_all=[], rmse_id=[], loss=[], guide_loss=[], groups=[])
    it0, t_prev, t_hit, t_hit_all = 0, 0.0, None, None
    if state is not None:
        params.copy_(torch.as_tensor(state["params"], device="cuda"))
        m.copy_(torch.as_tensor(state["m"], device="cuda"))
        v.copy_(torch.as_tensor(state["v"], device="cuda"))
        it0, t_prev = int(state["it"]), float(state["t"])
        hist = state["hist"]
        t_hit, t_hit_all = state.get("t_hit"), state.get("t_hit_all")
        if gd is not None and state.get("guide_w") is not None:
            gd.set_weights(state["guide_w"])
            if state.get("guide_rec") is not None and len(state["guide_rec"]):
                gd.add_records(state["guide_rec"])
            if cached:
                gd.cache_build(gd.cell_area)
    it_end = iters if stop_after is None else min(iters, it0 + stop_after)
    torch.cuda.synchronize()
    t0 = time.time() - t_prev
    for it in range(it0, it_end):
        mix = guide_mix if (gd is not None and it >= warmup) else 0.0
        kw = dict(seed=1000 * seed + 11, iteration=it, spp=spp, max_depth=D, rr_depth=rr, mis=mis)
        co = ipt.render_opts(stream_tag=TAG_A, guide=gd if mix > 0 else None, guide_mix=mix, guide_cached=cached, **kw)
        go = ipt.render_opts(stream_tag=TAG_B, guide=gd, guide_mix=mix, guide_cached=cached, **kw)
        g.loss_grad(dc, params, target, co, go, 0, loss=loss, grad=grad)
        # constant, or cosine decay from lr0 to lr_final (default lr0/20) over the run
        lr_end = lr_final if lr_final is not None else lr0 / 20
        lr_it = lr0 if lr_schedule == "const" else lr_end + (lr0 - lr_end) * 0.5 * (1 + np.cos(np.pi * it / iters))
        ipt.sgd_step(params, grad, m, v, it + 1, lr=lr_it, beta2=beta2, scale=scale, lo=lo, hi=hi, trainable=tr)
        gl = None
        if gd is not None and it % guide_every == 0 and gd.records() >= guide_batch:
            gl = gd.train(guide_steps, want_loss=(it % 10 == 0))
            if cached:
                gd.cache_build(gd.cell_area)
        r = param_rmse(params, p_true, scale, m_head)   # synchronises
        t = time.time() - t0
        hist["it"].append(it)
        hist["t"].append(t)
        hist["rmse"].append(r)
        hist["rmse_all"].append(param_rmse(params, p_true, scale, tr_all))
        hist["rmse_id"].append(param_rmse(params, p_true, scale, m_id))
        hist["loss"].append(float(loss.cpu()))
        hist["guide_loss"].append(gl)
        hist["groups"].append(group_rmse(params, p_true, scale, tr, sc["num_segments"], params_per_segment(sc))
                              if (it % log_every == 0 or it == iters - 1) else None)
        if t_hit_all is None and hist["rmse_all"][-1] <= target_rmse:
            t_hit_all = t
        if t_hit is None and r <= target_rmse:
            t_hit = t
            if stop_at_target:
                break
        if log and (it % log_every == 0 or it == iters - 1):
            gr = " ".join("%s %.3f" % kv for kv in hist["groups"][-1].items())
            log("it %4d  t %7.2fs  loss %.5f  rmse all %.4f (headline subset %.4f, identifiable %.4f; %s)%s" % (
                it, t, hist["loss"][-1], hist["rmse_all"][-1], r, hist["rmse_id"][-1], gr,
                "" if gl is None else "  guide loss %.4f" % gl))
    err = ((params - p_true) / scale).cpu().numpy()
    worst = [(int(i), float(err[i])) for i in np.argsort(-np.abs(err * masks[0]))[:8]]
    optimize.last = dict(params=params, guide=gd, target=target, g=g, dc=dc, fixed=fixed,
                         init=torch.as_tensor(p0, device="cuda"))
    out_state = None
    if want_state:
        out_state = dict(params=params.cpu().numpy(), m=m.cpu().numpy(), v=v.cpu().numpy(), it=it_end,
                         t=hist["t"][-1] if hist["t"] else 0.0, hist=hist, t_hit=t_hit, t_hit_all=t_hit_all,
                         guide_w=None if gd is None else gd.get_weights(),
                         guide_rec=None if gd is None else gd.read_records(
                             min(gd.records(), gd.capacity, STATE_RECORDS)).cpu().numpy())
    return dict(history=hist, time_to_target=t_hit, time_to_target_all=t_hit_all, final_rmse=hist["rmse"][-1],
                final_rmse_all=hist["rmse_all"][-1], final_rmse_id=hist["rmse_id"][-1], seconds=hist["t"][-1],
                iters=len(hist["it"]), guide=guide, seed=seed, n_head=int(masks[0].sum()),
                n_id=int(masks[1].sum()), worst=worst, done=it_end >= iters, state=out_state)


# training records kept in a saved state (a part of the ring: 16 MiB)
STATE_RECORDS = 1 << 18


def save_state(path, st):
    """A run's state for resuming: arrays in path.arrays (numpy's zip
    format), the rest in path.json."""
    arrays = {k: np.asarray(st[k]) for k in ("params", "m", "v", "guide_w", "guide_rec") if st.get(k) is not None}
    with open(path + ".arrays", "wb") as f:
        np.savez(f, **arrays)
    meta = {k: st[k] for k in ("it", "t", "hist", "t_hit", "t_hit_all")}
    with open(path + ".json", "w") as f:
        json.dump(meta, f)


def load_state(path):
    if not (os.path.exists(path + ".arrays") and os.path.exists(path + ".json")):
        return None
    with np.load(path + ".arrays") as z:
        st = {k: z[k] for k in z.files}
    with open(path + ".json") as f:
        st.update(json.load(f))
    return st


def paper_setting_masks(sc, cov, sigma=None, max_sigma=2.5e-3):
    """(fixed, head) for the all-emissive setting.  Held at their true values:
    every parameter of a segment seen in fewer than 100 pixels (16 for the
    scene's own emitters) and the reflectance of those emitters.  Headline:
    albedo of the seen segments that do not emit and emission of every seen
    segment (zero for all but the scene's own emitters), restricted, with
    sigma (target_precision over the free set), to the parameters the target
    pins to sigma <= max_sigma.  With every segment free to emit, an
    indirectly lit surface's albedo and its own emission explain its pixels
    almost equally well, so its albedo is often not pinned."""
    S = sc["num_segments"]
    true_emit = set(int(x) for x in sc.get("true_emitters", sc["emitter_seg"]))
    fixed = np.zeros(sc["params"].size, bool)
    head = np.zeros(sc["params"].size, bool)
    for s_ in range(S):
        seen = cov[s_] >= 100 or (s_ in true_emit and cov[s_] >= 16)
        if not seen:
            fixed[7 * s_:7 * s_ + 7] = True
            fixed[7 * S + 3 * s_:7 * S + 3 * s_ + 3] = True
            continue
        if s_ in true_emit:
            fixed[7 * s_:7 * s_ + 7] = True
        else:
            head[7 * s_:7 * s_ + 3] = True
        head[7 * S + 3 * s_:7 * S + 3 * s_ + 3] = True
    head &= sc["trainable"].astype(bool) & ~fixed
    if sigma is not None:
        head &= sigma <= max_sigma
    return fixed, head


def optimize_paper_setting(sc, iters=2000, seed=7, batch=8, spp=512, grad_spp=1, lr=5e-3, lam=1e-3, beta2=0.999,
                           target=None, g=None, log=None, log_every=100, target_rmse=1e-2, cov=None, loss_kind=1,
                           masks=None, max_depth=None, mis=2, time_budget=None):
    """The paper's own optimisation setting (Sec. 4.5, "Optimization Parameters";
    App. E): every segment emissive (scenes.all_emissive), albedo and
    emission initialised to zero, each iteration a batch of `batch` pixels
    drawn uniformly from all pixels of all views, `spp` paths per pixel for
    the colour estimate and `grad_spp` (one, the split Sec. 4 finds best) for
    the independent derivative estimate, the L1 loss and its sign adjoint, an
    L1 regulariser of weight `lam` (per unit of normalised emission) on every
    emission, Adam at lr 5e-3.  masks: (fixed, head) from
    paper_setting_masks (coverage only when None).  max_depth / mis override
    the workload's; time_budget (seconds) ends the run early."""
    cfg = sc["render"]
    D, rr = max_depth or cfg["max_depth"], cfg["rr_depth"]
    g = g or ipt.Scene.from_dict(sc)
    dc = ipt.make_cameras(sc["cams"])
    npix = dc["num_views"] * dc["width"] * dc["height"]
    S = sc["num_segments"]
    p_true = torch.as_tensor(sc["params"], device="cuda")
    if target is None:
        target = render_target(g, dc, p_true, cfg["target_spp"], D, rr)
    if masks is None:
        masks = paper_setting_masks(sc, coverage(g, sc) if cov is None else cov)
    fixed, head = masks
    tr_np = sc["trainable"].astype(bool)
    p0 = np.where(tr_np & ~fixed, 0.0, sc["params"]).astype(np.float32)
    # ks and roughness (when trainable) start at the middle of their range
    for s_ in range(S):
        if not fixed[7 * s_] and tr_np[7 * s_ + 3]:
            p0[7 * s_ + 3:7 * s_ + 6] = 0.5
            p0[7 * s_ + 6] = 0.5
    params = torch.as_tensor(p0, device="cuda")
    scale = torch.as_tensor(sc["scale"], device="cuda")
    lo = torch.as_tensor(sc["lo"], device="cuda")
    hi = torch.as_tensor(sc["hi"], device="cuda")
    tr = torch.as_tensor((tr_np & ~fixed).astype(np.uint8), device="cuda")
    m_head = torch.as_tensor(head.astype(np.uint8), device="cuda")
    w_l1 = np.zeros(sc["params"].size, np.float32)
    w_l1[7 * S:] = lam / sc["scale"][7 * S:]
    w_l1[fixed] = 0.0
    w_l1 = torch.as_tensor(w_l1, device="cuda")
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.zeros_like(params)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    pix0 = torch.zeros(batch, dtype=torch.int64, device="cuda")
    g.workspace(dc, ipt.render_opts(spp=spp, max_depth=D, rr_depth=rr, pixel_list=pix0))
    hist = dict(it=[], t=[], rmse=[], loss=[])
    torch.cuda.synchronize()
    t0 = time.time()
    t_hit = None
    for it in range(iters):
        pix = torch.randint(0, npix, (batch,), generator=gen, device="cuda")
        tgt = target.index_select(0, pix).contiguous()
        kw = dict(seed=1000 * seed + 17, iteration=it, max_depth=D, rr_depth=rr, mis=mis, pixel_list=pix)
        g.loss_grad(dc, params, tgt, ipt.render_opts(stream_tag=TAG_A, spp=spp, **kw),
                    ipt.render_opts(stream_tag=TAG_B, spp=grad_spp, **kw), loss_kind, loss=loss, grad=grad)
        ipt.l1_reg(params, grad, w_l1, loss)
        ipt.sgd_step(params, grad, m, v, it + 1, lr=lr, beta2=beta2, scale=scale, lo=lo, hi=hi, trainable=tr)
        if it % 10 == 0 or it == iters - 1:
            r = param_rmse(params, p_true, scale, m_head)
            t = time.time() - t0
            hist["it"].append(it)
            hist["t"].append(t)
            hist["rmse"].append(r)
            hist["loss"].append(float(loss.cpu()))
            if t_hit is None and r <= target_rmse:
                t_hit = t
            if log and (it % log_every == 0 or it == iters - 1):
                log("it %5d  t %7.2fs  batch loss %.5f  rmse %.4f" % (it, t, hist["loss"][-1], r))
            if time_budget is not None and t >= time_budget:
                iters = it + 1
                break
    err = ((params - p_true) / scale).cpu().numpy()
    worst = [(int(i), float(err[i])) for i in np.argsort(-np.abs(err * head))[:6]]
    free = tr_np & ~fixed
    return dict(history=hist, time_to_target=t_hit, final_rmse=hist["rmse"][-1], seconds=hist["t"][-1],
                final_rmse_free=float(np.sqrt(np.mean(err[free] ** 2))),
                iters=iters, seed=seed, n_head=int(head.sum()), worst=worst, batch=batch, spp=spp, grad_spp=grad_spp,
                lr=lr, lam=lam,
                loss_kind=loss_kind, beta2=beta2)


# The paper's optimiser ablations (Sec. 4, "Optimizer Ablation"; supplement:
# batch size, variance reduction, number of bounces), each as variants of the
# pixel-batch optimiser under one wall-clock budget.  Fixed: L1 loss, Adam lr
# 5e-3, the workload's emitters (not all-emissive), zero init.
ABLATIONS = {
    # paths per pixel of the colour estimate (one derivative path)
    "spp": [dict(spp=s, grad_spp=1) for s in (1, 8, 128, 1024)],
    # a budget of 128 paths per pixel split between colour and derivative
    "split": [dict(spp=128 - d, grad_spp=d) for d in (1, 32, 64, 96, 127)],
    # pixels per batch at 128 + 1 paths per pixel
    "batch": [dict(batch=b, spp=128, grad_spp=1) for b in (1, 8, 64, 512)],
    # light sampling + MIS against BRDF sampling only
    "mis": [dict(mis=2, spp=128, grad_spp=1), dict(mis=0, spp=128, grad_spp=1)],
    # bounces used by the optimiser, against a 10-bounce target
    "bounces": [dict(max_depth=d, spp=128, grad_spp=1) for d in (1, 2, 3)],
}


def run_ablation(sc, kind, budget, seeds, target_spp=4096, log=None, lam=1e-3):
    """Headline RMSE of each variant per seed: at a quarter of the budget and
    averaged over its second half (at a constant learning rate the iterate
    keeps fluctuating, so a single final value is noisy).  The bounce
    ablation renders its target with 10 bounces."""
    cfg = sc["render"]
    g = ipt.Scene.from_dict(sc)
    dc = ipt.make_cameras(sc["cams"])
    tD = 10 if kind == "bounces" else cfg["max_depth"]
    target, tvar = render_target(g, dc, torch.as_tensor(sc["params"], device="cuda"), target_spp, tD,
                                 cfg["rr_depth"], return_var=True)
    cov = coverage(g, sc)
    fixed, _ = paper_setting_masks(sc, cov)
    sigma = target_precision(g, dc, sc, tvar, free=sc["trainable"].astype(bool) & ~fixed)
    masks = paper_setting_masks(sc, cov, sigma=sigma)
    out = []
    for v in ABLATIONS[kind]:
        row = dict(variant=v, final=[], quarter=[], late_mean=[], iters=[])
        for seed in seeds:
            kw = dict(batch=8, spp=128, grad_spp=1)
            kw.update(v)
            res = optimize_paper_setting(sc, iters=10 ** 7, seed=seed, lr=5e-3, lam=lam, beta2=0.999, target=target,
                                         g=g, masks=masks, time_budget=budget, **kw)
            h = res["history"]
            t = np.asarray(h["t"])
            r = np.asarray(h["rmse"])
            row["final"].append(res["final_rmse"])
            row["quarter"].append(float(r[min(len(r) - 1, int(np.searchsorted(t, budget / 4)))]))
            row["late_mean"].append(float(r[t >= budget / 2].mean()))
            row["iters"].append(res["iters"])
        if log:
            log("ablation %s %s: rmse at %.1fs median %.4f; mean over [%.1fs, %.1fs] median %.4f (seeds %s); "
                "iterations %d" % (kind, v, budget / 4, np.median(row["quarter"]), budget / 2, budget,
                                   np.median(row["late_mean"]), np.round(row["late_mean"], 4).tolist(),
                                   int(np.median(row["iters"]))))
        out.append(row)
    return out


def train_guide_at(g, dc, sc, params, target, iters=100, warmup=5, guide_steps=10, guide_mix=0.5, seed=7,
                   guide_cells=0, guide_lr=2e-3, guide_batch=16384, spp=None, mis=2):
    """A guide trained online at fixed parameters: every iteration a gradient
    pass writes records (sampling the guide after `warmup` iterations) and
    the guide takes `guide_steps` training steps; the parameters do not
    change.  Returns the guide (its cached rows refilled when guide_cells)."""
    cfg = sc["render"]
    spp = spp or cfg["spp"]
    D, rr = cfg["max_depth"], cfg["rr_depth"]
    npix = dc["num_views"] * dc["width"] * dc["height"]
    stride = max(1, (npix * spp * 3) // (1 << 20))
    gd = ipt.Guide(g, seed=seed, lr=guide_lr, batch=guide_batch, ring_capacity=1 << 21, record_stride=stride)
    cached = 0
    if guide_cells:
        gd.cache_build(cell_area_for(sc, guide_cells))
        cached = 1
    for it in range(iters):
        mix = guide_mix if it >= warmup else 0.0
        kw = dict(seed=1000 * seed + 13, iteration=it, spp=spp, max_depth=D, rr_depth=rr, mis=mis)
        co = ipt.render_opts(stream_tag=TAG_A, **kw)
        go = ipt.render_opts(stream_tag=TAG_B, guide=gd, guide_mix=mix, guide_cached=cached, **kw)
        g.loss_grad(dc, params, target, co, go, 0)
        if gd.records() >= guide_batch:
            gd.train(guide_steps, want_loss=False)
            if cached:
                gd.cache_build(gd.cell_area)
    torch.cuda.synchronize()
    return gd


def pixel_triangles(g, sc):
    """Input triangle hit by the centre ray of every pixel of every view, in
    the images' pixel order (-1: none)."""
    cams = sc["cams"]
    W, H = int(cams["width"]), int(cams["height"])
    c2w = np.asarray(cams["cam_to_world"], np.float64)
    fov = np.asarray(cams["fov_y"], np.float64).reshape(-1)
    ys, xs = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    out = []
    for v in range(c2w.shape[0]):
        t = np.tan(0.5 * fov[v])
        d = np.stack([(2 * xs / W - 1) * t * W / H, (1 - 2 * ys / H) * t, -np.ones_like(xs)], -1).reshape(-1, 3)
        d = d @ c2w[v, :3, :3].T
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        o = np.ascontiguousarray(np.broadcast_to(c2w[v, :3, 3], d.shape))
        tri, _ = g.trace_rays(torch.as_tensor(o, dtype=torch.float32, device="cuda").contiguous(),
                              torch.as_tensor(d, dtype=torch.float32, device="cuda").contiguous())
        out.append(tri.cpu().numpy().astype(np.int64))
    return np.concatenate(out)


def triangle_errors(image, target, pix_tri, T):
    """Mean l2 error (mean over channels of (image - target)^2) of the pixels
    each triangle covers (the refinement criterion of the paper's textured
    scenes, supplement Sec. "Results on Scenes with Textures"), and the pixel
    count per triangle."""
    e = ((image - target) ** 2).mean(dim=1).double().cpu().numpy()
    m = pix_tri >= 0
    cnt = np.bincount(pix_tri[m], minlength=T)
    tot = np.bincount(pix_tri[m], weights=e[m], minlength=T)
    return np.where(cnt > 0, tot / np.maximum(cnt, 1), 0.0), cnt


def texture_rmse(sc, params, tri_kd, cnt):
    """Albedo error per triangle (each triangle's own or its segment's kd
    against its true kd), RMSE weighted by the pixels each triangle covers."""
    p = params.cpu().numpy() if torch.is_tensor(params) else np.asarray(params)
    seg = np.asarray(sc["tri_seg"], np.int64)
    kd = p[7 * seg[:, None] + np.arange(3)[None, :]]
    w = cnt.astype(np.float64)
    return float(np.sqrt((w[:, None] * (kd - tri_kd) ** 2).sum() / (3 * w.sum())))


def _refined_scene(sc0, refined, tri_vals, emission):
    """sc0 with one material per triangle in `refined` (values tri_vals [T, 7])
    and, for every other triangle, its object's current material (shared by
    the object's unrefined triangles)."""
    S0 = sc0["num_segments"]
    p = np.array(sc0["params"], np.float32)
    seg = np.asarray(sc0["tri_seg"], np.int64)
    rest = np.setdiff1d(np.arange(seg.size), refined)
    for s_ in range(S0):
        t = rest[seg[rest] == s_]
        if t.size:
            p[7 * s_:7 * s_ + 7] = tri_vals[t[0]]
    p[7 * S0:] = emission
    return scenes.per_triangle(dict(sc0, params=p), tris=refined, tri_params=tri_vals)


def coarse_to_fine(sc, iters_coarse=300, iters_fine=200, rounds=3, seed=7, spp=None, refine="excess", log=None,
                   lr=1e-2, beta2=0.9):
    """Coarse-to-fine optimisation on a textured scene (App. E; App. B,
    scenes with textures): one material per object first; then, `rounds`
    times, every triangle whose covered pixels carry a mean l2 re-rendering
    error above a threshold gets a material of its own and the optimisation
    continues from the current estimate.  refine="above_mean": the mean over
    all covered pixels; refine="excess" (default): the error expected from
    Monte Carlo noise alone (half the mean squared difference of two
    independent renders of the estimate, plus the target's variance) by more
    than 3 standard errors; refine="all": every seen triangle at once (the
    comparison arm).  Emission stays
    trainable.  sc: a per-object scene with `tri_params` (true per-triangle
    materials).  Returns the texture RMSE (albedo per triangle, weighted by
    covered pixels) and image error after each phase."""
    cfg = sc["render"]
    D, rr = cfg["max_depth"], cfg["rr_depth"]
    spp = spp or cfg["spp"]
    tri_true = np.asarray(sc["tri_params"], np.float32)
    tri_kd = tri_true[:, :3].astype(np.float64)
    T = sc["tris"].shape[0]
    S0 = sc["num_segments"]
    gt = scenes.per_triangle(sc, tri_params=tri_true)
    g_gt = ipt.Scene.from_dict(gt)
    dc = ipt.make_cameras(sc["cams"])
    target, tvar = render_target(g_gt, dc, torch.as_tensor(gt["params"], device="cuda"), cfg["target_spp"], D, rr,
                                 return_var=True)
    del g_gt
    g = ipt.Scene.from_dict(sc)
    pix_tri = pixel_triangles(g, sc)
    eval_opts = ipt.render_opts(seed=5, stream_tag=1, spp=64, max_depth=D, rr_depth=rr, mis=2)
    eval_opts2 = ipt.render_opts(seed=6, stream_tag=1, spp=64, max_depth=D, rr_depth=rr, mis=2)

    def excess_pick(g_, p, img):
        # per triangle: mean squared error against the target, against what
        # noise alone gives (render variance from two independent renders,
        # plus the target's variance); refine where it is 3 standard errors above
        img2 = g_.render(dc, p, eval_opts2)
        e, cnt_ = triangle_errors(img, target, pix_tri, T)
        nv = ((img - img2) ** 2).mean(dim=1) / 2 + tvar.mean(dim=1)
        m = pix_tri >= 0
        noise = np.bincount(pix_tri[m], weights=nv.double().cpu().numpy()[m], minlength=T) / np.maximum(cnt_, 1)
        e2 = ((img - target) ** 2).mean(dim=1).double().cpu().numpy()
        sq = np.bincount(pix_tri[m], weights=e2[m] ** 2, minlength=T) / np.maximum(cnt_, 1)
        se = np.sqrt(np.maximum(sq - e ** 2, 0.0) / np.maximum(cnt_, 1))
        return np.nonzero((cnt_ > 0) & (e - noise > 3.0 * se))[0]

    def run(scene, truth, g_, iters, p_init, it_seed):
        fixed = np.zeros(scene["params"].size, bool)
        for s_ in scene["emitter_seg"]:
            fixed[7 * int(s_):7 * int(s_) + 7] = True
        head = scene["trainable"].astype(bool) & ~fixed
        res = optimize(dict(scene, params=truth), iters=iters, seed=it_seed, target=target, g=g_, spp=spp, lr=lr,
                       lr_schedule="cos", masks=(head, head), fixed=fixed, beta2=beta2, log=log, log_every=100,
                       p_init=p_init)
        p = optimize.last["params"]
        img = g_.render(dc, p, eval_opts)
        return p, img, res["seconds"]

    phases = []
    p_c, img, sec = run(sc, sc["params"], g, iters_coarse, None, seed)
    g_cur, p_cur = g, p_c
    err, cnt = triangle_errors(img, target, pix_tri, T)
    phases.append(dict(phase="objects", segments=S0, texture_rmse=texture_rmse(sc, p_c, tri_kd, cnt),
                       image_l2=float(((img - target) ** 2).mean()), seconds=sec))
    pc = p_c.cpu().numpy()
    tri_vals = pc[7 * np.asarray(sc["tri_seg"], np.int64)[:, None] + np.arange(7)[None, :]].astype(np.float32)
    emission = pc[7 * S0:]
    refined = np.zeros(0, np.int64)
    for r in range(1 if refine == "all" else rounds):
        if refine == "all":
            new = np.nonzero(cnt > 0)[0]
        elif refine == "excess":
            new = excess_pick(g_cur, p_cur, img)
        else:
            mean_err = (err * cnt).sum() / max(cnt.sum(), 1)
            new = np.nonzero((cnt > 0) & (err > mean_err))[0]
        refined = np.union1d(refined, new)
        scene = _refined_scene(sc, refined, tri_vals, emission)
        truth = scenes.per_triangle(sc, tris=refined, tri_params=tri_true)["params"]
        g2 = ipt.Scene.from_dict(scene)
        iters = iters_fine * (rounds if refine == "all" else 1)
        p_f, img, sec = run(scene, truth, g2, iters, scene["params"], seed + 1 + r)
        err, _ = triangle_errors(img, target, pix_tri, T)
        pf = p_f.cpu().numpy()
        tri_vals = pf[7 * np.asarray(scene["tri_seg"], np.int64)[:, None] + np.arange(7)[None, :]].astype(np.float32)
        emission = pf[7 * scene["num_segments"]:]
        phases.append(dict(phase="refine %d" % (r + 1), segments=scene["num_segments"], refined=int(refined.size),
                           texture_rmse=texture_rmse(scene, p_f, tri_kd, cnt),
                           image_l2=float(((img - target) ** 2).mean()), seconds=sec,
                           params_global=int(g2.info()["params_global"])))
        g_cur, p_cur = g2, p_f
    return dict(phases=phases, seen_triangles=int((cnt > 0).sum()), refine=refine)


def fine_texture(n_gt=24, n_opt=6, rounds=2, iters_objects=300, iters=300, seed=7, lr=1e-2, beta2=0.9, spp=None,
                 log=None):
    """Texture finer than the mesh (supplement, scenes with textures): the
    target comes from walls tessellated n_gt x n_gt with one albedo per
    triangle; the optimisation starts from an n_opt x n_opt mesh with one
    material per object, then gives every triangle its own material, then
    `rounds` times splits the triangles whose re-rendering error exceeds the
    noise floor (R-31) into four (scenes.subdivide) and continues.  The
    measure is the albedo seen at each pixel (the estimate of the triangle
    the pixel's centre ray hits against the ground truth's)."""
    tex_gt = scenes.textured_cornell(n=n_gt)
    cfg = tex_gt["render"]
    D, rr = cfg["max_depth"], cfg["rr_depth"]
    spp = spp or cfg["spp"]
    gt = scenes.per_triangle(tex_gt, tri_params=tex_gt["tri_params"])
    g_gt = ipt.Scene.from_dict(gt)
    dc = ipt.make_cameras(tex_gt["cams"])
    target, tvar = render_target(g_gt, dc, torch.as_tensor(gt["params"], device="cuda"), cfg["target_spp"], D, rr,
                                 return_var=True)
    pix_gt = pixel_triangles(g_gt, gt)
    del g_gt
    seen = pix_gt >= 0
    kd_gt = np.asarray(tex_gt["tri_params"], np.float64)[np.maximum(pix_gt, 0), :3]
    eval1 = ipt.render_opts(seed=5, stream_tag=1, spp=64, max_depth=D, rr_depth=rr, mis=2)
    eval2 = ipt.render_opts(seed=6, stream_tag=1, spp=64, max_depth=D, rr_depth=rr, mis=2)

    def pixel_albedo_rmse(scene, g_, p):
        pt = pixel_triangles(g_, scene)
        ok = seen & (pt >= 0)
        pp = p.cpu().numpy()
        seg = np.asarray(scene["tri_seg"], np.int64)[np.maximum(pt, 0)]
        kd = pp[7 * seg[:, None] + np.arange(3)[None, :]]
        return float(np.sqrt(((kd - kd_gt)[ok] ** 2).mean())), pt

    def run(scene, g_, iters_, p_init, it_seed):
        fixed = np.zeros(scene["params"].size, bool)
        for s_ in scene["emitter_seg"]:
            fixed[7 * int(s_):7 * int(s_) + 7] = True
        head = scene["trainable"].astype(bool) & ~fixed
        # the progress RMSE is against the estimate's own start (no per-parameter truth exists here)
        res = optimize(scene, iters=iters_, seed=it_seed, target=target, g=g_, spp=spp, lr=lr, lr_schedule="cos",
                       masks=(head, head), fixed=fixed, beta2=beta2, log=None, p_init=p_init)
        return optimize.last["params"], res["seconds"]

    def noisy_tris(scene, g_, p, pt):
        img = g_.render(dc, p, eval1)
        img2 = g_.render(dc, p, eval2)
        T = scene["tris"].shape[0]
        e, cnt = triangle_errors(img, target, pt, T)
        nv = ((img - img2) ** 2).mean(dim=1) / 2 + tvar.mean(dim=1)
        m = pt >= 0
        noise = np.bincount(pt[m], weights=nv.double().cpu().numpy()[m], minlength=T) / np.maximum(cnt, 1)
        e2 = ((img - target) ** 2).mean(dim=1).double().cpu().numpy()
        sq = np.bincount(pt[m], weights=e2[m] ** 2, minlength=T) / np.maximum(cnt, 1)
        se = np.sqrt(np.maximum(sq - e ** 2, 0.0) / np.maximum(cnt, 1))
        return np.nonzero((cnt > 0) & (e - noise > 3.0 * se))[0], float(((img - target) ** 2).mean())

    phases = []
    scene = scenes.textured_cornell(n=n_opt)
    scene.pop("tri_params", None)
    scene.pop("albedo_at", None)
    g = ipt.Scene.from_dict(scene)
    p, sec = run(scene, g, iters_objects, None, seed)
    r, pt = pixel_albedo_rmse(scene, g, p)
    _, l2 = noisy_tris(scene, g, p, pt)
    phases.append(dict(phase="objects", triangles=int(scene["tris"].shape[0]), segments=scene["num_segments"],
                       pixel_albedo_rmse=r, image_l2=l2, seconds=sec))
    # one material per triangle
    scene = scenes.per_triangle(dict(scene, params=p.cpu().numpy()))
    g = ipt.Scene.from_dict(scene)
    p, sec = run(scene, g, iters, scene["params"], seed + 1)
    r, pt = pixel_albedo_rmse(scene, g, p)
    pick, l2 = noisy_tris(scene, g, p, pt)
    phases.append(dict(phase="per triangle", triangles=int(scene["tris"].shape[0]), segments=scene["num_segments"],
                       pixel_albedo_rmse=r, image_l2=l2, seconds=sec))
    for k in range(rounds):
        if pick.size == 0:
            break
        sub = scenes.subdivide(dict(scene, params=p.cpu().numpy()), pick)
        children = np.nonzero(np.isin(sub["parent_tri"], pick))[0]
        scene = scenes.per_triangle(sub, tris=children)
        g = ipt.Scene.from_dict(scene)
        p, sec = run(scene, g, iters, scene["params"], seed + 2 + k)
        r, pt = pixel_albedo_rmse(scene, g, p)
        pick, l2 = noisy_tris(scene, g, p, pt)
        phases.append(dict(phase="subdivide %d" % (k + 1), split=int(children.size // 4),
                           triangles=int(scene["tris"].shape[0]), segments=scene["num_segments"],
                           pixel_albedo_rmse=r, image_l2=l2, seconds=sec,
                           params_global=int(g.info()["params_global"])))
        if log:
            log("fine texture: %s" % phases[-1])
    return dict(phases=phases, n_gt=n_gt, n_opt=n_opt)


def gradient_variance(g, dc, sc, params, target, guide, free, K=32, spp=None, guide_mix=0.5, seed=555, cached=0,
                      mis=2):
    """Per-parameter variance of the loss gradient over K independent seeds at
    fixed parameters, with plain BRDF sampling and with the learned proposal
    (one-sample MIS at guide_mix), plus the mean time per gradient of each.
    Returns a dict of summary statistics over the free parameters."""
    cfg = sc["render"]
    spp = spp or cfg["spp"]
    D, rr = cfg["max_depth"], cfg["rr_depth"]
    out = {}
    for arm, gd, mix in (("brdf", None, 0.0), ("guided", guide, guide_mix)):
        G = []
        torch.cuda.synchronize()
        t0 = time.time()
        for k in range(K):
            kw = dict(seed=seed + k, iteration=k, spp=spp, max_depth=D, rr_depth=rr, mis=mis)
            co = ipt.render_opts(stream_tag=TAG_A, guide=gd, guide_mix=mix, guide_cached=cached if gd else 0, **kw)
            go = ipt.render_opts(stream_tag=TAG_B, guide=gd, guide_mix=mix, guide_cached=cached if gd else 0, **kw)
            _, gr = g.loss_grad(dc, params, target, co, go, 0)
            G.append(gr.double().clone())
        torch.cuda.synchronize()
        dt = (time.time() - t0) / K
        G = torch.stack(G).cpu().numpy()[:, free]
        out[arm] = dict(var=G.var(axis=0, ddof=1), mean=G.mean(axis=0), sec=dt)
    vb, vg = out["brdf"]["var"], out["guided"]["var"]
    ok = vb > 0
    ratio = vb[ok] / np.maximum(vg[ok], 1e-300)
    return dict(K=K, n_params=int(ok.sum()), sec_per_grad_brdf=out["brdf"]["sec"],
                sec_per_grad_guided=out["guided"]["sec"], var_ratio_median=float(np.median(ratio)),
                var_ratio_gmean=float(np.exp(np.mean(np.log(ratio)))),
                frac_params_lower_var_guided=float((ratio > 1).mean()),
                total_var_brdf=float(vb.sum()), total_var_guided=float(vg.sum()),
                efficiency_gain=float(vb.sum() * out["brdf"]["sec"] / (vg.sum() * out["guided"]["sec"])),
                mean_shift_z_median=float(np.median(np.abs(out["brdf"]["mean"] - out["guided"]["mean"]) /
                                                    np.sqrt((vb + vg) / K + 1e-300))))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="apartment", choices=sorted(scenes.WORKLOADS))
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--seeds", type=int, nargs="+", default=[7])
    ap.add_argument("--guide", action="store_true")
    ap.add_argument("--guide-mix", type=float, default=0.5)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--guide-steps", type=int, default=10)
    ap.add_argument("--guide-cells", type=int, default=0,
                    help="> 0: sample the cached proposal with about this many cells per side")
    ap.add_argument("--guide-every", type=int, default=1, help="train the guide every this many iterations")
    ap.add_argument("--mis", type=int, default=2, choices=[0, 1, 2, 3],
                    help="light transport: 0 BRDF sampling only, 1 light sampling only, 2 balance MIS, 3 power")
    ap.add_argument("--target-rmse", type=float, default=1e-2)
    ap.add_argument("--lr", type=float, default=None)
    ap.add_argument("--spp", type=int, default=None)
    ap.add_argument("--lr-final", type=float, default=None)
    ap.add_argument("--target-spp", type=int, default=None)
    ap.add_argument("--beta2", type=float, default=0.999)
    ap.add_argument("--variance", type=int, default=0,
                    help="after the run (with --guide), compare the gradient variance of K seeds with and "
                         "without the trained proposal at the final parameters")
    ap.add_argument("--log-every", type=int, default=10)
    ap.add_argument("--lr-schedule", default="const", choices=["const", "cos"])
    ap.add_argument("--out", default=None, help="JSON lines file for the histories")
    ap.add_argument("--material", default="ggx", choices=["ggx", "disney"],
                    help="material model: the workload's Lambert + GGX, or the Disney model (seeded parameters)")
    ap.add_argument("--state-dir", default=None,
                    help="resume each seed's run from its state file there, if present, and save it after this call")
    ap.add_argument("--stop-after", type=int, default=None,
                    help="iterations in this call (the schedule still spans --iters); with --state-dir")
    ap.add_argument("--paper-setting", action="store_true",
                    help="the paper's setting: every segment emissive, zero init, batches of --batch pixels at "
                         "--spp paths each, L1 loss, L1 emission regulariser --lam, Adam lr 5e-3")
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lam", type=float, default=1e-3)
    ap.add_argument("--loss", default="l1", choices=["l1", "l2"], help="image loss of the paper setting")
    ap.add_argument("--grad-spp", type=int, default=1, help="paper setting: paths per pixel of the derivative estimate")
    ap.add_argument("--ablation", default=None, choices=sorted(ABLATIONS),
                    help="the paper's optimiser ablations on the workload, --budget seconds per run")
    ap.add_argument("--budget", type=float, default=5.0)
    ap.add_argument("--precision", default="projections", choices=["projections", "fd"],
                    help="target precision (headline set): random projections of the adjoint (full inverse up to "
                         "256 free parameters, else the diagonal), or the full Gauss-Newton inverse from central "
                         "differences on a pixel sample")
    ap.add_argument("--fine-texture", action="store_true",
                    help="texture finer than the mesh: per-object, per-triangle, then subdivision where the "
                         "re-rendering error exceeds the noise")
    ap.add_argument("--coarse-to-fine", action="store_true",
                    help="textured Cornell: per-object optimisation, then per-triangle refinement where the "
                         "re-rendering error is high")
    a = ap.parse_args(argv)
    torch.cuda.set_device(0)
    sc = scenes.WORKLOADS[a.workload]()
    if a.material == "disney":
        sc = scenes.disney(sc, seed=11)
    if a.fine_texture:
        log = lambda s: print("[optimize] " + s, file=sys.stderr, flush=True)
        for seed in a.seeds:
            r = fine_texture(seed=seed, iters=a.iters or 300)
            for ph in r["phases"]:
                log("fine texture (seed %d, ground truth %dx%d per wall, mesh %dx%d): %s" % (
                    seed, r["n_gt"], r["n_gt"], r["n_opt"], r["n_opt"], json.dumps(ph)))
            if a.out:
                with open(a.out, "a") as f:
                    f.write(json.dumps(dict(workload="textured_cornell", mode="fine_texture", seed=seed, **r)) + "\n")
        return
    if a.coarse_to_fine:
        log = lambda s: print("[optimize] " + s, file=sys.stderr, flush=True)
        for seed in a.seeds:
            for mode in ("excess", "above_mean", "all"):
                r = coarse_to_fine(scenes.textured_cornell(), iters_coarse=a.iters or 300, iters_fine=a.iters or 200,
                                   seed=seed, refine=mode)
                for ph in r["phases"]:
                    log("coarse to fine (seed %d, refine %s, %d seen triangles): %s" % (
                        seed, mode, r["seen_triangles"], json.dumps(ph)))
                if a.out:
                    with open(a.out, "a") as f:
                        f.write(json.dumps(dict(workload="textured_cornell", mode="coarse_to_fine", seed=seed,
                                                **r)) + "\n")
        return
    if a.ablation:
        log = lambda s: print("[optimize] " + s, file=sys.stderr, flush=True)
        rows = run_ablation(sc, a.ablation, a.budget, a.seeds, target_spp=a.target_spp or 4096, log=log, lam=a.lam)
        if a.out:
            with open(a.out, "a") as f:
                f.write(json.dumps(dict(workload=sc["name"], ablation=a.ablation, budget=a.budget, rows=rows)) + "\n")
        return
    if a.paper_setting:
        log = lambda s: print("[optimize] " + s, file=sys.stderr, flush=True)
        sc = scenes.all_emissive(sc)
        cfg = sc["render"]
        g = ipt.Scene.from_dict(sc)
        dc = ipt.make_cameras(sc["cams"])
        target, tvar = render_target(g, dc, torch.as_tensor(sc["params"], device="cuda"),
                                     a.target_spp or cfg["target_spp"], cfg["max_depth"], cfg["rr_depth"],
                                     return_var=True)
        cov = coverage(g, sc)
        fixed, _ = paper_setting_masks(sc, cov)
        fr = sc["trainable"].astype(bool) & ~fixed
        sigma = target_precision(g, dc, sc, tvar, free=fr)
        masks = paper_setting_masks(sc, cov, sigma=sigma)
        log("paper setting: %d free parameters, %d headline (target precision <= 2.5e-3); not pinned: %s" % (
            fr.sum(), masks[1].sum(), [(int(i), float("%.3g" % sigma[i])) for i in
                                       np.nonzero(paper_setting_masks(sc, cov)[1] & ~masks[1])[0]]))
        for seed in a.seeds:
            res = optimize_paper_setting(sc, iters=a.iters or 2000, seed=seed, batch=a.batch, spp=a.spp or 512,
                                         grad_spp=a.grad_spp, lr=a.lr or 5e-3, lam=a.lam, beta2=a.beta2,
                                         target=target, g=g, log=log, log_every=a.log_every,
                                         target_rmse=a.target_rmse, masks=masks,
                                         loss_kind=1 if a.loss == "l1" else 0)
            if a.out:
                with open(a.out, "a") as f:
                    f.write(json.dumps(dict(workload=sc["name"], mode="paper_setting", **res)) + "\n")
            log("seed %d: final rmse %.4f (all free %.4f) after %d iters in %.1fs over %d headline parameters; "
                "time to %.0e: %s; worst %s" % (seed, res["final_rmse"], res["final_rmse_free"], res["iters"],
                                                res["seconds"], res["n_head"], a.target_rmse, res["time_to_target"],
                                                [(i, round(e, 3)) for i, e in res["worst"]]))
        return
    g = ipt.Scene.from_dict(sc)
    dc = ipt.make_cameras(sc["cams"])
    cfg = sc["render"]
    log = lambda s: print("[optimize] " + s, file=sys.stderr, flush=True)
    t0 = time.time()
    target, tvar = render_target(g, dc, torch.as_tensor(sc["params"], device="cuda"),
                                 a.target_spp or cfg["target_spp"], cfg["max_depth"], cfg["rr_depth"], return_var=True)
    cov = coverage(g, sc)
    fixed = unrecoverable_mask(sc, cov)
    tr = sc["trainable"].astype(bool)
    fr = tr & ~fixed
    if a.precision == "fd":
        sigma = target_precision_fd(g, dc, sc, tvar, fr)
    else:
        sigma = target_precision(g, dc, sc, tvar, free=fr)
    masks = identifiable_masks(sc, cov, sigma=sigma)
    log("target %d spp, precision in %.1fs; target precision of the free parameters: median %.2e, p90 %.2e, "
        "worst %s" % (a.target_spp or cfg["target_spp"], time.time() - t0, np.median(sigma[fr]),
                      np.percentile(sigma[fr], 90), [(int(i), float("%.3g" % sigma[i])) for i in
                                                      np.argsort(-np.where(fr, sigma, 0))[:5]]))
    log("coverage: %d of %d segments seen in >= 100 pixels; emitter pixels: %s; headline set %d params, "
        "identifiable %d of %d trainable, %d held at their true values" % (
            (cov >= 100).sum(), cov.size, cov[sc["emitter_seg"]].tolist(), masks[0].sum(), masks[1].sum(),
            sc["trainable"].sum(), (fixed & tr).sum()))
    # parameters the target cannot pin even to 0.25 (normalised) move little
    # from their random start: their initial errors' share of the
    # all-parameter RMSE is about where that RMSE levels off
    undetermined = fr & ~(sigma <= 0.25)
    for seed in a.seeds:
        log("workload %s seed %d guide %s" % (a.workload, seed, a.guide))
        e0 = (scenes.init_theta(sc, cfg["init"], seed=seed).astype(np.float64) - sc["params"]) / sc["scale"]
        log("initial-error share of the %d free parameters the target does not determine (sigma > 0.25): "
            "RMSE %.4f over the %d trainable parameters (they move little)" % (
                undetermined.sum(), np.sqrt(np.sum(e0[undetermined] ** 2) / max(1, tr.sum())), tr.sum()))
        st_path = None
        state = None
        if a.state_dir:
            os.makedirs(a.state_dir, exist_ok=True)
            st_path = os.path.join(a.state_dir, "state_%s_seed%d_%s" % (a.workload, seed, "guide" if a.guide else "brdf"))
            state = load_state(st_path)
            if state is not None:
                log("resuming from %s at iteration %d (%.1f s elapsed)" % (st_path, state["it"], state["t"]))
        res = optimize(sc, iters=a.iters, seed=seed, guide=a.guide, guide_mix=a.guide_mix, warmup=a.warmup,
                       guide_steps=a.guide_steps, target_rmse=a.target_rmse, target=target, g=g, log=log,
                       lr=a.lr, lr_schedule=a.lr_schedule, masks=masks, spp=a.spp, lr_final=a.lr_final,
                       log_every=a.log_every, fixed=fixed, beta2=a.beta2, guide_cells=a.guide_cells,
                       guide_every=a.guide_every, mis=a.mis, state=state, stop_after=a.stop_after,
                       want_state=st_path is not None)
        if st_path is not None:
            save_state(st_path, res["state"])
        res.pop("state")
        if not res["done"]:
            log("seed %d: stopped at iteration %d of %d (%.1f s); state saved to %s" % (
                seed, res["iters"], a.iters or sc["render"]["iters"], res["seconds"], st_path))
            continue
        if a.variance and a.guide:
            L = optimize.last
            vs = gradient_variance(g, dc, sc, L["params"], target, L["guide"], tr & ~fixed, K=a.variance,
                                   spp=a.spp, cached=1 if a.guide_cells else 0, guide_mix=a.guide_mix, mis=a.mis)
            res["variance"] = vs
            log("gradient variance over %d seeds at the final parameters (guide trained online over the %d "
                "iterations): %s" % (a.variance, res["iters"], json.dumps(vs)))
            # at the initial parameters, with a guide trained online at those parameters
            gi = train_guide_at(g, dc, sc, L["init"], target, iters=100, guide_steps=a.guide_steps,
                                guide_mix=a.guide_mix, seed=seed, guide_cells=a.guide_cells, spp=a.spp, mis=a.mis)
            vs = gradient_variance(g, dc, sc, L["init"], target, gi, tr & ~fixed, K=a.variance, spp=a.spp,
                                   cached=1 if a.guide_cells else 0, guide_mix=a.guide_mix, mis=a.mis)
            res["variance_init"] = vs
            log("gradient variance over %d seeds at the initial parameters (guide trained there for 100 "
                "iterations): %s" % (a.variance, json.dumps(vs)))
        line = json.dumps(dict(workload=a.workload, **res))
        if a.out:
            with open(a.out, "a") as f:
                f.write(line + "\n")
        log("seed %d: final rmse over all trainable parameters %.4f (headline subset %.4f, identifiable %.4f) "
            "after %d iters in %.1fs; time to %.0e: all %s, subset %s; worst %s" % (
                seed, res["final_rmse_all"], res["final_rmse"], res["final_rmse_id"], res["iters"], res["seconds"],
                a.target_rmse, res["time_to_target_all"], res["time_to_target"], res["worst"]))


if __name__ == "__main__":
    main()
