"""Helpers shared by the GPU parity tests: the same seeded scene goes to the
HIP library (through the C ABI) and to the FP64 oracle, and results are
compared on the paths whose event hashes agree."""
import math
import sys

import numpy as np
import torch

from oracle import oracle
from paper_1903_07145_amd import ipt, scenes


def banner(msg):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


def both(sc):
    g = ipt.Scene.from_dict(sc)
    o = oracle.Scene(sc["verts"], sc["tris"], sc["tri_seg"], sc["num_segments"], sc["emitter_seg"],
                     sc["normals"], material=sc.get("material", 0))
    return g, o


def dev(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def gpu_render(g, dc, params, opts_kw, pixel_list=None, sampling_params=None, mask=None, want_path_L=False):
    npix = dc["num_views"] * dc["width"] * dc["height"] if pixel_list is None else pixel_list.size
    spp = opts_kw.get("spp", 4)
    hsh = torch.zeros(npix * spp, dtype=torch.int64, device="cuda")
    pl = None if pixel_list is None else dev(pixel_list, torch.int64)
    pm = None if mask is None else dev(np.asarray(mask).reshape(-1).astype(np.uint8), torch.uint8)
    pL = torch.zeros((npix * spp, 3), dtype=torch.float32, device="cuda") if want_path_L else None
    o = ipt.render_opts(pixel_list=pl, debug_path_hash=hsh, path_mask=pm, debug_path_radiance=pL, **opts_kw)
    img = g.render(dc, dev(params), o, sampling_params=None if sampling_params is None else dev(sampling_params))
    torch.cuda.synchronize()
    out = (img.cpu().numpy().astype(np.float64), hsh.cpu().numpy().view(np.uint64).reshape(npix, spp))
    if want_path_L:
        out = out + (pL.cpu().numpy().astype(np.float64).reshape(npix, spp, 3),)
    return out


def gpu_grad(g, dc, params, w, opts_kw, pixel_list=None, mask=None, sampling_params=None,
             workspace_bytes=None):
    pl = None if pixel_list is None else dev(pixel_list, torch.int64)
    pm = None if mask is None else dev(mask.reshape(-1).astype(np.uint8), torch.uint8)
    o = ipt.render_opts(pixel_list=pl, path_mask=pm, **opts_kw)
    gr = g.render_grad(dc, dev(params), dev(np.asarray(w, np.float32).reshape(-1, 3)), o,
                       sampling_params=None if sampling_params is None else dev(sampling_params),
                       workspace_bytes=workspace_bytes)
    torch.cuda.synchronize()
    return gr.cpu().numpy().astype(np.float64)


def oracle_opts(kw):
    keys = ("seed", "stream_tag", "iteration", "spp", "max_depth", "rr_depth", "mis",
            "emission_profile", "jitter")
    return {k: v for k, v in kw.items() if k in keys}


NEAR_TIE = 1e-5   # relative margin under which float32 and float64 may legitimately disagree
ILL_COND = 1e-3   # path radiance change under 1e-6 relative perturbations at every vertex
GRAD_ILL_COND = 1e-2   # the same for a path's gradient contribution (10x the 1e-3 gradient bar,
                       # as ILL_COND is 10x the 1e-4 pixel bar)


# Paths whose events differ between float32 and float64 without being a hard
# mismatch: near-ties (a decision within NEAR_TIE of its threshold) and, with
# the conditioning probe, ill-conditioned paths (rounding at one vertex grows
# along the path until a later decision flips).  Each kind is bounded on its
# own, per path and per scattering vertex (a path of depth D takes about D
# times as many decisions as one of depth 1).
NEAR_TIE_MISMATCH_PER_VERTEX = 1e-3
ILL_COND_MISMATCH_PER_VERTEX = 1e-3


def mismatch_breakdown(hash_g, r):
    """Paths whose event hashes differ, split into near-ties, ill-conditioned
    paths that are not near-ties (when r holds the conditioning probe) and
    hard mismatches (neither).  Returns a dict of counts and fractions."""
    mism = hash_g != r["hash"]
    near = mism & (r["margin"] < NEAR_TIE) if r.get("margin") is not None else np.zeros_like(mism)
    ill = mism & ~near & (r["cond"] > ILL_COND) if r.get("cond") is not None else np.zeros_like(mism)
    hard = mism & ~near & ~ill
    n = hash_g.size
    return dict(paths=n, mismatch=int(mism.sum()), near_tie=int(near.sum()), ill_cond=int(ill.sum()),
                hard=int(hard.sum()), f_near_tie=near.sum() / n, f_ill_cond=ill.sum() / n)


def check_mismatches(hash_g, r, rays_per_path, ray_bar=1e-5, label="", depth=3, near_tie_bar=None):
    """Prints the breakdown and asserts each bar: hard mismatches <= ray_bar
    of the rays; near-tie and ill-conditioned mismatches each <= 1e-3 of the
    paths per scattering vertex of the depth (near_tie_bar overrides the
    near-tie one where a workload takes many more threshold decisions, e.g.
    a light table of tens of thousands of entries)."""
    b = mismatch_breakdown(hash_g, r)
    banner("%s paths %d: mismatching %d = near-tie %d + ill-conditioned %d + hard %d" % (
        label, b["paths"], b["mismatch"], b["near_tie"], b["ill_cond"], b["hard"]))
    assert b["hard"] <= ray_bar * rays_per_path * b["paths"], b
    assert b["f_near_tie"] <= (near_tie_bar or NEAR_TIE_MISMATCH_PER_VERTEX * depth), b
    assert b["f_ill_cond"] <= ILL_COND_MISMATCH_PER_VERTEX * depth, b
    return b


def mismatch_stats(hash_g, hash_o, margin, cond=None):
    """(paths mismatching, of which neither near-tie nor ill-conditioned)."""
    mism = hash_g != hash_o
    hard = mism & (margin >= NEAR_TIE)
    if cond is not None:
        hard &= cond <= ILL_COND
    return int(mism.sum()), int(hard.sum())


# Tiers of the paths whose events agree, by the oracle's conditioning probe
# (the largest relative change of the path's radiance, or of its gradient
# contribution, under 1e-6 relative perturbations; infinite if an event
# changes).  Float32 rounding injects ~1e-7 per vertex; the measured float32
# error of a path is 0.1 to 2 times its probe value, so each tier admits
# probe values of half its bar or less:
#   tight      cond <= 5e-5: pixels at 1e-4;
#   tight_g    cond and gcond <= 1e-3: gradient at 1e-3 (relative to
#              max(|g|, 1e-2 rms g); a sum over many paths);
#   loose      cond (and gcond) <= 5e-3, not tight: 1e-2;
#   irregular  the rest: float32 and float64 follow different trajectories.
#              Their mean radiance must agree statistically (|z| <= 5 per
#              channel), and on the GPU their emission gradient must satisfy
#              linearity in emission.
# With use_margin a near-tie (a decision within NEAR_TIE of its threshold)
# also makes a path irregular: where a discontinuity exists that the events
# do not record (the cell of a cached proposal), the two sides may lie on
# either side of it with the same events.  Without one the probe sees the
# rest: a tangent frame's sign convention switching on a curved surface
# changes the events under the probe's shifts.
PIX_COND = 5e-5
TIGHT_GCOND = 1e-3
LOOSE_COND = 5e-3


def mask_report(hash_g, r, gcond=None, label="", use_margin=True):
    """Masks of the tiers among the paths whose events agree, and the
    fraction of paths each one holds ('tight', 'loose', 'irregular'; with
    gcond also 'tight_g', 'loose_g', 'irregular_g' for the gradient)."""
    same = hash_g == r["hash"]
    cond = r["cond"]
    regular = same & (r["margin"] >= NEAR_TIE) if (use_margin and r.get("margin") is not None) else same
    tight = regular & (cond <= PIX_COND)
    loose = regular & ~tight & (cond <= LOOSE_COND)
    out = dict(same=same, tight=tight, loose=loose, irregular=same & ~tight & ~loose,
               f_mismatch=1.0 - same.mean())
    msg = "%s tiers: events differ %.3f%%, tight %.2f%%, loose %.2f%%, irregular %.2f%%" % (
        label, 100 * out["f_mismatch"], 100 * tight.mean(), 100 * loose.mean(), 100 * out["irregular"].mean())
    if gcond is not None:
        tg = regular & (cond <= TIGHT_GCOND) & (gcond <= TIGHT_GCOND)
        lg = regular & ~tg & (cond <= LOOSE_COND) & (gcond <= LOOSE_COND)
        out.update(tight_g=tg, loose_g=lg, irregular_g=same & ~tg & ~lg)
        msg += "; gradient: tight %.2f%%, loose %.2f%%, irregular %.2f%%" % (
            100 * tg.mean(), 100 * lg.mean(), 100 * out["irregular_g"].mean())
    for k in ("tight", "loose", "irregular", "tight_g", "loose_g", "irregular_g"):
        if k in out:
            out["f_" + k] = out[k].mean()
    banner(msg)
    return out


def emission_linearity(w, img, grad, params, S, label="", nm=7):
    """The estimate is linear in the emission: per path, sum_k e_k dL/de_k = L,
    so for any subset of paths sum_j w_j . I_j = sum_k e_k g_k with the
    gradient g of sum_j w_j . I_j.  Exact up to float32 rounding; it holds
    path by path, so it applies to paths whose float32 trajectory departs
    from float64's as well."""
    lhs = float(np.dot(np.asarray(params, np.float64)[nm * S:], grad[nm * S:]))
    rhs = float(np.sum(np.asarray(w, np.float64) * img))
    scale = float(np.sum(np.abs(np.asarray(w, np.float64) * img))) + 1e-30
    banner("%s emission linearity: sum e dI/de %.6e vs w.I %.6e (rel %.1e of sum |w I|)" % (
        label, lhs, rhs, abs(lhs - rhs) / scale))
    assert abs(lhs - rhs) <= 1e-4 * scale, (lhs, rhs, scale)


def chaotic_agreement(Lg, Lo, z_bar=5.0, label=""):
    """Irregular paths: the means of their radiance must agree within z_bar
    standard errors per channel (where the float32 and float64 trajectories
    separate, the two sides are two draws of the same estimator)."""
    if Lg.shape[0] < 2:
        return 0.0
    zmax = 0.0
    for c in range(3):
        d = Lg[:, c].mean() - Lo[:, c].mean()
        se = math.sqrt((Lg[:, c].var() + Lo[:, c].var()) / Lg.shape[0]) + 1e-30
        zmax = max(zmax, abs(d) / se)
    banner("%s %d irregular paths: mean radiance |z| max %.2f (bar %.0f)" % (label, Lg.shape[0], zmax, z_bar))
    assert zmax <= z_bar, zmax
    return zmax


LOOSE_REL = 1e-2   # bar for the paths the tight comparison leaves out


def rel_err(a, ref, floor):
    return np.abs(a - ref) / np.maximum(np.abs(ref), floor)


def comparable(hash_g, r):
    """Paths whose float32 radiance is expected to match float64 to 1e-4:
    same events, not a near-tie (a discontinuity that the events do not
    record, such as the cell of a cached proposal, may lie between the two
    sides), and well conditioned."""
    ok = hash_g == r["hash"]
    if r.get("margin") is not None:
        ok &= r["margin"] >= NEAR_TIE
    if r.get("cond") is not None:
        ok &= r["cond"] <= ILL_COND
    return ok


def image_parity(img_g, img_o, hash_g, hash_o, rel=1e-4):
    """Per-pixel check on pixels whose paths all agree.  Returns (ok_pixels,
    path mismatch fraction, max relative error)."""
    match = hash_g == hash_o
    pix_ok = match.all(axis=1)
    mean = np.abs(img_o).mean() + 1e-30
    denom = np.maximum(np.abs(img_o), 1e-4 * mean)
    err = np.abs(img_g - img_o) / denom
    err_ok = err[pix_ok]
    return pix_ok, 1.0 - match.mean(), (err_ok.max() if err_ok.size else 0.0), err
