"""Helpers shared by the GPU parity tests: the same seeded scene goes to the
HIP library (through the C ABI) and to the FP64 oracle, and results are
compared on the paths whose event hashes agree."""
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
                     sc["normals"])
    return g, o


def dev(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def gpu_render(g, dc, params, opts_kw, pixel_list=None, sampling_params=None, mask=None):
    npix = dc["num_views"] * dc["width"] * dc["height"] if pixel_list is None else pixel_list.size
    spp = opts_kw.get("spp", 4)
    hsh = torch.zeros(npix * spp, dtype=torch.int64, device="cuda")
    pl = None if pixel_list is None else dev(pixel_list, torch.int64)
    pm = None if mask is None else dev(np.asarray(mask).reshape(-1).astype(np.uint8), torch.uint8)
    o = ipt.render_opts(pixel_list=pl, debug_path_hash=hsh, path_mask=pm, **opts_kw)
    img = g.render(dc, dev(params), o, sampling_params=None if sampling_params is None else dev(sampling_params))
    torch.cuda.synchronize()
    return img.cpu().numpy().astype(np.float64), hsh.cpu().numpy().view(np.uint64).reshape(npix, spp)


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


def mismatch_stats(hash_g, hash_o, margin, cond=None):
    """(paths mismatching, of which neither near-tie nor ill-conditioned)."""
    mism = hash_g != hash_o
    hard = mism & (margin >= NEAR_TIE)
    if cond is not None:
        hard &= cond <= ILL_COND
    return int(mism.sum()), int(hard.sum())


def comparable(hash_g, r):
    """Paths whose float32 radiance is expected to match float64 to 1e-4:
    same events, not a near-tie, and well conditioned."""
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
