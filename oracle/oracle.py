"""Python wrapper of the FP64 CPU oracle (``oracle/ipt_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are its only users.  It imports nothing from the GPU package
and the GPU package never imports it.

The oracle follows the paper "Inverse Path Tracing for Joint Material and
Lighting Estimation" (CVPR 2019): Eq. 1-2 (Sec. 3.1) for the pixel estimate,
Eq. 3-6 (Sec. 3.2-3.3) for the loss and the product-rule derivatives, Adam
(Sec. 4.5), MIS of BRDF and light sampling (Appendix A.2, Appendix E).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ipt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force=False):
    """Compile the oracle with gcc (-O2, OpenMP, strict IEEE: no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-fno-fast-math", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.orc_scene_create.restype = P
        L.orc_scene_create.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_int64,
                                       ctypes.c_int32, P, ctypes.c_int32]
        L.orc_scene_free.argtypes = [P]
        L.orc_scene_set_material.argtypes = [P, ctypes.c_int32]
        L.orc_disney_eval.argtypes = [P, P, P, P, P, P]
        L.orc_disney_sample.restype = ctypes.c_int
        L.orc_disney_sample.argtypes = [P, P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
        L.orc_scene_diag.restype = ctypes.c_double
        L.orc_scene_diag.argtypes = [P]
        L.orc_scene_num_light_tris.restype = ctypes.c_int64
        L.orc_scene_num_light_tris.argtypes = [P]
        L.orc_run.restype = ctypes.c_int64
        L.orc_run.argtypes = [P, P, P, P, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_ray_triangle.restype = ctypes.c_int
        L.orc_ray_triangle.argtypes = [P, P, P, P, P, ctypes.c_double, ctypes.c_double, P]
        L.orc_closest_hit.restype = ctypes.c_int
        L.orc_closest_hit.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int32, ctypes.c_int, P, P]
        L.orc_camera_ray.argtypes = [P, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_double, P]
        L.orc_brdf_eval.argtypes = [P, P, P, P, P]
        L.orc_brdf_sample.restype = ctypes.c_int
        L.orc_brdf_sample.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, P]
        L.orc_light_probs.argtypes = [P, P, P]
        L.orc_loss_adjoint.restype = ctypes.c_double
        L.orc_loss_adjoint.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, P]
        L.orc_adam.argtypes = [P, P, P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double, P, P, P, P]
        L.orc_guide_eval.argtypes = [P, P, P, ctypes.c_int64, P]
        L.orc_mixture_pdf.restype = ctypes.c_double
        L.orc_mixture_pdf.argtypes = [P, P]
        L.orc_mixture_sample.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
        L.orc_set_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_cell_query.restype = ctypes.c_int
        L.orc_cell_query.argtypes = [P, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                     ctypes.c_float, P]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class _Opts(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("stream_tag", ctypes.c_uint32),
                ("iteration", ctypes.c_uint32), ("spp", ctypes.c_int32),
                ("max_depth", ctypes.c_int32), ("rr_depth", ctypes.c_int32),
                ("mis", ctypes.c_int32), ("emission_profile", ctypes.c_int32),
                ("jitter", ctypes.c_int32), ("brute_force", ctypes.c_int32),
                ("pixel_list", ctypes.c_void_p), ("num_pixels", ctypes.c_int64),
                ("guide_w", ctypes.c_void_p), ("guide_mix", ctypes.c_double),
                ("bb_lo", ctypes.c_double * 3), ("bb_inv", ctypes.c_double * 3),
                ("guide_cell_area", ctypes.c_double)]


class _Cams(ctypes.Structure):
    _fields_ = [("num_views", ctypes.c_int32), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("cam_to_world", ctypes.c_void_p),
                ("fov_y", ctypes.c_void_p)]


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def ray_triangle(o, d, p0, p1, p2, tmin=0.0, tmax=np.inf):
    arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (o, d, p0, p1, p2)]
    out = np.zeros(3)
    h = lib().orc_ray_triangle(*[_ptr(x) for x in arr], tmin, tmax, _ptr(out))
    return (out if h else None)


def camera_ray(c2w, fov_y, W, H, px, py):
    m = np.ascontiguousarray(c2w, dtype=np.float32).reshape(16)
    out = np.zeros(6)
    lib().orc_camera_ray(_ptr(m), float(fov_y), int(W), int(H), float(px), float(py), _ptr(out))
    return out[:3], out[3:]


def brdf_eval(mp, n, wo, wi):
    """Returns (f[3], pdf, spec, dspec/dalpha) for mp = [kd3, ks3, alpha]."""
    arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (mp, n, wo, wi)]
    out = np.zeros(6)
    lib().orc_brdf_eval(*[_ptr(x) for x in arr], _ptr(out))
    return out[:3].copy(), out[3], out[4], out[5]


def brdf_sample(mp, n, wo, u3, u4, u5):
    arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (mp, n, wo)]
    out = np.zeros(3)
    lobe = lib().orc_brdf_sample(*[_ptr(x) for x in arr], float(u3), float(u4), float(u5),
                                 _ptr(out))
    return lobe, out


DISNEY_PARAMS = ("base_r", "base_g", "base_b", "subsurface", "metallic", "specular", "specular_tint",
                 "roughness", "anisotropic", "sheen", "sheen_tint", "clearcoat", "clearcoat_gloss")


def disney_eval(mp, n, x, wo, wi):
    """Disney model (13 parameters mp): (f[3], pdf, df [13, 3]) with df the
    derivatives of f by complex-step differentiation; x is the tangent hint
    (projected onto the plane of n)."""
    arr = [np.ascontiguousarray(v, dtype=np.float64) for v in (mp, n, x, wo, wi)]
    out = np.zeros(4 + 3 * 13)
    lib().orc_disney_eval(*[_ptr(v) for v in arr], _ptr(out))
    return out[:3].copy(), out[3], out[4:].reshape(13, 3).copy()


def disney_sample(mp, n, x, wo, u3, u4, u5):
    """(lobe or -1, wi) of the Disney sampler."""
    arr = [np.ascontiguousarray(v, dtype=np.float64) for v in (mp, n, x, wo)]
    out = np.zeros(3)
    lobe = lib().orc_disney_sample(*[_ptr(v) for v in arr], float(u3), float(u4), float(u5), _ptr(out))
    return lobe, out


def guide_eval(weights, feat, seg):
    """Mixture parameters [n, 40] (per lobe mu xyz, kappa, weight) of the
    guide network with float32 weights, evaluated in float64."""
    w = np.ascontiguousarray(weights, dtype=np.float32)
    f = np.ascontiguousarray(feat, dtype=np.float64).reshape(-1, 9)
    sg = np.ascontiguousarray(seg, dtype=np.int32)
    out = np.zeros((f.shape[0], 40))
    lib().orc_guide_eval(_ptr(w), _ptr(f), _ptr(sg), f.shape[0], _ptr(out))
    return out


def set_threads(n):
    """OpenMP threads of the oracle's loops; returns the previous setting."""
    return lib().orc_set_threads(int(n))


def mixture_pdf(mix, w):
    m = np.ascontiguousarray(mix, dtype=np.float64)
    return lib().orc_mixture_pdf(_ptr(m), _ptr(np.ascontiguousarray(w, dtype=np.float64)))


def mixture_sample(mix, u3, u4, u5):
    m = np.ascontiguousarray(mix, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_mixture_sample(_ptr(m), float(u3), float(u4), float(u5), _ptr(out))
    return out


def loss_adjoint(img, target, kind=0):
    a = np.ascontiguousarray(img, dtype=np.float64).reshape(-1)
    b = np.ascontiguousarray(target, dtype=np.float64).reshape(-1)
    w = np.zeros_like(a)
    E = lib().orc_loss_adjoint(_ptr(a), _ptr(b), a.size, int(kind), _ptr(w))
    return E, w.reshape(np.shape(img))


def adam(params, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8, scale=None, lo=None,
         hi=None, trainable=None):
    """In-place projected Adam on float64 arrays."""
    conv = lambda x, dt: None if x is None else np.ascontiguousarray(x, dtype=dt)
    sc, l, h = conv(scale, np.float64), conv(lo, np.float64), conv(hi, np.float64)
    tr = conv(trainable, np.uint8)
    lib().orc_adam(_ptr(params), _ptr(np.ascontiguousarray(grad, dtype=np.float64)), _ptr(m),
                   _ptr(v), params.size, int(step), lr, b1, b2, eps, _ptr(sc), _ptr(l), _ptr(h),
                   _ptr(tr))


class Scene:
    """Oracle-side scene: positions, optional per-vertex normals, triangles,
    per-triangle segment ids, and the emitter segments (Sec. 4.2-4.3).
    material 0: Lambert + GGX, 7 parameters per segment; 1: the Disney model
    of Sec. 4.1, 13 parameters per segment (DISNEY_PARAMS)."""

    def __init__(self, verts, tris, tri_seg, num_segments, emitter_seg, normals=None, material=0):
        self._keep = [np.ascontiguousarray(verts, dtype=np.float32),
                      None if normals is None else np.ascontiguousarray(normals, dtype=np.float32),
                      np.ascontiguousarray(tris, dtype=np.int32),
                      np.ascontiguousarray(tri_seg, dtype=np.int32),
                      np.ascontiguousarray(emitter_seg, dtype=np.int32)]
        v, n, t, s, e = self._keep
        self.num_segments = int(num_segments)
        self.num_emitters = int(e.size)
        self.material = int(material)
        self.nm = 13 if self.material == 1 else 7
        self.P = self.nm * self.num_segments + 3 * self.num_emitters
        self.h = lib().orc_scene_create(_ptr(v), v.shape[0], _ptr(n), _ptr(t), _ptr(s),
                                        t.shape[0], self.num_segments, _ptr(e), e.size)
        lib().orc_scene_set_material(self.h, self.material)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_scene_free(self.h)
            self.h = None

    @property
    def diag(self):
        return lib().orc_scene_diag(self.h)

    @property
    def num_light_tris(self):
        return lib().orc_scene_num_light_tris(self.h)

    def closest_hit(self, o, d, tmin=0.0, tmax=np.inf, skip=-1, brute=False, want_margin=False):
        """(input triangle id or -1, [t, u, v]) and, with want_margin, the
        near-tie margin of the query (small: a float32 caster may disagree)."""
        o = np.ascontiguousarray(o, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.float64)
        out = np.zeros(3)
        mg = np.zeros(1)
        tri = lib().orc_closest_hit(self.h, _ptr(o), _ptr(d), tmin, tmax, skip, int(brute),
                                    _ptr(out), _ptr(mg) if want_margin else None)
        if want_margin:
            return tri, out, float(mg[0])
        return tri, out

    def cell_query(self, tri, u, v, back, cell_area):
        """Cached-proposal cell of barycentrics (u, v) on input triangle tri:
        (subdivision n, query position [3], query normal [3])."""
        out = np.zeros(6)
        n = lib().orc_cell_query(self.h, int(tri), float(u), float(v), int(bool(back)),
                                 float(np.float32(cell_area)), _ptr(out))
        return n, out[:3], out[3:]

    def light_probs(self, sampling_params):
        sp = np.ascontiguousarray(sampling_params, dtype=np.float64)
        out = np.zeros(self.num_light_tris)
        lib().orc_light_probs(self.h, _ptr(sp), _ptr(out))
        return out

    def run(self, cams, params, sampling_params=None, *, seed=0, stream_tag=1, iteration=0,
            spp=4, max_depth=3, rr_depth=-1, mis=2, emission_profile=0, jitter=1,
            brute_force=False, pixel_list=None, w=None, path_mask=None, want_grad=False,
            want_hash=False, want_path_L=False, want_margin=False, want_cond=False,
            want_vertices=False, guide_w=None, guide_mix=0.0, bb_lo=None, bb_inv=None, guide_cell_area=0.0):
        """Render (and optionally differentiate) pixels.

        cams: dict with cam_to_world [V,4,4] float32, fov_y [V], width, height.
        Returns dict(image [npix,3], grad [P] or None, hash [npix,spp] or None,
        path_L, margin [npix,spp] (near-tie margin of each path), cond
        [npix,spp] (relative radiance change when every vertex and direction
        is perturbed by 1e-6 relative; inf if an event changes), gcond (the
        same for the path's gradient contribution, when w is given), vertices
        [npix,spp,D+1,16] (per vertex: triangle id, u, v, t, radiance so far
        after its emission and light sample, light flag; for a vertex that
        continues: product of continuation weights up to it (RGB), density
        of the sampled direction, the direction, 1),
        dropped).
        """
        c2w = np.ascontiguousarray(cams["cam_to_world"], dtype=np.float32)
        fov = np.ascontiguousarray(cams["fov_y"], dtype=np.float32)
        V = c2w.shape[0]
        W, H = int(cams["width"]), int(cams["height"])
        pl = None if pixel_list is None else np.ascontiguousarray(pixel_list, dtype=np.int64)
        npix = V * W * H if pl is None else pl.size
        C = _Cams(V, W, H, _ptr(c2w), _ptr(fov))
        gw = None if guide_w is None else np.ascontiguousarray(guide_w, dtype=np.float32)
        O = _Opts(seed, stream_tag, iteration, spp, max_depth, rr_depth, mis, emission_profile,
                  jitter, int(brute_force), _ptr(pl), 0 if pl is None else pl.size, _ptr(gw),
                  float(guide_mix), (ctypes.c_double * 3)(*(bb_lo if bb_lo is not None else (0, 0, 0))),
                  (ctypes.c_double * 3)(*(bb_inv if bb_inv is not None else (1, 1, 1))),
                  float(np.float32(guide_cell_area)))
        p = np.ascontiguousarray(params, dtype=np.float64)
        sp = None if sampling_params is None else np.ascontiguousarray(sampling_params,
                                                                         dtype=np.float64)
        ww = None if w is None else np.ascontiguousarray(w, dtype=np.float64).reshape(npix, 3)
        pm = None if path_mask is None else np.ascontiguousarray(path_mask, dtype=np.uint8)
        img = np.zeros((npix, 3))
        grad = np.zeros(self.P) if want_grad else None
        hsh = np.zeros((npix, spp), dtype=np.uint64) if want_hash else None
        pL = np.zeros((npix, spp, 3)) if want_path_L else None
        mg = np.zeros((npix, spp)) if want_margin else None
        cd = np.zeros((npix, spp)) if want_cond else None
        vx = np.zeros((npix, spp, max_depth + 1, 16)) if want_vertices else None
        gcd = np.zeros((npix, spp)) if (want_cond and ww is not None) else None
        dropped = lib().orc_run(self.h, ctypes.byref(C), _ptr(p), _ptr(sp), ctypes.byref(O),
                                _ptr(ww), _ptr(pm), _ptr(img), _ptr(grad), _ptr(hsh), _ptr(pL),
                                _ptr(mg), _ptr(cd), _ptr(vx), _ptr(gcd))
        return dict(image=img, grad=grad, hash=hsh, path_L=pL, margin=mg, cond=cd, vertices=vx,
                    gcond=gcd, dropped=int(dropped))
