"""ctypes binding of libipt.so (the C ABI in include/ipt.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
libipt.so.  Device buffers are torch tensors on the current HIP device; the
work is enqueued on torch's current stream.  There is no CPU fallback: if the
library is missing or no GPU is present, calls raise.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# IPT_LIB_PATH selects another build of the same library (A/B comparisons of build variants)
LIB_PATH = os.environ.get("IPT_LIB_PATH", os.path.join(_HERE, "libipt.so"))

IPT_OK = 0
_STATUS = {0: "IPT_OK", 1: "IPT_ERR_INVALID_ARG", 2: "IPT_ERR_BAD_SCENE", 3: "IPT_ERR_OUT_OF_MEMORY",
           4: "IPT_ERR_WORKSPACE_TOO_SMALL", 5: "IPT_ERR_HIP", 6: "IPT_ERR_NOT_SUPPORTED"}

EXPORTS = ["ipt_scene_build", "ipt_scene_build_ex", "ipt_scene_free", "ipt_scene_info", "ipt_workspace_query", "ipt_render",
           "ipt_render_static",
           "ipt_render_grad", "ipt_loss_grad", "ipt_sgd_step", "ipt_l1_reg", "ipt_trace_rays", "ipt_guide_create",
           "ipt_guide_free", "ipt_guide_eval", "ipt_guide_train", "ipt_guide_weights", "ipt_guide_records",
           "ipt_guide_loss_grad", "ipt_guide_add_records", "ipt_guide_read_records", "ipt_guide_cache_build",
           "ipt_profile_enable", "ipt_profile_read",
           "ipt_profile_reset", "ipt_last_error"]


class IPTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS.get(status, status), msg))
        self.status = status


class Cameras(ctypes.Structure):
    _fields_ = [("num_views", ctypes.c_int32), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("cam_to_world", ctypes.c_void_p), ("fov_y", ctypes.c_void_p)]


class RenderOpts(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("stream_tag", ctypes.c_uint32), ("iteration", ctypes.c_uint32),
                ("spp", ctypes.c_int32), ("max_depth", ctypes.c_int32), ("rr_depth", ctypes.c_int32),
                ("mis", ctypes.c_int32), ("emission_profile", ctypes.c_int32), ("jitter", ctypes.c_int32),
                ("replay_traverse", ctypes.c_int32), ("pixel_list", ctypes.c_void_p),
                ("num_pixels", ctypes.c_int64), ("guide", ctypes.c_void_p), ("guide_mix", ctypes.c_float),
                ("guide_fp32", ctypes.c_int32), ("debug_path_hash", ctypes.c_void_p), ("path_mask", ctypes.c_void_p),
                ("debug_path_radiance", ctypes.c_void_p), ("debug_vertices", ctypes.c_void_p),
                ("guide_cached", ctypes.c_int32)]


class AdamOpts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


class SceneInfo(ctypes.Structure):
    _fields_ = [("num_triangles", ctypes.c_int64), ("num_vertices", ctypes.c_int64),
                ("num_nodes", ctypes.c_int64), ("num_light_triangles", ctypes.c_int64),
                ("num_segments", ctypes.c_int32), ("num_emitters", ctypes.c_int32),
                ("bvh_depth", ctypes.c_int32), ("has_normals", ctypes.c_int32),
                ("sah_cost", ctypes.c_double), ("build_ms", ctypes.c_double), ("scene_diag", ctypes.c_float),
                ("nonfinite_paths", ctypes.c_uint64), ("stack_overflows", ctypes.c_uint64),
                ("bvh_builder", ctypes.c_int32), ("params_global", ctypes.c_int32),
                ("node_bytes", ctypes.c_int32), ("material_model", ctypes.c_int32),
                ("params_per_segment", ctypes.c_int32), ("node_width", ctypes.c_int32)]


class BuildOpts(ctypes.Structure):
    _fields_ = [("bvh_builder", ctypes.c_int32), ("param_storage", ctypes.c_int32),
                ("material_model", ctypes.c_int32)]


BVH_GPU, BVH_HOST = 0, 1
PARAMS_AUTO, PARAMS_GLOBAL = 0, 1
MATERIAL_GGX, MATERIAL_DISNEY = 0, 1
PARAMS_PER_SEGMENT = {MATERIAL_GGX: 7, MATERIAL_DISNEY: 13}


class KernelProfile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double), ("rays", ctypes.c_uint64),
                ("nodes", ctypes.c_uint64), ("tris", ctypes.c_uint64), ("paths", ctypes.c_uint64),
                ("vertices", ctypes.c_uint64), ("units", ctypes.c_uint64)]


KERNELS = {0: "colour", 1: "grad_forward", 2: "adjoint_replay"}


class GuideOpts(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("lr", ctypes.c_float), ("batch", ctypes.c_int32),
                ("ring_capacity", ctypes.c_int32), ("record_stride", ctypes.c_int32)]


_lib = None


def lib():
    """Load libipt.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libipt.so not built: run __graft_entry__.build() or "
                               "python -m paper_1903_07145_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        sig = {
            "ipt_scene_build": [P, I64, P, P, P, I64, I32, P, I32, P, P],
            "ipt_scene_build_ex": [P, I64, P, P, P, I64, I32, P, I32, P, P, P],
            "ipt_scene_free": [P],
            "ipt_scene_info": [P, P],
            "ipt_workspace_query": [P, P, P, P, P],
            "ipt_render": [P, P, P, P, P, P, P, SZ, P],
            "ipt_render_static": [P, P, P, P, P, P, P],
            "ipt_render_grad": [P, P, P, P, P, P, P, P, SZ, P],
            "ipt_loss_grad": [P, P, P, P, P, P, I32, P, P, P, P, SZ, P],
            "ipt_sgd_step": [P, P, P, P, I32, I32, P, P, P, P, P, P],
            "ipt_l1_reg": [P, P, P, I32, P, P],
            "ipt_trace_rays": [P, P, P, P, I64, ctypes.c_float, I32, P, P, P],
            "ipt_guide_create": [P, P, P, P],
            "ipt_guide_free": [P],
            "ipt_guide_eval": [P, P, P, I64, I32, P, P],
            "ipt_guide_train": [P, I32, P, P],
            "ipt_guide_weights": [P, P, I32, I64],
            "ipt_guide_records": [P, P],
            "ipt_guide_loss_grad": [P, P, I64, P, P, P],
            "ipt_guide_add_records": [P, P, I64, P],
            "ipt_guide_read_records": [P, P, I64, P],
            "ipt_guide_cache_build": [P, P, ctypes.c_float, I32, P, P],
            "ipt_profile_enable": [P, I32],
            "ipt_profile_read": [P, I32, P],
            "ipt_profile_reset": [P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.ipt_last_error.restype = ctypes.c_char_p
        L.ipt_last_error.argtypes = []
        _lib = L
    return _lib


def _check(status):
    if status != IPT_OK:
        raise IPTError(status, lib().ipt_last_error().decode(errors="replace"))


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if not t.is_cuda:
            raise ValueError("expected a device tensor")
        if not t.is_contiguous():
            raise ValueError("expected a contiguous tensor")
        return ctypes.c_void_p(t.data_ptr())
    return t


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(x, dtype):
    if isinstance(x, torch.Tensor):
        return x.to(device="cuda", dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda").contiguous()


def make_cameras(cams):
    """Device copies of a camera dict (cam_to_world [V,4,4], fov_y [V], width, height)."""
    c2w = _dev(np.asarray(cams["cam_to_world"], np.float32).reshape(-1, 16), torch.float32)
    fov = _dev(np.asarray(cams["fov_y"], np.float32).reshape(-1), torch.float32)
    return dict(c2w=c2w, fov=fov, num_views=int(c2w.shape[0]), width=int(cams["width"]),
                height=int(cams["height"]))


def _cams_struct(dc):
    return Cameras(dc["num_views"], dc["width"], dc["height"], dc["c2w"].data_ptr(), dc["fov"].data_ptr())


def render_opts(seed=0, stream_tag=1, iteration=0, spp=4, max_depth=3, rr_depth=-1, mis=2,
                emission_profile=0, jitter=1, replay_traverse=0, pixel_list=None, guide=None,
                guide_mix=0.0, guide_fp32=0, debug_path_hash=None, path_mask=None,
                debug_path_radiance=None, debug_vertices=None, guide_cached=0):
    o = RenderOpts()
    o.seed, o.stream_tag, o.iteration = int(seed), int(stream_tag), int(iteration)
    o.spp, o.max_depth, o.rr_depth, o.mis = int(spp), int(max_depth), int(rr_depth), int(mis)
    o.emission_profile, o.jitter, o.replay_traverse = int(emission_profile), int(jitter), int(replay_traverse)
    o.pixel_list = None if pixel_list is None else pixel_list.data_ptr()
    o.num_pixels = 0 if pixel_list is None else int(pixel_list.numel())
    o.guide = None if guide is None else guide.handle
    o.guide_mix = float(guide_mix)
    o.guide_fp32 = int(guide_fp32)
    o.guide_cached = int(guide_cached)
    o.debug_path_hash = None if debug_path_hash is None else debug_path_hash.data_ptr()
    o.path_mask = None if path_mask is None else path_mask.data_ptr()
    o.debug_path_radiance = None if debug_path_radiance is None else debug_path_radiance.data_ptr()
    o.debug_vertices = None if debug_vertices is None else debug_vertices.data_ptr()
    o._keep = (pixel_list, debug_path_hash, path_mask, debug_path_radiance, debug_vertices)
    return o


class Scene:
    """A built scene on the current device (ipt_scene_build)."""

    def __init__(self, verts, tris, tri_seg, num_segments, emitter_seg, normals=None, bvh_builder=BVH_GPU,
                 param_storage=PARAMS_AUTO, material=MATERIAL_GGX):
        v = np.ascontiguousarray(verts, np.float32)
        t = np.ascontiguousarray(tris, np.int32)
        s = np.ascontiguousarray(tri_seg, np.int32)
        e = np.ascontiguousarray(emitter_seg, np.int32)
        n = None if normals is None else np.ascontiguousarray(normals, np.float32)
        self.num_segments = int(num_segments)
        self.num_emitters = int(e.size)
        self.material = int(material)
        if self.material not in PARAMS_PER_SEGMENT:
            raise ValueError("unknown material model %r" % (material,))
        self.P = PARAMS_PER_SEGMENT[self.material] * self.num_segments + 3 * self.num_emitters
        h = ctypes.c_void_p()
        torch.cuda.init()
        bo = BuildOpts(int(bvh_builder), int(param_storage), self.material)
        _check(lib().ipt_scene_build_ex(v.ctypes.data_as(ctypes.c_void_p), v.shape[0],
                                        None if n is None else n.ctypes.data_as(ctypes.c_void_p),
                                        t.ctypes.data_as(ctypes.c_void_p), s.ctypes.data_as(ctypes.c_void_p),
                                        t.shape[0], self.num_segments, e.ctypes.data_as(ctypes.c_void_p),
                                        e.size, ctypes.byref(bo), _stream(), ctypes.byref(h)))
        self.handle = h
        self._ws = None

    @classmethod
    def from_dict(cls, sc, bvh_builder=BVH_GPU, param_storage=PARAMS_AUTO):
        return cls(sc["verts"], sc["tris"], sc["tri_seg"], sc["num_segments"], sc["emitter_seg"],
                   sc.get("normals"), bvh_builder=bvh_builder, param_storage=param_storage,
                   material=sc.get("material", MATERIAL_GGX))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.ipt_scene_free(self.handle)
            self.handle = None

    def info(self):
        inf = SceneInfo()
        _check(lib().ipt_scene_info(self.handle, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in SceneInfo._fields_}

    def profile(self, enable=True):
        _check(lib().ipt_profile_enable(self.handle, int(bool(enable))))

    def profile_reset(self):
        _check(lib().ipt_profile_reset(self.handle))

    def profile_read(self, kernel):
        kp = KernelProfile()
        _check(lib().ipt_profile_read(self.handle, int(kernel), ctypes.byref(kp)))
        return {k: getattr(kp, k) for k, _ in KernelProfile._fields_}

    def workspace_query(self, dcams, opts):
        mn, full = ctypes.c_size_t(), ctypes.c_size_t()
        C = _cams_struct(dcams)
        _check(lib().ipt_workspace_query(self.handle, ctypes.byref(C), ctypes.byref(opts), ctypes.byref(mn),
                                         ctypes.byref(full)))
        return mn.value, full.value

    def workspace(self, dcams, opts, budget=48 << 30):
        mn, full = self.workspace_query(dcams, opts)
        need = max(mn, min(full, budget))
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            torch.cuda.empty_cache()
            self._ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        return self._ws

    def render(self, dcams, params, opts, sampling_params=None, out=None):
        npix = opts.num_pixels or dcams["num_views"] * dcams["width"] * dcams["height"]
        img = out if out is not None else torch.empty((npix, 3), dtype=torch.float32, device="cuda")
        ws = self.workspace(dcams, opts)
        C = _cams_struct(dcams)
        _check(lib().ipt_render(self.handle, ctypes.byref(C), _ptr(params), _ptr(sampling_params),
                                ctypes.byref(opts), _ptr(img), _ptr(ws), ws.numel(), _stream()))
        return img

    def render_static(self, dcams, params, opts, sampling_params=None, out=None):
        """ipt_render_static: the colour estimate without a workspace (the
        library's fixed device scratch; nothing is allocated by the call)."""
        npix = opts.num_pixels or dcams["num_views"] * dcams["width"] * dcams["height"]
        img = out if out is not None else torch.empty((npix, 3), dtype=torch.float32, device="cuda")
        C = _cams_struct(dcams)
        _check(lib().ipt_render_static(self.handle, ctypes.byref(C), _ptr(params), _ptr(sampling_params),
                                       ctypes.byref(opts), _ptr(img), _stream()))
        return img

    def render_grad(self, dcams, params, w, opts, sampling_params=None, out=None, workspace_bytes=None):
        grad = out if out is not None else torch.empty(self.P, dtype=torch.float32, device="cuda")
        ws = self.workspace(dcams, opts)
        nb = ws.numel() if workspace_bytes is None else min(ws.numel(), int(workspace_bytes))
        C = _cams_struct(dcams)
        _check(lib().ipt_render_grad(self.handle, ctypes.byref(C), _ptr(params), _ptr(sampling_params),
                                     ctypes.byref(opts), _ptr(w), _ptr(grad), _ptr(ws), nb, _stream()))
        return grad

    def loss_grad(self, dcams, params, target, color_opts, grad_opts, loss_kind=0, loss=None, grad=None,
                  image=None):
        loss = loss if loss is not None else torch.empty(1, dtype=torch.float32, device="cuda")
        grad = grad if grad is not None else torch.empty(self.P, dtype=torch.float32, device="cuda")
        ws = self.workspace(dcams, grad_opts)
        C = _cams_struct(dcams)
        _check(lib().ipt_loss_grad(self.handle, ctypes.byref(C), _ptr(params), _ptr(target),
                                   ctypes.byref(color_opts), ctypes.byref(grad_opts), int(loss_kind), _ptr(loss),
                                   _ptr(grad), _ptr(image), _ptr(ws), ws.numel(), _stream()))
        return loss, grad

    def trace_rays(self, origins, dirs, skip=None, tmin=0.0, brute_force=False):
        n = origins.shape[0]
        tri = torch.empty(n, dtype=torch.int32, device="cuda")
        tuv = torch.empty((n, 3), dtype=torch.float32, device="cuda")
        _check(lib().ipt_trace_rays(self.handle, _ptr(origins), _ptr(dirs), _ptr(skip), n, float(tmin),
                                    int(brute_force), _ptr(tri), _ptr(tuv), _stream()))
        return tri, tuv


def sgd_step(params, grad, m, v, step, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8, scale=None, lo=None,
             hi=None, trainable=None):
    """Projected Adam step on the device (ipt_sgd_step), in place."""
    a = AdamOpts(lr, beta1, beta2, eps)
    _check(lib().ipt_sgd_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(), int(step),
                              ctypes.byref(a), _ptr(scale), _ptr(lo), _ptr(hi), _ptr(trainable), _stream()))


def l1_reg(params, grad, weight, loss):
    """Adds the L1 emission regulariser to grad and loss in place (ipt_l1_reg)."""
    _check(lib().ipt_l1_reg(_ptr(params), _ptr(grad), _ptr(weight), params.numel(), _ptr(loss), _stream()))


class Guide:
    """A learned path-guiding proposal attached to a scene (ipt_guide_create)."""

    NUM_NET = 16744
    NUM_EMB = 16

    def __init__(self, scene, seed=1, lr=2e-3, batch=4096, ring_capacity=1 << 20, record_stride=1):
        o = GuideOpts(int(seed), float(lr), int(batch), int(ring_capacity), int(record_stride))
        h = ctypes.c_void_p()
        _check(lib().ipt_guide_create(scene.handle, ctypes.byref(o), _stream(), ctypes.byref(h)))
        self.handle = h
        self.scene = scene
        self.capacity = int(ring_capacity)
        self.num_params = self.NUM_NET + self.NUM_EMB * scene.num_segments

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.ipt_guide_free(h)
            self.handle = None

    def eval(self, feat, seg, mode=0):
        """Mixture parameters [n, 40] of feature rows feat [n, 9] (device) and segments seg [n]."""
        feat = _dev(feat, torch.float32)
        seg = _dev(seg, torch.int32)
        n = int(seg.numel())
        out = torch.empty((n, 40), dtype=torch.float32, device="cuda")
        _check(lib().ipt_guide_eval(self.handle, _ptr(feat), _ptr(seg), n, int(mode), _ptr(out), _stream()))
        return out

    def cache_build(self, cell_area, mode=0):
        """Builds (first call) or refills the cached proposal of the guide's
        scene (ipt_guide_cache_build); returns the number of cells per side."""
        n = ctypes.c_int64(0)
        _check(lib().ipt_guide_cache_build(self.handle, self.scene.handle, float(cell_area), int(mode),
                                           ctypes.byref(n), _stream()))
        self.cell_area = float(cell_area)
        return int(n.value)

    def train(self, steps=1, want_loss=True):
        loss = ctypes.c_float(0.0)
        _check(lib().ipt_guide_train(self.handle, int(steps), ctypes.byref(loss) if want_loss else None,
                                     _stream()))
        return float(loss.value) if want_loss else None

    def get_weights(self):
        w = np.zeros(self.num_params, np.float32)
        _check(lib().ipt_guide_weights(self.handle, w.ctypes.data_as(ctypes.c_void_p), 1, w.size))
        return w

    def set_weights(self, w):
        w = np.ascontiguousarray(w, np.float32)
        if w.size != self.num_params:
            raise ValueError("expected %d parameters" % self.num_params)
        _check(lib().ipt_guide_weights(self.handle, w.ctypes.data_as(ctypes.c_void_p), 0, w.size))

    def loss_grad(self, rec):
        """(loss, grad) of records rec [n, 16] (float32, ring layout) without training."""
        rec = _dev(rec, torch.float32)
        n = int(rec.shape[0])
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        grad = torch.zeros(self.num_params, dtype=torch.float32, device="cuda")
        _check(lib().ipt_guide_loss_grad(self.handle, _ptr(rec), n, _ptr(loss), _ptr(grad), _stream()))
        return loss, grad

    def add_records(self, rec):
        rec = _dev(rec, torch.float32)
        _check(lib().ipt_guide_add_records(self.handle, _ptr(rec), int(rec.shape[0]), _stream()))

    def read_records(self, n=None):
        """Ring slots [0, n) as a device tensor [n, 16] (default: the filled part)."""
        if n is None:
            n = min(self.records(), self.capacity)
        out = torch.zeros((int(n), 16), dtype=torch.float32, device="cuda")
        _check(lib().ipt_guide_read_records(self.handle, _ptr(out), int(n), _stream()))
        return out

    def records(self):
        c = ctypes.c_int64(0)
        _check(lib().ipt_guide_records(self.handle, ctypes.byref(c)))
        return int(c.value)


# ---------------------------------------------------------------------------
# torch.autograd integration (Sec. 3.3: the gradient is estimated from paths
# independent of the colour estimate).
# ---------------------------------------------------------------------------
class _RenderFn(torch.autograd.Function):
    """image = ipt_render(params) with stream-A options; the vector-Jacobian
    product with an image cotangent w is ipt_render_grad(w) with the stream-B
    options (the adjoint kernel: independent paths replayed from their
    Philox counters, Eq. 5-6)."""

    @staticmethod
    def forward(ctx, params, scene, dcams, color_opts, grad_opts, sampling_params):
        ctx.scene, ctx.dcams, ctx.grad_opts, ctx.sampling_params = scene, dcams, grad_opts, sampling_params
        ctx.save_for_backward(params)
        return scene.render(dcams, params.detach().contiguous(), color_opts, sampling_params=sampling_params)

    @staticmethod
    def backward(ctx, w):
        (params,) = ctx.saved_tensors
        g = ctx.scene.render_grad(ctx.dcams, params.detach().contiguous(), w.contiguous().float(), ctx.grad_opts,
                                  sampling_params=ctx.sampling_params)
        return g, None, None, None, None, None


def render(scene, dcams, params, color_opts, grad_opts, sampling_params=None):
    """Differentiable image [pixels, 3]: forward by ipt_render (color_opts),
    backward by ipt_render_grad (grad_opts, an independent stream)."""
    return _RenderFn.apply(params, scene, dcams, color_opts, grad_opts, sampling_params)


class _LossFn(torch.autograd.Function):
    """loss = ipt_loss_grad(params): the L2 (or L1) image loss of the stream-A
    estimate against the target; its gradient is the stream-B estimate that
    the same call computes, scaled by the incoming cotangent."""

    @staticmethod
    def forward(ctx, params, scene, dcams, target, color_opts, grad_opts, loss_kind):
        loss, grad = scene.loss_grad(dcams, params.detach().contiguous(), target, color_opts, grad_opts, loss_kind)
        ctx.save_for_backward(grad)
        return loss.reshape(())

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g * grad, None, None, None, None, None, None


def loss(scene, dcams, params, target, color_opts, grad_opts, loss_kind=0):
    """Differentiable scalar image loss (one ipt_loss_grad call)."""
    return _LossFn.apply(params, scene, dcams, target, color_opts, grad_opts, loss_kind)
