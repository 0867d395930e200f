"""Python binding of libnif.so (ctypes).

Argument marshalling only: every step of a query or training step runs in the
library's HIP kernels.  PyTorch supplies device memory (tensors) and the
stream (torch.cuda.current_stream()).  If the library is missing, loading it
raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnif.so")

NIF_F32, NIF_F16, NIF_BF16, NIF_FP8_E4M3 = 0, 1, 2, 3
NIF_OPT_ORDER = 1
NIF_OPT_GRID_IMAGE = 2
NIF_OPT_WINDOW_SORT = 3
NIF_OPT_TILE_SHAPE = 4
NIF_OPT_ORDER_BITS = 5
NIF_FLAG_INVALID_RAY = 1
NIF_FLAG_BAD_OBJECT = 2
DTYPES = {"f32": NIF_F32, "f16": NIF_F16, "bf16": NIF_BF16, "fp8": NIF_FP8_E4M3}
NIF_OK, NIF_ERR_INVALID_ARG, NIF_ERR_UNSUPPORTED, NIF_ERR_WORKSPACE, NIF_ERR_HIP, NIF_ERR_STATE = 0, -1, -2, -3, -4, -5
STATUS = {0: "NIF_OK", -1: "NIF_ERR_INVALID_ARG", -2: "NIF_ERR_UNSUPPORTED", -3: "NIF_ERR_WORKSPACE",
          -4: "NIF_ERR_HIP", -5: "NIF_ERR_STATE"}

# every symbol include/nif.h declares
EXPORTS = ["nif_create", "nif_destroy", "nif_param_layout", "nif_set_object", "nif_set_mlp", "nif_set_fp8_scales",
           "nif_calibrate_fp8", "nif_get_error_flags", "nif_pairs_workspace_bytes",
           "nif_expand_pairs", "nif_combine_pairs", "nif_expand_pairs_round", "nif_combine_pairs_and",
           "nif_expand_pairs_packed", "nif_order_keys", "nif_build_image", "nif_expand_pairs_by_object", "nif_init_grid", "nif_prepare", "nif_workspace_bytes", "nif_query", "nif_query_noalloc", "nif_encode", "nif_mlp",
           "nif_encode16", "nif_mlp16",
           "nif_set_option", "nif_image_bytes", "nif_set_image", "nif_order_workspace_bytes", "nif_order", "nif_query_ordered",
           "nif_order_packed", "nif_query_packed",
           "nif_plan_workspace_bytes", "nif_plan_create", "nif_plan_launch", "nif_plan_tuning", "nif_plan_destroy",
           "nif_set_object_train", "nif_set_mlp_train", "nif_train_step", "nif_backward", "nif_touched_bytes",
           "nif_train_step_depth", "nif_depth_from_visibility",
           "nif_bvh_create", "nif_bvh_destroy", "nif_bvh_num_nodes", "nif_bvh_anyhit", "nif_bvh_closest",
           "nif_paper_mlp_params", "nif_paper_grid_elems", "nif_paper_create", "nif_paper_destroy",
           "nif_paper_set_object", "nif_paper_init_grid", "nif_paper_set_mlp", "nif_paper_prepare", "nif_paper_query",
           "nif_paper_set_train", "nif_paper_set_object_train", "nif_paper_train_workspace_bytes",
           "nif_paper_train_step", "nif_paper_backward", "nif_light_create", "nif_light_destroy", "nif_light_sample",
           "nif_last_error", "nif_version"]


class NifError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


class ModelDesc(C.Structure):
    _fields_ = [("levels", C.c_int32), ("res_min", C.c_int32), ("res_max", C.c_int32), ("feats", C.c_int32),
                ("grid_dtype", C.c_int32), ("hidden_layers", C.c_int32), ("width", C.c_int32)]


class Adam(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


_lib = None


def lib():
    """Open libnif.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2306_07191_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        sig = {
            "nif_create": (i32, [vp, i32, i32, vp]),
            "nif_destroy": (None, [vp]),
            "nif_param_layout": (i32, [vp, vp, vp, vp, vp]),
            "nif_set_object": (i32, [vp, i32, vp, vp, i32]),
            "nif_set_mlp": (i32, [vp, i32, vp]),
            "nif_set_fp8_scales": (i32, [vp, i32, vp]),
            "nif_get_error_flags": (i32, [vp, vp, i32, vp]),
            "nif_pairs_workspace_bytes": (sz, [vp, i64]),
            "nif_expand_pairs": (i32, [vp, vp, vp, i64, i64, vp, vp, vp, vp, vp, vp, sz, vp]),
            "nif_combine_pairs": (i32, [vp, vp, vp, i64, i64, vp, vp]),
            "nif_expand_pairs_round": (i32, [vp, vp, vp, i64, i32, vp, i64, vp, vp, vp, vp, vp, vp, sz, vp]),
            "nif_expand_pairs_packed": (i32, [vp, vp, vp, i64, i64, vp, vp, vp, vp, vp, sz, vp]),
            "nif_order_keys": (i32, [vp, vp, i64, vp, vp, sz, vp]),
            "nif_build_image": (i32, [vp, i32, vp]),
            "nif_expand_pairs_by_object": (i32, [vp, vp, vp, i64, i64, vp, vp, vp, vp, vp, sz, vp]),
            "nif_combine_pairs_and": (i32, [vp, vp, vp, i64, i64, vp, vp]),
            "nif_calibrate_fp8": (i32, [vp, i32, vp, vp, vp, i64, vp, vp, sz, vp]),
            "nif_init_grid": (i32, [vp, i32, C.c_uint64, C.c_float, vp]),
            "nif_prepare": (i32, [vp, i32, vp]),
            "nif_workspace_bytes": (sz, [vp, i64, i32]),
            "nif_set_option": (i32, [vp, i32, i64]),
            "nif_image_bytes": (sz, [vp]),
            "nif_set_image": (i32, [vp, i32, vp, sz]),
            "nif_order_workspace_bytes": (sz, [vp, i64]),
            "nif_order": (i32, [vp, vp, vp, vp, i64, vp, vp, sz, vp]),
            "nif_query_ordered": (i32, [vp, i32, vp, vp, vp, vp, i64, vp, vp, vp]),
            "nif_order_packed": (i32, [vp, vp, vp, vp, i64, vp, vp, vp, sz, vp]),
            "nif_query_packed": (i32, [vp, i32, vp, vp, i64, vp, vp, vp]),
            "nif_query": (i32, [vp, i32, vp, vp, vp, i64, vp, vp, vp, sz, vp]),
            "nif_query_noalloc": (i32, [vp, i32, vp, vp, vp, i64, vp, vp, vp]),
            "nif_plan_workspace_bytes": (sz, [vp, i64]),
            "nif_plan_create": (i32, [vp, i32, vp, vp, vp, i64, vp, vp, vp, sz, C.c_char_p, vp, vp]),
            "nif_plan_launch": (i32, [vp, vp]),
            "nif_plan_tuning": (i32, [vp, vp, sz]),
            "nif_plan_destroy": (None, [vp]),
            "nif_encode": (i32, [vp, vp, vp, vp, i64, vp, vp, vp]),
            "nif_mlp": (i32, [vp, i32, i32, vp, i64, vp, vp]),
            "nif_encode16": (i32, [vp, i32, vp, vp, vp, i64, vp, vp, vp]),
            "nif_mlp16": (i32, [vp, i32, i32, vp, i64, vp, vp]),
            "nif_set_object_train": (i32, [vp, i32, vp, vp, vp, vp]),
            "nif_set_mlp_train": (i32, [vp, i32, vp, vp]),
            "nif_train_step": (i32, [vp, i32, vp, vp, vp, vp, i64, i32, vp, vp, vp, vp, sz, vp]),
            "nif_backward": (i32, [vp, i32, vp, vp, vp, vp, i64, vp, vp, sz, vp]),
            "nif_train_step_depth": (i32, [vp, i32, vp, vp, vp, vp, i64, i32, vp, vp, vp, vp, sz, vp]),
            "nif_depth_from_visibility": (i32, [vp, vp, vp, vp, vp, i64, vp, vp]),
            "nif_touched_bytes": (sz, [vp]),
            "nif_bvh_create": (i32, [vp, i64, vp]),
            "nif_bvh_destroy": (None, [vp]),
            "nif_bvh_num_nodes": (i64, [vp]),
            "nif_bvh_anyhit": (i32, [vp, vp, vp, i64, vp, vp]),
            "nif_bvh_closest": (i32, [vp, vp, vp, i64, vp, vp]),
            "nif_paper_mlp_params": (i64, [i32]),
            "nif_paper_grid_elems": (i64, [i32]),
            "nif_paper_create": (i32, [i32, vp]),
            "nif_paper_destroy": (None, [vp]),
            "nif_paper_set_object": (i32, [vp, i32, vp, vp, vp]),
            "nif_paper_init_grid": (i32, [vp, i32, i32, C.c_uint64, C.c_float, vp]),
            "nif_paper_set_mlp": (i32, [vp, i32, vp, vp]),
            "nif_paper_prepare": (i32, [vp, i32, vp]),
            "nif_paper_query": (i32, [vp, i32, vp, vp, vp, i64, vp, vp, vp]),
            "nif_paper_set_train": (i32, [vp, i32, vp, vp, vp, vp]),
            "nif_paper_set_object_train": (i32, [vp, i32, i32, vp, vp, vp]),
            "nif_paper_train_workspace_bytes": (sz, [vp, i32, i64]),
            "nif_paper_train_step": (i32, [vp, i32, vp, vp, vp, vp, i64, i32, vp, vp, vp, vp, sz, vp]),
            "nif_paper_backward": (i32, [vp, i32, vp, vp, vp, vp, i64, vp, vp, sz, vp]),
            "nif_light_create": (i32, [vp, vp, i64, vp]),
            "nif_light_destroy": (None, [vp]),
            "nif_light_sample": (i32, [vp, vp, vp, i64, vp, vp, vp, vp, vp]),
            "nif_last_error": (C.c_char_p, []),
            "nif_version": (C.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != 0:
        raise NifError(status, where, lib().nif_last_error().decode())


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


class BVH:
    """GPU BVH for any-hit shadow-ray casting (built on the host, traversed on the device)."""

    def __init__(self, tris):
        t = np.ascontiguousarray(tris, np.float32).reshape(-1, 9)
        h = C.c_void_p()
        _check(lib().nif_bvh_create(t.ctypes.data, t.shape[0], C.byref(h)), "nif_bvh_create")
        self.h = h
        self.num_nodes = int(lib().nif_bvh_num_nodes(self.h))

    def anyhit(self, rays, tmax, out=None):
        import torch
        n = tmax.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.uint8, device=rays.device)
        _check(lib().nif_bvh_anyhit(self.h, _ptr(rays), _ptr(tmax), n, _ptr(out), _stream()), "nif_bvh_anyhit")
        return out

    def closest(self, rays, tmax, out=None):
        """Closest-hit distance per ray (float32, +inf when none)."""
        import torch
        n = tmax.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=rays.device)
        _check(lib().nif_bvh_closest(self.h, _ptr(rays), _ptr(tmax), n, _ptr(out), _stream()), "nif_bvh_closest")
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().nif_bvh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Light:
    """Light importance sampling table (flux CDF) of emitting triangles."""

    def __init__(self, tris, radiance):
        t = np.ascontiguousarray(tris, np.float32).reshape(-1, 9)
        r = np.ascontiguousarray(radiance, np.float32).reshape(-1)
        h = C.c_void_p()
        _check(lib().nif_light_create(t.ctypes.data, r.ctypes.data, t.shape[0], C.byref(h)), "nif_light_create")
        self.h = h

    def sample(self, points, u, want_pdf: bool = True, want_tri: bool = True):
        """(rays [n, 6], t_max [n], pdf [n] or None, tri [n] or None) on the device."""
        import torch
        n = points.shape[0]
        rays = torch.empty((n, 6), dtype=torch.float32, device=points.device)
        tmax = torch.empty(n, dtype=torch.float32, device=points.device)
        pdf = torch.empty(n, dtype=torch.float32, device=points.device) if want_pdf else None
        tri = torch.empty(n, dtype=torch.int32, device=points.device) if want_tri else None
        _check(lib().nif_light_sample(self.h, _ptr(points), _ptr(u), n, _ptr(rays), _ptr(tmax), _ptr(pdf), _ptr(tri),
                                      _stream()), "nif_light_sample")
        return rays, tmax, pdf, tri

    def close(self):
        if getattr(self, "h", None):
            lib().nif_light_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PaperModel:
    """The paper's own outer and inner networks (spherical 2D grids, leaky-ReLU
    MLPs shared by all objects) over num_objects objects; grid buffers are
    binary16 torch tensors owned here."""

    def __init__(self, num_objects: int = 1, device: str = "cuda"):
        import torch
        self.torch = torch
        self.device = device
        h = C.c_void_p()
        _check(lib().nif_paper_create(num_objects, C.byref(h)), "nif_paper_create")
        self.h = h
        self.K = num_objects
        self.grids = [[None, None] for _ in range(num_objects)]
        self._w = [None, None]

    @staticmethod
    def mlp_params(network: int) -> int:
        return int(lib().nif_paper_mlp_params(network))

    @staticmethod
    def grid_elems(network: int) -> int:
        return int(lib().nif_paper_grid_elems(network))

    def set_object(self, obj: int, aabb, grids=None):
        t = self.torch
        if grids is None:
            grids = [t.zeros(self.grid_elems(n), dtype=t.float16, device=self.device) for n in (0, 1)]
        self.grids[obj] = list(grids)
        box = (C.c_float * 6)(*[float(v) for v in np.asarray(aabb, np.float32).ravel()])
        _check(lib().nif_paper_set_object(self.h, obj, box, _ptr(grids[0]), _ptr(grids[1])), "nif_paper_set_object")

    def init_grid(self, obj: int, network: int, seed: int, amp: float):
        _check(lib().nif_paper_init_grid(self.h, obj, network, seed, amp, _stream()), "nif_paper_init_grid")

    def set_mlp(self, network: int, w):
        t = self.torch
        w = t.as_tensor(np.asarray(w, np.float32) if not isinstance(w, t.Tensor) else w).to(self.device, t.float32)
        self._w[network] = w.contiguous()
        _check(lib().nif_paper_set_mlp(self.h, network, _ptr(self._w[network]), _stream()), "nif_paper_set_mlp")

    def prepare(self, dtype: str):
        _check(lib().nif_paper_prepare(self.h, DTYPES[dtype], _stream()), "nif_paper_prepare")

    def query(self, rays, ids, tmax, dtype: str = "f32", out=None, logits=None):
        t = self.torch
        n = ids.shape[0]
        if out is None:
            out = t.empty(n, dtype=t.float32, device=self.device)
        _check(lib().nif_paper_query(self.h, DTYPES[dtype], _ptr(rays), _ptr(ids), _ptr(tmax), n, _ptr(out),
                                     _ptr(logits), _stream()), "nif_paper_query")
        return out

    def setup_training(self, network: int, w=None):
        """Training buffers of `network`: binary32 master (from w, or the weights
        given to set_mlp), zero Adam moments, and per object the latent gradient
        and moments.  Returns the master tensor (updated in place by Adam)."""
        t = self.torch
        if w is None:
            w = self._w[network]
        master = t.as_tensor(np.asarray(w, np.float32) if not isinstance(w, t.Tensor) else w).to(
            self.device, t.float32).clone().contiguous()
        m, v = t.zeros_like(master), t.zeros_like(master)
        self._train = getattr(self, "_train", {})
        self._train[network] = {"w": master, "m": m, "v": v, "grids": []}
        _check(lib().nif_paper_set_train(self.h, network, _ptr(master), _ptr(m), _ptr(v), _stream()),
               "nif_paper_set_train")
        n = self.grid_elems(network)
        for k in range(self.K):
            bufs = [t.zeros(n, dtype=t.float32, device=self.device) for _ in range(3)]
            self._train[network]["grids"].append(bufs)
            _check(lib().nif_paper_set_object_train(self.h, k, network, _ptr(bufs[0]), _ptr(bufs[1]), _ptr(bufs[2])),
                   "nif_paper_set_object_train")
        return master

    def grid_grad(self, obj: int, network: int):
        return self._train[network]["grids"][obj][0]

    def train_step(self, network: int, rays, ids, tmax, labels, step: int = 1, adam=None, mlp_grad=None, ws=None):
        """One step; returns the loss tensor (device scalar).  adam: (lr, beta1,
        beta2, eps) or None for gradients only."""
        t = self.torch
        n = ids.shape[0]
        if ws is None:
            ws = t.empty(max(1, int(lib().nif_paper_train_workspace_bytes(self.h, network, n))), dtype=t.uint8,
                         device=self.device)
        loss = t.zeros(1, dtype=t.float32, device=self.device)
        ad = None if adam is None else C.byref(Adam(*[float(a) for a in adam]))
        _check(lib().nif_paper_train_step(self.h, network, _ptr(rays), _ptr(ids), _ptr(tmax), _ptr(labels), n, step,
                                          ad, _ptr(loss), _ptr(mlp_grad), _ptr(ws), ws.numel(), _stream()),
               "nif_paper_train_step")
        return loss

    def backward(self, network: int, rays, ids, tmax, grad_y, mlp_grad=None):
        """Gradients of a given dL/dy through `network` (MLP into mlp_grad, latents
        into each object's grid_grad buffer)."""
        t = self.torch
        n = ids.shape[0]
        ws = t.empty(max(1, int(lib().nif_paper_train_workspace_bytes(self.h, network, n))), dtype=t.uint8,
                     device=self.device)
        _check(lib().nif_paper_backward(self.h, network, _ptr(rays), _ptr(ids), _ptr(tmax), _ptr(grad_y), n,
                                        _ptr(mlp_grad), _ptr(ws), ws.numel(), _stream()), "nif_paper_backward")

    def close(self):
        if getattr(self, "h", None):
            lib().nif_paper_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """A tuned, graph-captured query over fixed buffers (see nif_plan_create)."""

    def __init__(self, ctx, rays, ids, tmax, dtype: str = "bf16", out=None, logits=None, tuning: str | None = None):
        import torch
        n = ids.shape[0]
        self.ctx = ctx
        self.out = torch.empty(n, dtype=torch.float32, device=rays.device) if out is None else out
        self.logits = logits
        self.bufs = (rays, ids, tmax)
        self.ws = torch.empty(max(1, int(lib().nif_plan_workspace_bytes(ctx.h, n))), dtype=torch.uint8,
                              device=rays.device)
        h = C.c_void_p()
        _check(lib().nif_plan_create(ctx.h, DTYPES[dtype], _ptr(rays), _ptr(ids), _ptr(tmax), n, _ptr(self.out),
                                     _ptr(logits), _ptr(self.ws), self.ws.numel(),
                                     None if tuning is None else tuning.encode(), _stream(), C.byref(h)),
               "nif_plan_create")
        self.h = h

    def launch(self):
        _check(lib().nif_plan_launch(self.h, _stream()), "nif_plan_launch")
        return self.out

    def tuning(self) -> str:
        buf = C.create_string_buffer(1024)
        _check(lib().nif_plan_tuning(self.h, buf, 1024), "nif_plan_tuning")
        return buf.value.decode()

    def close(self):
        if getattr(self, "h", None):
            lib().nif_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """A nif_ctx plus the device buffers the caller owns (torch tensors).

    shape: synth.ModelShape-like object (levels, res_min, res_max, feats,
    hidden, width, grid_dtype "f32"/"f16")."""

    def __init__(self, shape, num_objects: int = 1, num_mlps: int = 1, device: str = "cuda"):
        import torch
        self.torch = torch
        self.shape = shape
        self.K, self.M = num_objects, num_mlps
        self.device = device
        d = ModelDesc(shape.levels, shape.res_min, shape.res_max, shape.feats,
                      NIF_F16 if shape.grid_dtype == "f16" else NIF_F32, shape.hidden, shape.width)
        h = C.c_void_p()
        _check(lib().nif_create(C.byref(d), num_objects, num_mlps, C.byref(h)), "nif_create")
        self.h = h
        ge = C.c_int64()
        mp = C.c_int64()
        off = np.zeros(3 * shape.levels + 1, np.int64)
        res = np.zeros(shape.levels, np.int32)
        _check(lib().nif_param_layout(self.h, C.byref(ge), off.ctypes.data, res.ctypes.data, C.byref(mp)),
               "nif_param_layout")
        self.grid_elems, self.mlp_params = ge.value, mp.value
        self.table_offsets, self.level_res = off, res
        self.grids = [None] * num_objects
        self.mlps = [None] * num_mlps
        self.mlp_index = np.zeros(num_objects, np.int32)
        self.aabb = np.zeros((num_objects, 6), np.float32)
        # query images (NIF_OPT_GRID_IMAGE) are the caller's: allocated here,
        # registered with nif_set_image at the next prepare; on by default for
        # binary16 grids (the y-pair image, twice the grid's memory)
        self.image_mode = 0
        self.images = [None] * num_objects
        if shape.grid_dtype == "f16":
            self.set_option(NIF_OPT_GRID_IMAGE, 1)

    def close(self):
        if getattr(self, "h", None):
            lib().nif_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- parameters ----------------------------------------------------
    def alloc_grid(self):
        t = self.torch
        dt = t.float16 if self.shape.grid_dtype == "f16" else t.float32
        return t.empty(self.grid_elems, dtype=dt, device=self.device)

    def set_object(self, k: int, aabb, grid, mlp: int = 0):
        a = np.ascontiguousarray(aabb, np.float32).reshape(6)
        self.aabb[k] = a
        self.grids[k] = grid
        self.mlp_index[k] = mlp
        _check(lib().nif_set_object(self.h, k, a.ctypes.data, _ptr(grid), mlp), "nif_set_object")

    def set_mlp(self, m: int, weights):
        self.mlps[m] = weights
        _check(lib().nif_set_mlp(self.h, m, _ptr(weights)), "nif_set_mlp")

    def set_fp8_scales(self, m: int, scales):
        s = np.ascontiguousarray(scales, np.float32)
        _check(lib().nif_set_fp8_scales(self.h, m, s.ctypes.data), "nif_set_fp8_scales")

    def expand_pairs(self, rays, tmax, max_pairs=None, round: int = 0, ray_visible=None):
        """(pair_rays, pair_tmax, pair_ids, pair_ray) of the rays' AABB hits, ray order.
        round 1 / 2: the early-out form's rounds (nif_expand_pairs_round)."""
        t = self.torch
        n = tmax.shape[0]
        ws = t.empty(max(1, int(lib().nif_pairs_workspace_bytes(self.h, n))), dtype=t.uint8, device=self.device)
        cnt = t.zeros(1, dtype=t.int64, device=self.device)
        for _ in range(2):
            m = max(1, n if max_pairs is None else max_pairs)
            pr = t.empty((m, 6), dtype=t.float32, device=self.device)
            pt = t.empty(m, dtype=t.float32, device=self.device)
            pi = t.empty(m, dtype=t.int32, device=self.device)
            pray = t.empty(m, dtype=t.int32, device=self.device)
            if round:
                _check(lib().nif_expand_pairs_round(self.h, _ptr(rays), _ptr(tmax), n, round, _ptr(ray_visible), m,
                                                    _ptr(pr), _ptr(pt), _ptr(pi), _ptr(pray), _ptr(cnt), _ptr(ws),
                                                    ws.numel(), _stream()), "nif_expand_pairs_round")
            else:
                _check(lib().nif_expand_pairs(self.h, _ptr(rays), _ptr(tmax), n, m, _ptr(pr), _ptr(pt), _ptr(pi),
                                              _ptr(pray), _ptr(cnt), _ptr(ws), ws.numel(), _stream()), "nif_expand_pairs")
            total = int(cnt.item())
            if total <= m:
                return pr[:total], pt[:total], pi[:total], pray[:total]
            max_pairs = total
        raise RuntimeError("pair count changed between calls")

    def expand_pairs_packed(self, rays, tmax, max_pairs=None, keys: bool = True):
        """(packed [P, 8] float32 query records, pair_ray, keys or None) of the
        rays' AABB hits in ray order (nif_expand_pairs_packed)."""
        t = self.torch
        n = tmax.shape[0]
        ws = t.empty(max(1, int(lib().nif_pairs_workspace_bytes(self.h, n))), dtype=t.uint8, device=self.device)
        cnt = t.zeros(1, dtype=t.int64, device=self.device)
        for _ in range(2):
            m = max(1, n if max_pairs is None else max_pairs)
            rec = t.empty((m, 8), dtype=t.float32, device=self.device)
            pray = t.empty(m, dtype=t.int32, device=self.device)
            key = t.empty(m, dtype=t.int32, device=self.device) if keys else None
            _check(lib().nif_expand_pairs_packed(self.h, _ptr(rays), _ptr(tmax), n, m, _ptr(rec), _ptr(pray), _ptr(key),
                                                 _ptr(cnt), _ptr(ws), ws.numel(), _stream()), "nif_expand_pairs_packed")
            total = int(cnt.item())
            if total <= m:
                return rec[:total], pray[:total], None if key is None else key[:total]
            max_pairs = total
        raise RuntimeError("pair count changed between calls")

    def expand_pairs_by_object(self, rays, tmax, max_pairs=None):
        """(packed [P, 8] float32 query records grouped by object, pair_ray,
        obj_offsets [K + 1] int64) of the rays' AABB hits
        (nif_expand_pairs_by_object)."""
        t = self.torch
        n = tmax.shape[0]
        ws = t.empty(max(1, int(lib().nif_pairs_workspace_bytes(self.h, n))), dtype=t.uint8, device=self.device)
        cnt = t.zeros(1, dtype=t.int64, device=self.device)
        off = t.empty(self.K + 1, dtype=t.int64, device=self.device)
        for _ in range(2):
            m = max(1, n if max_pairs is None else max_pairs)
            rec = t.empty((m, 8), dtype=t.float32, device=self.device)
            pray = t.empty(m, dtype=t.int32, device=self.device)
            _check(lib().nif_expand_pairs_by_object(self.h, _ptr(rays), _ptr(tmax), n, m, _ptr(rec), _ptr(pray),
                                                    _ptr(cnt), _ptr(off), _ptr(ws), ws.numel(), _stream()),
                   "nif_expand_pairs_by_object")
            total = int(cnt.item())
            if total <= m:
                return rec[:total], pray[:total], off
            max_pairs = total
        raise RuntimeError("pair count changed between calls")

    def order_keys(self, keys, perm=None, ws=None):
        """Ordering from the keys of expand_pairs_packed (nif_order_keys): perm."""
        t = self.torch
        n = keys.shape[0]
        if perm is None:
            perm = t.empty(n, dtype=t.int32, device=self.device)
        if ws is None:
            ws = t.empty(max(1, int(lib().nif_order_workspace_bytes(self.h, n))), dtype=t.uint8, device=self.device)
        _check(lib().nif_order_keys(self.h, _ptr(keys), n, _ptr(perm), _ptr(ws), ws.numel(), _stream()),
               "nif_order_keys")
        return perm

    def combine_pairs(self, pair_ray, visibility, n_rays, out=None, accumulate: bool = False):
        """Per-ray visibility (uint8): 0 iff some pair of the ray is below 0.5.
        accumulate: only clear rays of occluded pairs in out (nif_combine_pairs_and)."""
        t = self.torch
        if out is None:
            out = t.empty(n_rays, dtype=t.uint8, device=self.device)
        f = lib().nif_combine_pairs_and if accumulate else lib().nif_combine_pairs
        _check(f(self.h, _ptr(pair_ray), _ptr(visibility), pair_ray.shape[0], n_rays, _ptr(out), _stream()),
               "nif_combine_pairs")
        return out

    def error_flags(self, clear: bool = True) -> int:
        """Domain-error bits of the queries since the last clear (1 invalid ray, 2 bad object id)."""
        f = C.c_uint32(0)
        _check(lib().nif_get_error_flags(self.h, C.byref(f), 1 if clear else 0, _stream()), "nif_get_error_flags")
        return int(f.value)

    def calibrate_fp8(self, rays, ids, tmax, mlp: int = 0, ws=None):
        """Per-layer FP8 scales of MLP `mlp` from the given queries; returns them (s_W then s_x)."""
        t = self.torch
        n = ids.shape[0]
        if ws is None:
            ws = t.empty(max(1, self.workspace_bytes(n, 2)), dtype=t.uint8, device=self.device)
        out = np.zeros(2 * self.shape.hidden, np.float32)
        _check(lib().nif_calibrate_fp8(self.h, mlp, _ptr(rays), _ptr(ids), _ptr(tmax), n, out.ctypes.data, _ptr(ws),
                                       ws.numel(), _stream()), "nif_calibrate_fp8")
        return out

    def init_grid(self, k: int, seed: int, amp: float = 1e-4):
        _check(lib().nif_init_grid(self.h, k, seed, amp, _stream()), "nif_init_grid")

    def build_image(self, k: int):
        """Allocate (if needed) and build object k's query image now."""
        t = self.torch
        if self.images[k] is None:
            nb = int(lib().nif_image_bytes(self.h))
            self.images[k] = t.empty(nb, dtype=t.uint8, device=self.device)
            _check(lib().nif_set_image(self.h, k, _ptr(self.images[k]), nb), "nif_set_image")
        _check(lib().nif_build_image(self.h, k, _stream()), "nif_build_image")

    def drop_grid(self, k: int):
        """Answer object k from its built query image alone; its grid tensor is released."""
        _check(lib().nif_set_object(self.h, k, self.aabb[k].ctypes.data, None, int(self.mlp_index[k])),
               "nif_set_object")
        self.grids[k] = None

    def prepare(self, dtype: str):
        if self.image_mode:
            t = self.torch
            nb = int(lib().nif_image_bytes(self.h))
            for k in range(self.K):
                if self.images[k] is None:
                    self.images[k] = t.empty(nb, dtype=t.uint8, device=self.device)
                    _check(lib().nif_set_image(self.h, k, _ptr(self.images[k]), nb), "nif_set_image")
        _check(lib().nif_prepare(self.h, DTYPES[dtype], _stream()), "nif_prepare")

    def set_option(self, option: int, value: int):
        _check(lib().nif_set_option(self.h, option, value), "nif_set_option")
        if option == NIF_OPT_GRID_IMAGE and value != self.image_mode:
            self.image_mode = value
            self.images = [None] * self.K  # the library forgot them; sizes differ between kinds

    def workspace_bytes(self, n: int, mode: int = 0) -> int:
        return int(lib().nif_workspace_bytes(self.h, n, mode))

    # ---- queries -------------------------------------------------------
    def query(self, rays, ids, tmax, dtype: str = "f32", out=None, logits=None, ws=None):
        t = self.torch
        n = ids.shape[0]
        if out is None:
            out = t.empty(n, dtype=t.float32, device=self.device)
        wsb = self.workspace_bytes(n, 0)
        if ws is None and wsb > 0:
            ws = t.empty(wsb, dtype=t.uint8, device=self.device)
        _check(lib().nif_query(self.h, DTYPES[dtype], _ptr(rays), _ptr(ids), _ptr(tmax), n, _ptr(out),
                               _ptr(logits), _ptr(ws), 0 if ws is None else ws.numel(), _stream()), "nif_query")
        return out

    def query_noalloc(self, rays, ids, tmax, dtype: str = "f32", out=None, logits=None):
        """nif_query_noalloc: as query, with the library's static scratch instead of a workspace."""
        n = ids.shape[0]
        if out is None:
            out = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
        _check(lib().nif_query_noalloc(self.h, DTYPES[dtype], _ptr(rays), _ptr(ids), _ptr(tmax), n, _ptr(out),
                                       _ptr(logits), _stream()), "nif_query_noalloc")
        return out

    def order(self, rays, ids, tmax, perm=None, ws=None):
        """Ordering step alone: a permutation of [0, n) (int32 tensor, uint32 values)."""
        t = self.torch
        n = ids.shape[0]
        if perm is None:
            perm = t.empty(n, dtype=t.int32, device=self.device)
        if ws is None:
            ws = t.empty(max(1, int(lib().nif_order_workspace_bytes(self.h, n))), dtype=t.uint8, device=self.device)
        _check(lib().nif_order(self.h, _ptr(rays), _ptr(ids), _ptr(tmax), n, _ptr(perm), _ptr(ws), ws.numel(),
                               _stream()), "nif_order")
        return perm

    def query_ordered(self, rays, ids, tmax, perm, dtype: str = "f32", out=None, logits=None):
        t = self.torch
        n = ids.shape[0]
        if out is None:
            out = t.empty(n, dtype=t.float32, device=self.device)
        _check(lib().nif_query_ordered(self.h, DTYPES[dtype], _ptr(rays), _ptr(ids), _ptr(tmax), _ptr(perm), n,
                                       _ptr(out), _ptr(logits), _stream()), "nif_query_ordered")
        return out

    def order_packed(self, rays, ids, tmax, perm=None, packed=None, ws=None):
        """Ordering step that also stores every query as a 32-byte record:
        (perm, packed [n, 8] float32 rows o, d, t_max, object id bits)."""
        t = self.torch
        n = ids.shape[0]
        if perm is None:
            perm = t.empty(n, dtype=t.int32, device=self.device)
        if packed is None:
            packed = t.empty((n, 8), dtype=t.float32, device=self.device)
        if ws is None:
            ws = t.empty(max(1, int(lib().nif_order_workspace_bytes(self.h, n))), dtype=t.uint8, device=self.device)
        _check(lib().nif_order_packed(self.h, _ptr(rays), _ptr(ids), _ptr(tmax), n, _ptr(perm), _ptr(packed),
                                      _ptr(ws), ws.numel(), _stream()), "nif_order_packed")
        return perm, packed

    def query_packed(self, packed, perm, dtype: str = "f32", out=None, logits=None):
        """Query on the records of order_packed, in the order perm (None: the
        records' own order); outputs in query order."""
        t = self.torch
        n = packed.shape[0] if perm is None else perm.shape[0]
        if out is None:
            out = t.empty(n, dtype=t.float32, device=self.device)
        _check(lib().nif_query_packed(self.h, DTYPES[dtype], _ptr(packed), _ptr(perm), n, _ptr(out),
                                      _ptr(logits), _stream()), "nif_query_packed")
        return out

    def encode16(self, rays, ids, tmax, fmt: str = "bf16"):
        """Grid stage alone with 16-bit features: (features [n, din] int16 bit
        patterns of fmt, status [n])."""
        t = self.torch
        n = ids.shape[0]
        f = t.empty((n, self.shape.din), dtype=t.int16, device=self.device)
        st = t.empty(n, dtype=t.int32, device=self.device)
        _check(lib().nif_encode16(self.h, DTYPES[fmt], _ptr(rays), _ptr(ids), _ptr(tmax), n, _ptr(f), _ptr(st),
                                  _stream()), "nif_encode16")
        return f, st

    def mlp16(self, features, dtype: str = "bf16", mlp: int = 0, out=None):
        """Inference stage on 16-bit features of format dtype; logits [n]."""
        t = self.torch
        n = features.shape[0]
        if out is None:
            out = t.empty(n, dtype=t.float32, device=self.device)
        _check(lib().nif_mlp16(self.h, DTYPES[dtype], mlp, _ptr(features), n, _ptr(out), _stream()), "nif_mlp16")
        return out

    def encode(self, rays, ids, tmax):
        """Grid stage alone: (features [n, din], status [n])."""
        t = self.torch
        n = ids.shape[0]
        f = t.empty((n, self.shape.din), dtype=t.float32, device=self.device)
        st = t.empty(n, dtype=t.int32, device=self.device)
        _check(lib().nif_encode(self.h, _ptr(rays), _ptr(ids), _ptr(tmax), n, _ptr(f), _ptr(st), _stream()),
               "nif_encode")
        return f, st

    def mlp(self, features, dtype: str = "f32", mlp: int = 0):
        """Inference stage alone: logits of MLP `mlp` on features [n, din]."""
        t = self.torch
        n = features.shape[0]
        z = t.empty(n, dtype=t.float32, device=self.device)
        _check(lib().nif_mlp(self.h, DTYPES[dtype], mlp, _ptr(features), n, _ptr(z), _stream()), "nif_mlp")
        return z

    # ---- training --------------------------------------------------------
    def setup_training(self, shared: bool = False):
        """Allocate and register zeroed training buffers for every object and MLP.
        shared=True registers one set of latent buffers for every object (objects
        trained one MLP at a time; zero the moments before moving to the next)."""
        t = self.torch
        tb = int(lib().nif_touched_bytes(self.h))
        self.train_bufs = []
        for k in range(self.K):
            if shared and k > 0:
                g, m, v, tch = self.train_bufs[0]
            else:
                g = t.zeros(self.grid_elems, dtype=t.float32, device=self.device)
                m = t.zeros_like(g)
                v = t.zeros_like(g)
                tch = t.zeros((tb + 3) // 4, dtype=t.int32, device=self.device)
            self.train_bufs.append((g, m, v, tch))
            _check(lib().nif_set_object_train(self.h, k, _ptr(g), _ptr(m), _ptr(v), _ptr(tch)),
                   "nif_set_object_train")
        self.mlp_moments = []
        for mi in range(self.M):
            m = t.zeros(self.mlp_params, dtype=t.float32, device=self.device)
            v = t.zeros_like(m)
            self.mlp_moments.append((m, v))
            _check(lib().nif_set_mlp_train(self.h, mi, _ptr(m), _ptr(v)), "nif_set_mlp_train")

    def train_step(self, rays, ids, tmax, labels, step: int, mlp: int = 0, adam=(1e-2, 0.9, 0.99, 1e-15),
                   loss=None, mlp_grad=None, ws=None):
        """One training step; adam=None computes gradients only."""
        t = self.torch
        n = ids.shape[0]
        if ws is None:
            ws = t.empty(max(1, self.workspace_bytes(n, 1)), dtype=t.uint8, device=self.device)
        a = None if adam is None else Adam(*adam)
        _check(lib().nif_train_step(self.h, mlp, _ptr(rays), _ptr(ids), _ptr(tmax), _ptr(labels), n, step,
                                    None if a is None else C.byref(a), _ptr(loss), _ptr(mlp_grad), _ptr(ws),
                                    ws.numel(), _stream()), "nif_train_step")

    def train_step_depth(self, rays, ids, tmax, t_hit, step: int, mlp: int = 0, adam=(1e-2, 0.9, 0.99, 1e-15),
                         loss=None, mlp_grad=None, ws=None):
        """One training step of the depth output (L2 on the normalised closest-hit depth)."""
        t = self.torch
        n = ids.shape[0]
        if ws is None:
            ws = t.empty(max(1, self.workspace_bytes(n, 1)), dtype=t.uint8, device=self.device)
        a = None if adam is None else Adam(*adam)
        _check(lib().nif_train_step_depth(self.h, mlp, _ptr(rays), _ptr(ids), _ptr(tmax), _ptr(t_hit), n, step,
                                          None if a is None else C.byref(a), _ptr(loss), _ptr(mlp_grad), _ptr(ws),
                                          ws.numel(), _stream()), "nif_train_step_depth")

    def depth_from_visibility(self, rays, ids, tmax, visibility, out=None):
        """t_a + y (t_b - t_a) per query (+inf for a miss, NaN for an invalid query)."""
        n = ids.shape[0]
        if out is None:
            out = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
        _check(lib().nif_depth_from_visibility(self.h, _ptr(rays), _ptr(ids), _ptr(tmax), _ptr(visibility), n,
                                               _ptr(out), _stream()), "nif_depth_from_visibility")
        return out

    def backward(self, rays, ids, tmax, grad_y, mlp: int = 0, mlp_grad=None, ws=None):
        """dL/dW (into mlp_grad) and dL/dlatent (added to the registered grid gradient
        buffers) for an upstream gradient grad_y = dL/dvisibility."""
        t = self.torch
        n = ids.shape[0]
        if ws is None:
            ws = t.empty(max(1, self.workspace_bytes(n, 1)), dtype=t.uint8, device=self.device)
        _check(lib().nif_backward(self.h, mlp, _ptr(rays), _ptr(ids), _ptr(tmax), _ptr(grad_y), n, _ptr(mlp_grad),
                                  _ptr(ws), ws.numel(), _stream()), "nif_backward")
