"""ctypes front-end of the CPU oracle (nif_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark; never by the product path.  The heavy
per-query loops are in C (binary64, binary32 only where a float decides a
grid cell); what is here is marshalling plus the two steps that are plain
elementwise formulas: the binary cross-entropy of a vector of logits and the
Adam update.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nif_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

QUANT = {"f32": 0, "exact": 0, "bf16": 1, "f16": 2, "fp8": 3}
FMT = {"f32": 0, "f16": 1, "bf16": 2, "e4m3": 3}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (binary64, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-Wall",
                               "-shared", "-fPIC", "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Model(C.Structure):
    _fields_ = [("levels", C.c_int32), ("res_min", C.c_int32), ("res_max", C.c_int32), ("feats", C.c_int32),
                ("hidden", C.c_int32), ("width", C.c_int32), ("num_objects", C.c_int32),
                ("grid_dtype", C.c_int32), ("quant", C.c_int32), ("coord_mode", C.c_int32),
                ("aabb", C.c_void_p), ("grids", C.c_void_p), ("grid_seed", C.c_void_p),
                ("grid_amp", C.c_void_p), ("mlp_index", C.c_void_p), ("mlps", C.c_void_p),
                ("fp8_scales", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        sig = {
            "orc_round_fmt": (d, [d, C.c_int]),
            "orc_midpoint_distance": (d, [d, C.c_int]),
            "orc_f16_to_f64": (d, [C.c_uint16]),
            "orc_bf16_to_f64": (d, [C.c_uint16]),
            "orc_e4m3_to_f64": (d, [C.c_uint8]),
            "orc_f64_to_f16_bits": (C.c_uint16, [d]),
            "orc_f64_to_e4m3_bits": (C.c_uint8, [d]),
            "orc_philox4x64_10": (None, [vp, vp, vp]),
            "orc_init_value_f32": (C.c_float, [C.c_uint64, C.c_uint64, C.c_uint64, C.c_float]),
            "orc_init_fill": (None, [C.c_uint64, C.c_uint64, C.c_float, C.c_int, i64, i64, vp]),
            "orc_din": (i32, [vp]),
            "orc_mlp_params": (i64, [vp]),
            "orc_level_res": (None, [i32, i32, i32, vp]),
            "orc_grid_offsets": (i64, [vp, vp]),
            "orc_forward": (None, [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_int]),
            "orc_query_detail": (C.c_int, [vp, vp, i32, C.c_float, vp, vp, vp, vp]),
            "orc_mlp_only": (None, [vp, i32, i64, vp, vp, vp, vp, vp]),
            "orc_status": (None, [vp, i64, vp, vp, vp, vp]),
            "orc_segment": (None, [vp, i64, vp, vp, vp, vp, vp]),
            "orc_backward": (i64, [vp, i32, i64, vp, vp, vp, vp, vp, vp, vp, C.c_int]),
            "orc_backward_given": (i64, [vp, i32, i64, vp, vp, vp, vp, vp, vp, C.c_int]),
            "orc_grid_grad_dense": (None, [vp, i32, i64, vp, vp, vp, vp, vp]),
            "orc_grid_grad_at": (None, [vp, i32, i64, vp, vp, vp, vp, i64, vp, vp]),
            "orc_ray_tri": (C.c_int, [vp, vp, d, vp]),
            "orc_anyhit_brute": (None, [i64, vp, i64, vp, vp, vp, C.c_int]),
            "orc_bvh_build": (vp, [i64, vp]),
            "orc_bvh_free": (None, [vp]),
            "orc_anyhit_bvh": (None, [vp, i64, vp, vp, vp, C.c_int]),
            "orc_ray_tri_t": (C.c_int, [vp, vp, d, vp, vp]),
            "orc_closest_brute": (None, [i64, vp, i64, vp, vp, vp, C.c_int]),
            "orc_closest_bvh": (None, [vp, i64, vp, vp, vp, C.c_int]),
            "orc_ray_tri32_t": (C.c_int, [vp, vp, C.c_float, vp, vp]),
            "orc_trace_brute32": (None, [i64, vp, i64, vp, vp, vp, vp, C.c_int]),
            "orc_trace_bvh32": (None, [vp, i64, vp, vp, vp, vp, C.c_int]),
            "orc_default_threads": (C.c_int, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# --------------------------------------------------------------------------
# number formats and the latent generator
# --------------------------------------------------------------------------

def round_fmt(x: float, fmt: str) -> float:
    return lib().orc_round_fmt(float(x), FMT[fmt])


def round_fmt_array(a, fmt: str) -> np.ndarray:
    f = lib().orc_round_fmt
    k = FMT[fmt]
    return np.array([f(float(v), k) for v in np.asarray(a, np.float64).ravel()]).reshape(np.shape(a))


def philox4x64_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def init_grid(seed: int, obj: int, amp: float, grid_dtype: str, count: int, begin: int = 0) -> np.ndarray:
    """Initial latents [begin, begin+count) of object obj's grid buffer."""
    dt = np.uint16 if grid_dtype == "f16" else np.float32
    out = np.empty(count, dt)
    lib().orc_init_fill(seed, obj, amp, 1 if grid_dtype == "f16" else 0, begin, count, _p(out))
    return out


# --------------------------------------------------------------------------
# model
# --------------------------------------------------------------------------

class Model:
    """Owns the arrays an orc_model points at.

    shape: synth.ModelShape.  aabb: float32 [K, 6].  grids: list of K arrays
    (float32, or uint16 binary16 bits) or None entries for generated grids.
    mlps: [M, P] weights (binary64 copies are made).  quant: "exact", "bf16",
    "f16" or "fp8".  fp8_scales: [M, 2H] (s_W for layers 1..H, then s_x)."""

    def __init__(self, shape, aabb, mlps, mlp_index=None, grids=None, grid_seed=0, grid_amp=1e-4,
                 quant="exact", coord_mode=0, fp8_scales=None):
        self.shape = shape
        self.aabb = np.ascontiguousarray(aabb, np.float32).reshape(-1, 6)
        K = self.aabb.shape[0]
        self.K = K
        self.mlps64 = np.ascontiguousarray(np.asarray(mlps, np.float64).reshape(-1, shape.mlp_params))
        self.M = self.mlps64.shape[0]
        self.mlp_index = np.ascontiguousarray(
            np.zeros(K, np.int32) if mlp_index is None else np.asarray(mlp_index, np.int32))
        grids = [None] * K if grids is None else list(grids)
        self._grids = [None if g is None else np.ascontiguousarray(g) for g in grids]
        self._gptr = (C.c_void_p * K)(*[None if g is None else g.ctypes.data for g in self._grids])
        self.grid_seed = np.ascontiguousarray(np.broadcast_to(np.asarray(grid_seed, np.uint64), (K,)).copy())
        self.grid_amp = np.ascontiguousarray(np.broadcast_to(np.asarray(grid_amp, np.float32), (K,)).copy())
        self._mptr = (C.c_void_p * self.M)(*[self.mlps64[i].ctypes.data for i in range(self.M)])
        self.fp8 = None
        self._sptr = None
        if fp8_scales is not None:
            self.fp8 = np.ascontiguousarray(np.asarray(fp8_scales, np.float64).reshape(self.M, -1))
            self._sptr = (C.c_void_p * self.M)(*[self.fp8[i].ctypes.data for i in range(self.M)])
        self.s = _Model(shape.levels, shape.res_min, shape.res_max, shape.feats, shape.hidden, shape.width,
                        K, 1 if shape.grid_dtype == "f16" else 0, QUANT[quant], coord_mode,
                        self.aabb.ctypes.data, C.cast(self._gptr, C.c_void_p).value,
                        self.grid_seed.ctypes.data, self.grid_amp.ctypes.data, self.mlp_index.ctypes.data,
                        C.cast(self._mptr, C.c_void_p).value,
                        None if self._sptr is None else C.cast(self._sptr, C.c_void_p).value)

    @property
    def ref(self):
        return C.byref(self.s)

    def with_(self, **kw):
        args = dict(shape=self.shape, aabb=self.aabb, mlps=self.mlps64, mlp_index=self.mlp_index,
                    grids=self._grids, grid_seed=self.grid_seed, grid_amp=self.grid_amp,
                    quant={v: k for k, v in QUANT.items() if k not in ("f32",)}[self.s.quant],
                    coord_mode=self.s.coord_mode, fp8_scales=self.fp8)
        args.update(kw)
        return Model(**args)

    # ---- layout --------------------------------------------------------
    def level_res(self):
        r = np.zeros(self.shape.levels, np.int32)
        lib().orc_level_res(self.shape.levels, self.shape.res_min, self.shape.res_max, _p(r))
        return r

    def grid_offsets(self):
        off = np.zeros(3 * self.shape.levels + 1, np.int64)
        lib().orc_grid_offsets(self.ref, _p(off))
        return off

    @property
    def grid_elems(self) -> int:
        return int(self.grid_offsets()[-1])

    # ---- forward -------------------------------------------------------
    def forward(self, rays, ids, tmax, nthreads: int = 0, want_x: bool = False):
        rays = np.ascontiguousarray(rays, np.float32)
        ids = np.ascontiguousarray(ids, np.int32)
        tmax = np.ascontiguousarray(tmax, np.float32)
        n = ids.shape[0]
        z = np.empty(n)
        y = np.empty(n)
        st = np.empty(n, np.int32)
        ztol = np.empty(n)
        yb = np.empty(n)
        fl = np.empty(n, np.int32)
        x = np.zeros((n, self.shape.din)) if want_x else None
        lib().orc_forward(self.ref, n, _p(rays), _p(ids), _p(tmax), _p(z), _p(y), _p(st), _p(ztol), _p(yb),
                          _p(fl), _p(x), nthreads)
        out = dict(z=z, y=y, status=st, ztol=ztol, ybound=yb, flags=fl)
        if want_x:
            out["x"] = x
        return out

    def status(self, rays, ids, tmax):
        """Clip status only: 1 the segment meets the AABB, 0 miss, -1 invalid."""
        rays = np.ascontiguousarray(rays, np.float32)
        ids = np.ascontiguousarray(ids, np.int32)
        tmax = np.ascontiguousarray(tmax, np.float32)
        st = np.empty(ids.shape[0], np.int32)
        lib().orc_status(self.ref, ids.shape[0], _p(rays), _p(ids), _p(tmax), _p(st))
        return st

    def segment(self, rays, ids, tmax):
        """[t_a, t_b] of every query (+inf for a miss, NaN for an invalid one)."""
        rays = np.ascontiguousarray(rays, np.float32)
        ids = np.ascontiguousarray(ids, np.int32)
        tmax = np.ascontiguousarray(tmax, np.float32)
        n = ids.shape[0]
        ta, tb = np.empty(n), np.empty(n)
        lib().orc_segment(self.ref, n, _p(rays), _p(ids), _p(tmax), _p(ta), _p(tb))
        return ta, tb

    # ---- depth output for primary rays (Sec. 7: the network can encode the
    # ---- depth of the first hit instead of visibility) ------------------
    def depth_targets(self, rays, ids, tmax, t_hit):
        """Normalised depth s = (t_hit - t_a) / (t_b - t_a) clamped to [0, 1] of
        the queries that meet their AABB, whose closest hit is finite and whose
        segment has t_b > t_a; NaN elsewhere (no target)."""
        ta, tb = self.segment(rays, ids, tmax)
        t_hit = np.asarray(t_hit, np.float64)
        ok = np.isfinite(ta) & np.isfinite(tb) & np.isfinite(t_hit) & (tb > ta)
        s = np.full(ta.shape, np.nan)
        s[ok] = np.clip((t_hit[ok] - ta[ok]) / (tb[ok] - ta[ok]), 0.0, 1.0)
        return s

    def depth_loss_backward(self, rays, ids, tmax, t_hit, nthreads: int = 0):
        """L2 depth loss (the paper trains with L2, Sec. 5 "Training") over the B
        queries with a target: L = (1/B) sum (y - s)^2, y = sigmoid(z); its
        gradients through the upstream-gradient backward with dL/dy = 2 (y - s) / B.
        Returns (loss, B, mlp_grads [M, P], gx [n, din])."""
        s = self.depth_targets(rays, ids, tmax, t_hit)
        f = self.forward(rays, ids, tmax, nthreads=nthreads)
        ok = np.isfinite(s) & (f["status"] == 1)
        B = int(ok.sum())
        gy = np.zeros(s.shape[0])
        if B:
            gy[ok] = 2.0 * (f["y"][ok] - s[ok]) / B
        _, g, gx = self.backward_given(rays, ids, tmax, gy, nthreads=nthreads)
        loss = float(((f["y"][ok] - s[ok]) ** 2).mean()) if B else 0.0
        return loss, B, g, gx

    def depth(self, rays, ids, tmax, nthreads: int = 0):
        """Predicted closest-hit distance t_a + y (t_b - t_a) (+inf for a miss)."""
        ta, tb = self.segment(rays, ids, tmax)
        y = self.forward(rays, ids, tmax, nthreads=nthreads)["y"]
        t = ta + y * (tb - ta)
        t[np.isinf(ta)] = np.inf
        return t

    def expand_pairs(self, rays, tmax):
        """(Sec. 4.1) The (ray, object) pairs whose segment meets the object's AABB,
        in ray order and objects ascending: (pair_ray, pair_obj)."""
        n, K = tmax.shape[0], self.K
        rr = np.repeat(np.arange(n, dtype=np.int64), K)
        kk = np.tile(np.arange(K, dtype=np.int32), n)
        st = self.status(np.asarray(rays)[rr], kk, np.asarray(tmax)[rr])
        hit = st == 1
        return rr[hit], kk[hit]

    def detail(self, ray, obj, tmax):
        L = self.shape.levels
        u = np.zeros(9)
        x = np.zeros(self.shape.din)
        ce = np.zeros(3 * L * 8, np.int64)
        cw = np.zeros(3 * L * 8)
        r = np.ascontiguousarray(ray, np.float32)
        st = lib().orc_query_detail(self.ref, _p(r), int(obj), float(tmax), _p(u), _p(x), _p(ce), _p(cw))
        return st, u.reshape(3, 3), x, ce.reshape(3 * L, 8), cw.reshape(3 * L, 8)

    def mlp_only(self, x, mlp: int = 0, want_acts: bool = False, want_tol: bool = False):
        """Logits of MLP `mlp` on features x [n, din]; with want_acts also the
        pre-activation outputs a_j = W_j h_{j-1} of the hidden layers [n, H, width];
        with want_tol a dict with z, ztol and ybound (as forward's)."""
        x = np.ascontiguousarray(x, np.float64).reshape(-1, self.shape.din)
        n = x.shape[0]
        z = np.empty(n)
        acts = np.empty((n, self.shape.hidden, self.shape.width)) if want_acts else None
        ztol = np.empty(n) if want_tol else None
        yb = np.empty(n) if want_tol else None
        lib().orc_mlp_only(self.ref, mlp, n, _p(x), _p(z), _p(acts), _p(ztol), _p(yb))
        if want_tol:
            return dict(z=z, ztol=ztol, ybound=yb)
        return (z, acts) if want_acts else z

    def fp8_calibrate(self, rays, ids, tmax, mlp: int = 0):
        """Per-layer E4M3 scales of MLP `mlp` (the paper's networks run in reduced
        precision, Sec. 4.2; per-layer scaling is the reading for E4M3): s_W[j] =
        max|W_j| / 448 and s_x[j] = max |input of layer j| / 448 over the queries
        that meet their AABB and whose object uses `mlp`, the inputs taken from
        the binary64 forward pass (x for layer 1, h_{j-1} after ReLU for layer
        j); 1 where the maximum is 0.  Returns [s_W..., s_x...]."""
        exact = self.with_(quant="exact")
        f = exact.forward(rays, ids, tmax, want_x=True)
        ids = np.asarray(ids)
        sel = f["status"] == 1
        sel[sel] &= self.mlp_index[ids[sel]] == mlp
        H, W, din = self.shape.hidden, self.shape.width, self.shape.din
        w = self.mlps64[mlp]
        amax_w, amax_x = [], []
        off = 0
        for j in range(H):
            kin = din if j == 0 else W
            amax_w.append(np.abs(w[off:off + W * kin]).max(initial=0.0))
            off += W * kin
        x = f["x"][sel]
        amax_x.append(np.abs(x).max(initial=0.0))
        if H > 1:
            _, acts = exact.mlp_only(x, mlp, want_acts=True)
            for j in range(1, H):
                amax_x.append(np.maximum(acts[:, j - 1, :], 0.0).max(initial=0.0))  # acts: pre-ReLU
        return np.array([a / 448.0 if a > 0 else 1.0 for a in amax_w + amax_x])

    # ---- training ------------------------------------------------------
    def backward(self, rays, ids, tmax, labels, nthreads: int = 0, want_gx: bool = True):
        """Returns (loss, B, mlp_grads [M, P], gx [n, din])."""
        rays = np.ascontiguousarray(rays, np.float32)
        ids = np.ascontiguousarray(ids, np.int32)
        tmax = np.ascontiguousarray(tmax, np.float32)
        labels = np.ascontiguousarray(labels, np.uint8)
        n = ids.shape[0]
        loss = C.c_double(0.0)
        g = np.zeros((self.M, self.shape.mlp_params))
        gx = np.zeros((n, self.shape.din)) if want_gx else None
        B = lib().orc_backward(self.ref, self.M, n, _p(rays), _p(ids), _p(tmax), _p(labels), C.byref(loss),
                               _p(g), _p(gx), nthreads)
        return loss.value, int(B), g, gx

    def backward_given(self, rays, ids, tmax, grad_y, nthreads: int = 0):
        """Gradients of sum_i grad_y[i] * y_i: returns (B, mlp_grads [M, P], gx [n, din])."""
        rays = np.ascontiguousarray(rays, np.float32)
        ids = np.ascontiguousarray(ids, np.int32)
        tmax = np.ascontiguousarray(tmax, np.float32)
        gy = np.ascontiguousarray(grad_y, np.float64)
        n = ids.shape[0]
        g = np.zeros((self.M, self.shape.mlp_params))
        gx = np.zeros((n, self.shape.din))
        B = lib().orc_backward_given(self.ref, self.M, n, _p(rays), _p(ids), _p(tmax), _p(gy), _p(g), _p(gx),
                                     nthreads)
        return int(B), g, gx

    def grid_grad_dense(self, obj, rays, ids, tmax, gx):
        out = np.zeros(self.grid_elems)
        lib().orc_grid_grad_dense(self.ref, obj, ids.shape[0], _p(np.ascontiguousarray(rays, np.float32)),
                                  _p(np.ascontiguousarray(ids, np.int32)),
                                  _p(np.ascontiguousarray(tmax, np.float32)), _p(np.ascontiguousarray(gx)),
                                  _p(out))
        return out

    def grid_grad_at(self, obj, rays, ids, tmax, gx, elems):
        elems = np.ascontiguousarray(np.sort(np.asarray(elems, np.int64)))
        out = np.zeros(elems.shape[0])
        lib().orc_grid_grad_at(self.ref, obj, ids.shape[0], _p(np.ascontiguousarray(rays, np.float32)),
                               _p(np.ascontiguousarray(ids, np.int32)),
                               _p(np.ascontiguousarray(tmax, np.float32)), _p(np.ascontiguousarray(gx)),
                               elems.shape[0], _p(elems), _p(out))
        return elems, out


# --------------------------------------------------------------------------
# elementwise steps
# --------------------------------------------------------------------------

def combine_pairs(pair_ray, visibility, n_rays):
    """(Sec. 4.1) A ray is visible iff every one of its pairs is visible
    (visibility >= 0.5); a ray without pairs is visible.  Returns uint8 [n_rays]."""
    out = np.ones(n_rays, np.uint8)
    for r, v in zip(np.asarray(pair_ray).tolist(), np.asarray(visibility).tolist()):
        if v < 0.5:
            out[r] = 0
    return out


def bce_with_logits(z, t):
    """mean(softplus(z) - t z) and its derivative (sigmoid(z) - t) / B."""
    z = np.asarray(z, np.float64)
    t = np.asarray(t, np.float64)
    sp = np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))
    B = z.shape[0]
    return (sp - t * z).mean(), (1.0 / (1.0 + np.exp(-z)) - t) / B


def adam_step(theta, m, v, g, step, lr, beta1, beta2, eps, lazy: bool):
    """One bias-corrected Adam step (Kingma & Ba 2015, Algorithm 1) in binary64.
    lazy=True leaves entries with g == 0 exactly untouched (m, v, theta)."""
    theta = np.asarray(theta, np.float64).copy()
    m = np.asarray(m, np.float64).copy()
    v = np.asarray(v, np.float64).copy()
    g = np.asarray(g, np.float64)
    sel = (g != 0.0) if lazy else np.ones(g.shape, bool)
    m[sel] = beta1 * m[sel] + (1.0 - beta1) * g[sel]
    v[sel] = beta2 * v[sel] + (1.0 - beta2) * g[sel] ** 2
    mh = m[sel] / (1.0 - beta1 ** step)
    vh = v[sel] / (1.0 - beta2 ** step)
    theta[sel] = theta[sel] - lr * mh / (np.sqrt(vh) + eps)
    return theta, m, v


# --------------------------------------------------------------------------
# exact labels
# --------------------------------------------------------------------------

def ray_tri(o, d, tmax, tri) -> bool:
    o = np.ascontiguousarray(o, np.float64)
    d = np.ascontiguousarray(d, np.float64)
    t = np.ascontiguousarray(tri, np.float32).reshape(9)
    return bool(lib().orc_ray_tri(_p(o), _p(d), float(tmax), _p(t)))


def anyhit_brute(tris, rays, tmax, nthreads: int = 0) -> np.ndarray:
    tris = np.ascontiguousarray(tris, np.float32)
    rays = np.ascontiguousarray(rays, np.float32)
    tmax = np.ascontiguousarray(tmax, np.float32)
    vis = np.empty(rays.shape[0], np.uint8)
    lib().orc_anyhit_brute(tris.shape[0], _p(tris), rays.shape[0], _p(rays), _p(tmax), _p(vis), nthreads)
    return vis


def ray_tri_t(o, d, tmax, tri):
    """Hit distance of the watertight test (binary64), or None for a miss."""
    o = np.ascontiguousarray(o, np.float64)
    d = np.ascontiguousarray(d, np.float64)
    t = np.ascontiguousarray(tri, np.float32).reshape(9)
    out = C.c_double(0.0)
    return out.value if lib().orc_ray_tri_t(_p(o), _p(d), float(tmax), _p(t), C.byref(out)) else None


def closest_brute(tris, rays, tmax, nthreads: int = 0) -> np.ndarray:
    """Closest-hit distance per ray (binary64; +inf when no hit with 0 < t < t_max)."""
    tris = np.ascontiguousarray(tris, np.float32)
    rays = np.ascontiguousarray(rays, np.float32)
    tmax = np.ascontiguousarray(tmax, np.float32)
    t = np.empty(rays.shape[0])
    lib().orc_closest_brute(tris.shape[0], _p(tris), rays.shape[0], _p(rays), _p(tmax), _p(t), nthreads)
    return t


def trace_brute32(tris, rays, tmax, nthreads: int = 0):
    """(visible uint8, closest-hit float32) of the binary32 watertight test over
    every triangle: the GPU caster's decisions, for exact comparison."""
    tris = np.ascontiguousarray(tris, np.float32)
    rays = np.ascontiguousarray(rays, np.float32)
    tmax = np.ascontiguousarray(tmax, np.float32)
    vis = np.empty(rays.shape[0], np.uint8)
    t = np.empty(rays.shape[0], np.float32)
    lib().orc_trace_brute32(tris.shape[0], _p(tris), rays.shape[0], _p(rays), _p(tmax), _p(vis), _p(t), nthreads)
    return vis, t


class BVH:
    def __init__(self, tris):
        self.tris = np.ascontiguousarray(tris, np.float32)
        self.h = lib().orc_bvh_build(self.tris.shape[0], _p(self.tris))

    def anyhit(self, rays, tmax, nthreads: int = 0) -> np.ndarray:
        rays = np.ascontiguousarray(rays, np.float32)
        tmax = np.ascontiguousarray(tmax, np.float32)
        vis = np.empty(rays.shape[0], np.uint8)
        lib().orc_anyhit_bvh(self.h, rays.shape[0], _p(rays), _p(tmax), _p(vis), nthreads)
        return vis

    def trace32(self, rays, tmax, nthreads: int = 0):
        """trace_brute32 through the BVH (same answer)."""
        rays = np.ascontiguousarray(rays, np.float32)
        tmax = np.ascontiguousarray(tmax, np.float32)
        vis = np.empty(rays.shape[0], np.uint8)
        t = np.empty(rays.shape[0], np.float32)
        lib().orc_trace_bvh32(self.h, rays.shape[0], _p(rays), _p(tmax), _p(vis), _p(t), nthreads)
        return vis, t

    def closest(self, rays, tmax, nthreads: int = 0) -> np.ndarray:
        rays = np.ascontiguousarray(rays, np.float32)
        tmax = np.ascontiguousarray(tmax, np.float32)
        t = np.empty(rays.shape[0])
        lib().orc_closest_bvh(self.h, rays.shape[0], _p(rays), _p(tmax), _p(t), nthreads)
        return t

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_bvh_free(self.h)
            self.h = None


def default_threads() -> int:
    return int(lib().orc_default_threads())
