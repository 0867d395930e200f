"""The C-ABI library loads, exports every symbol include/nif.h declares, and
validates arguments on the host (no GPU needed: these calls return before any
device work)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2306_07191_amd import nif
from paper_2306_07191_amd import synth as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "nif.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nif_[a-z_0-9]+)\s*\(", src)))


def test_header_and_exports_agree():
    assert _declared() == sorted(nif.EXPORTS)


def test_library_exports_every_symbol():
    L = nif.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert b"gfx950" in L.nif_version()


def _desc(**kw):
    d = dict(levels=4, res_min=4, res_max=32, feats=2, grid_dtype=0, hidden_layers=3, width=64)
    d.update(kw)
    return nif.ModelDesc(**d)


@pytest.mark.parametrize("bad,code", [(dict(feats=3), -2), (dict(width=48), -2), (dict(levels=5), -2),
                                      (dict(hidden_layers=0), -2), (dict(res_max=2), -2), (dict(grid_dtype=2), -2),
                                      (dict(res_max=2048), -2)])
def test_create_rejects_unsupported(bad, code):
    h = C.c_void_p()
    assert nif.lib().nif_create(C.byref(_desc(**bad)), 1, 1, C.byref(h)) == code
    assert len(nif.lib().nif_last_error()) > 0


def test_validation_before_device_work():
    L = nif.lib()
    h = C.c_void_p()
    assert L.nif_create(None, 1, 1, C.byref(h)) == -1
    assert L.nif_create(C.byref(_desc()), 0, 1, C.byref(h)) == -1
    assert L.nif_create(C.byref(_desc()), 2, 1, C.byref(h)) == 0
    try:
        ge, mp = C.c_int64(), C.c_int64()
        off = np.zeros(13, np.int64)
        res = np.zeros(4, np.int32)
        assert L.nif_param_layout(h, C.byref(ge), off.ctypes.data, res.ctypes.data, C.byref(mp)) == 0
        assert list(res) == [4, 8, 16, 32] and mp.value == S.TINY.mlp_params
        assert ge.value == off[-1] == 3 * 2 * sum((r + 1) ** 3 for r in res)
        box = np.array([0, 0, 0, 1, 1, 1], np.float32)
        flat = np.array([0, 0, 0, 1, 0, 1], np.float32)  # zero extent on y
        fake = C.c_void_p(4096)
        assert L.nif_set_object(h, 2, box.ctypes.data, fake, 0) == -1  # object out of range
        assert L.nif_set_object(h, 0, box.ctypes.data, fake, 1) == -1  # MLP out of range
        assert L.nif_set_object(h, 0, flat.ctypes.data, fake, 0) == -1  # degenerate box
        assert L.nif_set_object(h, 0, box.ctypes.data, None, 0) == -5  # no grid and no built query image
        assert L.nif_set_object(h, 0, box.ctypes.data, fake, 0) == 0
        assert L.nif_query(h, 0, fake, fake, fake, -1, fake, None, None, 0, None) == -1  # n < 0
        assert L.nif_query(h, 0, fake, fake, fake, 0, fake, None, None, 0, None) == 0   # n = 0: no-op
        assert L.nif_query(h, 0, None, fake, fake, 10, fake, None, None, 0, None) == -1  # NULL rays
        assert L.nif_query(h, 7, fake, fake, fake, 10, fake, None, None, 0, None) == -2  # unknown dtype
        assert L.nif_query(h, 0, fake, fake, fake, 10, fake, None, None, 0, None) == -5  # not prepared
        assert L.nif_query_noalloc(h, 0, fake, fake, fake, -1, fake, None, None) == -1  # n < 0
        assert L.nif_query_noalloc(h, 0, fake, fake, fake, 0, fake, None, None) == 0   # n = 0: no-op
        assert L.nif_query_noalloc(h, 0, fake, None, fake, 10, fake, None, None) == -1  # NULL ids
        assert L.nif_query_noalloc(h, 0, fake, fake, fake, 10, fake, None, None) == -5  # not prepared
        # more queries than the static scratch holds: refused, whatever the state
        assert L.nif_workspace_bytes(h, 2_000_000, 0) > 64 * 1024 * 1024
        assert L.nif_query_noalloc(h, 0, fake, fake, fake, 2_000_000, fake, None, None) == -2
        assert b"scratch" in L.nif_last_error()
        assert L.nif_prepare(h, 0, None) == -5  # object 1 and the MLP are not registered
        sc = np.array([1, 1, 1, 0, 1, 1], np.float32)
        assert L.nif_set_fp8_scales(h, 0, sc.ctypes.data) == -1  # zero scale
        assert L.nif_calibrate_fp8(h, 1, fake, fake, fake, 10, None, fake, 1 << 30, None) == -1  # MLP out of range
        assert L.nif_calibrate_fp8(h, 0, None, fake, fake, 10, None, fake, 1 << 30, None) == -1  # NULL rays
        assert L.nif_calibrate_fp8(h, 0, fake, fake, fake, 10, None, fake, 1 << 30, None) == -5  # MLP not set
        assert L.nif_last_error() != b""
    finally:
        L.nif_destroy(h)


def test_image_only_objects_validation_on_the_host():
    """nif_build_image and nif_set_object without a grid are refused unless the
    image mode is on, the object has an image buffer and a grid to build from,
    and (for no grid) its image was built; all before any device work."""
    L = nif.lib()
    h = C.c_void_p()
    assert L.nif_create(C.byref(_desc(grid_dtype=1)), 2, 1, C.byref(h)) == 0
    try:
        fake, img = C.c_void_p(4096), C.c_void_p(1 << 20)
        box = np.array([0, 0, 0, 1, 1, 1], np.float32)
        assert L.nif_build_image(h, 0, None) == -1  # object not registered
        assert L.nif_set_object(h, 0, box.ctypes.data, fake, 0) == 0
        assert L.nif_build_image(h, 2, None) == -1  # out of range
        assert L.nif_build_image(h, 0, None) == -5  # image mode 0
        assert L.nif_set_object(h, 0, box.ctypes.data, None, 0) == -5  # no image at all
        assert L.nif_set_option(h, 2, 1) == 0
        assert L.nif_build_image(h, 0, None) == -5  # no image buffer
        assert L.nif_set_image(h, 0, img, L.nif_image_bytes(h)) == 0
        assert L.nif_set_object(h, 0, box.ctypes.data, None, 0) == -5  # image registered, not built
        assert L.nif_last_error() != b""
        assert L.nif_set_option(h, 5, 5) == -1 and L.nif_set_option(h, 5, -2) == -1  # NIF_OPT_ORDER_BITS range
        assert L.nif_set_option(h, 5, 0) == 0 and L.nif_set_option(h, 5, -1) == 0
    finally:
        L.nif_destroy(h)


def test_paper_network_and_light_validation_on_the_host():
    """The paper's networks, light sampling and the 16-bit stages reject bad
    arguments before any device work."""
    L = nif.lib()
    assert L.nif_paper_mlp_params(0) == 4544 and L.nif_paper_mlp_params(1) == 5280
    assert L.nif_paper_mlp_params(2) == -1 and L.nif_paper_grid_elems(-1) == -1
    assert L.nif_paper_grid_elems(0) == 2 * 256 * 256 * 3 and L.nif_paper_grid_elems(1) == 2 * 128 * 128 * 5 + 128 * 3
    h = C.c_void_p()
    assert L.nif_paper_create(0, C.byref(h)) == -1
    assert L.nif_paper_create(1, C.byref(h)) == 0
    try:
        fake = C.c_void_p(4096)
        box = np.array([0, 0, 0, 1, 1, 1], np.float32)
        flat = np.array([0, 0, 0, 1, 0, 1], np.float32)
        assert L.nif_paper_set_object(h, 1, box.ctypes.data, fake, fake) == -1   # object out of range
        assert L.nif_paper_set_object(h, 0, flat.ctypes.data, fake, fake) == -1  # degenerate box
        assert L.nif_paper_set_object(h, 0, box.ctypes.data, None, fake) == -1
        assert L.nif_paper_set_object(h, 0, box.ctypes.data, fake, fake) == 0
        assert L.nif_paper_prepare(h, 3, None) == -2      # no FP8 form
        assert L.nif_paper_prepare(h, 0, None) == -5      # no weights yet
        assert L.nif_paper_query(h, 0, fake, fake, fake, 10, fake, None, None) == -5  # not prepared
        assert L.nif_paper_query(h, 0, fake, fake, fake, 0, fake, None, None) == 0    # n = 0
        assert L.nif_paper_train_step(h, 2, fake, fake, fake, fake, 10, 1, None, None, None, fake, 1 << 30, None) == -1
        assert L.nif_paper_train_step(h, 0, fake, fake, fake, fake, 10, 1, None, None, None, fake, 1 << 30, None) == -5
        assert L.nif_paper_set_object_train(h, 0, 2, fake, fake, fake) == -1
    finally:
        L.nif_paper_destroy(h)
    lh = C.c_void_p()
    tri = np.array([[0, 5, 0, 1, 5, 0, 0, 5, 1]], np.float32)
    line = np.array([[0, 5, 0, 1, 5, 0, 2, 5, 0]], np.float32)
    one = np.ones(1, np.float32)
    assert L.nif_light_create(line.ctypes.data, one.ctypes.data, 1, C.byref(lh)) == -1          # zero area
    assert L.nif_light_create(tri.ctypes.data, (-one).ctypes.data, 1, C.byref(lh)) == -1       # negative
    assert L.nif_light_create(tri.ctypes.data, np.zeros(1, np.float32).ctypes.data, 1, C.byref(lh)) == -1  # no flux
    assert L.nif_light_create(tri.ctypes.data, one.ctypes.data, 0, C.byref(lh)) == -1           # no triangles
    c = C.c_void_p()
    assert L.nif_create(C.byref(_desc()), 1, 1, C.byref(c)) == 0
    try:
        fake = C.c_void_p(4096)
        assert L.nif_encode16(c, 0, fake, fake, fake, 10, fake, None, None) == -2  # binary32 is not a 16-bit format
        assert L.nif_encode16(c, 2, fake, fake, fake, 10, C.c_void_p(4098), None, None) == -1  # misaligned
        assert L.nif_mlp16(c, 3, 0, fake, 10, fake, None) == -2                    # FP8 is not 16-bit
        assert L.nif_order_packed(c, fake, fake, fake, 10, fake, C.c_void_p(4100), fake, 1 << 30, None) == -1  # misaligned
    finally:
        L.nif_destroy(c)


def test_query_image_is_caller_owned():
    """NIF_OPT_GRID_IMAGE images live in caller buffers: nif_image_bytes gives
    their size for the mode (kind 1: (N+1) x N x (N+1) entries of 4 latents
    per table; kind 2: (N+1) x N x N entries of 8), nif_set_image checks the
    buffer, and nif_prepare refuses while an object has none."""
    L = nif.lib()
    h = C.c_void_p()
    assert L.nif_create(C.byref(_desc(grid_dtype=1)), 2, 1, C.byref(h)) == 0
    try:
        res = [4, 8, 16, 32]
        fake = C.c_void_p(1 << 20)
        assert L.nif_image_bytes(h) == 0                       # default: no image
        assert L.nif_set_image(h, 0, fake, 1 << 30) == -5       # mode 0 has no image
        for kind, per in ((1, lambda N: (N + 1) * N * (N + 1) * 4), (2, lambda N: (N + 1) * N * N * 8)):
            assert L.nif_set_option(h, 2, kind) == 0
            need = 3 * sum(per(N) for N in res) * 2
            assert L.nif_image_bytes(h) == need
            assert L.nif_set_image(h, 2, fake, need) == -1           # object out of range
            assert L.nif_set_image(h, 0, None, need) == -1
            assert L.nif_set_image(h, 0, C.c_void_p((1 << 20) + 64), need) == -1  # not 256-byte aligned
            assert L.nif_set_image(h, 0, fake, need - 1) == -3       # too small
            assert L.nif_set_image(h, 0, fake, need) == 0
        box = np.array([0, 0, 0, 1, 1, 1], np.float32)
        w = C.c_void_p(1 << 21)
        for k in range(2):
            assert L.nif_set_object(h, k, box.ctypes.data, w, 0) == 0
        assert L.nif_set_mlp(h, 0, w) == 0
        assert L.nif_prepare(h, 0, None) == -5  # object 1 has no image buffer
        assert b"nif_set_image" in L.nif_last_error()
        # binary32 grids have no image form
        h2 = C.c_void_p()
        assert L.nif_create(C.byref(_desc()), 1, 1, C.byref(h2)) == 0
        assert L.nif_set_option(h2, 2, 1) == -2
        L.nif_destroy(h2)
    finally:
        L.nif_destroy(h)


def test_expand_pairs_total_stays_32_bit():
    """The pair counts are scanned in 32 bits: a call whose rays x objects could
    reach 2^32 pairs is refused on the host."""
    L = nif.lib()
    h = C.c_void_p()
    assert L.nif_create(C.byref(_desc()), 4096, 1, C.byref(h)) == 0
    try:
        fake = C.c_void_p(4096)
        cnt = C.c_void_p(8192)
        n = (1 << 32) // 4096  # n x K = 2^32
        assert L.nif_expand_pairs(h, fake, fake, n, 0, None, None, None, None, cnt, fake, 1 << 40, None) == -2
        assert b"2^32" in L.nif_last_error()
    finally:
        L.nif_destroy(h)
