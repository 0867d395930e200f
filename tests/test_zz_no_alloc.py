"""nif_query_noalloc (the query entry point that allocates nothing, for callers
that cannot allocate device memory) against nif_query with a caller workspace:
bit-identical outputs on two calls in a row, the second smaller, so that the
second call runs over the scratch the first one left behind."""
import numpy as np
import pytest

from paper_2306_07191_amd import synth as S

from gpu_util import make_pair

pytestmark = pytest.mark.gpu


def _inputs(w, n):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(w["rays"][:n])).cuda(),
            torch.from_numpy(np.ascontiguousarray(w["ids"][:n])).cuda(),
            torch.from_numpy(np.ascontiguousarray(w["tmax"][:n])).cuda())


def _max_queries(ctx, limit):
    lo, hi = 1, 1 << 24
    while lo < hi:  # largest n whose workspace fits the scratch
        mid = (lo + hi + 1) // 2
        if ctx.workspace_bytes(mid, 0) <= limit:
            lo = mid
        else:
            hi = mid - 1
    return lo


@pytest.mark.parametrize("case", ["tiny", "frame"])
def test_noalloc_matches_query_on_two_calls(case):
    import torch
    from paper_2306_07191_amd import nif
    limit = 64 * 1024 * 1024
    if case == "tiny":
        w = S.tiny_workload(n_rays=400000)
        dtypes, sizes = ("f32", "bf16"), (400000, 70001)
    else:
        w = S.frame_workload(n_rays=1 << 20, with_mesh=False)
        dtypes, sizes = ("f16", "fp8"), (1 << 20, 99999)
    scales = None
    if "fp8" in dtypes:
        scales = np.ones((1, 2 * w["shape"].hidden), np.float64)
        scales[0, :w["shape"].hidden] = np.abs(w["mlps"][0]).max() / 448
    ctx, _ = make_pair(w, 0.5, fp8_scales=scales)
    try:
        ctx.set_option(nif.NIF_OPT_ORDER, 1)  # always order, so that every call uses the scratch
        if case == "frame":
            ctx.set_option(nif.NIF_OPT_GRID_IMAGE, 2)
        nmax = _max_queries(ctx, limit)
        print(f"{case}: at most {nmax} queries fit the {limit >> 20} MiB scratch", flush=True)
        assert 1_000_000 < nmax < 2_000_000
        for dtype in dtypes:
            ctx.prepare(dtype)
            for n in sizes:
                assert ctx.workspace_bytes(n, 0) > 0
                rays, ids, tmax = _inputs(w, n)
                y0, z0 = torch.empty(n, device="cuda"), torch.empty(n, device="cuda")
                y1, z1 = torch.full((n,), -7.0, device="cuda"), torch.full((n,), -7.0, device="cuda")
                ctx.query(rays, ids, tmax, dtype=dtype, out=y0, logits=z0)
                ctx.query_noalloc(rays, ids, tmax, dtype=dtype, out=y1, logits=z1)
                torch.cuda.synchronize()
                a, b = y0.cpu().numpy(), y1.cpu().numpy()
                print(f"{case} {dtype} n={n}: {int((a.view(np.uint32) != b.view(np.uint32)).sum())} differing bits",
                      flush=True)
                assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
                assert np.array_equal(z0.cpu().numpy().view(np.uint32), z1.cpu().numpy().view(np.uint32))
                assert np.isfinite(a).all() and ((a >= 0) & (a <= 1)).all()
        # beyond the scratch: refused on the host before anything is enqueued
        rays, ids, tmax = _inputs(w, 16)
        y = torch.empty(16, device="cuda")
        L = nif.lib()
        st = L.nif_query_noalloc(ctx.h, nif.DTYPES[dtypes[0]], rays.data_ptr(), ids.data_ptr(), tmax.data_ptr(),
                                 nmax + 1, y.data_ptr(), None, None)
        assert st == -2 and b"scratch" in L.nif_last_error()
    finally:
        ctx.close()
