"""Parity of the training step (nif_train_step through the C ABI) with the
oracle's binary64 gradients and Adam update."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2306_07191_amd import synth as S

from gpu_util import GRID_SEED, make_pair

pytestmark = pytest.mark.gpu


def _tiny_labelled(n=4096, gain=2.0):
    w = S.tiny_workload(n_rays=n)
    w["mlps"] = (w["mlps"].astype(np.float64) * gain).astype(np.float32)
    w["labels"] = O.BVH(w["tris"]).anyhit(w["rays"], w["tmax"])
    return w


def _cuda(w, *keys):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(w[k])).cuda() for k in keys]


def _grad_close(g, g64, rel_norm=1e-4, rel_max=1e-3):
    err = np.abs(g - g64)
    nrm = np.linalg.norm(err) / max(np.linalg.norm(g64), 1e-300)
    assert nrm <= rel_norm, f"relative norm error {nrm}"
    assert err.max() <= rel_max * np.abs(g64).max(), f"max error {err.max()} vs max |g| {np.abs(g64).max()}"
    return nrm, err.max()


@pytest.mark.parametrize("order", [0, 1])
def test_gradients_match_oracle(order):
    import torch
    from paper_2306_07191_amd import nif
    w = _tiny_labelled()
    ctx, model = make_pair(w, grid_amp=0.5)
    ctx.set_option(nif.NIF_OPT_ORDER, order)
    ctx.prepare("f32")
    ctx.setup_training()
    rays, ids, tmax, labels = _cuda(w, "rays", "ids", "tmax", "labels")
    loss = torch.zeros(1, device="cuda")
    g = torch.zeros(ctx.mlp_params, device="cuda")
    ctx.train_step(rays, ids, tmax, labels, step=1, adam=None, loss=loss, mlp_grad=g)
    torch.cuda.synchronize()
    L64, B, gW, gx = model.backward(w["rays"], w["ids"], w["tmax"], w["labels"])
    assert abs(loss.item() - L64) <= 1e-5 * abs(L64)
    st = _grad_close(g.cpu().numpy().astype(np.float64), gW[0])
    gg64 = model.grid_grad_dense(0, w["rays"], w["ids"], w["tmax"], gx)
    gg = ctx.train_bufs[0][0].cpu().numpy().astype(np.float64)
    sg = _grad_close(gg, gg64)
    assert ((gg != 0) == (gg64 != 0)).mean() > 0.999  # same touched set (bar exact cancellations)
    assert (ctx.train_bufs[0][3].cpu().numpy() == 0).all()  # bitmap cleared
    print("mlp grad err", st, "grid grad err", sg, "B", B)


def test_adam_step_matches_oracle():
    """One Adam step (step 3) from a seeded non-zero state of latents, weights and moments."""
    import torch
    w = _tiny_labelled()
    ctx, model = make_pair(w, grid_amp=0.5)
    ctx.prepare("f32")
    ctx.setup_training()
    g_ = np.random.default_rng(21)
    P, E = ctx.mlp_params, ctx.grid_elems
    mm = g_.normal(0, 1e-3, P).astype(np.float32)
    vv = g_.uniform(1e-7, 1e-5, P).astype(np.float32)
    gm = g_.normal(0, 1e-4, E).astype(np.float32)
    gv = g_.uniform(1e-9, 1e-7, E).astype(np.float32)
    ctx.mlp_moments[0][0].copy_(torch.from_numpy(mm))
    ctx.mlp_moments[0][1].copy_(torch.from_numpy(vv))
    ctx.train_bufs[0][1].copy_(torch.from_numpy(gm))
    ctx.train_bufs[0][2].copy_(torch.from_numpy(gv))
    theta0 = ctx.grids[0].cpu().numpy().astype(np.float64)
    W0 = w["mlps"][0].astype(np.float64)
    rays, ids, tmax, labels = _cuda(w, "rays", "ids", "tmax", "labels")
    hp = dict(lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15)
    ctx.train_step(rays, ids, tmax, labels, step=3, adam=(hp["lr"], hp["beta1"], hp["beta2"], hp["eps"]))
    torch.cuda.synchronize()
    # oracle: same state, binary64
    m_grid = O.Model(w["shape"], w["aabb"], w["mlps"], grids=[theta0.astype(np.float32)])
    L64, B, gW, gx = m_grid.backward(w["rays"], w["ids"], w["tmax"], w["labels"])
    gg64 = m_grid.grid_grad_dense(0, w["rays"], w["ids"], w["tmax"], gx)
    W1, mW, vW = O.adam_step(W0, mm, vv, gW[0], 3, lazy=False, **hp)
    T1, mT, vT = O.adam_step(theta0, gm, gv, gg64, 3, lazy=True, **hp)
    Wg = ctx.mlps[0].cpu().numpy().astype(np.float64)
    Tg = ctx.grids[0].cpu().numpy().astype(np.float64)
    # Element by element.  Adam is smooth in g here (v > 0), so the device's
    # update differs from the oracle's by at most |d step / d g| times the
    # gradient's binary32 error (bounded by the gradient parity criterion:
    # 1e-3 of the largest |g|), plus the rounding of the stored value: a few
    # binary32 ulps for the weights, one binary16 ulp for the latents.
    def sens(theta, m, v, g):
        h = 1e-6 * np.maximum(np.abs(g), 1e-12)
        up = O.adam_step(theta, m, v, g + h, 3, lazy=False, **hp)[0]
        dn = O.adam_step(theta, m, v, g - h, 3, lazy=False, **hp)[0]
        return np.abs(up - dn) / (2 * h)
    dgW = 1e-3 * np.abs(gW[0]).max()
    tolW = sens(W0, mm, vv, gW[0]) * dgW + 4 * np.spacing(np.abs(W1).astype(np.float32)).astype(np.float64)
    errW = np.abs(Wg - W1)
    print("MLP Adam: max err / tol", (errW / tolW).max())
    assert (errW <= tolW).all()
    touched = gg64 != 0
    dgT = 1e-3 * np.abs(gg64).max()
    ulp16 = np.spacing(np.abs(T1[touched]).astype(np.float16)).astype(np.float64)
    tolT = sens(theta0[touched], gm[touched], gv[touched], gg64[touched]) * dgT + ulp16
    errT = np.abs(Tg[touched] - T1[touched])
    print("latent Adam: max err / tol", (errT / tolT).max())
    assert (errT <= tolT).all()
    assert (Tg[~touched] == theta0[~touched]).all()  # lazy rule: untouched latents keep their value
    np.testing.assert_allclose(ctx.train_bufs[0][1].cpu().numpy()[~touched], gm[~touched])
    assert (ctx.train_bufs[0][0].cpu().numpy() == 0).all()  # gradient left zero


def test_loss_decreases():
    import torch
    w = _tiny_labelled(n=8192, gain=1.0)
    ctx, model = make_pair(w, grid_amp=1e-4)
    ctx.prepare("f32")
    ctx.setup_training()
    rays, ids, tmax, labels = _cuda(w, "rays", "ids", "tmax", "labels")
    loss = torch.zeros(1, device="cuda")
    losses = []
    for step in range(1, 31):
        ctx.train_step(rays, ids, tmax, labels, step=step, loss=loss)
        losses.append(loss.item())
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.7 * losses[0], losses


def test_frame_batch_gradients_sampled():
    """Full-size training batch of the frame scene (262,144 rays, 8 levels up to 512,
    binary16 latents): MLP gradient and sampled latent gradients vs the oracle."""
    import torch
    w = S.frame_workload(with_mesh=False, n_rays=16)
    rays, tmax = S.train_batch(0)
    n = rays.shape[0]
    w.update(rays=rays, tmax=tmax, ids=np.zeros(n, np.int32))
    w["labels"] = (np.random.default_rng(4).uniform(size=n) < 0.6).astype(np.uint8)
    ctx, model = make_pair(w, grid_amp=0.25)
    ctx.prepare("f32")
    ctx.setup_training()
    r, i, t, lab = _cuda(w, "rays", "ids", "tmax", "labels")
    loss = torch.zeros(1, device="cuda")
    g = torch.zeros(ctx.mlp_params, device="cuda")
    ctx.train_step(r, i, t, lab, step=1, adam=None, loss=loss, mlp_grad=g)
    torch.cuda.synchronize()
    L64, B, gW, gx = model.backward(w["rays"], w["ids"], w["tmax"], w["labels"])
    assert abs(loss.item() - L64) <= 1e-5 * abs(L64)
    _grad_close(g.cpu().numpy().astype(np.float64), gW[0])
    gg = ctx.train_bufs[0][0]
    nz = torch.nonzero(gg).flatten().cpu().numpy()
    sel = np.random.default_rng(5).choice(nz, 2000, replace=False)
    el, ref = model.grid_grad_at(0, w["rays"], w["ids"], w["tmax"], gx, sel)
    got = gg[torch.from_numpy(el).cuda()].cpu().numpy().astype(np.float64)
    err = np.abs(got - ref)
    assert np.linalg.norm(err) <= 1e-4 * np.linalg.norm(ref) and err.max() <= 1e-3 * np.abs(ref).max()
    del ctx
    torch.cuda.empty_cache()


def test_backward_upstream_gradient_matches_oracle():
    """nif_backward: gradients of sum_i c_i y_i vs the oracle's binary64 chain rule."""
    import torch
    w = _tiny_labelled()
    ctx, model = make_pair(w, grid_amp=0.5)
    ctx.prepare("f32")
    ctx.setup_training()
    c = np.random.default_rng(12).normal(size=w["ids"].shape[0]).astype(np.float32)
    rays, ids, tmax = _cuda(w, "rays", "ids", "tmax")
    g = torch.zeros(ctx.mlp_params, device="cuda")
    ctx.backward(rays, ids, tmax, torch.from_numpy(c).cuda(), mlp_grad=g)
    torch.cuda.synchronize()
    B, gW, gx = model.backward_given(w["rays"], w["ids"], w["tmax"], c.astype(np.float64))
    _grad_close(g.cpu().numpy().astype(np.float64), gW[0])
    gg64 = model.grid_grad_dense(0, w["rays"], w["ids"], w["tmax"], gx)
    _grad_close(ctx.train_bufs[0][0].cpu().numpy().astype(np.float64), gg64)
    assert (ctx.train_bufs[0][3].cpu().numpy() == 0).all()


def test_autograd_function():
    """torch.autograd through the query: weight and latent gradients of sum_i c_i y_i."""
    import torch
    from paper_2306_07191_amd.autograd import visibility
    w = _tiny_labelled()
    ctx, model = make_pair(w, grid_amp=0.5)
    ctx.setup_training()
    ctx.mlps[0].requires_grad_(True)
    ctx.grids[0].requires_grad_(True)
    rays, ids, tmax = _cuda(w, "rays", "ids", "tmax")
    c = np.random.default_rng(13).normal(size=w["ids"].shape[0]).astype(np.float32)
    y = visibility(ctx, rays, ids, tmax)
    ref = model.forward(w["rays"], w["ids"], w["tmax"])
    hit = ref["status"] == 1
    yc = y.detach().cpu().numpy().astype(np.float64)
    assert (np.abs(yc[hit] - ref["y"][hit]) <= 1e-5 * ref["y"][hit]).all()
    (y * torch.from_numpy(c).cuda()).sum().backward()
    B, gW, gx = model.backward_given(w["rays"], w["ids"], w["tmax"], c.astype(np.float64))
    _grad_close(ctx.mlps[0].grad.cpu().numpy().astype(np.float64), gW[0])
    gg64 = model.grid_grad_dense(0, w["rays"], w["ids"], w["tmax"], gx)
    _grad_close(ctx.grids[0].grad.cpu().numpy().astype(np.float64), gg64)
