"""Pins for the oracle's probability model, adjoint and Adam.

The forward pass is checked against PyTorch's own FP64 library routines
(embedding, linear, bmm, layer_norm, exact-erf gelu, softmax) -- a second,
independent implementation of the paper's Eqs. 9-16 and Eq. 1.  The adjoint is
checked against central finite differences of the oracle's own loss and
against torch.autograd; Adam against its first-step closed form and
torch.optim.Adam.
"""

import math

import numpy as np
import pytest
import torch
import torch.nn.functional as Fnn

from oracle.model import Config, Model, gelu, gelu_grad, layer_norm, softmax

TINY = Config(context=3, embed=4, latent=5, blocks=2, hidden=6, branches=2)
# the "w/o LTE" ablation of Table 4: F x F FDM, no W1 / W2
TINY_NO_LTE = Config(context=3, embed=4, latent=12, blocks=2, hidden=6, branches=2, lte=False)
# the "low-rank factorization" ablation of Table 4: per-instance A_s, U_s, B_s
TINY_LOW_RANK = Config(context=3, embed=4, latent=5, blocks=2, hidden=6, branches=2,
                       low_rank=True)


def _rand_model(cfg, n_slots, seed=0, scale=0.5):
    m = Model(cfg, n_slots)
    r = np.random.default_rng(seed)
    for k in m.p:
        m.p[k] = m.p[k] + scale * r.standard_normal(m.p[k].shape) * 0.3
    m.U = m.U + 0.3 * r.standard_normal(m.U.shape)
    if cfg.low_rank:
        m.A = m.A + 0.3 * r.standard_normal(m.A.shape)
        m.B = m.B + 0.3 * r.standard_normal(m.B.shape)
    return m


def _torch_forward(m: Model, ctx, slots, targets):
    cfg = m.cfg
    P = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in m.p.items()}
    U = torch.tensor(m.U, dtype=torch.float64, requires_grad=True)
    c = torch.tensor(ctx, dtype=torch.long)
    n = c.shape[0]
    sl = torch.tensor(slots)
    X = Fnn.embedding(c, P["emb"]).reshape(n, cfg.feat)
    if cfg.low_rank:
        P["A"] = torch.tensor(m.A, dtype=torch.float64, requires_grad=True)
        P["B"] = torch.tensor(m.B, dtype=torch.float64, requires_grad=True)
        X1 = torch.bmm(X[:, None, :], P["A"][sl].contiguous())[:, 0, :]
    else:
        X1 = Fnn.linear(X, P["w1"], P["b1"]) if cfg.lte else X
    Y = torch.bmm(X1[:, None, :], U[sl].contiguous())[:, 0, :]
    if cfg.low_rank:
        H = torch.bmm(Y[:, None, :], P["B"][sl].contiguous())[:, 0, :]
    else:
        H = Fnn.linear(Y, P["w2"], P["b2"]) if cfg.lte else Y
    for j in range(cfg.blocks):
        X0 = Fnn.layer_norm(H, (cfg.feat,), P[f"ln{j}.gamma"], P[f"ln{j}.beta"], eps=1e-5)
        Xf = None
        for i in range(cfg.branches):
            Xi = Fnn.linear(X0, P[f"blk{j}.w{i}"], P[f"blk{j}.b{i}"])
            Xf = Xi if Xf is None else Xf * Xi
        H = Fnn.linear(Fnn.gelu(Xf, approximate="none"), P[f"blk{j}.wo"], P[f"blk{j}.bo"]) + H
    z = Fnn.linear(H, P["wh"], P["bh"])
    p = torch.softmax(z, dim=1)
    loss = Fnn.cross_entropy(z, torch.tensor(targets, dtype=torch.long))
    return P, U, p, loss


@pytest.mark.parametrize("branches", [1, 2, 3])
def test_forward_matches_torch_fp64(branches):
    cfg = TINY.with_(branches=branches)
    m = _rand_model(cfg, 6, seed=branches)
    r = np.random.default_rng(1)
    ctx = r.integers(0, 256, size=(4, cfg.context))
    slots = np.array([5, 0, 3, 1])
    tgt = r.integers(0, 256, size=4)
    c = m.forward(ctx, slots)
    _, _, p_t, loss_t = _torch_forward(m, ctx, slots, tgt)
    np.testing.assert_allclose(c["p"], p_t.detach().numpy(), rtol=1e-12, atol=1e-15)
    assert abs(Model.loss(c, tgt) - loss_t.item()) < 1e-12


@pytest.mark.parametrize("branches", [1, 2, 3])
def test_adjoint_matches_torch_autograd(branches):
    cfg = TINY.with_(branches=branches)
    m = _rand_model(cfg, 6, seed=10 + branches)
    r = np.random.default_rng(2)
    ctx = r.integers(0, 256, size=(5, cfg.context))
    ctx[1] = ctx[0]  # repeated bytes exercise the embedding scatter-add
    slots = np.array([2, 4, 0, 5, 1])
    tgt = r.integers(0, 256, size=5)
    c = m.forward(ctx, slots)
    g, dU = m.backward(c, tgt)
    P, U, _, loss_t = _torch_forward(m, ctx, slots, tgt)
    loss_t.backward()
    for k in m.p:
        np.testing.assert_allclose(g[k], P[k].grad.numpy(), rtol=1e-9, atol=1e-13, err_msg=k)
    full = U.grad.numpy()
    np.testing.assert_allclose(dU, full[slots], rtol=1e-9, atol=1e-13)
    others = np.setdiff1d(np.arange(6), slots)
    assert not full[others].any()


def test_without_lte_matches_torch_fp64():
    cfg = TINY_NO_LTE
    m = _rand_model(cfg, 4, seed=21)
    assert not any(k in m.p for k in ("w1", "b1", "w2", "b2"))
    assert m.U.shape == (4, cfg.feat, cfg.feat)
    r = np.random.default_rng(4)
    ctx = r.integers(0, 256, size=(5, cfg.context))
    ctx = ctx[:4]
    ctx[3] = ctx[1]  # repeated bytes exercise the embedding scatter-add
    slots, tgt = np.array([3, 0, 2, 1]), r.integers(0, 256, size=4)
    c = m.forward(ctx, slots)
    g, dU = m.backward(c, tgt)
    P, U, p_t, loss_t = _torch_forward(m, ctx, slots, tgt)
    np.testing.assert_allclose(c["p"], p_t.detach().numpy(), rtol=1e-12, atol=1e-15)
    loss_t.backward()
    for k in m.p:
        np.testing.assert_allclose(g[k], P[k].grad.numpy(), rtol=1e-9, atol=1e-13, err_msg=k)
    np.testing.assert_allclose(dU, U.grad.numpy()[slots], rtol=1e-9, atol=1e-13)


def test_without_lte_is_the_lte_with_identity_maps():
    # Eqs. 14 and 16 with W1 = W2 = I and zero biases leave the features
    # unchanged, so the F x F ablation must reproduce that model exactly
    cfg_n = TINY_NO_LTE
    cfg_l = cfg_n.with_(lte=True)
    n = _rand_model(cfg_n, 3, seed=5)
    lte = Model(cfg_l, 3, shared=dict(n.p, w1=np.eye(cfg_l.feat), b1=np.zeros(cfg_l.feat),
                                      w2=np.eye(cfg_l.feat), b2=np.zeros(cfg_l.feat)),
                fdm=n.U)
    r = np.random.default_rng(6)
    ctx = r.integers(0, 256, size=(3, cfg_n.context))
    slots, tgt = np.array([2, 0, 1]), r.integers(0, 256, size=3)
    # one step: the update moves W1, W2 away from the identity afterwards
    cn, _, gn, dUn = n.step(ctx, tgt, slots)
    cl, _, gl, dUl = lte.step(ctx, tgt, slots)
    np.testing.assert_array_equal(cn["p"], cl["p"])
    np.testing.assert_array_equal(dUn, dUl)
    for k in n.p:
        np.testing.assert_array_equal(gn[k], gl[k], err_msg=k)
        np.testing.assert_array_equal(n.p[k], lte.p[k], err_msg=k)
    np.testing.assert_array_equal(n.U, lte.U)


def test_low_rank_matches_torch_fp64():
    cfg = TINY_LOW_RANK
    m = _rand_model(cfg, 5, seed=31)
    assert not any(k in m.p for k in ("w1", "b1", "w2", "b2"))
    assert m.A.shape == (5, cfg.feat, cfg.latent) and m.B.shape == (5, cfg.latent, cfg.feat)
    r = np.random.default_rng(8)
    ctx = r.integers(0, 256, size=(4, cfg.context))
    ctx[2] = ctx[0]
    slots, tgt = np.array([4, 1, 0, 2]), r.integers(0, 256, size=4)
    c = m.forward(ctx, slots)
    g, dU = m.backward(c, tgt)
    P, U, p_t, loss_t = _torch_forward(m, ctx, slots, tgt)
    np.testing.assert_allclose(c["p"], p_t.detach().numpy(), rtol=1e-12, atol=1e-15)
    loss_t.backward()
    for k in m.p:
        np.testing.assert_allclose(g[k], P[k].grad.numpy(), rtol=1e-9, atol=1e-13, err_msg=k)
    np.testing.assert_allclose(dU, U.grad.numpy()[slots], rtol=1e-9, atol=1e-13)
    for k in ("A", "B"):
        full = P[k].grad.numpy()
        np.testing.assert_allclose(g[k], full[slots], rtol=1e-9, atol=1e-13, err_msg=k)
        assert not full[3].any()  # slot 3 is not in the batch


def test_low_rank_with_identity_factors_is_without_lte():
    # with latent = F and A_s = B_s = I the three factors collapse to the
    # per-instance F x F matrix U_s of the "w/o LTE" ablation; the Adam step
    # on A_s, B_s must leave U_s's trajectory unchanged in the first step
    cfg_n = TINY_NO_LTE
    cfg_r = cfg_n.with_(lte=True, low_rank=True)
    n = _rand_model(cfg_n, 3, seed=9)
    lr = Model(cfg_r, 3, shared=dict(n.p), fdm=n.U)
    eye = np.broadcast_to(np.eye(cfg_n.feat), (3, cfg_n.feat, cfg_n.feat))
    lr.A, lr.B = eye.copy(), eye.copy()
    r = np.random.default_rng(12)
    ctx = r.integers(0, 256, size=(3, cfg_n.context))
    slots, tgt = np.array([1, 2, 0]), r.integers(0, 256, size=3)
    cn, ln_, gn, dUn = n.step(ctx, tgt, slots)
    cr, lr_, gr, dUr = lr.step(ctx, tgt, slots)
    np.testing.assert_array_equal(cn["p"], cr["p"])
    assert ln_ == lr_
    np.testing.assert_array_equal(dUn, dUr)
    for k in n.p:
        np.testing.assert_array_equal(n.p[k], lr.p[k], err_msg=k)
    np.testing.assert_array_equal(n.U, lr.U)


def test_low_rank_requires_lte():
    with pytest.raises(ValueError):
        TINY_LOW_RANK.with_(lte=False)


def test_without_lte_requires_square_fdm():
    with pytest.raises(ValueError):
        TINY_NO_LTE.with_(latent=5)


def test_adjoint_matches_central_differences():
    cfg = TINY
    m = _rand_model(cfg, 3, seed=7)
    r = np.random.default_rng(3)
    ctx = r.integers(0, 256, size=(3, cfg.context))
    ctx[2, 0] = ctx[0, 1]
    slots = np.array([1, 2, 0])
    tgt = r.integers(0, 256, size=3)
    g, dU = m.backward(m.forward(ctx, slots), tgt)

    def loss_at():
        return Model.loss(m.forward(ctx, slots), tgt)

    eps = 1e-5
    for k in m.p:
        flat = m.p[k].reshape(-1)
        gflat = g[k].reshape(-1)
        idx = r.choice(flat.size, size=min(6, flat.size), replace=False)
        if k == "emb":  # make sure touched rows are checked
            idx = np.concatenate([idx, [ctx[0, 0] * cfg.embed, ctx[0, 1] * cfg.embed + 1]])
        for i in idx:
            old = flat[i]
            flat[i] = old + eps
            lp = loss_at()
            flat[i] = old - eps
            lm = loss_at()
            flat[i] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - gflat[i]) <= 1e-7 + 1e-6 * abs(fd), (k, i, fd, gflat[i])
    for row, s in enumerate(slots):
        for (a, b) in [(0, 1), (4, 2), (3, 3)]:
            old = m.U[s, a, b]
            m.U[s, a, b] = old + eps
            lp = loss_at()
            m.U[s, a, b] = old - eps
            lm = loss_at()
            m.U[s, a, b] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - dU[row, a, b]) <= 1e-7 + 1e-6 * abs(fd)


def test_fdm_orientation_row_vector_times_matrix():
    # Eq. 15, Y = bmm(X', U) with X' a row per instance: with U_s = e_a e_b^T,
    # y_s = x'_s[a] e_b.
    cfg = TINY
    m = Model(cfg, 2)
    m.U[:] = 0.0
    m.U[1, 2, 4] = 1.0
    ctx = np.array([[1, 2, 3]])
    c = m.forward(ctx, np.array([1]))
    y = c["Y"][0]
    assert y[4] == c["X1"][0, 2]
    assert np.count_nonzero(y) == 1


def test_zero_head_gives_uniform_probabilities():
    cfg = TINY.with_(zero_head=True)
    m = Model(cfg, 2)
    c = m.forward(np.array([[9, 8, 7], [1, 1, 1]]), np.array([0, 1]))
    assert np.all(c["p"] == 1.0 / 256.0)


def test_elementwise_definitions():
    x = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(gelu(x), Fnn.gelu(torch.tensor(x)).numpy(), rtol=1e-14, atol=1e-15)
    assert gelu(np.array([0.0]))[0] == 0.0
    assert gelu_grad(np.array([0.0]))[0] == 0.5
    h = 1e-6
    np.testing.assert_allclose(gelu_grad(x), (gelu(x + h) - gelu(x - h)) / (2 * h), atol=1e-8)
    z = np.random.default_rng(0).standard_normal((3, 256))
    np.testing.assert_allclose(softmax(z), softmax(z + 123.0), rtol=1e-12)
    np.testing.assert_allclose(softmax(z).sum(1), 1.0, rtol=1e-14)
    hconst = np.full((2, 8), 3.25)
    gamma = np.arange(8.0)
    beta = np.linspace(-1, 1, 8)
    out, xhat, _ = layer_norm(hconst, gamma, beta)
    np.testing.assert_array_equal(out, np.broadcast_to(beta, (2, 8)))
    hr = np.random.default_rng(1).standard_normal((4, 8))
    ref = Fnn.layer_norm(torch.tensor(hr), (8,), torch.tensor(gamma), torch.tensor(beta), eps=1e-5)
    np.testing.assert_allclose(layer_norm(hr, gamma, beta)[0], ref.numpy(), rtol=1e-12, atol=1e-13)


def test_adam_first_step_closed_form():
    cfg = TINY.with_(lr=1e-3)
    m = Model(cfg, 2)
    before = {k: v.copy() for k, v in m.p.items()}
    U0 = m.U.copy()
    r = np.random.default_rng(4)
    g = {k: r.standard_normal(v.shape) for k, v in m.p.items()}
    dU = r.standard_normal((1,) + m.U.shape[1:])
    m.adam(g, dU, np.array([1]))
    for k in m.p:
        expect = before[k] - cfg.lr * g[k] / (np.abs(g[k]) + cfg.eps)
        np.testing.assert_allclose(m.p[k], expect, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m.U[1], U0[1] - cfg.lr * dU[0] / (np.abs(dU[0]) + cfg.eps), rtol=1e-12)
    assert np.array_equal(m.U[0], U0[0])  # inactive slot untouched


def test_adam_matches_torch_optim():
    cfg = TINY
    m = Model(cfg, 1)
    w = torch.tensor(m.p["w1"].copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=cfg.lr, betas=(cfg.beta1, cfg.beta2), eps=cfg.eps)
    r = np.random.default_rng(5)
    for _ in range(7):
        g = {k: np.zeros_like(v) for k, v in m.p.items()}
        g["w1"] = r.standard_normal(m.p["w1"].shape)
        m.adam(g, np.zeros((1,) + m.U.shape[1:]), np.array([0]))
        w.grad = torch.tensor(g["w1"])
        opt.step()
    np.testing.assert_allclose(m.p["w1"], w.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_step_lowers_loss_on_repeated_batch():
    cfg = TINY.with_(lr=1e-2)
    m = Model(cfg, 2)
    ctx = np.array([[1, 2, 3], [4, 5, 6]])
    tgt = np.array([7, 8])
    first = m.step(ctx, tgt, np.array([0, 1]))[1]
    for _ in range(20):
        last = m.step(ctx, tgt, np.array([0, 1]))[1]
    assert last < first - 0.5
    assert math.isfinite(last)
