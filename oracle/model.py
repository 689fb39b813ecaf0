"""FP64 probability model, cross-entropy adjoint and Adam (oracle side).

Test infrastructure only.  Follows the paper's equations in their order:

* byte embedding of the t previous bytes, concatenated oldest first, giving
  the feature vector of width F = t * E (the embedding is not spelled out in
  the paper; this is the reading that makes F = C * E);
* Latent Transformation Engine (Sec. 3.2): down-projection X' = W1 X + b1
  (Eq. 14), per-instance Feature Distribution Matrix Y = bmm(X', U)
  (Eq. 15, row vector times matrix, U of shape [b, F', F']), up-projection
  X'' = W2 Y + b2 (Eq. 16); no activation inside the LTE;
* the "w/o LTE" ablation (Table 4, Sec. 4.4.1), ``lte=False``: no W1, b1, W2,
  b2; the per-instance FDM acts on the F-wide features directly, Y = bmm(X, U)
  with U of shape [b, F, F], and Y feeds the first block (latent must be F);
* the "low-rank factorization" ablation (Table 4), ``low_rank=True``: the
  per-instance F x F matrix of "w/o LTE" is replaced by three per-instance
  factors, X' = X A_s (A_s: [F, F']), Y = X' U_s, X'' = Y B_s (B_s: [F', F]),
  with no shared W1, b1, W2, b2 and no biases; A_s and B_s are updated only on
  steps where their stream is in the batch, like U_s.  Reading: the shared LTE
  is made per instance and loses its biases, which the parameter count of
  Table 4 fixes (4096 * (2 * 256 * 64 + 64 * 64) more than the shared part,
  with per-instance biases it would be 1.3e6 more);
* ``blocks`` Multi-path Byte Refinement Blocks (Sec. 3.1.2, Eqs. 9-13):
  X0 = LN(X); X_i = Linear_i(X0), i = 1..k; X_fused = X_1 * ... * X_k;
  X_ff = GeLU(X_fused) (exact erf form); X_out = Linear_out(X_ff) + X;
  LayerNorm with biased variance, eps 1e-5, affine gamma/beta;
* head Linear(F -> 256) and softmax: Pr(i) = P(x_i | x_{i-t} .. x_{i-1})
  (Eq. 1);
* loss = mean over the rows of CrossEntropy(Pr(i), x_i) (Eq. 2, natural log),
  gradients by a hand-derived adjoint (backpropagation, Sec. 2.1);
* Adam (Kingma & Ba 2015; lr 1e-3, Sec. 4.1) with beta1 0.9, beta2 0.999,
  eps 1e-8, bias correction, no weight decay.  The FDM slice U_s of a stream
  is updated only on steps where that stream is in the batch.

Parity pins (tests/test_oracle_model.py): forward against PyTorch's own FP64
modules (layer_norm, gelu, softmax, linear) on random weights; special cases
(one-hot FDM, constant-row LayerNorm, zero head); the adjoint against central
finite differences and against torch.autograd in FP64; Adam against the
first-step closed form and against torch.optim.Adam.  The "w/o LTE" ablation:
forward and adjoint against the same PyTorch modules, one step against the LTE
model with identity W1, W2 and zero biases, and its parameter count against
the difference printed in Table 4.  The low-rank ablation: forward and
adjoint against torch.autograd in FP64, one step against the "w/o LTE" model
with identity factors (latent = F), and its parameter count against Table 4.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np
from scipy.special import erf

from . import rng

LN_EPS = 1e-5
V = 256  # alphabet size

# Tensor ids used by the counter-based initialiser.
TID_EMB, TID_W1, TID_B1, TID_U, TID_W2, TID_B2, TID_WH, TID_BH = 1, 2, 3, 4, 5, 6, 7, 8
TID_LR_A, TID_LR_B = 9, 10  # per-instance factors of the low-rank ablation


def tid_branch_w(j, i):
    return 16 + 16 * j + 2 * i


def tid_branch_b(j, i):
    return 17 + 16 * j + 2 * i


def tid_out_w(j):
    return 16 + 16 * j + 14


def tid_out_b(j):
    return 16 + 16 * j + 15


@dataclass(frozen=True)
class Config:
    context: int = 16
    embed: int = 16
    latent: int = 64
    blocks: int = 2
    hidden: int = 128
    branches: int = 2
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    seed: int = 0
    cdf_bits: int = 16
    zero_head: bool = False  # test special case: head weights and bias start at 0
    lte: bool = True  # False: the "w/o LTE" ablation (Table 4), latent == feat
    low_rank: bool = False  # True: the "low-rank factorization" ablation (Table 4)

    def __post_init__(self):
        if not self.lte and self.latent != self.feat:
            raise ValueError("without the LTE the FDM is F x F: latent must equal feat")
        if self.low_rank and not self.lte:
            raise ValueError("the low-rank ablation factorises the LTE: lte must be set")

    @property
    def feat(self) -> int:
        return self.context * self.embed

    @classmethod
    def from_dict(cls, d: dict) -> "Config":
        keys = {f for f in cls.__dataclass_fields__}
        return cls(**{k: v for k, v in d.items() if k in keys})

    def with_(self, **kw) -> "Config":
        return replace(self, **kw)


def param_specs(cfg: Config):
    """(name, shape, tensor_id or None, bound or constant) in storage order."""
    F, E, L, H = cfg.feat, cfg.embed, cfg.latent, cfg.hidden
    specs = [("emb", (V, E), TID_EMB, math.sqrt(3.0))]
    if cfg.lte and not cfg.low_rank:
        specs += [
            ("w1", (L, F), TID_W1, 1.0 / math.sqrt(F)),
            ("b1", (L,), TID_B1, 1.0 / math.sqrt(F)),
            ("w2", (F, L), TID_W2, 1.0 / math.sqrt(L)),
            ("b2", (F,), TID_B2, 1.0 / math.sqrt(L)),
        ]
    for j in range(cfg.blocks):
        specs.append((f"ln{j}.gamma", (F,), None, 1.0))
        specs.append((f"ln{j}.beta", (F,), None, 0.0))
        for i in range(cfg.branches):
            specs.append((f"blk{j}.w{i}", (H, F), tid_branch_w(j, i), 1.0 / math.sqrt(F)))
            specs.append((f"blk{j}.b{i}", (H,), tid_branch_b(j, i), 1.0 / math.sqrt(F)))
        specs.append((f"blk{j}.wo", (F, H), tid_out_w(j), 1.0 / math.sqrt(H)))
        specs.append((f"blk{j}.bo", (F,), tid_out_b(j), 1.0 / math.sqrt(H)))
    hb = 0.0 if cfg.zero_head else 1.0 / math.sqrt(F)
    specs.append(("wh", (V, F), None if cfg.zero_head else TID_WH, hb))
    specs.append(("bh", (V,), None if cfg.zero_head else TID_BH, hb))
    return specs


def init_shared(cfg: Config) -> dict:
    out = {}
    for name, shape, tid, bound in param_specs(cfg):
        if tid is None:
            out[name] = np.full(shape, bound, dtype=np.float32)
        else:
            out[name] = rng.init_tensor(cfg.seed, tid, shape, bound)
    return out


def init_fdm(cfg: Config, slots) -> np.ndarray:
    """FP32 U_s for the given stream slots: [len(slots), L, L], U(+-1/sqrt(L))."""
    L = cfg.latent
    bound = 1.0 / math.sqrt(L)
    out = np.empty((len(slots), L, L), dtype=np.float32)
    for r, s in enumerate(slots):
        out[r] = rng.init_tensor(cfg.seed, TID_U, (L, L), bound, start=int(s) * L * L)
    return out


def init_low_rank(cfg: Config, slots):
    """FP32 per-instance factors (A_s [F, L], U(+-1/sqrt(F)); B_s [L, F],
    U(+-1/sqrt(L))) of the low-rank ablation, slot s drawing the counter range
    that starts at s times the factor's size (the layout of U)."""
    F, L = cfg.feat, cfg.latent
    A = np.empty((len(slots), F, L), dtype=np.float32)
    B = np.empty((len(slots), L, F), dtype=np.float32)
    for r, s in enumerate(slots):
        A[r] = rng.init_tensor(cfg.seed, TID_LR_A, (F, L), 1.0 / math.sqrt(F), start=int(s) * F * L)
        B[r] = rng.init_tensor(cfg.seed, TID_LR_B, (L, F), 1.0 / math.sqrt(L), start=int(s) * L * F)
    return A, B


# --------------------------------------------------------------------------
# elementwise pieces
# --------------------------------------------------------------------------

def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    cdf = 0.5 * (1.0 + erf(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def softmax(z):
    zm = z - z.max(axis=1, keepdims=True)
    e = np.exp(zm)
    return e / e.sum(axis=1, keepdims=True)


def layer_norm(h, gamma, beta):
    mu = h.mean(axis=1, keepdims=True)
    var = ((h - mu) ** 2).mean(axis=1, keepdims=True)
    rstd = 1.0 / np.sqrt(var + LN_EPS)
    xhat = (h - mu) * rstd
    return xhat * gamma + beta, xhat, rstd


# --------------------------------------------------------------------------
# the model
# --------------------------------------------------------------------------

class Model:
    """Shared parameters + per-stream FDM slices + Adam state, all FP64.

    ``slots`` is the number of FDM slices (one per stream).
    """

    def __init__(self, cfg: Config, n_slots: int, shared: dict | None = None,
                 fdm: np.ndarray | None = None):
        self.cfg = cfg
        self.n_slots = n_slots
        sh = init_shared(cfg) if shared is None else shared
        self.p = {k: np.asarray(v, dtype=np.float64).copy() for k, v in sh.items()}
        U = init_fdm(cfg, range(n_slots)) if fdm is None else fdm
        self.U = np.asarray(U, dtype=np.float64).copy()
        self.m = {k: np.zeros_like(v) for k, v in self.p.items()}
        self.v = {k: np.zeros_like(v) for k, v in self.p.items()}
        self.mU = np.zeros_like(self.U)
        self.vU = np.zeros_like(self.U)
        if cfg.low_rank:
            A, B = init_low_rank(cfg, range(n_slots))
            self.A = np.asarray(A, dtype=np.float64)
            self.B = np.asarray(B, dtype=np.float64)
            self.mA, self.vA = np.zeros_like(self.A), np.zeros_like(self.A)
            self.mB, self.vB = np.zeros_like(self.B), np.zeros_like(self.B)
        self.tau = 0

    # ---- forward: Eq. 1 via Eqs. 14-16 and 9-13 ------------------------
    def forward(self, ctx: np.ndarray, slots: np.ndarray) -> dict:
        cfg, P = self.cfg, self.p
        n = ctx.shape[0]
        c = {"ctx": ctx, "slots": np.asarray(slots)}
        X = P["emb"][ctx].reshape(n, cfg.feat)                       # embed, oldest first
        if cfg.low_rank:
            X1 = np.matmul(X[:, None, :], self.A[c["slots"]])[:, 0, :]   # X A_s
        else:
            X1 = X @ P["w1"].T + P["b1"] if cfg.lte else X           # Eq. 14
        Us = self.U[c["slots"]]
        Y = np.matmul(X1[:, None, :], Us)[:, 0, :]                   # Eq. 15
        if cfg.low_rank:
            H = np.matmul(Y[:, None, :], self.B[c["slots"]])[:, 0, :]    # Y B_s
        else:
            H = Y @ P["w2"].T + P["b2"] if cfg.lte else Y            # Eq. 16
        c.update(X=X, X1=X1, Y=Y, H0=H)
        blocks = []
        for j in range(cfg.blocks):
            X0, xhat, rstd = layer_norm(H, P[f"ln{j}.gamma"], P[f"ln{j}.beta"])   # Eq. 9
            Xi = [X0 @ P[f"blk{j}.w{i}"].T + P[f"blk{j}.b{i}"]
                  for i in range(cfg.branches)]                      # Eq. 10
            Xf = Xi[0].copy()
            for i in range(1, cfg.branches):
                Xf = Xf * Xi[i]                                      # Eq. 11
            Xff = gelu(Xf)                                           # Eq. 12
            Hn = Xff @ P[f"blk{j}.wo"].T + P[f"blk{j}.bo"] + H       # Eq. 13
            blocks.append(dict(Hin=H, X0=X0, xhat=xhat, rstd=rstd, Xi=Xi, Xf=Xf, Xff=Xff))
            H = Hn
        z = H @ P["wh"].T + P["bh"]
        c.update(blocks=blocks, Hn=H, z=z, p=softmax(z))
        return c

    @staticmethod
    def loss(c: dict, target: np.ndarray) -> float:
        """Mean cross entropy (Eq. 2), natural log."""
        p = c["p"]
        return float(-np.log(p[np.arange(len(target)), target]).mean())

    # ---- adjoint of the mean cross entropy --------------------------------
    def backward(self, c: dict, target: np.ndarray):
        cfg, P = self.cfg, self.p
        n = len(target)
        g = {}
        dz = c["p"].copy()
        dz[np.arange(n), target] -= 1.0
        dz /= n
        g["wh"] = dz.T @ c["Hn"]
        g["bh"] = dz.sum(0)
        dH = dz @ P["wh"]
        for j in reversed(range(cfg.blocks)):
            b = c["blocks"][j]
            g[f"blk{j}.wo"] = dH.T @ b["Xff"]
            g[f"blk{j}.bo"] = dH.sum(0)
            dXff = dH @ P[f"blk{j}.wo"]
            dXf = dXff * gelu_grad(b["Xf"])
            dX0 = np.zeros_like(b["X0"])
            for i in range(cfg.branches):
                dXi = dXf.copy()
                for k2 in range(cfg.branches):
                    if k2 != i:
                        dXi = dXi * b["Xi"][k2]
                g[f"blk{j}.w{i}"] = dXi.T @ b["X0"]
                g[f"blk{j}.b{i}"] = dXi.sum(0)
                dX0 += dXi @ P[f"blk{j}.w{i}"]
            g[f"ln{j}.gamma"] = (dX0 * b["xhat"]).sum(0)
            g[f"ln{j}.beta"] = dX0.sum(0)
            dxhat = dX0 * P[f"ln{j}.gamma"]
            dln = b["rstd"] * (dxhat - dxhat.mean(1, keepdims=True)
                               - b["xhat"] * (dxhat * b["xhat"]).mean(1, keepdims=True))
            dH = dH + dln                                           # residual path of Eq. 13
        if cfg.low_rank:
            g["B"] = c["Y"][:, :, None] * dH[:, None, :]            # dB_s = y_s (x) dx''_s
            dY = np.matmul(self.B[c["slots"]], dH[:, :, None])[:, :, 0]
        elif cfg.lte:
            g["w2"] = dH.T @ c["Y"]
            g["b2"] = dH.sum(0)
            dY = dH @ P["w2"]
        else:
            dY = dH
        Us = self.U[c["slots"]]
        dU = c["X1"][:, :, None] * dY[:, None, :]                    # dU_s = x'_s (x) dy_s
        dX1 = np.matmul(Us, dY[:, :, None])[:, :, 0]                  # U_s dy_s
        if cfg.low_rank:
            g["A"] = c["X"][:, :, None] * dX1[:, None, :]           # dA_s = x_s (x) dx'_s
            dX1 = np.matmul(self.A[c["slots"]], dX1[:, :, None])[:, :, 0]
        elif cfg.lte:
            g["w1"] = dX1.T @ c["X"]
            g["b1"] = dX1.sum(0)
            dX1 = dX1 @ P["w1"]
        dX = dX1.reshape(n, cfg.context, cfg.embed)
        dEmb = np.zeros_like(P["emb"])
        np.add.at(dEmb, c["ctx"], dX)
        g["emb"] = dEmb
        return g, dU

    # ---- Adam --------------------------------------------------------------
    def adam(self, g: dict, dU: np.ndarray, slots: np.ndarray):
        cfg = self.cfg
        self.tau += 1
        b1, b2 = cfg.beta1, cfg.beta2
        bc1 = 1.0 - b1 ** self.tau
        bc2 = 1.0 - b2 ** self.tau

        def upd(theta, m, v, grad):
            m *= b1
            m += (1.0 - b1) * grad
            v *= b2
            v += (1.0 - b2) * grad * grad
            theta -= cfg.lr * (m / bc1) / (np.sqrt(v / bc2) + cfg.eps)

        for k in self.p:
            upd(self.p[k], self.m[k], self.v[k], g[k])
        slots = np.asarray(slots)
        Us, mU, vU = self.U[slots], self.mU[slots], self.vU[slots]
        upd(Us, mU, vU, dU)
        self.U[slots], self.mU[slots], self.vU[slots] = Us, mU, vU
        if cfg.low_rank:
            for name, key in (("A", "A"), ("B", "B")):
                th, m, v = (getattr(self, n)[slots] for n in (name, "m" + name, "v" + name))
                upd(th, m, v, g[key])
                getattr(self, name)[slots] = th
                getattr(self, "m" + name)[slots] = m
                getattr(self, "v" + name)[slots] = v

    def step(self, ctx, target, slots, update: bool = True):
        """forward -> loss -> adjoint -> (Adam); returns (cache, loss, grads, dU)."""
        c = self.forward(ctx, slots)
        lval = self.loss(c, target)
        g, dU = self.backward(c, target)
        if update:
            self.adam(g, dU, slots)
        return c, lval, g, dU

    # ---- state exchange ------------------------------------------------------
    def state_f32(self) -> dict:
        """Every tensor rounded to FP32 (for loading into another implementation)."""
        out = {f"param.{k}": v.astype(np.float32) for k, v in self.p.items()}
        out.update({f"m.{k}": v.astype(np.float32) for k, v in self.m.items()})
        out.update({f"v.{k}": v.astype(np.float32) for k, v in self.v.items()})
        out["param.U"] = self.U.astype(np.float32)
        out["m.U"] = self.mU.astype(np.float32)
        out["v.U"] = self.vU.astype(np.float32)
        if self.cfg.low_rank:
            for n in ("A", "B"):
                out[f"param.{n}"] = getattr(self, n).astype(np.float32)
                out[f"m.{n}"] = getattr(self, "m" + n).astype(np.float32)
                out[f"v.{n}"] = getattr(self, "v" + n).astype(np.float32)
        return out

    def round_to_f32(self):
        """Round every tensor to FP32 in place (values stay FP64 arrays)."""
        for d in (self.p, self.m, self.v):
            for k in d:
                d[k] = d[k].astype(np.float32).astype(np.float64)
        names = ["U", "mU", "vU"]
        if self.cfg.low_rank:
            names += ["A", "mA", "vA", "B", "mB", "vB"]
        for name in names:
            setattr(self, name, getattr(self, name).astype(np.float32).astype(np.float64))

    def n_shared_params(self) -> int:
        return int(sum(v.size for v in self.p.values()))
