"""GPU parity of the mutual-information tool of Sec. 3.1.1 (Kraskov's
estimator, Eq. 7, and the IFR ratio, Eq. 8) against the oracle.

The neighbour distances (eps) and counts are decided in FP32 on both sides
and must agree bit for bit; the estimate, formed from those integers in
FP64, within 1e-10.  The block activations the tool reads back are compared
with the oracle's forward pass (FP32 path: 1e-5 of their scale)."""

import os

import numpy as np
import pytest

import gen
from oracle.ifr import ifr, ksg_counts, ksg_mi
from oracle.model import Model as OModel
from tests.gpu_util import banner, lib_cfg, load_oracle_state, oracle_cfg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SMALL = gen.WORKLOADS["small"].model
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ksg_handworked.txt")


@pytest.fixture(scope="module")
def E():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_18969_amd as E
    E.lib()
    return E


@pytest.fixture(autouse=True)
def _name(request):
    banner(request.node.nodeid)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to("cuda")


def _gpu(E, z, y, v):
    c = z.shape[0]
    counts = torch.empty((c, 2), dtype=torch.int32, device="cuda")
    eps = torch.empty(c, dtype=torch.float32, device="cuda")
    mi = E.edpc_mutual_info(_dev(z), _dev(y), v, counts, eps)
    torch.cuda.synchronize()
    return mi, eps.cpu().numpy(), counts.cpu().numpy()


CASES = {
    # name: (samples, dims of z, dims of y, data)
    "gauss_300x7x5": (300, 7, 5, "gauss"),
    "grid_300x3x2": (300, 3, 2, "grid"),      # ties and duplicated points
    "gauss_1000x64x64": (1000, 64, 64, "gauss"),
    "corr_777x33x40": (777, 33, 40, "corr"),
}


def _data(kind, c, dz, dy, seed):
    r = np.random.default_rng(seed)
    if kind == "grid":
        return ((r.integers(0, 8, size=(c, dz)) / 4.0).astype(np.float32),
                (r.integers(0, 8, size=(c, dy)) / 4.0).astype(np.float32))
    z = r.standard_normal((c, dz)).astype(np.float32)
    y = r.standard_normal((c, dy)).astype(np.float32)
    if kind == "corr":  # y shares most of z's first coordinates
        k = min(dz, dy)
        y[:, :k] = 0.8 * z[:, :k] + 0.6 * y[:, :k]
    return z, y


@pytest.mark.parametrize("v", [1, 3, 16])
@pytest.mark.parametrize("case", sorted(CASES))
def test_counts_bit_exact_and_estimate(E, case, v):
    c, dz, dy, kind = CASES[case]
    z, y = _data(kind, c, dz, dy, seed=len(case) + v)
    mi, eps, counts = _gpu(E, z, y, v)
    eps_o, cz_o, cy_o = ksg_counts(z, y, v)
    assert np.array_equal(eps.view(np.uint32), eps_o.view(np.uint32))
    assert np.array_equal(counts[:, 0], cz_o) and np.array_equal(counts[:, 1], cy_o)
    assert abs(mi - ksg_mi(z, y, v)) < 1e-10


def test_handworked_case(E):
    g = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                g[line[0]] = [float(x) for x in line[1:]]
    z = np.array(g["z"], dtype=np.float32)[:, None]
    y = np.array(g["y"], dtype=np.float32)[:, None]
    mi, eps, counts = _gpu(E, z, y, int(g["v"][0]))
    assert list(eps) == g["eps"]
    assert list(counts[:, 0]) == g["cz"] and list(counts[:, 1]) == g["cy"]
    assert abs(mi - 5.0 / 24.0) < 1e-12


def test_rejects_bad_sizes(E):
    z = np.zeros((4, 2), np.float32)
    for v in (0, 4, 17):
        with pytest.raises(E.EdpcError):
            E.edpc_mutual_info(_dev(z), _dev(z), v)
    with pytest.raises(E.EdpcError):
        E.edpc_mutual_info(_dev(z[:1]), _dev(z[:1]), 1)


@pytest.mark.parametrize("branches", [1, 2, 3])
def test_block_activations_and_ifr_inputs(E, branches):
    # the FP32 block inputs read back after a step equal the oracle's forward
    # pass; the block mutual information of Sec. 3.1.1 is then the estimator
    # above applied to consecutive block inputs
    model = dict(SMALL, branches=branches)
    rows, C = 256, model["context"]
    data, _ = gen.make_streams("mid_fp32", prefix=C + 9, n_streams=rows)
    st = np.frombuffer(data.tobytes(), dtype=np.uint8).reshape(rows, -1)
    om = OModel(oracle_cfg(model), rows)
    for i in range(C, C + 8):
        om.step(st[:, i - C:i].astype(np.int64), st[:, i].astype(np.int64), np.arange(rows))
    om.round_to_f32()
    m = E.Model(lib_cfg(E, model), rows, rows)
    load_oracle_state(m, om)
    ctx, tgt = st[:, 8:8 + C], st[:, 8 + C]
    c = om.forward(ctx.astype(np.int64), np.arange(rows))
    d_ctx = torch.as_tensor(np.ascontiguousarray(ctx)).to("cuda")
    d_tgt = torch.as_tensor(np.ascontiguousarray(tgt)).to("cuda")
    mis = E.block_mutual_info(m, d_ctx, d_tgt, np.arange(rows), v=3)
    F = model["context"] * model["embed"]
    oracle_h = [b["Hin"] for b in c["blocks"]] + [c["Hn"]]
    for j in range(model["blocks"] + 1):
        h = m.edpc_model_activation(j, torch.empty((rows, F), dtype=torch.float32, device="cuda"))
        torch.cuda.synchronize()
        ho = oracle_h[j]
        assert np.abs(h.cpu().numpy() - ho).max() <= 1e-5 * (np.abs(ho).max() + 1.0), j
    assert len(mis) == model["blocks"] and all(np.isfinite(mis))
    assert ifr(mis[0], mis[0]) == 1.0


def test_row_block_step_has_no_fp32_head_input(E):
    m = E.Model(lib_cfg(E, SMALL, "bf16"), 8, 8)
    ctx = torch.zeros((8, SMALL["context"]), dtype=torch.uint8, device="cuda")
    m.edpc_model_step(ctx, ctx[:, 0].contiguous(), np.arange(8))
    F = SMALL["context"] * SMALL["embed"]
    m.edpc_model_activation(0, torch.empty((8, F), dtype=torch.float32, device="cuda"))
    with pytest.raises(E.EdpcError) as ei:
        m.edpc_model_activation(SMALL["blocks"], torch.empty((8, F), dtype=torch.float32,
                                                             device="cuda"))
    assert ei.value.status == -6
