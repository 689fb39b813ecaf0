"""GPU parity: the HIP path, called through the C ABI, against the oracle.

Tolerances: FP32 path probabilities within 1e-5 absolute, BF16 within 2e-3;
integer work (coder bytes, CDF sums, round trips) bit-exact; compressed size
within 0.5 % of the oracle's.
"""

import json
import os

import numpy as np
import pytest

import gen
import oracle
from oracle.codec import split_streams
from oracle.model import Model as OModel
from oracle.model import init_fdm, init_low_rank, init_shared
from oracle.quantize import cumulative, quantize
from oracle.rangecoder import RangeEncoder
from tests.gpu_util import banner, lib_cfg, load_oracle_state, oracle_cfg, parse_container

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_sizes.json")
SMALL = gen.WORKLOADS["small"].model
MID = gen.WORKLOADS["mid_fp32"].model


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


def _dev(a, dtype=torch.uint8):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


# ---------------------------------------------------------------- coder lanes

def test_range_coder_lanes_bit_exact(E):
    r = np.random.default_rng(7)
    n_steps, n_streams = 700, 37
    z = r.standard_normal((n_steps, n_streams, 256)) * r.choice([0.3, 3.0, 12.0], size=(n_steps, n_streams, 1))
    p = np.exp(z - z.max(-1, keepdims=True))
    p /= p.sum(-1, keepdims=True)
    q = quantize(p.reshape(-1, 256)).reshape(n_steps, n_streams, 256)
    cum = cumulative(q.reshape(-1, 256)).reshape(n_steps, n_streams, 257)
    sym = np.array([[r.choice(256, p=p[t, s]) for s in range(n_streams)] for t in range(n_steps)],
                   dtype=np.uint8)
    expect = []
    for s in range(n_streams):
        e = RangeEncoder()
        for t in range(n_steps):
            x = int(sym[t, s])
            e.encode(int(cum[t, s, x]), int(q[t, s, x]))
        expect.append(e.finish())
    d_cum = _dev(cum.astype(np.uint32), torch.int32)
    d_sym = _dev(sym)
    out, lens = E.edpc_rc_encode(d_cum, d_sym, 2 * n_steps + 2)
    got = out.cpu().numpy()
    for s in range(n_streams):
        assert got[s, : lens[s]].tobytes() == expect[s]
    back = E.edpc_rc_decode(d_cum, out, lens).cpu().numpy()
    assert np.array_equal(back, sym)


# ---------------------------------------------------------------- model step

def test_initial_parameters_bit_identical(E):
    cfg = lib_cfg(E, SMALL)
    m = E.Model(cfg, 8, 8)
    ref = init_shared(oracle_cfg(SMALL))
    for k, v in ref.items():
        assert np.array_equal(m.edpc_model_read(k), v.reshape(-1)), k
    assert np.array_equal(m.edpc_model_read("U"), init_fdm(oracle_cfg(SMALL), range(8)).reshape(-1))


def _step_case(E, model, precision, rows, pos, om_steps=0, n_slots=None, prefix=None, wl="small",
               kernel_id=0, **over):
    data, lens = gen.make_streams(wl, prefix=prefix or (pos + 1), n_streams=rows)
    st = np.frombuffer(data.tobytes(), dtype=np.uint8).reshape(rows, -1)
    C = model["context"]
    ocfg = oracle_cfg(model)
    om = OModel(ocfg, n_slots or rows)
    # advance the oracle on this input, then start both sides from its state
    for i in range(C, C + om_steps):
        om.step(st[:, i - C:i].astype(np.int64), st[:, i].astype(np.int64), np.arange(rows))
    om.round_to_f32()
    cfg = lib_cfg(E, model, precision, **over)
    m = E.Model(cfg, n_slots or rows, rows, kernel_id)
    if om_steps:
        load_oracle_state(m, om)
    ctx = st[:, pos - C:pos]
    tgt = st[:, pos]
    return om, m, ctx, tgt


def _compare_step(E, om, m, ctx, tgt, p_tol, g_rtol):
    rows = ctx.shape[0]
    slots = np.arange(rows)
    c = om.forward(ctx.astype(np.int64), slots)
    loss_o = OModel.loss(c, tgt.astype(np.int64))
    g_o, dU_o = om.backward(c, tgt.astype(np.int64))
    d_ctx, d_tgt = _dev(ctx), _dev(tgt)
    probs = torch.empty((rows, 256), dtype=torch.float32, device="cuda")
    cum = torch.empty((rows, 257), dtype=torch.int32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    m.edpc_model_step(d_ctx, d_tgt, slots, probs, cum, loss,
                      flags=E.EDPC_STEP_BACKWARD | E.EDPC_STEP_KEEP_FDM_GRAD)
    torch.cuda.synchronize()
    p_g = probs.cpu().numpy()
    assert np.abs(p_g - c["p"]).max() <= p_tol
    assert abs(loss.item() - loss_o) <= 1e-5 * max(1.0, abs(loss_o)) + p_tol
    cg = cum.cpu().numpy().astype(np.int64)
    assert np.all(cg[:, 0] == 0) and np.all(cg[:, 256] == 65536)
    qg = np.diff(cg, axis=1)
    assert qg.min() >= 1
    # the GPU's CDF is the quantisation of its own FP32 probabilities
    fl = 1 + np.floor(p_g.astype(np.float32) * np.float32(65280.0)).astype(np.int64)
    am = np.argmax(qg, axis=1)
    mask = np.ones_like(qg, dtype=bool)
    mask[np.arange(rows), am] = False
    assert np.array_equal(qg[mask], fl[mask])
    # and, away from the remainder bin, within what the probability gap allows
    # under q = 1 + floor(p (2^16 - 256)): one count plus 65280 |dp|
    qo = quantize(c["p"])
    dp = np.abs(p_g.astype(np.float64) - c["p"]).max()
    assert np.abs(qg - qo)[mask].max() <= 1 + np.floor(dp * 65280.0)
    for k in om.p:
        gg = m.edpc_model_read(k, kind=E.EDPC_KIND_GRAD)
        go = g_o[k].reshape(-1)
        scale = np.abs(go).max() + 1e-30
        err = np.abs(gg - go).max() / scale
        assert err <= g_rtol, (k, err)
    dU = m.edpc_model_read("U", kind=E.EDPC_KIND_GRAD).reshape(om.U.shape)
    for r in range(rows):
        scale = np.abs(dU_o[r]).max() + 1e-30
        assert np.abs(dU[r] - dU_o[r]).max() / scale <= g_rtol
    return c, g_o, dU_o


def _compare_update(E, om, m, ctx, tgt, g_o, dU_o, tol):
    rows = ctx.shape[0]
    slots = np.arange(rows)
    d_ctx, d_tgt = _dev(ctx), _dev(tgt)
    m.edpc_model_step(d_ctx, d_tgt, slots, flags=E.EDPC_STEP_UPDATE)
    torch.cuda.synchronize()
    before = {k: v.copy() for k, v in om.p.items()}
    om.adam(g_o, dU_o, slots)
    for k in om.p:
        new_g = m.edpc_model_read(k)
        new_o = om.p[k].reshape(-1)
        # elements whose gradient stands clear of rounding noise must move
        # exactly like the oracle's; near-zero gradients may differ in sign
        g = np.abs(g_o[k].reshape(-1))
        clear = g > 1e-3 * (g.max() + 1e-30)
        d = np.abs(new_g - new_o)[clear]
        assert d.size == 0 or d.max() <= tol, (k, d.max())
        # Adam's effective step is bounded by lr (1 - beta1) / sqrt(1 - beta2)
        # (Kingma & Ba 2015, Sec. 2.1); on the first step it is lr itself
        c = om.cfg
        bound = c.lr * max(1.0, (1 - c.beta1) / np.sqrt(1 - c.beta2))
        assert np.abs(new_g - before[k].reshape(-1)).max() <= 1.01 * bound
    assert m.edpc_model_get_step() == om.tau


# positions C, C + 1, C + 24, 64 and 1024 of the 16-byte-context model
@pytest.mark.parametrize("om_steps", [0, 1, 24, 48, 1008])
def test_one_step_fp32_small(E, om_steps):
    om, m, ctx, tgt = _step_case(E, SMALL, "fp32", rows=8, pos=16 + om_steps, om_steps=om_steps,
                                 prefix=16 + om_steps + 1)
    _, g_o, dU_o = _compare_step(E, om, m, ctx, tgt, p_tol=1e-5, g_rtol=1e-4)
    _compare_update(E, om, m, ctx, tgt, g_o, dU_o, tol=1e-6)


def test_one_step_fp32_ragged_rows_and_slots(E):
    # 5 rows mapped to scattered slots of a 13-slot model: tails of every tile
    data, lens = gen.make_streams("small", prefix=40, n_streams=8)
    st = np.frombuffer(data.tobytes(), dtype=np.uint8).reshape(8, -1)
    ocfg = oracle_cfg(SMALL)
    om = OModel(ocfg, 13)
    cfg = lib_cfg(E, SMALL)
    m = E.Model(cfg, 13, 5)
    slots = np.array([12, 3, 7, 0, 9])
    ctx = st[:5, 20:36]
    tgt = st[:5, 36]
    c = om.forward(ctx.astype(np.int64), slots)
    probs = torch.empty((5, 256), dtype=torch.float32, device="cuda")
    m.edpc_model_step(_dev(ctx), _dev(tgt), slots, probs, flags=E.EDPC_STEP_BACKWARD)
    torch.cuda.synchronize()
    assert np.abs(probs.cpu().numpy() - c["p"]).max() <= 1e-5


@pytest.mark.parametrize("fused", ["1", "0"])
@pytest.mark.parametrize("om_steps", [0, 1008])
def test_one_step_bf16_small(E, fused, om_steps):
    # BF16 row-block fused step (default) and layer-by-layer products, from the
    # initial state and from the oracle's state at position 1024
    om, m, ctx, tgt = _step_case(E, SMALL, "bf16", rows=8, pos=16 + om_steps, om_steps=om_steps,
                                 prefix=16 + om_steps + 1, layerwise=fused == "0")
    _compare_step(E, om, m, ctx, tgt, p_tol=2e-3, g_rtol=3e-2)


@pytest.mark.parametrize("precision,fused", [("bf16", "1"), ("bf16", "0"), ("fp32", "0")])
def test_one_step_mid_ragged_row_blocks(E, precision, fused):
    # mid model (F = 512, L = 128, H = 256): 40 rows = two full 16-row blocks
    # and a ragged one, after 8 oracle steps
    om, m, ctx, tgt = _step_case(E, MID, precision, rows=40, pos=40, prefix=41, om_steps=8,
                                  wl="mid_bf16", layerwise=fused == "0")
    if precision == "fp32":
        _compare_step(E, om, m, ctx, tgt, p_tol=1e-5, g_rtol=1e-4)
    else:
        _compare_step(E, om, m, ctx, tgt, p_tol=2e-3, g_rtol=3e-2)


def test_mid_first_step_sampled_rows_full_batch(E):
    # full 1024-stream batch in the encoder's launch configuration; the
    # oracle checks sampled rows one by one (at the first model step a row's
    # probabilities depend only on its own context and U_s)
    rows = 1024
    C = MID["context"]
    data, lens = gen.make_streams("mid_fp32", prefix=C + 1)
    st = np.frombuffer(data.tobytes(), dtype=np.uint8).reshape(rows, -1)
    cfg = lib_cfg(E, MID)
    m = E.Model(cfg, rows, rows)
    probs = torch.empty((rows, 256), dtype=torch.float32, device="cuda")
    m.edpc_model_step(_dev(st[:, :C]), _dev(st[:, C]), np.arange(rows), probs)
    torch.cuda.synchronize()
    pg = probs.cpu().numpy()
    ocfg = oracle_cfg(MID)
    sample = np.random.default_rng(3).choice(rows, size=12, replace=False)
    shared = init_shared(ocfg)
    for s in sample:
        om = OModel(ocfg, 1, shared=shared, fdm=init_fdm(ocfg, [s]))
        c = om.forward(st[s:s + 1, :C].astype(np.int64), np.array([0]))
        assert np.abs(pg[s] - c["p"][0]).max() <= 1e-5


# ---------------------------------------------------------------- codec

def _encode(E, cfg, data, lens):
    d = _dev(data)
    cont = E.edpc_encode(cfg, d, lens)
    torch.cuda.synchronize()
    return cont


def test_identity_case_payload_is_the_stream(E):
    data, lens = gen.make_streams("small", prefix=300, n_streams=5)
    cfg = lib_cfg(E, SMALL, lr=0.0, zero_head=True)
    cont = _encode(E, cfg, data, lens).cpu().numpy().tobytes()
    _, pays = parse_container(cont)
    for s, p in zip(split_streams(data, lens), pays):
        assert p == s + b"\x00"


def test_roundtrip_ragged_empty_short(E):
    data, lens = gen.make_streams("small", prefix=160, n_streams=8)
    st = split_streams(data, lens)
    cuts = [160, 0, 5, 16, 17, 100, 1, 159]
    st = [s[:c] for s, c in zip(st, cuts)]
    flat = np.frombuffer(b"".join(st), dtype=np.uint8)
    cfg = lib_cfg(E, SMALL)
    cont = _encode(E, cfg, flat, cuts)
    out, lens_back = E.edpc_decode(cont)
    assert list(lens_back) == cuts
    assert out.cpu().numpy().tobytes() == b"".join(st)
    _, pays = parse_container(cont.cpu().numpy().tobytes())
    pay_o, _ = oracle.encode(st, oracle_cfg(SMALL))
    for s, p, po in zip(st, pays, pay_o):
        k = min(len(s), SMALL["context"])
        assert p[:k] == s[:k]
        assert len(p) == 0 if len(s) == 0 else abs(len(p) - len(po)) <= 2


def test_roundtrip_many_ragged_streams(E):
    # 600 streams of 91 different lengths (0 .. 90): the per-step count of
    # active streams takes more than one round of the schedule's 256-way search
    data, lens = gen.make_streams("mid_fp32", prefix=90, n_streams=600)
    cuts = np.random.default_rng(1031).integers(0, 91, size=600)
    st = [s[:c] for s, c in zip(split_streams(data, lens), cuts)]
    flat = np.frombuffer(b"".join(st), dtype=np.uint8)
    cont = _encode(E, lib_cfg(E, SMALL), flat, cuts)
    out, lens_back = E.edpc_decode(cont)
    assert list(lens_back) == list(cuts)
    assert out.cpu().numpy().tobytes() == b"".join(st)
    _, pays = parse_container(cont.cpu().numpy().tobytes())
    pay_o, _ = oracle.encode(st, oracle_cfg(SMALL))
    for s, p, po in zip(st, pays, pay_o):
        assert len(p) == 0 if len(s) == 0 else abs(len(p) - len(po)) <= 2


def test_small_full_roundtrip_determinism_and_size(E):
    data, lens = gen.make_streams("small")
    cfg = lib_cfg(E, SMALL)
    cont1 = _encode(E, cfg, data, lens)
    cont2 = _encode(E, cfg, data, lens)
    assert torch.equal(cont1, cont2)
    out, _ = E.edpc_decode(cont1)
    assert out.cpu().numpy().tobytes() == data.tobytes()
    _, pays = parse_container(cont1.cpu().numpy().tobytes())
    with open(GOLDEN) as f:
        gold = json.load(f)["small_full"]
    g = sum(map(len, pays))
    o = sum(gold["payload_bytes"])
    assert abs(g - o) / o <= 0.005, (g, o)


def test_decoder_rejects_corruption(E):
    data, lens = gen.make_streams("small", prefix=200, n_streams=3)
    cfg = lib_cfg(E, SMALL)
    cont = _encode(E, cfg, data, lens)
    bad = cont.clone()
    hl = 96 + 20 * 3
    bad[hl + 5] ^= 0x5A  # inside stream 0's verbatim prefix
    with pytest.raises(E.EdpcError) as ei:
        E.edpc_decode(bad)
    assert ei.value.status == -5
    hdr = cont.clone()
    hdr[20] ^= 1
    with pytest.raises(E.EdpcError) as ei:
        E.edpc_decode(hdr)
    assert ei.value.status == -5
    with pytest.raises(E.EdpcError) as ei:
        E.edpc_decode(cont[:-10])
    assert ei.value.status == -4


def test_autotuned_encode_roundtrip(E):
    data, lens = gen.make_streams("small", prefix=120, n_streams=8)
    cfg = lib_cfg(E, SMALL, autotune=True)
    cont = _encode(E, cfg, data, lens)
    kid = int.from_bytes(cont[76:84].cpu().numpy().tobytes(), "little")
    assert kid >> 48 == 7  # numerics revision
    out, _ = E.edpc_decode(cont)
    assert out.cpu().numpy().tobytes() == data.tobytes()


def test_bf16_roundtrip_and_size_vs_fp32(E):
    data, lens = gen.make_streams("small", prefix=1024)
    c32 = _encode(E, lib_cfg(E, SMALL), data, lens)
    c16 = _encode(E, lib_cfg(E, SMALL, "bf16"), data, lens)
    out, _ = E.edpc_decode(c16)
    assert out.cpu().numpy().tobytes() == data.tobytes()
    assert abs(c16.numel() - c32.numel()) / c32.numel() <= 0.005


def _without_graph_flag(cont):
    """The container with the EDPC_CFG_NO_GRAPHS bit of its configuration
    cleared (header CRC recomputed), so that payloads can be compared."""
    import struct
    import zlib
    b = bytearray(cont.cpu().numpy().tobytes())
    hl = struct.unpack_from("<I", b, 8)[0]
    flags = struct.unpack_from("<I", b, 48)[0]
    struct.pack_into("<I", b, 48, flags & ~0x20)
    struct.pack_into("<I", b, hl - 4, zlib.crc32(bytes(b[:hl - 4])))
    return bytes(b)


def test_graph_replay_matches_direct_launches(E):
    # same input through captured step windows and through direct launches:
    # identical payloads, and each container decodes
    data, lens = gen.make_streams("small", prefix=400, n_streams=8)
    lens = np.array([400, 400, 399, 250, 130, 129, 64, 17])
    st = split_streams(data, [400] * 8)
    flat = np.frombuffer(b"".join(s[:l] for s, l in zip(st, lens)), dtype=np.uint8)
    direct = _encode(E, lib_cfg(E, SMALL, graphs=False), flat, lens)
    graph = _encode(E, lib_cfg(E, SMALL), flat, lens)
    graph2 = _encode(E, lib_cfg(E, SMALL), flat, lens)
    assert torch.equal(graph, graph2)
    assert _without_graph_flag(direct) == graph.cpu().numpy().tobytes()
    for cont in (direct, graph):
        out, _ = E.edpc_decode(cont)
        assert out.cpu().numpy().tobytes() == flat.tobytes()


def test_fused_and_layerwise_containers_decode(E):
    # the container records which BF16 step encoded it (bit 47 of the kernel
    # configuration id); the decoder follows the container
    data, lens = gen.make_streams("small", prefix=300, n_streams=8)
    conts = {}
    for fused in ("1", "0"):
        conts[fused] = _encode(E, lib_cfg(E, SMALL, "bf16", layerwise=fused == "0"), data, lens)
        kid = int.from_bytes(conts[fused][76:84].cpu().numpy().tobytes(), "little")
        assert (kid >> 47) & 1 == int(fused)
    for fused, cont in conts.items():
        out, _ = E.edpc_decode(cont)
        assert out.cpu().numpy().tobytes() == data.tobytes()
    assert abs(conts["1"].numel() - conts["0"].numel()) / conts["0"].numel() <= 0.005


# smallest shapes the configuration accepts, and the widest feature vector
# (context 256 x embed 64); BF16 with shapes outside the row-block kernels
# runs the layer-by-layer products
EXTREMES = {
    "min": dict(SMALL, context=4, embed=16, latent=16, blocks=1, hidden=16),
    "widest": dict(SMALL, context=256, embed=64, latent=256, blocks=1, hidden=16),
    # a context that is not a multiple of 8: the embedding gradient's 8-pair
    # operand groups straddle rows
    "ctx12": dict(SMALL, context=12, embed=32, latent=32, blocks=1, hidden=16),
}


@pytest.mark.parametrize("shape", sorted(EXTREMES))
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_extreme_shapes_one_step_and_roundtrip(E, shape, precision):
    model = EXTREMES[shape]
    C = model["context"]
    om, m, ctx, tgt = _step_case(E, model, precision, rows=3, pos=C, prefix=C + 1)
    if precision == "fp32":
        _compare_step(E, om, m, ctx, tgt, p_tol=1e-5, g_rtol=1e-4)
    else:
        _compare_step(E, om, m, ctx, tgt, p_tol=2e-3, g_rtol=3e-2)
    del m
    data, _ = gen.make_streams("small", prefix=C + 40, n_streams=3)
    lens = np.array([C + 40, C + 1, 0])
    st = split_streams(data, [C + 40] * 3)
    flat = np.frombuffer(b"".join(s[:l] for s, l in zip(st, lens)), dtype=np.uint8)
    cont = _encode(E, lib_cfg(E, model, precision), flat, lens)
    out, _ = E.edpc_decode(cont)
    assert out.cpu().numpy().tobytes() == flat.tobytes()


LN_FOLD = 1 << 46  # kernel configuration bit: LayerNorm adjoint with its column sums


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_layernorm_adjoint_with_column_sums(E, precision):
    # the layer-by-layer LayerNorm adjoint that also forms its block's beta,
    # gamma and output-bias column sums over groups of 16 rows (the default
    # from 4096 rows), forced on 40 rows: two full groups and a ragged one
    cfg = lib_cfg(E, MID, precision, layerwise=True)
    kid = E.Model(cfg, 40, 40).edpc_model_kernel_id()
    assert not (kid >> 47) & 1 and not (kid >> 46) & 1
    assert (E.Model(cfg, 4096, 4096).edpc_model_kernel_id() >> 46) & 1
    om, m, ctx, tgt = _step_case(E, MID, precision, rows=40, pos=MID["context"] + 4, om_steps=4,
                                 prefix=MID["context"] + 5, wl="mid_bf16", kernel_id=kid | LN_FOLD,
                                 layerwise=True)
    assert m.edpc_model_kernel_id() == kid | LN_FOLD
    if precision == "fp32":
        _, g_o, dU_o = _compare_step(E, om, m, ctx, tgt, p_tol=1e-5, g_rtol=1e-4)
        _compare_update(E, om, m, ctx, tgt, g_o, dU_o, tol=1e-6)
    else:
        _compare_step(E, om, m, ctx, tgt, p_tol=2e-3, g_rtol=3e-2)


@pytest.mark.parametrize("branches", [1, 3])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_branch_count_variants(E, branches, precision):
    # refinement blocks with one or three branches (Eq. 11 with k = 1, 3; the
    # paper's three-branch ablation); BF16 runs the layer-by-layer products
    model = dict(SMALL, branches=branches)
    C = model["context"]
    om, m, ctx, tgt = _step_case(E, model, precision, rows=8, pos=C + 8, om_steps=8, prefix=C + 9)
    if precision == "fp32":
        _, g_o, dU_o = _compare_step(E, om, m, ctx, tgt, p_tol=1e-5, g_rtol=1e-4)
        _compare_update(E, om, m, ctx, tgt, g_o, dU_o, tol=1e-6)
    else:
        _compare_step(E, om, m, ctx, tgt, p_tol=2e-3, g_rtol=3e-2)
    del m
    data, lens = gen.make_streams("small", prefix=200, n_streams=4)
    cont = _encode(E, lib_cfg(E, model, precision), data, lens)
    out, _ = E.edpc_decode(cont)
    assert out.cpu().numpy().tobytes() == data.tobytes()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_without_lte_variant(E, precision):
    # the "w/o LTE" ablation of Table 4: a per-stream F x F FDM on the embedded
    # features (F = 256), no W1 / W2; BF16 runs the layer-by-layer products
    model = dict(SMALL, latent=256, lte=False)
    C = model["context"]
    m0 = E.Model(lib_cfg(E, model, precision), 3, 3)
    for k, v in init_shared(oracle_cfg(model)).items():
        assert np.array_equal(m0.edpc_model_read(k), v.reshape(-1)), k
    assert np.array_equal(m0.edpc_model_read("U"), init_fdm(oracle_cfg(model), range(3)).reshape(-1))
    del m0
    om, m, ctx, tgt = _step_case(E, model, precision, rows=8, pos=C + 8, om_steps=8, prefix=C + 9)
    assert om.U.shape[1:] == (256, 256)
    if precision == "fp32":
        _, g_o, dU_o = _compare_step(E, om, m, ctx, tgt, p_tol=1e-5, g_rtol=1e-4)
        _compare_update(E, om, m, ctx, tgt, g_o, dU_o, tol=1e-6)
    else:
        _compare_step(E, om, m, ctx, tgt, p_tol=2e-3, g_rtol=3e-2)
    del m
    data, lens = gen.make_streams("small", prefix=200, n_streams=4)
    cont = _encode(E, lib_cfg(E, model, precision), data, lens)
    out, _ = E.edpc_decode(cont)
    assert out.cpu().numpy().tobytes() == data.tobytes()
    _, pays = parse_container(cont.cpu().numpy().tobytes())
    pay_o, _ = oracle.encode(split_streams(data, lens), oracle_cfg(model))
    for p, po in zip(pays, pay_o):
        assert abs(len(p) - len(po)) <= 2


def test_without_lte_rejects_non_square_fdm(E):
    with pytest.raises(Exception):
        E.edpc_config_validate(lib_cfg(E, dict(SMALL, lte=False)))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_low_rank_variant(E, precision):
    # the "low-rank factorization" ablation of Table 4: per-stream factors
    # x' = x A_s, y = x' U_s, x'' = y B_s, no shared W1 / W2 or biases
    model = dict(SMALL, low_rank=True)
    C = model["context"]
    ocfg = oracle_cfg(model)
    m0 = E.Model(lib_cfg(E, model, precision), 3, 3)
    for k, v in init_shared(ocfg).items():
        assert np.array_equal(m0.edpc_model_read(k), v.reshape(-1)), k
    A0, B0 = init_low_rank(ocfg, range(3))
    assert np.array_equal(m0.edpc_model_read("A"), A0.reshape(-1))
    assert np.array_equal(m0.edpc_model_read("B"), B0.reshape(-1))
    del m0
    om, m, ctx, tgt = _step_case(E, model, precision, rows=8, pos=C + 8, om_steps=8, prefix=C + 9)
    assert om.A.shape[1:] == (256, 64) and om.B.shape[1:] == (64, 256)
    if precision == "fp32":
        _, g_o, dU_o = _compare_step(E, om, m, ctx, tgt, p_tol=1e-5, g_rtol=1e-4)
        _compare_update(E, om, m, ctx, tgt, g_o, dU_o, tol=1e-6)
        # the factors moved like the oracle's wherever their gradient stands
        # clear of rounding noise
        for n in ("A", "B"):
            new_g = m.edpc_model_read(n)
            new_o = getattr(om, n).reshape(-1)
            g = np.abs(g_o[n]).reshape(-1)
            clear = g > 1e-3 * (g.max() + 1e-30)
            assert clear.sum() > 0.5 * g.size, n
            assert np.abs(new_g - new_o)[clear].max() <= 1e-6, n
            mo = getattr(om, "m" + n).reshape(-1)
            mg = m.edpc_model_read(n, kind=E.EDPC_KIND_ADAM_M)
            assert np.abs(mg - mo).max() <= 1e-4 * (np.abs(mo).max() + 1e-30), n
    else:
        _compare_step(E, om, m, ctx, tgt, p_tol=2e-3, g_rtol=3e-2)
    del m
    data, lens = gen.make_streams("small", prefix=200, n_streams=4)
    cont = _encode(E, lib_cfg(E, model, precision), data, lens)
    out, _ = E.edpc_decode(cont)
    assert out.cpu().numpy().tobytes() == data.tobytes()
    _, pays = parse_container(cont.cpu().numpy().tobytes())
    pay_o, _ = oracle.encode(split_streams(data, lens), ocfg)
    for p, po in zip(pays, pay_o):
        assert abs(len(p) - len(po)) <= 2
