"""The host-to-host codec (edpc_encode_host / edpc_decode_host): the input
moves to the device in time chunks through a window of a few chunks per
stream, overlapped with the steps, and payload bytes come back as soon as no
carry can change them.  It must write exactly the container that the
device-resident edpc_encode writes, and decode any container back."""

import numpy as np
import pytest

import gen
from oracle.codec import split_streams
from tests.gpu_util import banner, lib_cfg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SMALL = gen.WORKLOADS["small"].model
MID = gen.WORKLOADS["mid_bf16"].model


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


def _device_encode(E, cfg, flat, lens):
    d = torch.as_tensor(np.ascontiguousarray(flat)).to("cuda")
    c = E.edpc_encode(cfg, d, lens)
    torch.cuda.synchronize()
    return c.cpu().numpy().tobytes()


def _ragged(workload, prefix, n, cuts):
    data, lens = gen.make_streams(workload, prefix=prefix, n_streams=n)
    st = [s[:c] for s, c in zip(split_streams(data, lens), cuts)]
    return np.frombuffer(b"".join(st), dtype=np.uint8).copy(), np.array(cuts, dtype=np.int64)


@pytest.mark.parametrize("chunk", [16, 50, 64, 1000])
def test_small_fp32_ragged_matches_device_encode(E, chunk):
    # ragged streams (empty, shorter than the context, shorter than a chunk,
    # ending inside a chunk); 16-step chunks give 25 chunks, 1000 one chunk
    cuts = [400, 0, 5, 16, 17, 130, 399, 64]
    flat, lens = _ragged("small", 400, 8, cuts)
    cfg = lib_cfg(E, SMALL)
    want = _device_encode(E, cfg, flat, lens)
    got = E.edpc_encode_host(cfg, flat, lens, chunk).tobytes()
    assert got == want
    for dchunk in (16, 77):
        out = E.edpc_decode_host(got, dchunk)
        assert out.tobytes() == flat.tobytes()


def test_bf16_row_block_step_pinned_input(E):
    # the fused BF16 step over 64 ragged streams of the 1024-stream model,
    # input in pinned host memory, 3+ chunks of 96 steps
    rng = np.random.default_rng(5)
    cuts = list(rng.integers(40, 400, size=64))
    cuts[0] = 400
    flat, lens = _ragged("mid_bf16", 400, 64, cuts)
    cfg = lib_cfg(E, MID, "bf16")
    want = _device_encode(E, cfg, flat, lens)
    pinned = torch.from_numpy(flat).pin_memory()
    got = E.edpc_encode_host(cfg, pinned, lens, 96).tobytes()
    assert got == want
    out = E.edpc_decode_host(got, 128)
    assert out.tobytes() == flat.tobytes()


def test_payload_runs_of_ff_are_held_back_and_flushed(E):
    # zero head, lr 0: every byte is coded with probability 1/256, so the
    # payload is the stream itself plus one 0x00; streams of 0xFF bytes give
    # payloads that are one long run of 0xFF, which no drain may release before
    # the end (a carry could still change them), and the final drain must take
    # several rounds (longer than one drain buffer)
    cfg = lib_cfg(E, SMALL, lr=0.0, zero_head=True)
    lens = np.array([900, 300, 900, 0], dtype=np.int64)
    flat = np.concatenate([np.full(900, 0xFF, np.uint8),
                           np.arange(300, dtype=np.uint8),
                           np.where(np.arange(900) % 97 == 5, 0x00, 0xFF).astype(np.uint8)])
    want = _device_encode(E, cfg, flat, lens)
    got = E.edpc_encode_host(cfg, flat, lens, 16).tobytes()
    assert got == want
    assert E.edpc_decode_host(got, 20).tobytes() == flat.tobytes()


def test_host_codec_errors(E):
    flat, lens = _ragged("small", 100, 2, [100, 60])
    cfg = lib_cfg(E, SMALL)
    with pytest.raises(E.EdpcError) as ei:  # chunk shorter than the context
        E.edpc_encode_host(cfg, flat, lens, 8)
    assert ei.value.status == -1
    cont = E.edpc_encode_host(cfg, flat, lens, 32)
    small = np.empty(16, dtype=np.uint8)
    import ctypes
    n = ctypes.c_size_t()
    st = E.lib().edpc_encode_host(ctypes.byref(cfg), E._host_ptr(flat),
                                  lens.astype(np.uint64).ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                  2, E._host_ptr(small), small.size, ctypes.byref(n), 32, None)
    assert st == -3 and n.value == len(cont)
    bad = cont.copy()
    bad[96 + 20 * 2 + 5] ^= 0x5A  # inside stream 0's verbatim prefix: its CRC fails
    with pytest.raises(E.EdpcError) as ei:
        E.edpc_decode_host(bad.tobytes(), 32)
    assert ei.value.status == -5


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_all_streams_empty(E, precision):
    # every stream empty: the container is the header alone (96 bytes with its
    # CRC, 20 per stream), with empty payloads, through the device-resident and
    # the host-to-host codecs alike, and it decodes to nothing
    cfg = lib_cfg(E, SMALL, precision)
    lens = np.zeros(3, dtype=np.int64)
    flat = np.zeros(0, dtype=np.uint8)
    dev = E.edpc_encode(cfg, torch.empty(0, dtype=torch.uint8, device="cuda"), lens)
    torch.cuda.synchronize()
    want = dev.cpu().numpy().tobytes()
    assert len(want) == 96 + 20 * 3
    got = E.edpc_encode_host(cfg, flat, lens, 32).tobytes()
    assert got == want
    _, lens_back, hl, total = E.edpc_decode_info(want)
    assert list(lens_back) == [0, 0, 0] and hl == len(want) and total == 0
    out, _ = E.edpc_decode(dev)
    assert out.numel() == 0
    assert E.edpc_decode_host(got, 32).size == 0
