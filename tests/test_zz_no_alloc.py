"""The allocation-free coder entry point against the allocating one.

edpc_rc_encode_noalloc keeps the per-stream payload lengths in a fixed
device array instead of a temporary allocation; everything else is the same
coder.  Two calls in a row (the second smaller, so that stale entries of the
first would show) must give the payload bytes and lengths of
edpc_rc_encode bit for bit, and sizes past the fixed array are refused
before any device work.
"""

import ctypes

import numpy as np
import pytest

from oracle.quantize import cumulative, quantize
from tests.gpu_util import banner

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_18969_amd as E
    E.lib()
    return E


def _tables(seed, n_steps, n_streams):
    r = np.random.default_rng(seed)
    z = r.standard_normal((n_steps, n_streams, 256)) * r.choice([0.3, 3.0, 12.0],
                                                                 size=(n_steps, n_streams, 1))
    p = np.exp(z - z.max(-1, keepdims=True))
    p /= p.sum(-1, keepdims=True)
    q = quantize(p.reshape(-1, 256))
    cum = cumulative(q).reshape(n_steps, n_streams, 257).astype(np.uint32)
    sym = r.integers(0, 256, size=(n_steps, n_streams)).astype(np.uint8)
    # symbols drawn from their tables where the tables are peaked
    top = np.argmax(q.reshape(n_steps, n_streams, 256), axis=-1).astype(np.uint8)
    pick = r.random((n_steps, n_streams)) < 0.6
    sym[pick] = top[pick]
    return cum, sym


def test_noalloc_matches_allocating_entry_twice(E):
    for call, (n_steps, n_streams) in enumerate([(120, 600), (60, 37)]):
        banner(f"rc_encode_noalloc call {call}: {n_steps} steps x {n_streams} streams")
        cum, sym = _tables(100 + call, n_steps, n_streams)
        d_cum = torch.as_tensor(cum.view(np.int32)).to("cuda")
        d_sym = torch.as_tensor(sym).to("cuda")
        cap = 2 * n_steps + 2
        ref, ref_lens = E.edpc_rc_encode(d_cum, d_sym, cap)
        out = torch.zeros((n_streams, cap), dtype=torch.uint8, device="cuda")
        lens = E.edpc_rc_encode_noalloc(d_cum, d_sym, out)
        torch.cuda.synchronize()
        assert np.array_equal(lens, ref_lens)
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        for s in range(n_streams):
            assert a[s, :lens[s]].tobytes() == b[s, :lens[s]].tobytes(), s
        back = E.edpc_rc_decode(d_cum, out, lens).cpu().numpy()
        assert np.array_equal(back, sym)


def test_noalloc_refuses_more_streams_than_its_array(E):
    t = torch.zeros(1024, dtype=torch.uint8, device="cuda")
    p = ctypes.c_void_p(t.data_ptr())
    lens = np.zeros(4, dtype=np.uint32)
    st = E.lib().edpc_rc_encode_noalloc(p, p, 1, E.EDPC_RC_NOALLOC_MAX_STREAMS + 1, p, 4,
                                        lens.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                        None)
    assert st == -1
    assert b"EDPC_RC_NOALLOC_MAX_STREAMS" in E.lib().edpc_last_error()
