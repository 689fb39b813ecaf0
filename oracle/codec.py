"""The autoregressive compression loop over many streams (oracle side).

Test infrastructure only.  Algorithm 1 of the paper, for b streams advanced
in lockstep with one shared model (the batch dimension b of Secs. 3.1-3.2):

* at step i the batch is the set A_i of streams with i < len_s, in stream
  order;
* steps i < t: every byte is coded "with equal probability" (freq 256 of
  2**16), with no model call and no update;
* steps i >= t: Pr(i) from the t previous bytes of each stream (Eq. 1),
  quantised to an integer CDF, the byte coded (or decoded, then appended to
  the stream's history), the mean cross entropy over A_i (Eq. 2)
  back-propagated and one Adam step taken on the shared weights and on U_s
  for s in A_i.

The decoder replays the same loop; its targets are the bytes it has just
decoded.  Returns per-stream payloads; the container format around them is
the library's business and not modelled here.
"""

from __future__ import annotations

import numpy as np

from .model import Config, Model
from .quantize import cumulative, quantize
from .rangecoder import RangeDecoder, RangeEncoder


def _run(cfg: Config, lens, streams=None, payloads=None, hook=None, max_steps=None):
    lens = [int(x) for x in lens]
    nst = len(lens)
    decoding = payloads is not None
    model = Model(cfg, nst)
    if decoding:
        coders = [RangeDecoder(payloads[s], cfg.cdf_bits) for s in range(nst)]
        hist = [np.zeros(lens[s], dtype=np.int64) for s in range(nst)]
    else:
        coders = [RangeEncoder(cfg.cdf_bits) for _ in range(nst)]
        hist = [np.frombuffer(bytes(streams[s]), dtype=np.uint8).astype(np.int64)
                for s in range(nst)]
    C = cfg.context
    uni = 1 << (cfg.cdf_bits - 8)
    maxlen = max(lens) if lens else 0
    if max_steps is not None:
        maxlen = min(maxlen, max_steps)
    ideal_bits = np.zeros(nst)
    losses = []
    for i in range(maxlen):
        act = np.array([s for s in range(nst) if lens[s] > i], dtype=np.int64)
        if i < C:
            for s in act:
                if decoding:
                    x = coders[s].decode([uni * v for v in range(257)])
                    hist[s][i] = x
                else:
                    coders[s].encode(uni * int(hist[s][i]), uni)
                ideal_bits[s] += 8.0
            continue
        ctx = np.stack([hist[s][i - C:i] for s in act])
        cache = model.forward(ctx, act)
        q = quantize(cache["p"], cfg.cdf_bits)
        cum = cumulative(q)
        target = np.empty(len(act), dtype=np.int64)
        for r, s in enumerate(act):
            if decoding:
                x = coders[s].decode(cum[r].tolist())
                hist[s][i] = x
            else:
                x = int(hist[s][i])
                coders[s].encode(int(cum[r, x]), int(q[r, x]))
            target[r] = x
            ideal_bits[s] += cfg.cdf_bits - np.log2(q[r, x])
        losses.append(model.loss(cache, target))
        g, dU = model.backward(cache, target)
        if hook is not None:
            hook(i, act, cache, q, model)
        model.adam(g, dU, act)
    info = dict(ideal_bits=ideal_bits, losses=losses, model=model)
    if decoding:
        return [hist[s].astype(np.uint8).tobytes() for s in range(nst)], info
    return [coders[s].finish() for s in range(nst)], info


def encode(streams, cfg: Config, hook=None):
    """Payloads (list of bytes) for a list of byte strings; and run info."""
    lens = [len(s) for s in streams]
    return _run(cfg, lens, streams=streams, hook=hook)


def decode(payloads, lens, cfg: Config, hook=None):
    """Decoded streams (list of bytes) from payloads and original lengths."""
    return _run(cfg, lens, payloads=payloads, hook=hook)


def split_streams(data: np.ndarray, lens) -> list:
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return [data[offs[s]:offs[s + 1]].tobytes() for s in range(len(lens))]
