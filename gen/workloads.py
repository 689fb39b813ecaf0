"""The five synthetic workloads, as plain data.

Each workload names its input (source kind, stream count, lengths) and the
model hyper-parameters it is coded with.  The model fields follow the
paper's notation: context t (here ``context``), embedding width, LTE latent
dimension F' (``latent``), number of refinement blocks, block hidden width,
branch count k (Sec. 3.1.2), Adam learning rate (Sec. 4.1).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import sources


@dataclass(frozen=True)
class Workload:
    name: str
    description: str
    source: str  # "markov2" | "mixture" | "skewed"
    n_streams: int
    stream_len: int | None  # equal-length streams; None for ragged
    total_bytes: int
    zipf_s: float
    model: dict = field(default_factory=dict)
    precision: str = "fp32"  # "fp32" | "bf16" (GEMM operand type)

    def lens(self) -> np.ndarray:
        if self.stream_len is not None:
            return np.full(self.n_streams, self.stream_len, dtype=np.int64)
        return sources.ragged_lengths(self.n_streams, self.total_bytes, 4096, 1 << 20)


def _model(context, embed, latent, blocks, hidden):
    return dict(context=context, embed=embed, latent=latent, blocks=blocks,
                hidden=hidden, branches=2, lr=1e-3, beta1=0.9, beta2=0.999,
                eps=1e-8, seed=0)


_SMALL = _model(16, 16, 64, 2, 128)
_MID = _model(32, 16, 128, 4, 256)
_LARGE = _model(64, 32, 256, 6, 512)

WORKLOADS = {
    "small": Workload(
        "small", "64 KiB order-2 Markov Zipf(1.2), 8 streams x 8 KiB; FP32",
        "markov2", 8, 8192, 8 * 8192, 1.2, _SMALL, "fp32"),
    "mid_fp32": Workload(
        "mid_fp32", "64 MiB order-2 Markov Zipf(1.2), 1024 streams x 64 KiB; FP32",
        "markov2", 1024, 65536, 1024 * 65536, 1.2, _MID, "fp32"),
    "mid_bf16": Workload(
        "mid_bf16", "64 MiB order-2 Markov Zipf(1.2), 1024 streams x 64 KiB; BF16 GEMMs",
        "markov2", 1024, 65536, 1024 * 65536, 1.2, _MID, "bf16"),
    "ragged": Workload(
        "ragged", "256 MiB mixture, 4096 log-uniform ragged streams; BF16 GEMMs",
        "mixture", 4096, None, 256 << 20, 1.1, _MID, "bf16"),
    "large": Workload(
        "large", "1 GiB order-2 Markov Zipf(1.2), 16384 streams x 64 KiB; BF16 GEMMs",
        "markov2", 16384, 65536, 16384 * 65536, 1.2, _LARGE, "bf16"),
    # a learnable stand-in (i.i.d. skewed bytes, 1.75 bits of entropy) on the
    # two models above, for size parity where the coded probabilities are
    # strongly peaked; not one of the benchmarked workloads
    "skewed_small": Workload(
        "skewed_small", "i.i.d. skewed 4-letter bytes, 8 streams x 2 KiB; small model, FP32",
        "skewed", 8, 2048, 8 * 2048, 0.0, _SMALL, "fp32"),
    "skewed_mid": Workload(
        "skewed_mid", "i.i.d. skewed 4-letter bytes, 1024 streams x 512 B; 1024-stream model",
        "skewed", 1024, 512, 1024 * 512, 0.0, _MID, "bf16"),
}


def make_streams(w: Workload | str, prefix: int | None = None,
                 n_streams: int | None = None):
    """Generate a workload's input.

    Returns ``(data, lens)``: ``data`` is the flat uint8 concatenation of the
    streams in order, ``lens`` their int64 lengths.  ``prefix`` truncates each
    stream to at most that many bytes (an exact prefix of the full input);
    ``n_streams`` keeps only the first streams.
    """
    if isinstance(w, str):
        w = WORKLOADS[w]
    nst = w.n_streams if n_streams is None else min(n_streams, w.n_streams)
    if w.source in ("markov2", "skewed"):
        length = w.stream_len if prefix is None else min(prefix, w.stream_len)
        if w.source == "markov2":
            arr = sources.markov2_streams(nst, length, w.zipf_s)
        else:
            arr = sources.skewed_streams(nst, length)
        return arr.reshape(-1), np.full(nst, length, dtype=np.int64)
    lens = w.lens()[:nst]
    return sources.mixture_streams(lens, w.zipf_s, prefix=prefix)


def truncate(data: np.ndarray, lens: np.ndarray, prefix: int):
    """Cut every stream of a flat concatenation to at most ``prefix`` bytes."""
    offs = np.concatenate([[0], np.cumsum(lens)])
    parts = [data[offs[s]:offs[s] + min(prefix, lens[s])] for s in range(len(lens))]
    new = np.minimum(lens, prefix)
    return (np.concatenate(parts) if parts else data[:0]), new
