"""Write the oracle's expected payload sizes for the GPU parity tests.

Calls only the CPU oracle (oracle/) on the seeded synthetic inputs (gen/);
nothing here touches the GPU library.  Output: tests/golden/oracle_sizes.json

    python tests/golden/make_oracle_golden.py [--only NAME]

Cases:
  small_full      the 8-stream x 8 KiB workload, every byte (8192 steps)
  small_zero_lr   the same input with lr = 0 (static random model), 2 KiB prefix
  mid_prefix      the 1024-stream x 64 KiB workload cut to its first 160 bytes
  mid_slice       4 streams x 512 bytes of the mid workload
  ragged_prefix   32 streams of the mixture source cut to seeded lengths in
                  [100, 1500] (ragged), mid model
  ragged_wide     all 4096 streams of the mixture workload cut to their first
                  96 bytes (64 model steps), mid model
  skewed_small    the learnable skewed source, 8 streams x 2 KiB, small model
  skewed_mid_64   the skewed source, 64 streams x 512 B, mid model
  skewed_wide     the skewed source, 1024 streams x 256 B, mid model (the
                  1024-row launch of the benchmarked configuration)
  ablation_*      the Table 4 / 5 variants (base, w/o LTE, low-rank, three
                  branches, one block) of the small model on 64 mixture
                  streams cut to 256 bytes
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gen  # noqa: E402
import oracle  # noqa: E402
from oracle.codec import split_streams  # noqa: E402
from oracle.model import Config  # noqa: E402

def ragged_prefix_input():
    """32 mixture streams cut to lengths drawn from a seeded generator."""
    import numpy as np
    data, lens = gen.make_streams("ragged", prefix=1500, n_streams=32)
    cut = np.random.default_rng(2507).integers(100, 1501, size=32)
    cut[0] = 1500
    cut = np.minimum(cut, lens)
    offs = np.concatenate([[0], np.cumsum(lens)])
    parts = [data[offs[s]:offs[s] + cut[s]] for s in range(32)]
    return np.concatenate(parts), cut.astype(np.int64)


CASES = {
    "small_full": ("small", None, None, {}),
    "small_zero_lr": ("small", 2048, None, {"lr": 0.0}),
    "mid_prefix": ("mid_fp32", 160, None, {}),
    "mid_slice": ("mid_fp32", 512, 4, {}),
    "ragged_prefix": ("ragged", "ragged_prefix", None, {}),
    "ragged_wide": ("ragged", 96, None, {}),
    "skewed_small": ("skewed_small", None, None, {}),
    "skewed_mid_64": ("skewed_mid", 512, 64, {}),
    "skewed_wide": ("skewed_mid", 256, None, {}),
}

# Table 4 / Table 5 variants on the small model, 64 streams of the ragged
# mixture cut to 256 bytes: base, w/o LTE (per-stream F x F FDM), per-stream
# low-rank factors, three branches, one block
_ABL_BASE = dict(context=16, embed=16, latent=64, blocks=2, hidden=128)
ABLATION_CASES = {
    "base": {},
    "wo_lte": {"latent": 256, "lte": False},
    "low_rank": {"low_rank": True},
    "k3": {"branches": 3},
    "one_block": {"blocks": 1},
}
for _name, _over in ABLATION_CASES.items():
    CASES["ablation_" + _name] = ("ragged", 256, 64, dict(_ABL_BASE, **_over))


def case_input(name):
    """(flat data, lengths, model dict with the case's overrides) of a case."""
    wl, prefix, nst, over = CASES[name]
    w = gen.WORKLOADS[wl]
    if prefix == "ragged_prefix":
        data, lens = ragged_prefix_input()
    else:
        data, lens = gen.make_streams(w, prefix=prefix, n_streams=nst)
    return data, lens, dict(w.model, **over)


def run_case(name):
    wl, prefix, nst, over = CASES[name]
    data, lens, model = case_input(name)
    cfg = Config.from_dict(model)
    t = time.time()
    pay, info = oracle.encode(split_streams(data, lens), cfg)
    return {
        "workload": wl, "prefix": prefix, "n_streams": int(len(lens)), "overrides": over,
        "lens": [int(x) for x in lens],
        "payload_bytes": [len(p) for p in pay],
        "ideal_bits": [float(b) for b in info["ideal_bits"]],
        "final_loss": float(info["losses"][-1]) if info["losses"] else None,
        "oracle_seconds": time.time() - t,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=None, help="comma list of case names")
    a = ap.parse_args()
    path = os.path.join(HERE, "oracle_sizes.json")
    out = {}
    if os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    for name in CASES:
        if a.only and name not in a.only.split(","):
            continue
        out[name] = run_case(name)
        print(name, sum(out[name]["payload_bytes"]), f"{out[name]['oracle_seconds']:.1f}s", flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
