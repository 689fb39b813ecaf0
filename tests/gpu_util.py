"""Helpers shared by the GPU tests: library handle, configs, oracle state
loading through the C ABI, container parsing."""

from __future__ import annotations

import struct
import sys

import numpy as np

import gen
from oracle.model import Config


def banner(msg: str):
    print(f"[gpu] {msg}", file=sys.stderr, flush=True)


def lib_cfg(E, model: dict, precision: str = "fp32", **over):
    d = dict(model)
    d.update(over)
    kw = {k: d[k] for k in ("context", "embed", "latent", "blocks", "hidden", "branches", "lr",
                            "beta1", "beta2", "eps", "seed") if k in d}
    return E.edpc_config_default(precision=precision, zero_head=d.get("zero_head", False),
                                 autotune=d.get("autotune", False), lte=d.get("lte", True),
                                 low_rank=d.get("low_rank", False),
                                 layerwise=d.get("layerwise", False),
                                 graphs=d.get("graphs", True), **kw)


def oracle_cfg(model: dict, **over) -> Config:
    return Config.from_dict(model).with_(**over)


def load_oracle_state(m, om, slots=None):
    """Write an oracle model's state (rounded to FP32) into a library model.
    The oracle is the source; nothing flows back."""
    for k in om.p:
        m.edpc_model_write(k, om.p[k].astype(np.float32))
        m.edpc_model_write(k, om.m[k].astype(np.float32), kind=2)
        m.edpc_model_write(k, om.v[k].astype(np.float32), kind=3)
    m.edpc_model_write("U", om.U.astype(np.float32))
    m.edpc_model_write("U", om.mU.astype(np.float32), kind=2)
    m.edpc_model_write("U", om.vU.astype(np.float32), kind=3)
    if om.cfg.low_rank:
        for n in ("A", "B"):
            m.edpc_model_write(n, getattr(om, n).astype(np.float32))
            m.edpc_model_write(n, getattr(om, "m" + n).astype(np.float32), kind=2)
            m.edpc_model_write(n, getattr(om, "v" + n).astype(np.float32), kind=3)
    m.edpc_model_set_step(om.tau)


def parse_container(buf: bytes):
    """Split a container into (per-stream lengths, payload byte strings).
    Follows the documented layout independently of the library."""
    assert buf[:4] == b"EDPC"
    hl, n = struct.unpack_from("<II", buf, 8)
    lens, plens = [], []
    for s in range(n):
        ln, pl, _ = struct.unpack_from("<QQI", buf, 92 + 20 * s)
        lens.append(ln)
        plens.append(pl)
    pays, o = [], hl
    for pl in plens:
        pays.append(buf[o:o + pl])
        o += pl
    assert o == len(buf)
    return lens, pays


def streams(workload: str, prefix=None, n=None):
    return gen.make_streams(workload, prefix=prefix, n_streams=n)
