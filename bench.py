"""Throughput of the online-adaptive byte-model codec on one MI355X.

A step is one pass of the whole hot path over one batch: for every one of
the 1024 streams, gather the context window, embed, LTE, refinement blocks,
softmax, integer CDF, range-code the byte, then the adjoint and the Adam
update (shared weights and each stream's FDM slice).  One step codes one
byte per stream.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--full]

Workload: 64 MiB of order-2 Markov Zipf(1.2) bytes in 1024 streams of 64
KiB; model context 32, embed 16, latent 128, 4 blocks of hidden 256.  The
input is resident in HBM before timing; each timed region covers K
consecutive steps of an encoder (and a decoder) session after W warm-up
steps, bracketed by device synchronisation and HIP events on the library's
stream.  Steady-state steps all cost the same, so K steps' rate is the rate
of the whole 65,536-step job (the first 32 bytes of each stream are coded
uniformly and are not timed).  --full also times a complete encode and
decode of the whole 64 MiB.

Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("encode/decode MB/s on 1 MI355X (BF16 vs FP32 path) at compressed bits/byte "
          "within 0.5% of oracle")
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3}  # dense MFMA peaks of MI355X
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_mid_1024x64KiB.txt")
KERNEL_TIMING_STEPS = 64
KERNEL_SOURCES = ["fused.hip", "fused.h", "kernels.hip", "kernels.h", "common.h", "head_row.h",
                  "rangecoder.h", "adam.h", "gemm.h", "gemm.hip"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def lib_cfg(E, model, precision):
    keys = ("context", "embed", "latent", "blocks", "hidden", "branches", "lr", "beta1",
            "beta2", "eps", "seed")
    return E.edpc_config_default(precision=precision, autotune=True,
                                 **{k: model[k] for k in keys})


def time_session(torch, sess, warmup, steps):
    if warmup:
        sess.edpc_session_run(warmup)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record()
    done = sess.edpc_session_run(steps)
    b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return done, a.elapsed_time(b), wall


def run_precision(torch, E, w, d_in, lens, data, precision, warmup, steps,
                  kernel_steps=KERNEL_TIMING_STEPS):
    cfg = lib_cfg(E, w.model, precision)
    rows = len(lens)
    log(f"{precision}: encoder session")
    enc = E.edpc_encoder_begin(cfg, d_in, lens)
    # per-kernel HIP-event times over kernel_steps steps right after the
    # warm-up (direct launches with events on the session stream), then the
    # timed steps (captured windows, no per-kernel events)
    enc.edpc_session_run(warmup)
    kern = enc.edpc_session_time_kernels(kernel_steps)
    done, ms, wall = time_session(torch, enc, 0, steps)
    enc.edpc_session_destroy()
    enc_mbps = done * rows / (ms * 1e-3) / 1e6
    log(f"{precision}: encode {enc_mbps:.3f} MB/s ({ms / done:.3f} ms/step)")

    # decoder: a container of the streams cut after the steps it will run
    C = w.model["context"]
    cut = C + warmup + steps + 16
    sub = np.ascontiguousarray(data.reshape(rows, -1)[:, :cut]).reshape(-1)
    d_sub = torch.as_tensor(sub).to("cuda")
    cont = E.edpc_encode(cfg, d_sub, np.full(rows, cut))
    kernel_id = int.from_bytes(cont[76:84].cpu().numpy().tobytes(), "little")
    out = torch.empty(rows * cut, dtype=torch.uint8, device="cuda")
    log(f"{precision}: decoder session")
    dec = E.edpc_decoder_begin(cont, out)
    ddone, dms, _ = time_session(torch, dec, warmup, steps)
    dec.edpc_decoder_finish()
    dec.edpc_session_destroy()
    torch.cuda.synchronize()
    assert torch.equal(out, d_sub), "decoder output differs from the input"
    dec_mbps = ddone * rows / (dms * 1e-3) / 1e6
    log(f"{precision}: decode {dec_mbps:.3f} MB/s ({dms / ddone:.3f} ms/step)")
    return dict(encode=enc_mbps, decode=dec_mbps, ms_per_step=ms / done,
                decode_ms_per_step=dms / ddone, wall_s=wall, kernels=kern, steps=done,
                kernel_steps=kernel_steps, kernel_id=kernel_id)


def full_job(torch, E, w, d_in, lens, precision):
    """A whole encode and decode of the workload (device buffers), and the same
    encode with the input copied from pinned host memory and the container
    copied back (the PCIe-inclusive rate)."""
    cfg = lib_cfg(E, w.model, precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cont = E.edpc_encode(cfg, d_in, lens)
    torch.cuda.synchronize()
    te = time.perf_counter() - t0
    t0 = time.perf_counter()
    out, _ = E.edpc_decode(cont)
    torch.cuda.synchronize()
    td = time.perf_counter() - t0
    ok = bool(torch.equal(out, d_in))
    n = int(d_in.numel())
    hdr = 96 + 20 * len(lens)
    h_in = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    h_in.copy_(d_in.cpu())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d2 = h_in.to("cuda", non_blocking=True)
    cont2 = E.edpc_encode(cfg, d2, lens)
    h_out = cont2.cpu()
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    # (each encode autotunes its tiles, so the two containers may differ in
    # summation order; both decode)
    return dict(encode_MBps=n / te / 1e6, decode_MBps=n / td / 1e6, roundtrip=ok,
                bits_per_byte=8.0 * (cont.numel() - hdr) / n,
                encode_with_pcie_MBps=n / tp / 1e6,
                pcie_run_bits_per_byte=8.0 * (h_out.numel() - hdr) / n)


def extra_workload(torch, E, name, warmup, steps):
    """Encoder steady-state rate of another workload in its own precision.
    Ragged: steps from the start of the model phase while all 4096 streams are
    active (the shortest stream is > 1 KiB long), so the rate is of full-batch
    steps; the tail with fewer active streams is slower per step but cheaper."""
    import gen
    w = gen.WORKLOADS[name]
    C = w.model["context"]
    prefix = C + warmup + steps + 8
    log(f"{name}: generating input (prefix {prefix} bytes per stream)")
    data, lens = gen.make_streams(w, prefix=prefix)
    d_in = torch.as_tensor(data).to("cuda")
    cfg = lib_cfg(E, w.model, w.precision)
    enc = E.edpc_encoder_begin(cfg, d_in, lens)
    done, ms, _ = time_session(torch, enc, warmup, steps)
    kern = enc.edpc_session_time_kernels(4)
    enc.edpc_session_destroy()
    rows = int((lens > C + warmup).sum())
    res = {"workload": w.description, "precision": w.precision, "streams": int(len(lens)),
           "encode_MBps": round(done * rows / (ms * 1e-3) / 1e6, 4),
           "ms_per_step": round(ms / done, 4), "steps": int(done)}
    if "fdm_bwd_adam" in kern:
        # (the stored counter readings belong to the 1024-stream workload)
        res["roofline_fdm_bwd_adam"] = fdm_roofline(w, kern, rows, stored=False)
    del d_in
    torch.cuda.empty_cache()
    return res


TILE_NAMES = ("32x32", "64x32", "32x64", "64x64", "128x64", "64x128", "128x128",
              "w128x128", "w256x128", "w128x256", "w256x256")


def kernel_tiles(kernel_id):
    """Tile shape per product class of a container's kernel configuration id
    (4 bits per product slot, slots in GEMM_CLASSES order)."""
    return {c: TILE_NAMES[(kernel_id >> (4 * i)) & 15] if ((kernel_id >> (4 * i)) & 15) < len(TILE_NAMES)
            else "?" for i, c in enumerate(GEMM_CLASSES)}


def copy_rate(torch, nbytes=4 << 30, reps=3):
    """Device-to-device copy rate of the HIP runtime (bytes read + written per
    second) on a buffer too large for any cache: the practical ceiling of a
    pass that reads and writes each byte once."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes": nbytes, "GB_per_s": round(gbs, 1)}


GEMM_CLASSES = ("gemm_lte_down", "gemm_lte_up", "gemm_branches_gelu", "gemm_block_out",
                "gemm_head", "gemm_head_bwd", "gemm_gelu_bwd", "gemm_branches_bwd",
                "gemm_lte_up_bwd", "gemm_lte_down_bwd", "gemm_weight_grads")


def gemm_flops_per_step(m, rows):
    """Algorithmic flops (2 per multiply-add) of each matrix-product class of
    the layer-by-layer step on `rows` active rows."""
    F, L, H, N, K = (m["context"] * m["embed"], m["latent"], m["hidden"], m["blocks"],
                     m["branches"])
    weights = L * F + F * L + N * (K * H * F + F * H) + 256 * F
    per = {"gemm_lte_down": L * F, "gemm_lte_up": F * L, "gemm_branches_gelu": N * K * H * F,
           "gemm_block_out": N * F * H, "gemm_head": 256 * F, "gemm_head_bwd": F * 256,
           "gemm_gelu_bwd": N * H * F, "gemm_branches_bwd": N * F * K * H,
           "gemm_lte_up_bwd": L * F, "gemm_lte_down_bwd": F * L, "gemm_weight_grads": weights}
    return {k: 2 * rows * v for k, v in per.items()}


def gemm_roofline(w, kern, rows, precision, n_steps):
    """MFMA roofline of the layer-by-layer step's matrix products: algorithmic
    flops over their summed HIP-event time, in total and per product class."""
    fl = gemm_flops_per_step(w.model, rows)
    peak = MFMA_PEAK_TFLOPS[precision]
    by, tot_f, tot_ms = {}, 0.0, 0.0
    for c in GEMM_CLASSES:
        ms, launches = kern.get(c, (0.0, 0))
        if not launches:
            continue
        f = fl[c] * n_steps
        tf = f / (ms * 1e-3) / 1e12
        by[c] = {"ms_per_step": round(ms / n_steps, 4), "tflops": round(tf, 1),
                 "frac": round(tf / peak, 4)}
        tot_f += f
        tot_ms += ms
    if not tot_ms:
        return None
    tf = tot_f / (tot_ms * 1e-3) / 1e12
    return {"kernels": "matrix products", "bound": "mfma", "achieved": round(tf, 1), "peak": peak,
            "unit": "TFLOP/s", "frac": round(tf / peak, 4), "ms_per_step": round(tot_ms / n_steps, 4),
            "by_class": by}


def large_workload(torch, E, precisions, warmup=8, kernel_steps=8, steps=24):
    """The 16384-stream large model: encoder and sequential-decoder steady
    state in each precision (a prefix of the input long enough for the steps
    timed; by causality those steps are the first steps of the whole job)."""
    import gen
    w = gen.WORKLOADS["large"]
    C = w.model["context"]
    prefix = C + warmup + kernel_steps + steps + 16
    log(f"large: generating input (prefix {prefix} bytes per stream)")
    data, lens = gen.make_streams(w, prefix=prefix)
    d_in = torch.as_tensor(data).to("cuda")
    rows = len(lens)
    out = {"workload": w.description, "streams": rows}
    for prec in precisions:
        r = run_precision(torch, E, w, d_in, lens, data, prec, warmup, steps, kernel_steps)
        kern = r["kernels"]
        out[prec] = {"encode_MBps": round(r["encode"], 4), "decode_MBps": round(r["decode"], 4),
                     "ms_per_step": round(r["ms_per_step"], 3),
                     "decode_ms_per_step": round(r["decode_ms_per_step"], 3),
                     "kernels_ms_per_step": {k: round(v[0] / kernel_steps, 4)
                                             for k, v in kern.items() if v[1]},
                     "roofline_fdm_bwd_adam": fdm_roofline(w, kern, rows, stored=False),
                     "roofline_gemm": gemm_roofline(w, kern, rows, prec, kernel_steps),
                     "tiles": kernel_tiles(r["kernel_id"])}
        log(f"large {prec}: {out[prec]['encode_MBps']} / {out[prec]['decode_MBps']} MB/s")
    if "bf16" in out and "fp32" in out:
        out["bf16_over_fp32_encode"] = round(out["bf16"]["encode_MBps"] / out["fp32"]["encode_MBps"], 3)
    del d_in
    torch.cuda.empty_cache()
    out["device_copy"] = copy_rate(torch)
    torch.cuda.empty_cache()
    return out


def ragged_full_job(torch, E):
    """The whole 256 MiB ragged mixture job: one encode and one decode of all
    4096 streams, including the tail of shrinking active sets."""
    import gen
    w = gen.WORKLOADS["ragged"]
    log("ragged_full: generating the 256 MiB input")
    data, lens = gen.make_streams(w)
    d_in = torch.as_tensor(data).to("cuda")
    cfg = lib_cfg(E, w.model, w.precision)
    n = int(d_in.numel())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cont = E.edpc_encode(cfg, d_in, lens)
    torch.cuda.synchronize()
    te = time.perf_counter() - t0
    log(f"ragged_full: encode {n / te / 1e6:.3f} MB/s")
    t0 = time.perf_counter()
    out, _ = E.edpc_decode(cont)
    torch.cuda.synchronize()
    td = time.perf_counter() - t0
    ok = bool(torch.equal(out, d_in))
    hdr = 96 + 20 * len(lens)
    res = {"workload": w.description, "streams": int(len(lens)), "bytes": n,
           "steps": int(lens.max()), "encode_MBps": round(n / te / 1e6, 4),
           "decode_MBps": round(n / td / 1e6, 4), "encode_s": round(te, 2),
           "decode_s": round(td, 2), "roundtrip": ok,
           "bits_per_byte": round(8.0 * (cont.numel() - hdr) / n, 4)}
    log(f"ragged_full: {res}")
    del d_in, out, cont
    torch.cuda.empty_cache()
    return res


def rows_sweep(torch, E, counts=(16, 64, 256, 1024, 2048, 4096), warmup=80, steps=400):
    """Step time of the 1024-stream model (BF16, row-block step) against the
    number of active streams, and the ragged job's time predicted from it: the
    ragged mixture runs the same model while its active set shrinks, so its
    rate follows from this curve and its row counts per step."""
    import gen
    w = gen.WORKLOADS["mid_bf16"]
    cfg = lib_cfg(E, w.model, "bf16")
    pts = []
    for rows in counts:
        # the workload has 1024 streams; larger sets repeat them (the step
        # time does not depend on the bytes)
        base, blens = gen.make_streams(w, prefix=w.model["context"] + warmup + steps + 16,
                                       n_streams=min(rows, len(w.lens())))
        rep = max(1, rows // len(blens))
        data = np.tile(base.reshape(len(blens), -1), (rep, 1)).reshape(-1)
        lens = np.tile(blens, rep)
        d_in = torch.as_tensor(data).to("cuda")
        enc = E.edpc_encoder_begin(cfg, d_in, lens)
        enc.edpc_session_run(warmup)
        done, ms, _ = time_session(torch, enc, 0, steps)
        enc.edpc_session_destroy()
        pts.append((int(len(lens)), ms / done))
        log(f"rows: {len(lens)} active streams: {ms / done:.4f} ms/step")
        del d_in
    r = gen.WORKLOADS["ragged"]
    ls = np.sort(r.lens())
    active = len(ls) - np.searchsorted(ls, np.arange(int(ls[-1])), side="right")
    t = np.interp(active, [p[0] for p in pts], [p[1] for p in pts])
    res = {"model": w.description, "precision": "bf16",
           "ms_per_step": {str(k): round(v, 4) for k, v in pts},
           "MBps": {str(k): round(k / (v * 1e-3) / 1e6, 3) for k, v in pts},
           "ragged_predicted_s": round(float(t.sum()) / 1e3, 1),
           "ragged_time_share_at_most_1024_rows": round(float(t[active <= 1024].sum() / t.sum()), 3),
           "ragged_byte_share_at_most_1024_rows": round(float(active[active <= 1024].sum()
                                                              / active.sum()), 3)}
    log(f"rows: {res}")
    torch.cuda.empty_cache()
    return res


def stream_job(torch, E, chunk=4096, precision="bf16"):
    """End-to-end host-to-host rate of the 1024-stream workload: the whole
    64 MiB encoded from pinned host memory into host memory and decoded back
    (edpc_encode_host / edpc_decode_host: input and output move through a
    device window of a few chunks per stream, overlapped with the steps)."""
    import gen
    w = gen.WORKLOADS["mid_bf16"]
    data, lens = gen.make_streams(w)
    h_in = torch.from_numpy(data).pin_memory()
    cfg = lib_cfg(E, w.model, precision)
    cap = E.edpc_encode_bound(cfg, lens)
    h_cont = torch.empty(cap, dtype=torch.uint8).pin_memory()
    n = int(data.size)
    t0 = time.perf_counter()
    clen = E.edpc_encode_host(cfg, h_in, lens, chunk, out=h_cont)
    te = time.perf_counter() - t0
    log(f"stream: encode {n / te / 1e6:.3f} MB/s")
    h_out = torch.empty(n, dtype=torch.uint8).pin_memory()
    t0 = time.perf_counter()
    got = E.edpc_decode_host(h_cont[:clen], chunk, out=h_out)
    td = time.perf_counter() - t0
    ok = got == n and bool(torch.equal(h_out, h_in))
    res = {"workload": w.description, "precision": precision, "chunk_steps": chunk,
           "encode_MBps": round(n / te / 1e6, 4), "decode_MBps": round(n / td / 1e6, 4),
           "encode_s": round(te, 2), "decode_s": round(td, 2), "roundtrip": ok,
           "bits_per_byte": round(8.0 * (clen - (96 + 20 * len(lens))) / n, 4)}
    log(f"stream: {res}")
    return res


def ifr_analysis(torch, E, train_steps=512, rows=1024, v=3):
    """The information-flow analysis of Sec. 3.1.1 on synthetic data: models
    with k = 1, 2, 3 branches per refinement block (context 16, embed 16,
    latent 64, 2 blocks x hidden 128, FP32) are trained online for
    `train_steps` steps over `rows` streams of the ragged mixture (the same
    update as the codec), then each block's I(S; S + X^(k)) is estimated on
    the next step's batch (Kraskov, v neighbours, one sample per stream) and
    IFR_{k1->k2} = I^(k1) / I^(k2) (Eq. 8) is formed per block."""
    import gen
    base = dict(gen.WORKLOADS["small"].model)
    C = base["context"]
    data, lens = gen.make_streams("ragged", prefix=C + train_steps + 1, n_streams=rows)
    st = np.frombuffer(data.tobytes(), dtype=np.uint8).reshape(rows, -1)
    slots = np.arange(rows)
    out = {"model": "context 16, embed 16, latent 64, 2 blocks x hidden 128, FP32",
           "train_steps": train_steps, "samples": rows, "neighbours": v,
           "source": "ragged mixture (Markov, uniform, runs, sine), first bytes of each stream"}
    mi = {}
    for k in (1, 2, 3):
        keys = ("context", "embed", "latent", "blocks", "hidden", "lr", "beta1", "beta2", "eps",
                "seed")
        cfg = E.edpc_config_default(precision="fp32", branches=k, **{x: base[x] for x in keys})
        m = E.Model(cfg, rows, rows)
        t0 = time.perf_counter()
        for i in range(C, C + train_steps):
            m.edpc_model_step(torch.as_tensor(np.ascontiguousarray(st[:, i - C:i])).to("cuda"),
                              torch.as_tensor(np.ascontiguousarray(st[:, i])).to("cuda"), slots,
                              flags=E.EDPC_STEP_UPDATE)
        torch.cuda.synchronize()
        i = C + train_steps
        ctx = torch.as_tensor(np.ascontiguousarray(st[:, i - C:i])).to("cuda")
        tgt = torch.as_tensor(np.ascontiguousarray(st[:, i])).to("cuda")
        mi[k] = E.block_mutual_info(m, ctx, tgt, slots, v)
        out[f"k{k}"] = {"mi_nats_per_block": [round(x, 5) for x in mi[k]],
                        "train_s": round(time.perf_counter() - t0, 2)}
        del m
    for a, b in ((1, 2), (1, 3), (2, 3)):
        out[f"IFR_{a}to{b}"] = [round(x / y, 4) for x, y in zip(mi[a], mi[b])]
    log(f"ifr: {out}")
    return out


GOLDEN_FILE = os.path.join(ROOT, "tests", "golden", "oracle_sizes.json")


def size_parity(torch, E, precisions, cases=("mid_prefix", "skewed_wide")):
    """Compressed size against the oracle's (the metric's qualifier): the
    benchmarked configuration encodes the inputs of stored oracle cases (the
    1024-stream workload's first 160 bytes per stream, and 1024 streams of a
    learnable skewed source) and its payload is compared with the oracle's
    payload, written by tests/golden/make_oracle_golden.py."""
    import gen
    with open(GOLDEN_FILE) as f:
        gold = json.load(f)
    out = {}
    worst = 0.0
    for case in cases:
        g = gold[case]
        data, lens = gen.make_streams(g["workload"], prefix=g["prefix"], n_streams=g["n_streams"])
        assert [int(x) for x in lens] == g["lens"], case
        w = gen.WORKLOADS[g["workload"]]
        d_in = torch.as_tensor(data).to("cuda")
        o_bytes = sum(g["payload_bytes"])
        res = {"streams": int(len(lens)), "bytes": int(lens.sum()),
               "oracle_bits_per_byte": round(8.0 * o_bytes / lens.sum(), 5)}
        for prec in precisions:
            cont = E.edpc_encode(lib_cfg(E, dict(w.model, **g["overrides"]), prec), d_in, lens)
            torch.cuda.synchronize()
            pay = cont.numel() - (96 + 20 * len(lens))
            rel = (pay - o_bytes) / o_bytes
            worst = max(worst, abs(rel))
            res[prec] = {"bits_per_byte": round(8.0 * pay / lens.sum(), 5),
                         "rel_diff": round(rel, 6)}
        out[case] = res
        log(f"size parity {case}: {res}")
    out["max_abs_rel_diff"] = round(worst, 6)
    out["within_0.5pct"] = bool(worst <= 0.005)
    return out


ABLATIONS = (
    # name, model overrides (Table 4 rows; F = context x embed = 256 so every
    # variant is accepted: w/o LTE needs latent = F, low-rank a power-of-two F)
    ("base", {}),
    ("wo_lte", {"latent": 256, "lte": False}),
    ("low_rank", {"low_rank": True}),
    ("k3", {"branches": 3}),
    ("one_block", {"blocks": 1}),
    # the base model on the layer-by-layer products, so that the speed column
    # compares the variants (which all run layer by layer) like with like
    ("base_layerwise", {"layerwise": True}),
)


def ablation_cfg(E, base, over, precision):
    """Library configuration of one ablation: the base model with `over` applied."""
    m = dict(base, **over)
    keys = ("context", "embed", "latent", "blocks", "hidden", "branches", "lr", "beta1",
            "beta2", "eps", "seed")
    return E.edpc_config_default(precision=precision, autotune=True,
                                 lte=m.get("lte", True), low_rank=m.get("low_rank", False),
                                 layerwise=m.get("layerwise", False),
                                 **{k: m[k] for k in keys})


def ablation_workload(torch, E, warmup, steps, precision="bf16", ratio_bytes=1024):
    """The Table 4 variants on one model (context 16, embed 16, latent 64,
    2 blocks x hidden 128, k = 2), each with
    * speed: encoder steady state over the 1024-stream order-2 Markov input;
    * memory: the session's device memory (free-memory drop from begin to
      after the first steps);
    * ratio: bits/byte of a whole encode of 1024 streams of the ragged
      mixture cut to `ratio_bytes` bytes (a source the model partly learns),
      and of the 64-stream x 256-byte mixture prefix whose oracle size is
      stored (tests/golden/oracle_sizes.json, ablation_* cases)."""
    import gen
    w = gen.WORKLOADS["mid_bf16"]
    base = dict(gen.WORKLOADS["small"].model)
    C = base["context"]
    prefix = C + warmup + steps + 8
    log(f"ablations: generating input (prefix {prefix} bytes per stream)")
    data, lens = gen.make_streams(w, prefix=prefix)
    d_in = torch.as_tensor(data).to("cuda")
    rows = int((lens > C + warmup).sum())
    mdata, mlens = gen.make_streams("ragged", prefix=ratio_bytes, n_streams=1024)
    d_mix = torch.as_tensor(mdata).to("cuda")
    with open(GOLDEN_FILE) as f:
        gold = json.load(f)
    out = {"model": "context 16, embed 16, latent 64, 2 blocks x hidden 128, k = 2",
           "streams": int(len(lens)), "precision": precision,
           "ratio_input": f"1024 mixture streams x {ratio_bytes} B"}
    for name, over in ABLATIONS:
        cfg = ablation_cfg(E, base, over, precision)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        enc = E.edpc_encoder_begin(cfg, d_in, lens)
        done, ms, _ = time_session(torch, enc, warmup, steps)
        free1 = torch.cuda.mem_get_info()[0]
        kern = enc.edpc_session_time_kernels(4)
        enc.edpc_session_destroy()
        torch.cuda.synchronize()
        cont = E.edpc_encode(cfg, d_mix, mlens)
        torch.cuda.synchronize()
        bpb = 8.0 * (cont.numel() - (96 + 20 * len(mlens))) / mlens.sum()
        out[name] = {"encode_MBps": round(done * rows / (ms * 1e-3) / 1e6, 4),
                     "ms_per_step": round(ms / done, 4), "steps": int(done),
                     "session_MB": round((free0 - free1) / 1e6, 1),
                     "row_block_step": kern["fused_rowblock_step"][1] > 0,
                     "bits_per_byte": round(bpb, 4)}
        g = gold.get("ablation_" + name.replace("_layerwise", ""))
        if g:
            gd, gl = gen.make_streams(g["workload"], prefix=g["prefix"], n_streams=g["n_streams"])
            c2 = E.edpc_encode(cfg, torch.as_tensor(gd).to("cuda"), gl)
            torch.cuda.synchronize()
            pay = c2.numel() - (96 + 20 * len(gl))
            o = sum(g["payload_bytes"])
            out[name]["prefix_bits_per_byte"] = round(8.0 * pay / gl.sum(), 4)
            out[name]["prefix_oracle_bits_per_byte"] = round(8.0 * o / gl.sum(), 4)
            out[name]["prefix_rel_diff"] = round((pay - o) / o, 6)
        log(f"ablation {name}: {out[name]}")
    del d_in, d_mix
    torch.cuda.empty_cache()
    return out


def source_code(text):
    """Kernel source text without comments and whitespace (a comment edit does
    not change the code the counter readings belong to)."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_digest(read=None):
    """Digest of the kernel sources the stored counter readings belong to."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        if read is None:
            with open(os.path.join(ROOT, "paper_2507_18969_amd", "csrc", name), "r") as f:
                text = f.read()
        else:
            text = read(name)
        h.update(source_code(text).encode())
    return h.hexdigest()[:16]


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE readings (already scaled by the copy-kernel factor), or None if
    there are none or the kernel sources changed since they were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            kv = dict(line.strip().split("=", 1) for line in f
                      if "=" in line and not line.startswith("#"))
    except OSError:
        return None
    if kv.get("source_digest") != source_digest():
        return None
    v = kv.get(f"{kernel}.hbm_bytes_per_launch")
    return int(float(v)) if v else None


def fdm_roofline(w, kern, rows, stored=True):
    """FDM adjoint + Adam kernel: U, m, v read and written per step (24 B per
    element of the active streams' L x L slices) plus the x', dy rows read and
    dx' written."""
    L = w.model["latent"]
    ms, launches = kern["fdm_bwd_adam"]
    per_launch_s = ms / launches * 1e-3
    algo = rows * L * L * 24 + rows * L * 4 * 3
    gbs = algo / per_launch_s / 1e9
    return {"kernel": "fdm_bwd_adam", "bound": "hbm", "achieved": round(gbs, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": stored_traffic("fdm_bwd_adam") if stored else None,
            "algorithmic_bytes_per_launch": algo,
            "avg_launch_us": round(per_launch_s * 1e6, 2)}


def dense_flops_per_row(m):
    """Multiply-adds per row of one pass through the shared dense layers the
    row-block step runs: LTE up, the blocks' branch and output linears, the head."""
    F, L, H, N, K = (m["context"] * m["embed"], m["latent"], m["hidden"], m["blocks"],
                     m["branches"])
    return F * L + N * (K * H * F + F * H) + 256 * F


def fused_roofline(w, kern, rows, precision):
    """Row-block fused step: forward products and the input adjoints of the
    same layers (2 passes x 2 flops per multiply-add) for every active row."""
    ms, launches = kern["fused_rowblock_step"]
    per_launch_s = ms / launches * 1e-3
    flops = rows * 4 * dense_flops_per_row(w.model)
    tf = flops / per_launch_s / 1e12
    peak = MFMA_PEAK_TFLOPS[precision]
    return {"kernel": "fused_rowblock_step", "bound": "mfma", "achieved": round(tf, 2),
            "peak": peak, "unit": "TFLOP/s", "frac": round(tf / peak, 4),
            "traffic": stored_traffic("fused_rowblock_step"),
            "algorithmic_flops_per_launch": flops, "avg_launch_us": round(per_launch_s * 1e6, 2)}


# Per-CU limit on L2 reads in flight and the mean L2 read latency the
# row-block kernel sees (rocprofv3 TCP_TCC_READ_REQ(_LATENCY) counters of the
# 1024-stream BF16 step): the rate at which one CU can stream operands from L2.
CU_L2_READS_IN_FLIGHT = 64
CU_L2_READ_LATENCY_CYCLES = 290
CLOCK_GHZ = 2.4


def fused_stream_bound(w, kern, rows):
    """The bound the row-block kernel actually meets: every workgroup (one
    per CU, 16 rows) streams each BF16 weight of its products twice (forward
    and adjoint orientation) from L2, and a CU can keep only so many L2 reads
    in flight.  Achieved = those bytes over the launch time, per CU clock."""
    if w.precision != "bf16" or "fused_rowblock_step" not in kern:
        return None
    ms, launches = kern["fused_rowblock_step"]
    per_launch_s = ms / launches * 1e-3
    weight_bytes = 2 * 2 * dense_flops_per_row(w.model)  # two orientations x 2 bytes
    achieved = weight_bytes / (per_launch_s * CLOCK_GHZ * 1e9)
    limit = CU_L2_READS_IN_FLIGHT * 128 / CU_L2_READ_LATENCY_CYCLES
    return {"kernel": "fused_rowblock_step", "bound": "per-CU L2 reads in flight",
            "achieved": round(achieved, 2), "limit": round(limit, 2), "unit": "B/clk/CU",
            "frac": round(achieved / limit, 3), "bytes_per_workgroup": weight_bytes,
            "workgroups": (rows + 15) // 16}


def dominant_roofline(w, kern, rows, precision):
    """Roofline of the kernel with the largest share of the step."""
    share = {k: v[0] for k, v in kern.items() if v[1]}
    top = max(share, key=share.get)
    if top == "fused_rowblock_step":
        return fused_roofline(w, kern, rows, precision)
    return fdm_roofline(w, kern, rows)


def cpu_baseline(w, data, lens, n_model_steps):
    """The CPU oracle on a bounded sample of the same workload: all 1024
    streams, the uniform prefix plus n_model_steps model steps."""
    import oracle
    from oracle.codec import _run
    from oracle.model import Config
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    C = w.model["context"]
    cut = C + n_model_steps
    rows = len(lens)
    sub = data.reshape(rows, -1)[:, :cut]
    streams = [sub[s].tobytes() for s in range(rows)]
    cfg = Config.from_dict(w.model)
    t0 = time.perf_counter()
    _run(cfg, [cut] * rows, streams=streams)
    dt = time.perf_counter() - t0
    del oracle
    return {"value": round(rows * cut / dt / 1e6, 6), "unit": "MB/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{rows} streams x {cut} bytes ({C} uniform + {n_model_steps} model steps), "
                      f"FP64 numpy, {dt:.1f} s"}


def run_extra(torch, E, a):
    extra = {}
    for name in [x for x in a.extra.split(",") if x and x != "none"]:
        if name == "ablations":
            extra[name] = ablation_workload(torch, E, a.warmup, min(a.steps, 200))
        elif name == "large":
            extra[name] = large_workload(torch, E, a.precisions.split(","))
        elif name == "ragged_full":
            extra[name] = ragged_full_job(torch, E)
        elif name == "stream":
            extra[name] = stream_job(torch, E)
        elif name == "ifr":
            extra[name] = ifr_analysis(torch, E)
        elif name == "rows":
            extra[name] = rows_sweep(torch, E)
        else:
            extra[name] = extra_workload(torch, E, name, a.warmup, min(a.steps, 200))
    return extra


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--full", action="store_true", help="also time a whole encode + decode")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=64)
    ap.add_argument("--precisions", default="bf16,fp32")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after timing, run a 256 MiB device copy (the reference kernel for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE readings)")
    ap.add_argument("--extra", default="large",
                    help="comma list of further workloads measured after the main one "
                         "(ragged, ragged_full, large, stream, ifr, ablations, rows; 'none' for "
                         "none); reported under extra_workloads.  Default: the 16384-stream "
                         "large model (encode and decode in both precisions, about 10 s)")
    ap.add_argument("--no-size-parity", action="store_true",
                    help="skip the compressed-size comparison with the oracle's stored sizes")
    ap.add_argument("--only-extra", action="store_true",
                    help="measure only the --extra workloads (no main line; for profiling)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (sharding the "
              "streams needs a fixed-order exchange of the shared-weight gradients every step, "
              "which is not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch

    import gen
    import paper_2507_18969_amd as E
    E.lib()
    if a.only_extra:
        print(json.dumps({"extra_workloads": run_extra(torch, E, a)}), flush=True)
        return
    w = gen.WORKLOADS["mid_bf16"]
    log("generating 64 MiB input")
    data, lens = gen.make_streams(w)
    d_in = torch.as_tensor(data).to("cuda")
    torch.cuda.synchronize()
    rows = len(lens)
    res = {}
    for prec in a.precisions.split(","):
        res[prec] = run_precision(torch, E, w, d_in, lens, data, prec, a.warmup, a.steps)
    main_p = "bf16" if "bf16" in res else list(res)[0]
    r = res[main_p]
    kern = {k: [round(v[0] / KERNEL_TIMING_STEPS, 4), v[1] // KERNEL_TIMING_STEPS]
            for k, v in r["kernels"].items() if v[1]}
    line = {
        "metric": METRIC, "value": round(r["encode"], 4), "unit": "MB/s", "n_gpus": 1,
        "steps": int(r["steps"]), "warmup": a.warmup, "kernel_timing_steps": KERNEL_TIMING_STEPS,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": main_p,
        "data": "synthetic",
        "config": {"workload": "64 MiB order-2 Markov Zipf(1.2), 1024 streams x 64 KiB; "
                               "context 32, embed 16, latent 128, 4 blocks x hidden 256",
                   "streams": rows, "stream_bytes": int(lens[0]), "bytes_per_step": rows,
                   "precision": main_p},
        "encode_MBps": {p: round(v["encode"], 4) for p, v in res.items()},
        "decode_MBps": {p: round(v["decode"], 4) for p, v in res.items()},
        "ms_per_step_by_precision": {p: round(v["ms_per_step"], 4) for p, v in res.items()},
        "kernels_ms_per_step": kern,
        "roofline": dominant_roofline(w, r["kernels"], rows, main_p),
        "roofline_hbm": fdm_roofline(w, r["kernels"], rows),
        "fused_stream_bound": fused_stream_bound(w, r["kernels"], rows),
    }
    if "bf16" in res and "fp32" in res:
        line["bf16_over_fp32_encode"] = round(res["bf16"]["encode"] / res["fp32"]["encode"], 3)
    extra = run_extra(torch, E, a)
    if not a.no_size_parity:
        line["size_parity_vs_oracle"] = size_parity(torch, E, list(res))
    if extra:
        line["extra_workloads"] = extra
    if a.full:
        line["full_job"] = {p: full_job(torch, E, w, d_in, lens, p) for p in res}
    if a.copy_probe:
        src = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not a.no_cpu:
        log("CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline(w, data, lens, a.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
