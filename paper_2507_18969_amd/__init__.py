"""Python binding of libedpc (MI355X / gfx950 HIP library).

Thin argument marshalling over the C ABI declared in include/edpc.h: every
function here has the name of the C entry point it calls; PyTorch tensors
provide device memory and the current HIP stream.  All computation happens
in the library's HIP kernels; if the built library is missing, loading fails
loudly (there is no fallback).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# EDPC_LIB names another build of the same library (the host-sanitizer build
# of build.py --sanitize); by default the in-tree libedpc.so is loaded
LIB_PATH = os.environ.get("EDPC_LIB") or os.path.join(_HERE, "libedpc.so")

EDPC_OK = 0
STATUS = {0: "EDPC_OK", -1: "EDPC_E_INVALID_ARG", -2: "EDPC_E_NOMEM", -3: "EDPC_E_CAPACITY",
          -4: "EDPC_E_CORRUPT", -5: "EDPC_E_CHECKSUM", -6: "EDPC_E_UNSUPPORTED",
          -7: "EDPC_E_DEVICE"}
EDPC_FP32, EDPC_BF16 = 0, 1
EDPC_CFG_ZERO_HEAD = 0x1
EDPC_CFG_AUTOTUNE = 0x2
EDPC_CFG_NO_LTE = 0x4
EDPC_CFG_LOW_RANK = 0x8
EDPC_CFG_LAYERWISE = 0x10
EDPC_CFG_NO_GRAPHS = 0x20
EDPC_MAX_STREAM_LEN = 0x7FFFFFFF
EDPC_MAX_STREAMS = 1 << 24
EDPC_RC_NOALLOC_MAX_STREAMS = 65536
EDPC_STEP_BACKWARD, EDPC_STEP_UPDATE, EDPC_STEP_KEEP_FDM_GRAD = 0x1, 0x2, 0x4
EDPC_KIND_PARAM, EDPC_KIND_GRAD, EDPC_KIND_ADAM_M, EDPC_KIND_ADAM_V = 0, 1, 2, 3
EDPC_KIND_OPERAND_NT, EDPC_KIND_OPERAND_NN = 4, 5
KCLASS_COUNT = 24

#: every symbol include/edpc.h declares
EXPORTS = [
    "edpc_status_string", "edpc_last_error", "edpc_abi_version", "edpc_config_default",
    "edpc_config_validate", "edpc_encode_bound", "edpc_encode", "edpc_decode_info",
    "edpc_decode", "edpc_encode_host", "edpc_decode_host", "edpc_encoder_begin", "edpc_decoder_begin", "edpc_session_run",
    "edpc_session_progress", "edpc_encoder_finish", "edpc_decoder_finish",
    "edpc_session_destroy", "edpc_session_time_kernels", "edpc_kclass_name", "edpc_model_create", "edpc_model_create_with_kernels", "edpc_model_kernel_id",
    "edpc_model_destroy", "edpc_model_step",
    "edpc_model_tensor_count", "edpc_model_tensor_info", "edpc_model_read", "edpc_model_write",
    "edpc_model_read_device", "edpc_model_write_device",
    "edpc_model_get_step", "edpc_model_set_step", "edpc_model_activation",
    "edpc_mutual_info", "edpc_model_get_state",
    "edpc_model_set_state", "edpc_rc_encode", "edpc_rc_decode", "edpc_rc_encode_noalloc",
    "edpc_rc_encode_host", "edpc_rc_decode_host",
]


class EdpcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class edpc_config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("context", ctypes.c_uint32),
                ("embed", ctypes.c_uint32), ("latent", ctypes.c_uint32),
                ("blocks", ctypes.c_uint32), ("hidden", ctypes.c_uint32),
                ("branches", ctypes.c_uint32), ("cdf_bits", ctypes.c_uint32),
                ("precision", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("seed", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_P = ctypes.c_void_p
_SZ = ctypes.c_size_t
_U64P = ctypes.POINTER(ctypes.c_uint64)
_U32P = ctypes.POINTER(ctypes.c_uint32)
_SZP = ctypes.POINTER(ctypes.c_size_t)


def lib() -> ctypes.CDLL:
    """Load libedpc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2507_18969_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    cfgp = ctypes.POINTER(edpc_config)
    sig = {
        "edpc_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "edpc_last_error": (ctypes.c_char_p, []),
        "edpc_abi_version": (ctypes.c_int, []),
        "edpc_config_default": (ctypes.c_int, [cfgp]),
        "edpc_config_validate": (ctypes.c_int, [cfgp]),
        "edpc_encode_bound": (ctypes.c_int, [cfgp, _U64P, _SZ, _SZP]),
        "edpc_encode": (ctypes.c_int, [cfgp, _P, _U64P, _SZ, _P, _SZ, _SZP, _P]),
        "edpc_decode_info": (ctypes.c_int, [_P, _SZ, cfgp, _SZP, _U64P, _SZ, _SZP, _SZP]),
        "edpc_decode": (ctypes.c_int, [_P, _SZ, _P, _SZ, _SZP, _P]),
        "edpc_encode_host": (ctypes.c_int, [cfgp, _P, _U64P, _SZ, _P, _SZ, _SZP,
                                             ctypes.c_uint32, _P]),
        "edpc_decode_host": (ctypes.c_int, [_P, _SZ, _P, _SZ, _SZP, ctypes.c_uint32, _P]),
        "edpc_encoder_begin": (ctypes.c_int, [cfgp, _P, _U64P, _SZ, _P, ctypes.POINTER(_P)]),
        "edpc_decoder_begin": (ctypes.c_int, [_P, _SZ, _P, _SZ, _P, ctypes.POINTER(_P)]),
        "edpc_session_run": (ctypes.c_int, [_P, ctypes.c_uint64, _U64P]),
        "edpc_session_progress": (ctypes.c_int, [_P, _U64P, _U64P]),
        "edpc_encoder_finish": (ctypes.c_int, [_P, _P, _SZ, _SZP]),
        "edpc_decoder_finish": (ctypes.c_int, [_P, _SZP]),
        "edpc_session_destroy": (None, [_P]),
        "edpc_session_time_kernels": (ctypes.c_int, [_P, ctypes.c_uint64, _P, _P]),
        "edpc_kclass_name": (ctypes.c_char_p, [ctypes.c_int]),
        "edpc_model_create": (ctypes.c_int, [cfgp, _SZ, _SZ, ctypes.POINTER(_P)]),
        "edpc_model_create_with_kernels": (ctypes.c_int, [cfgp, _SZ, _SZ, ctypes.c_uint64,
                                                           ctypes.POINTER(_P)]),
        "edpc_model_kernel_id": (ctypes.c_int, [_P, _U64P]),
        "edpc_model_destroy": (None, [_P]),
        "edpc_model_step": (ctypes.c_int, [_P, _P, _P, _U32P, _SZ, _P, _P, _P, ctypes.c_uint32, _P]),
        "edpc_model_tensor_count": (ctypes.c_int, [_P, _SZP]),
        "edpc_model_tensor_info": (ctypes.c_int, [_P, _SZ, ctypes.c_char_p, _SZ, _SZP]),
        "edpc_model_read": (ctypes.c_int, [_P, ctypes.c_uint32, _SZ, _P, _SZ]),
        "edpc_model_write": (ctypes.c_int, [_P, ctypes.c_uint32, _SZ, _P, _SZ]),
        "edpc_model_read_device": (ctypes.c_int, [_P, ctypes.c_uint32, _SZ, _P, _SZ, _P]),
        "edpc_model_write_device": (ctypes.c_int, [_P, ctypes.c_uint32, _SZ, _P, _SZ, _P]),
        "edpc_model_get_step": (ctypes.c_int, [_P, _U64P]),
        "edpc_model_set_step": (ctypes.c_int, [_P, ctypes.c_uint64]),
        "edpc_model_activation": (ctypes.c_int, [_P, ctypes.c_uint32, _P, _SZ, _P]),
        "edpc_mutual_info": (ctypes.c_int, [_P, _SZ, _P, _SZ, _SZ, ctypes.c_uint32,
                                             ctypes.POINTER(ctypes.c_double), _P, _P, _P]),
        "edpc_model_get_state": (ctypes.c_int, [_P, _P, _SZ, _SZP]),
        "edpc_model_set_state": (ctypes.c_int, [_P, _P, _SZ]),
        "edpc_rc_encode": (ctypes.c_int, [_P, _P, _SZ, _SZ, _P, _SZ, _U32P, _P]),
        "edpc_rc_encode_noalloc": (ctypes.c_int, [_P, _P, _SZ, _SZ, _P, _SZ, _U32P, _P]),
        "edpc_rc_decode": (ctypes.c_int, [_P, _P, _U32P, _SZ, _SZ, _SZ, _P, _P]),
        "edpc_rc_encode_host": (ctypes.c_int, [_P, _P, _SZ, _P, _SZ, _SZP]),
        "edpc_rc_decode_host": (ctypes.c_int, [_P, _P, _SZ, _SZ, _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(st: int):
    if st != EDPC_OK:
        raise EdpcError(st, lib().edpc_last_error().decode())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _np_ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def edpc_config_default(**overrides) -> edpc_config:
    c = edpc_config()
    _check(lib().edpc_config_default(ctypes.byref(c)))
    for k, v in overrides.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp32": EDPC_FP32, "bf16": EDPC_BF16}[v]
        if k in ("zero_head", "autotune", "lte", "low_rank", "layerwise", "graphs"):
            bit = {"zero_head": EDPC_CFG_ZERO_HEAD, "autotune": EDPC_CFG_AUTOTUNE,
                   "lte": EDPC_CFG_NO_LTE, "low_rank": EDPC_CFG_LOW_RANK,
                   "layerwise": EDPC_CFG_LAYERWISE, "graphs": EDPC_CFG_NO_GRAPHS}[k]
            # "lte" and "graphs" name the feature; their bits switch it off
            on = (not v) if k in ("lte", "graphs") else v
            c.flags = (c.flags | bit) if on else (c.flags & ~bit)
            continue
        setattr(c, k, v)
    return c


def edpc_config_validate(cfg: edpc_config):
    _check(lib().edpc_config_validate(ctypes.byref(cfg)))


def _lens(lens) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(lens, dtype=np.uint64))


def edpc_encode_bound(cfg: edpc_config, lens) -> int:
    ln = _lens(lens)
    out = ctypes.c_size_t()
    _check(lib().edpc_encode_bound(ctypes.byref(cfg), ln.ctypes.data_as(_U64P), len(ln),
                                   ctypes.byref(out)))
    return out.value


def edpc_encode(cfg: edpc_config, d_in, lens, stream=None):
    """Compress device bytes ``d_in`` (uint8 tensor, streams concatenated);
    returns the container as a uint8 device tensor."""
    import torch
    ln = _lens(lens)
    cap = edpc_encode_bound(cfg, ln)
    out = torch.empty(cap, dtype=torch.uint8, device=d_in.device)
    n = ctypes.c_size_t()
    _check(lib().edpc_encode(ctypes.byref(cfg), _dptr(d_in), ln.ctypes.data_as(_U64P), len(ln),
                             _dptr(out), cap, ctypes.byref(n), _stream(stream)))
    return out[: n.value]


def edpc_decode_info(h_in: bytes):
    """(config, lens, header_len, decoded_len) from container bytes in host memory."""
    buf = np.frombuffer(bytes(h_in), dtype=np.uint8)
    cfg = edpc_config()
    n = ctypes.c_size_t()
    hl = ctypes.c_size_t()
    dl = ctypes.c_size_t()
    _check(lib().edpc_decode_info(_np_ptr(buf), len(buf), ctypes.byref(cfg), ctypes.byref(n),
                                  None, 0, ctypes.byref(hl), ctypes.byref(dl)))
    lens = np.zeros(n.value, dtype=np.uint64)
    _check(lib().edpc_decode_info(_np_ptr(buf), len(buf), None, None,
                                  lens.ctypes.data_as(_U64P), len(lens), None, None))
    return cfg, lens.astype(np.int64), hl.value, dl.value


def _header_bytes(container) -> bytes:
    head = container[:16].cpu().numpy().tobytes()
    hl = int.from_bytes(head[8:12], "little")
    return container[: min(hl, container.numel())].cpu().numpy().tobytes()


def edpc_decode(container, stream=None):
    """Decompress a container held in a uint8 device tensor."""
    import torch
    _, lens, _, total = edpc_decode_info(_header_bytes(container))
    out = torch.empty(max(total, 1), dtype=torch.uint8, device=container.device)
    n = ctypes.c_size_t()
    _check(lib().edpc_decode(_dptr(container), container.numel(), _dptr(out), out.numel(),
                             ctypes.byref(n), _stream(stream)))
    return out[: n.value], lens


def _host_ptr(a):
    """Pointer of a host buffer: a numpy array or a (pinned) CPU torch tensor."""
    if isinstance(a, np.ndarray):
        return ctypes.c_void_p(a.ctypes.data)
    return ctypes.c_void_p(a.data_ptr())


def edpc_encode_host(cfg: edpc_config, h_in, lens, chunk_steps: int, out=None, stream=None):
    """Compress streams held in host memory (numpy uint8 array or CPU torch
    tensor, pinned for speed); returns the container as numpy bytes, or its
    length if ``out`` (a host buffer of at least edpc_encode_bound bytes) is
    given."""
    ln = _lens(lens)
    cap = edpc_encode_bound(cfg, ln)
    buf = np.empty(cap, dtype=np.uint8) if out is None else out
    n = ctypes.c_size_t()
    _check(lib().edpc_encode_host(ctypes.byref(cfg), _host_ptr(h_in), ln.ctypes.data_as(_U64P),
                                  len(ln), _host_ptr(buf), cap, ctypes.byref(n), chunk_steps,
                                  _stream(stream)))
    return buf[: n.value] if out is None else n.value


def edpc_decode_host(container, chunk_steps: int, out=None, stream=None):
    """Decompress a container held in host memory; returns the decoded bytes
    (numpy) or their count if ``out`` is given."""
    c = np.ascontiguousarray(np.frombuffer(bytes(container), dtype=np.uint8)) \
        if not hasattr(container, "data_ptr") and not isinstance(container, np.ndarray) else container
    head = bytes(np.asarray(c[:16] if isinstance(c, np.ndarray) else c[:16].numpy()))
    hl = int.from_bytes(head[8:12], "little")
    hdr = bytes(np.asarray(c[:hl] if isinstance(c, np.ndarray) else c[:hl].numpy()))
    _, _, _, total = edpc_decode_info(hdr)
    buf = np.empty(max(total, 1), dtype=np.uint8) if out is None else out
    n = ctypes.c_size_t()
    size = c.size if isinstance(c, np.ndarray) else c.numel()
    _check(lib().edpc_decode_host(_host_ptr(c), size, _host_ptr(buf), total, ctypes.byref(n),
                                  chunk_steps, _stream(stream)))
    return buf[: n.value] if out is None else n.value


class Session:
    """edpc_encoder_begin / edpc_decoder_begin ... edpc_session_destroy."""

    def __init__(self, handle, keep):
        self.h = handle
        self._keep = keep  # tensors the session reads until destroyed

    def edpc_session_run(self, n_steps: int) -> int:
        done = ctypes.c_uint64()
        _check(lib().edpc_session_run(self.h, n_steps, ctypes.byref(done)))
        return done.value

    def edpc_session_progress(self):
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().edpc_session_progress(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def edpc_encoder_finish(self, bound: int):
        import torch
        dev = self._keep[0].device
        out = torch.empty(bound, dtype=torch.uint8, device=dev)
        n = ctypes.c_size_t()
        _check(lib().edpc_encoder_finish(self.h, _dptr(out), bound, ctypes.byref(n)))
        return out[: n.value]

    def edpc_decoder_finish(self) -> int:
        n = ctypes.c_size_t()
        _check(lib().edpc_decoder_finish(self.h, ctypes.byref(n)))
        return n.value

    def edpc_session_time_kernels(self, n_steps: int) -> dict:
        """{class name: (total ms, launches)} over the next n_steps."""
        ms = np.zeros(KCLASS_COUNT, dtype=np.float32)
        la = np.zeros(KCLASS_COUNT, dtype=np.uint32)
        _check(lib().edpc_session_time_kernels(self.h, n_steps, _np_ptr(ms), _np_ptr(la)))
        return {lib().edpc_kclass_name(c).decode(): (float(ms[c]), int(la[c]))
                for c in range(KCLASS_COUNT)}

    def edpc_session_destroy(self):
        if self.h:
            lib().edpc_session_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.edpc_session_destroy()
        except Exception:
            pass


def edpc_encoder_begin(cfg: edpc_config, d_in, lens, stream=None) -> Session:
    ln = _lens(lens)
    h = ctypes.c_void_p()
    _check(lib().edpc_encoder_begin(ctypes.byref(cfg), _dptr(d_in), ln.ctypes.data_as(_U64P),
                                    len(ln), _stream(stream), ctypes.byref(h)))
    return Session(h, (d_in,))


def edpc_decoder_begin(container, d_out, stream=None) -> Session:
    h = ctypes.c_void_p()
    _check(lib().edpc_decoder_begin(_dptr(container), container.numel(), _dptr(d_out),
                                    d_out.numel(), _stream(stream), ctypes.byref(h)))
    return Session(h, (container, d_out))


class Model:
    """edpc_model_create ... edpc_model_destroy, with tensor access by name."""

    def __init__(self, cfg: edpc_config, n_slots: int, max_rows: int, kernel_id: int = 0):
        self.cfg = cfg
        h = ctypes.c_void_p()
        if kernel_id:
            _check(lib().edpc_model_create_with_kernels(ctypes.byref(cfg), n_slots, max_rows,
                                                        kernel_id, ctypes.byref(h)))
        else:
            _check(lib().edpc_model_create(ctypes.byref(cfg), n_slots, max_rows, ctypes.byref(h)))
        self.h = h
        self.n_slots = n_slots
        n = ctypes.c_size_t()
        _check(lib().edpc_model_tensor_count(self.h, ctypes.byref(n)))
        self.names, self.numel = [], []
        buf = ctypes.create_string_buffer(64)
        for i in range(n.value):
            ne = ctypes.c_size_t()
            _check(lib().edpc_model_tensor_info(self.h, i, buf, 64, ctypes.byref(ne)))
            self.names.append(buf.value.decode())
            self.numel.append(ne.value)

    def edpc_model_destroy(self):
        if self.h:
            lib().edpc_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.edpc_model_destroy()
        except Exception:
            pass

    def edpc_model_step(self, ctx, target, slots, probs=None, cum=None, loss=None, flags=0,
                        stream=None):
        sl = np.ascontiguousarray(np.asarray(slots, dtype=np.uint32))
        _check(lib().edpc_model_step(
            self.h, _dptr(ctx), _dptr(target) if target is not None else None,
            sl.ctypes.data_as(_U32P), len(sl),
            _dptr(probs) if probs is not None else None,
            _dptr(cum) if cum is not None else None,
            _dptr(loss) if loss is not None else None, flags, _stream(stream)))

    def index(self, name: str) -> int:
        return self.names.index(name)

    def edpc_model_read(self, name: str, kind: int = EDPC_KIND_PARAM) -> np.ndarray:
        i = self.index(name)
        out = np.empty(self.numel[i], dtype=np.float32)
        _check(lib().edpc_model_read(self.h, kind, i, _np_ptr(out), out.size))
        return out

    def edpc_model_write(self, name: str, values, kind: int = EDPC_KIND_PARAM):
        i = self.index(name)
        a = np.ascontiguousarray(np.asarray(values, dtype=np.float32).reshape(-1))
        _check(lib().edpc_model_write(self.h, kind, i, _np_ptr(a), a.size))

    def edpc_model_read_device(self, name: str, out, kind: int = EDPC_KIND_PARAM, stream=None):
        i = self.index(name)
        _check(lib().edpc_model_read_device(self.h, kind, i, _dptr(out), out.numel(),
                                            _stream(stream)))
        return out

    def edpc_model_write_device(self, name: str, src, kind: int = EDPC_KIND_PARAM, stream=None):
        i = self.index(name)
        _check(lib().edpc_model_write_device(self.h, kind, i, _dptr(src), src.numel(),
                                             _stream(stream)))

    def edpc_model_get_step(self) -> int:
        t = ctypes.c_uint64()
        _check(lib().edpc_model_get_step(self.h, ctypes.byref(t)))
        return t.value

    def edpc_model_set_step(self, tau: int):
        _check(lib().edpc_model_set_step(self.h, tau))

    def edpc_model_activation(self, block: int, out, stream=None):
        """FP32 input of refinement block `block` of the last step into the
        device tensor `out` [rows, context * embed]."""
        _check(lib().edpc_model_activation(self.h, block, _dptr(out), out.numel(),
                                           _stream(stream)))
        return out

    def edpc_model_kernel_id(self) -> int:
        k = ctypes.c_uint64()
        _check(lib().edpc_model_kernel_id(self.h, ctypes.byref(k)))
        return k.value

    def edpc_model_get_state(self) -> bytes:
        """The whole training state as one blob (layout in include/edpc.h)."""
        n = ctypes.c_size_t()
        st = lib().edpc_model_get_state(self.h, None, 0, ctypes.byref(n))
        if st != -3:
            _check(st)
        buf = np.empty(n.value, dtype=np.uint8)
        _check(lib().edpc_model_get_state(self.h, _np_ptr(buf), buf.size, ctypes.byref(n)))
        return buf.tobytes()

    def edpc_model_set_state(self, blob: bytes):
        buf = np.frombuffer(bytes(blob), dtype=np.uint8)
        _check(lib().edpc_model_set_state(self.h, _np_ptr(buf), buf.size))


def edpc_model_create(cfg: edpc_config, n_slots: int, max_rows: int) -> Model:
    return Model(cfg, n_slots, max_rows)


def edpc_rc_encode(d_cum, d_sym, cap_per_stream: int, stream=None):
    """Range-code [n_steps, n_streams] symbols with [n_steps, n_streams, 257]
    u32 CDFs; returns (payload tensor [n_streams, cap], lengths)."""
    import torch
    n_steps, n_streams = d_sym.shape
    out = torch.zeros((n_streams, cap_per_stream), dtype=torch.uint8, device=d_sym.device)
    lens = np.zeros(n_streams, dtype=np.uint32)
    _check(lib().edpc_rc_encode(_dptr(d_cum), _dptr(d_sym), n_steps, n_streams, _dptr(out),
                                cap_per_stream, lens.ctypes.data_as(_U32P), _stream(stream)))
    return out, lens


def edpc_mutual_info(d_z, d_y, v: int = 3, counts=None, eps=None, stream=None) -> float:
    """Kraskov estimate of I(Z; Y) in nats from FP32 device tensors [c, dz]
    and [c, dy] (rows are samples)."""
    c, dz = d_z.shape
    c2, dy = d_y.shape
    if c != c2:
        raise ValueError("z and y need the same number of samples")
    mi = ctypes.c_double()
    _check(lib().edpc_mutual_info(_dptr(d_z.contiguous()), dz, _dptr(d_y.contiguous()), dy, c, v,
                                  ctypes.byref(mi), _dptr(counts) if counts is not None else None,
                                  _dptr(eps) if eps is not None else None, _stream(stream)))
    return mi.value


def block_mutual_info(model, d_ctx, d_target, slots, v: int = 3):
    """I(S; S + X^(k)) of every refinement block on one batch (Sec. 3.1.1):
    runs a forward step on the contexts, then estimates the mutual
    information between each block's input (the skip connection S) and its
    output.  Returns a list with one value (nats) per block."""
    import torch
    model.edpc_model_step(d_ctx, d_target, slots)
    rows = len(np.asarray(slots))
    F = model.cfg.context * model.cfg.embed
    acts = [model.edpc_model_activation(j, torch.empty((rows, F), dtype=torch.float32,
                                                       device=d_ctx.device))
            for j in range(model.cfg.blocks + 1)]
    return [edpc_mutual_info(acts[j], acts[j + 1], v) for j in range(model.cfg.blocks)]


def edpc_rc_encode_noalloc(d_cum, d_sym, out, stream=None):
    """edpc_rc_encode into a caller-provided payload tensor ``out``
    [n_streams, cap] (uint8); the library allocates nothing.  Returns the
    lengths."""
    n_steps, n_streams = d_sym.shape
    lens = np.zeros(n_streams, dtype=np.uint32)
    _check(lib().edpc_rc_encode_noalloc(_dptr(d_cum), _dptr(d_sym), n_steps, n_streams,
                                        _dptr(out), out.shape[1], lens.ctypes.data_as(_U32P),
                                        _stream(stream)))
    return lens


def edpc_rc_decode(d_cum, d_payload, lens, stream=None):
    import torch
    n_steps, n_streams = d_cum.shape[0], d_cum.shape[1]
    sym = torch.empty((n_steps, n_streams), dtype=torch.uint8, device=d_cum.device)
    ln = np.ascontiguousarray(np.asarray(lens, dtype=np.uint32))
    _check(lib().edpc_rc_decode(_dptr(d_cum), _dptr(d_payload), ln.ctypes.data_as(_U32P),
                                d_payload.shape[1], n_steps, n_streams, _dptr(sym),
                                _stream(stream)))
    return sym


def edpc_rc_encode_host(cum: np.ndarray, sym: np.ndarray) -> bytes:
    cum = np.ascontiguousarray(cum, dtype=np.uint32)
    sym = np.ascontiguousarray(sym, dtype=np.uint8)
    cap = 2 * len(sym) + 2
    out = np.zeros(cap, dtype=np.uint8)
    n = ctypes.c_size_t()
    _check(lib().edpc_rc_encode_host(_np_ptr(cum), _np_ptr(sym), len(sym), _np_ptr(out), cap,
                                     ctypes.byref(n)))
    return out[: n.value].tobytes()


def edpc_rc_decode_host(cum: np.ndarray, payload: bytes, n_steps: int) -> np.ndarray:
    cum = np.ascontiguousarray(cum, dtype=np.uint32)
    buf = np.frombuffer(bytes(payload) + b"\0", dtype=np.uint8)
    sym = np.zeros(max(n_steps, 1), dtype=np.uint8)
    _check(lib().edpc_rc_decode_host(_np_ptr(cum), _np_ptr(buf), len(payload), n_steps,
                                     _np_ptr(sym)))
    return sym[:n_steps]


def _step_function():
    import torch

    class StepFunction(torch.autograd.Function):
        """Mean cross entropy of one model step (Eq. 2) as an autograd op.

        ``StepFunction.apply(model, ctx, target, slots, *tensors)`` where
        ``tensors`` are FP32 device tensors holding every model tensor in
        ``model.names`` order (the FDM "U" last, all slots).  Forward loads
        them into the model and runs the forward kernels; backward runs the
        library's hand-written adjoint kernels (no update) and returns their
        gradients scaled by the incoming gradient.
        """

        @staticmethod
        def forward(fctx, model, d_ctx, d_tgt, slots, *tensors):
            for name, t in zip(model.names, tensors):
                model.edpc_model_write_device(name, t.detach().contiguous())
            loss = torch.empty(1, dtype=torch.float32, device=d_ctx.device)
            model.edpc_model_step(d_ctx, d_tgt, slots, loss=loss,
                                  flags=EDPC_STEP_BACKWARD | EDPC_STEP_KEEP_FDM_GRAD)
            fctx.model = model
            fctx.shapes = [t.shape for t in tensors]
            return loss[0]

        @staticmethod
        def backward(fctx, g):
            m = fctx.model
            grads = []
            for name, shp in zip(m.names, fctx.shapes):
                out = torch.empty(shp, dtype=torch.float32, device=g.device)
                m.edpc_model_read_device(name, out, kind=EDPC_KIND_GRAD)
                grads.append(out * g)
            return (None, None, None, None, *grads)

    return StepFunction


def __getattr__(name):
    if name == "StepFunction":
        return _step_function()
    raise AttributeError(name)
