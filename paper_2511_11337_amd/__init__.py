"""BOA Constrictor hot path on MI355X: a byte-level Mamba predictor driving a
range coder over many independent byte streams, behind the C ABI of
``libboa.so`` (include/boa.h).

This module only marshals arguments; every step of compression,
decompression and training runs in the library's gfx950 kernels.  PyTorch is
used for device buffers and streams.  There is no CPU fallback: if
``libboa.so`` is missing the calls raise.

    m = Model(Config(d_model=256, n_layers=3), weights)      # float32 flat vector
    blob = compress(m, data, chunk_len=65536, dtype="f32")
    assert decompress(m, blob) == data
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib
from ._lib import BoaError, DTYPES  # noqa: F401

__all__ = ["Config", "Model", "compress", "decompress", "logits", "encode_dev", "decode_dev", "workspace_size",
           "code_tables", "decode_tables", "order2_encode", "order2_decode", "BoaError",
           "container_info", "numerics_id", "diagnostics",
           "StreamCompressor", "decompress_shards"]


@dataclass(frozen=True)
class Config:
    d_model: int = 64
    n_layers: int = 2
    d_state: int = 16
    d_conv: int = 4
    expand: int = 2
    ffn_mult: int = 0

    @staticmethod
    def of(obj) -> "Config":
        if isinstance(obj, Config):
            return obj
        keys = ("d_model", "n_layers", "d_state", "d_conv", "expand", "ffn_mult")
        if isinstance(obj, dict):
            return Config(**{k: int(obj[k]) for k in keys if k in obj})
        return Config(*(int(getattr(obj, k, 0)) for k in keys))

    def c(self) -> _lib.boa_config:
        return _lib.boa_config(self.d_model, self.n_layers, self.d_state, self.d_conv, self.expand, self.ffn_mult)

    @property
    def n_params(self) -> int:
        c = self.c()
        return int(_lib.load().boa_param_count(C.byref(c)))


def _dtype(d) -> int:
    if isinstance(d, int):
        return d
    return DTYPES[str(d).lower()]


def _stream_ptr(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


DECODE_KERNELS = {"auto": 0, "fused": 1, "steps": 2}


def _opts(dtype="f32", max_lanes=0, tile_t=0, use_graph=True, fallback=False, decode_groups=0,
          decode_kernel="auto", fused_lanes=0) -> _lib.boa_run_opts:
    o = _lib.boa_run_opts()
    o.decode_groups = int(decode_groups)
    o.decode_kernel = DECODE_KERNELS[decode_kernel] if isinstance(decode_kernel, str) else int(decode_kernel)
    o.fused_lanes = int(fused_lanes)
    o.dtype = _dtype(dtype)
    o.max_lanes = int(max_lanes)
    o.tile_t = int(tile_t)
    o.use_graph = 1 if use_graph else 2
    o.fallback = 1 if fallback else 0
    return o


class Model:
    """A predictor resident on one GPU (float32 master weights + derived copies)."""

    def __init__(self, cfg, weights: np.ndarray | None = None, device: int = 0, _handle=None):
        lib = _lib.load()
        self.cfg = Config.of(cfg)
        if _handle is not None:
            self._h = _handle
        else:
            w = np.ascontiguousarray(weights, dtype=np.float32)
            h = C.c_void_p()
            c = self.cfg.c()
            _lib.check(lib.boa_model_create(C.byref(c), w.ctypes.data, w.size, int(device), C.byref(h)))
            self._h = h
        self.device = device

    @classmethod
    def load(cls, path: str, device: int = 0) -> "Model":
        lib = _lib.load()
        h = C.c_void_p()
        _lib.check(lib.boa_model_load(path.encode(), int(device), C.byref(h)))
        c = _lib.boa_config()
        _lib.check(lib.boa_model_config(h, C.byref(c)))
        return cls(Config(c.d_model, c.n_layers, c.d_state, c.d_conv, c.expand, c.ffn_mult), device=device,
                   _handle=h)

    def save(self, path: str) -> None:
        _lib.check(_lib.load().boa_model_save(self._h, path.encode()))

    @property
    def handle(self):
        return self._h

    @property
    def n_params(self) -> int:
        return self.cfg.n_params

    @property
    def fingerprint(self) -> int:
        v = C.c_uint64()
        _lib.check(_lib.load().boa_model_fingerprint(self._h, C.byref(v)))
        return int(v.value)

    def get_weights(self) -> np.ndarray:
        w = np.empty(self.n_params, dtype=np.float32)
        _lib.check(_lib.load().boa_model_get_weights(self._h, w.ctypes.data, w.size))
        return w

    def set_weights(self, w: np.ndarray) -> None:
        w = np.ascontiguousarray(w, dtype=np.float32)
        _lib.check(_lib.load().boa_model_set_weights(self._h, w.ctypes.data, w.size))

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.load().boa_model_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _chunk_lens(n: int, chunk_lens=None, chunk_len: int = 65536) -> np.ndarray:
    if chunk_lens is not None:
        cl = np.asarray(chunk_lens, dtype=np.uint64)
        if int(cl.sum()) != n:
            raise ValueError("chunk lengths do not sum to the data length")
        return cl
    lib = _lib.load()
    k = C.c_uint64()
    _lib.check(lib.boa_split_fixed(n, int(chunk_len), None, 0, C.byref(k)))
    cl = np.zeros(k.value, dtype=np.uint64)
    _lib.check(lib.boa_split_fixed(n, int(chunk_len), cl.ctypes.data_as(_lib.U64P), cl.size, C.byref(k)))
    return cl


def compress(model: Model, data, chunk_lens=None, chunk_len: int = 65536, dtype="f32", max_lanes: int = 0,
             tile_t: int = 0, fallback: bool = False) -> bytes:
    """compress(model, bytes) -> .boa container (host memory in, host memory out)."""
    lib = _lib.load()
    buf = np.frombuffer(bytes(data), dtype=np.uint8) if not isinstance(data, np.ndarray) else \
        np.ascontiguousarray(data, dtype=np.uint8)
    cl = _chunk_lens(buf.size, chunk_lens, chunk_len)
    out = C.c_void_p()
    out_len = C.c_uint64()
    o = _opts(dtype, max_lanes, tile_t, True, fallback)
    _lib.check(lib.boa_compress(model.handle, buf.ctypes.data if buf.size else None,
                                cl.ctypes.data_as(_lib.U64P), cl.size, C.byref(o), C.byref(out), C.byref(out_len)))
    try:
        return C.string_at(out, out_len.value)
    finally:
        lib.boa_free(out)


def last_chunk_stats(n_chunks: int):
    """(payload bytes, coder id) per chunk of the last compress on this thread."""
    lib = _lib.load()
    pb = np.zeros(n_chunks, dtype=np.uint64)
    cd = np.zeros(n_chunks, dtype=np.uint32)
    _lib.check(lib.boa_last_chunk_stats(pb.ctypes.data_as(_lib.U64P), cd.ctypes.data_as(C.POINTER(C.c_uint32)),
                                        n_chunks))
    return pb, cd


def decompress(model: Model, blob: bytes, max_lanes: int = 0, use_graph: bool = True,
               decode_kernel="auto", fused_lanes: int = 0) -> bytes:
    lib = _lib.load()
    b = np.frombuffer(blob, dtype=np.uint8)
    out = C.c_void_p()
    out_len = C.c_uint64()
    o = _opts(0, max_lanes, 0, use_graph, decode_kernel=decode_kernel, fused_lanes=fused_lanes)
    _lib.check(lib.boa_decompress(model.handle, b.ctypes.data, b.size, C.byref(o), C.byref(out), C.byref(out_len)))
    try:
        return C.string_at(out, out_len.value) if out_len.value else b""
    finally:
        lib.boa_free(out)


def container_info(blob: bytes) -> dict:
    lib = _lib.load()
    b = np.frombuffer(blob, dtype=np.uint8)
    n, t, f, nid = C.c_uint64(), C.c_uint64(), C.c_uint64(), C.c_uint32()
    _lib.check(lib.boa_container_info(b.ctypes.data, b.size, C.byref(n), C.byref(t), C.byref(f), C.byref(nid)))
    return {"n_chunks": n.value, "total_len": t.value, "fingerprint": f.value, "numerics_id": nid.value}


def numerics_id(dtype="f32") -> int:
    return int(_lib.load().boa_numerics_id(_dtype(dtype)))


# --------------------------------------------------------------------------- device level
def logits(model: Model, seqs, dtype="f32", tile_t: int = 0, want_probs=False, want_tables=False, stream=None):
    """Teacher-forced logits [B, T-1, 256] of device uint8 sequences [B, T]."""
    import torch
    assert seqs.is_cuda and seqs.dtype == torch.uint8 and seqs.dim() == 2
    seqs = seqs.contiguous()
    B, T = seqs.shape
    dev = seqs.device
    lg = torch.empty((B, max(T - 1, 0), 256), dtype=torch.float32, device=dev)
    pr = torch.empty_like(lg) if want_probs else None
    tb = torch.empty((B, max(T - 1, 0), 256), dtype=torch.int16, device=dev) if want_tables else None
    _lib.check(_lib.load().boa_logits_dev(model.handle, seqs.data_ptr(), B, T, _dtype(dtype), int(tile_t),
                                          lg.data_ptr(), pr.data_ptr() if pr is not None else None,
                                          tb.data_ptr() if tb is not None else None, _stream_ptr(stream)))
    out = [lg]
    if want_probs:
        out.append(pr)
    if want_tables:
        out.append(tb)                      # int16 storage of the uint16 histogram
    return out[0] if len(out) == 1 else tuple(out)


def diagnostics(model: Model, seqs, dtype="f32", n_bins: int = 10, tile_t: int = 0, stream=None):
    """Predictor diagnostics of device uint8 sequences [B, T] (teacher-forced,
    the coder's probabilities): confusion [256, 256] ([true, predicted]),
    rank histogram [256] (Top-k = ranks < k), reliability bins [n_bins, 3]
    (count, correct, sum of conf * 2^32), and Top-1/5/10 and ECE from them."""
    import torch
    assert seqs.is_cuda and seqs.dtype == torch.uint8 and seqs.dim() == 2
    seqs = seqs.contiguous()
    B, T = seqs.shape
    dev = seqs.device
    conf = torch.empty((256, 256), dtype=torch.int32, device=dev)
    rank = torch.empty(256, dtype=torch.int32, device=dev)
    cal = torch.empty((max(int(n_bins), 1), 3), dtype=torch.int64, device=dev)
    _lib.check(_lib.load().boa_diagnostics_dev(model.handle, seqs.data_ptr(), B, T, _dtype(dtype), int(tile_t),
                                               int(n_bins), conf.data_ptr(), rank.data_ptr(), cal.data_ptr(),
                                               _stream_ptr(stream)))
    c = conf.cpu().numpy().view(np.uint32).astype(np.int64)
    h32 = np.ascontiguousarray(rank.cpu().numpy().view(np.uint32))
    k64 = np.ascontiguousarray(cal.cpu().numpy().view(np.uint64))
    topk = np.zeros(256, dtype=np.float64)
    ece, n = C.c_double(), C.c_uint64()
    _lib.check(_lib.load().boa_diagnostics_summary(h32.ctypes.data, k64.ctypes.data, int(n_bins), topk.ctypes.data,
                                                   C.byref(ece), C.byref(n)))
    return {"confusion": c, "rank_hist": h32.astype(np.int64), "calibration": k64.astype(np.int64),
            "positions": int(n.value), "topk": topk, "top1": float(topk[0]), "top5": float(topk[4]),
            "top10": float(topk[9]), "ece": float(ece.value)}


class StreamCompressor:
    """Streaming compress (host bytes in, shards out): push() bytes as they
    arrive; every lanes x chunk_len bytes become one shard (a .boa container)
    compressed by one of `workers` library threads while pushing continues;
    shards() yields them in input order.  finish() submits the partial last
    group."""

    def __init__(self, model: Model, chunk_len: int = 65536, lanes: int = 256, workers: int = 2, dtype="f32",
                 max_lanes: int = 0, tile_t: int = 0, fallback: bool = False):
        self._lib = _lib.load()
        self._model = model                       # the model must outlive the stream
        self._opts = _opts(dtype, max_lanes, tile_t, True, fallback)
        h = C.c_void_p()
        _lib.check(self._lib.boa_stream_open(model.handle, int(chunk_len), int(lanes), int(workers),
                                             C.byref(self._opts), C.byref(h)))
        self._h = h

    def push(self, data):
        buf = np.frombuffer(bytes(data), dtype=np.uint8) if not isinstance(data, np.ndarray) else \
            np.ascontiguousarray(data, dtype=np.uint8)
        _lib.check(self._lib.boa_stream_push(self._h, buf.ctypes.data if buf.size else None, buf.size))

    def finish(self):
        _lib.check(self._lib.boa_stream_finish(self._h))

    def next_shard(self, wait: bool = True):
        """The next shard in input order, or None (none ready / none in flight)."""
        out = C.c_void_p()
        n = C.c_uint64()
        _lib.check(self._lib.boa_stream_next_shard(self._h, 1 if wait else 0, C.byref(out), C.byref(n)))
        if not out.value:
            return None
        try:
            return C.string_at(out, n.value)
        finally:
            self._lib.boa_free(out)

    def shards(self, wait: bool = True):
        while True:
            sh = self.next_shard(wait)
            if sh is None:
                return
            yield sh

    def close(self):
        if self._h is not None and self._h.value:
            self._lib.boa_stream_close(self._h)
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def decompress_shards(model: Model, shards, **kw) -> bytes:
    """The bytes of a stream from its shards, in order."""
    return b"".join(decompress(model, sh, **kw) for sh in shards)


def _layout(chunk_lens):
    """(lengths, chunk offsets, payload offsets, payload capacities) from the library."""
    cl = np.ascontiguousarray(chunk_lens, dtype=np.uint64)
    off, poff, cap = (np.zeros(cl.size, dtype=np.uint64) for _ in range(3))
    tot = C.c_uint64()
    _lib.check(_lib.load().boa_payload_layout(cl.ctypes.data_as(_lib.U64P), cl.size, off.ctypes.data_as(_lib.U64P),
                                              poff.ctypes.data_as(_lib.U64P), cap.ctypes.data_as(_lib.U64P),
                                              C.byref(tot)))
    return cl, off, poff, cap


WS_ENCODE, WS_DECODE = 0, 1


def workspace_size(model: Model, chunk_lens, mode: str, dtype="f32", max_lanes=0, tile_t=0, decode_kernel="auto",
                   fused_lanes=0) -> int:
    """Device bytes encode_dev (mode "encode") or decode_dev ("decode") needs as
    its workspace for these chunks and options."""
    cl = np.ascontiguousarray(chunk_lens, dtype=np.uint64)
    o = _opts(dtype, max_lanes, tile_t, decode_kernel=decode_kernel, fused_lanes=fused_lanes)
    b = C.c_uint64()
    _lib.check(_lib.load().boa_workspace_size(model.handle, cl.ctypes.data_as(_lib.U64P), cl.size, C.byref(o),
                                              WS_ENCODE if mode == "encode" else WS_DECODE, C.byref(b)))
    return int(b.value)


def plan_lanes(chunk_lens, max_lanes=0) -> int:
    """Lanes the library schedules these chunks on (max_lanes 0: its own
    choice, see boa_plan_lanes)."""
    cl = np.ascontiguousarray(chunk_lens, dtype=np.uint64)
    n = C.c_uint32()
    _lib.check(_lib.load().boa_plan_lanes(cl.ctypes.data_as(_lib.U64P), cl.size, int(max_lanes), C.byref(n)))
    return int(n.value)


def _ws(workspace):
    if workspace is None:
        return None, 0
    return workspace.data_ptr(), workspace.numel() * workspace.element_size()


def encode_dev(model: Model, d_data, chunk_lens, dtype="f32", max_lanes=0, tile_t=0, ideal=True, stream=None,
               workspace=None):
    """Encode device-resident chunks.  Returns (payload, pay_off, pay_len, ideal_bits)
    with payload a device uint8 tensor, pay_off a host uint64 array, pay_len a
    device int32 tensor (0xFFFFFFFF = overflow) and ideal_bits a device float64
    tensor (or None).  workspace: optional device tensor of at least
    workspace_size(model, chunk_lens, "encode", ...) bytes (else the library
    allocates for the call)."""
    import torch
    cl, off, poff, cap = _layout(chunk_lens)
    dev = d_data.device
    payload = torch.empty(int(cap.sum()) if cap.size else 1, dtype=torch.uint8, device=dev)
    pay_len = torch.empty(max(cl.size, 1), dtype=torch.int32, device=dev)
    ib = torch.empty(max(cl.size, 1), dtype=torch.float64, device=dev) if ideal else None
    o = _opts(dtype, max_lanes, tile_t)
    wp, wn = _ws(workspace)
    _lib.check(_lib.load().boa_encode_dev(
        model.handle, d_data.data_ptr(), off.ctypes.data_as(_lib.U64P), cl.ctypes.data_as(_lib.U64P), cl.size,
        C.byref(o), payload.data_ptr(), poff.ctypes.data_as(_lib.U64P), cap.ctypes.data_as(_lib.U64P),
        pay_len.data_ptr(), ib.data_ptr() if ib is not None else None, wp, wn, _stream_ptr(stream)))
    return payload, poff.astype(np.int64), pay_len, ib


def decode_dev(model: Model, payload, pay_off, pay_len, first, chunk_lens, dtype="f32", max_lanes=0,
               use_graph=True, out=None, stream=None, decode_groups=0, decode_kernel="auto", fused_lanes=0,
               workspace=None):
    """Decode device payloads into a device uint8 tensor of the concatenated chunks.

    decode_kernel: "fused" runs every step of a lane in one persistent kernel
    (fused_lanes lanes per workgroup, 0 = auto), "steps" launches the per-step
    kernel chain (captured step graph when use_graph), "auto" picks fused.
    workspace: optional device tensor of at least workspace_size(model,
    chunk_lens, "decode", ...) bytes."""
    import torch
    cl, off, _, _ = _layout(chunk_lens)
    pl = np.ascontiguousarray(pay_len, dtype=np.uint64)
    po = np.ascontiguousarray(pay_off, dtype=np.uint64)
    fb = np.ascontiguousarray(first, dtype=np.uint8)
    if out is None:
        out = torch.empty(max(int(cl.sum()), 1), dtype=torch.uint8, device=payload.device)
    o = _opts(dtype, max_lanes, 0, use_graph, decode_groups=decode_groups, decode_kernel=decode_kernel,
              fused_lanes=fused_lanes)
    wp, wn = _ws(workspace)
    _lib.check(_lib.load().boa_decode_dev(
        model.handle, payload.data_ptr(), po.ctypes.data_as(_lib.U64P), pl.ctypes.data_as(_lib.U64P),
        fb.ctypes.data, off.ctypes.data_as(_lib.U64P), cl.ctypes.data_as(_lib.U64P), cl.size, C.byref(o),
        out.data_ptr(), wp, wn, _stream_ptr(stream)))
    return out


class QModel:
    """The integer-only predictor converted from a Model's current weights
    (boa_qmodel_create); its tables and coded bytes do not depend on the device."""

    def __init__(self, model: Model):
        h = C.c_void_p()
        _lib.check(_lib.load().boa_qmodel_create(model.handle, C.byref(h)))
        self._h = h
        self.cfg = model.cfg

    @property
    def handle(self):
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            _lib.load().boa_qmodel_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def int_tables(q: QModel, d_seqs, stream=None):
    """(tables uint16 viewed as int16, logits int32 Q12), both [B, T-1, 256] on
    the device, for device sequences d_seqs uint8 [B, T]."""
    import torch
    B, T = d_seqs.shape
    tb = torch.empty((B, max(T - 1, 0), 256), dtype=torch.int16, device=d_seqs.device)
    lg = torch.empty((B, max(T - 1, 0), 256), dtype=torch.int32, device=d_seqs.device)
    _lib.check(_lib.load().boa_int_tables_dev(q.handle, d_seqs.data_ptr(), B, T, tb.data_ptr(), lg.data_ptr(),
                                              _stream_ptr(stream)))
    return tb, lg


def int_encode_dev(q: QModel, d_data, chunk_lens, stream=None):
    """Encode device-resident chunks with the integer pipeline: (payload,
    pay_off host int64, pay_len device int32)."""
    import torch
    cl, off, poff, cap = _layout(chunk_lens)
    dev = d_data.device
    payload = torch.empty(int(cap.sum()) if cap.size else 1, dtype=torch.uint8, device=dev)
    pay_len = torch.empty(max(cl.size, 1), dtype=torch.int32, device=dev)
    _lib.check(_lib.load().boa_int_encode_dev(
        q.handle, d_data.data_ptr(), off.ctypes.data_as(_lib.U64P), cl.ctypes.data_as(_lib.U64P), cl.size,
        payload.data_ptr(), poff.ctypes.data_as(_lib.U64P), cap.ctypes.data_as(_lib.U64P), pay_len.data_ptr(),
        _stream_ptr(stream)))
    return payload, poff.astype(np.int64), pay_len


def int_decode_dev(q: QModel, payload, pay_off, pay_len, first, chunk_lens, stream=None):
    """Decode what int_encode_dev wrote into a device uint8 tensor of the
    concatenated chunks."""
    import torch
    cl, off, _, _ = _layout(chunk_lens)
    pl = np.ascontiguousarray(pay_len, dtype=np.uint64)
    po = np.ascontiguousarray(pay_off, dtype=np.uint64)
    fb = np.ascontiguousarray(first, dtype=np.uint8)
    out = torch.empty(max(int(cl.sum()), 1), dtype=torch.uint8, device=payload.device)
    _lib.check(_lib.load().boa_int_decode_dev(
        q.handle, payload.data_ptr(), po.ctypes.data_as(_lib.U64P), pl.ctypes.data_as(_lib.U64P), fb.ctypes.data,
        off.ctypes.data_as(_lib.U64P), cl.ctypes.data_as(_lib.U64P), cl.size, out.data_ptr(), _stream_ptr(stream)))
    return out


def code_tables(sym, freq, nsym, stream=None):
    """Range-code explicit integer tables on the GPU.  sym: device uint8 [S];
    freq: device int16/uint16 [S, 256]; nsym: per-lane symbol counts.
    Returns (payload device uint8, pay_off np.uint64, pay_len device int32)."""
    import torch
    ns = np.asarray(nsym, dtype=np.uint64)
    cap = 4 * ns + 64
    poff = np.zeros(ns.size, dtype=np.uint64)
    if ns.size:
        poff[1:] = np.cumsum(cap)[:-1]
    payload = torch.empty(max(int(cap.sum()), 1), dtype=torch.uint8, device=sym.device)
    pay_len = torch.empty(max(ns.size, 1), dtype=torch.int32, device=sym.device)
    _lib.check(_lib.load().boa_code_tables_dev(
        sym.data_ptr(), freq.data_ptr(), ns.ctypes.data_as(_lib.U64P), ns.size, payload.data_ptr(),
        poff.ctypes.data_as(_lib.U64P), cap.ctypes.data_as(_lib.U64P), pay_len.data_ptr(), _stream_ptr(stream)))
    return payload, poff.astype(np.int64), pay_len


def decode_tables(payload, pay_off, pay_len, freq, nsym, stream=None):
    import torch
    ns = np.asarray(nsym, dtype=np.uint64)
    po = np.asarray(pay_off, dtype=np.uint64)
    pl = np.asarray(pay_len, dtype=np.uint64)
    sym = torch.empty(max(int(ns.sum()), 1), dtype=torch.uint8, device=payload.device)
    _lib.check(_lib.load().boa_decode_tables_dev(
        payload.data_ptr(), po.ctypes.data_as(_lib.U64P), pl.ctypes.data_as(_lib.U64P), freq.data_ptr(),
        ns.ctypes.data_as(_lib.U64P), ns.size, sym.data_ptr(), _stream_ptr(stream)))
    return sym


def order2_encode(d_data, chunk_lens, stream=None):
    import torch
    cl, off, poff, cap = _layout(chunk_lens)
    dev = d_data.device
    payload = torch.empty(max(int(cap.sum()), 1), dtype=torch.uint8, device=dev)
    pay_len = torch.empty(max(cl.size, 1), dtype=torch.int32, device=dev)
    ib = torch.empty(max(cl.size, 1), dtype=torch.float64, device=dev)
    _lib.check(_lib.load().boa_order2_encode_dev(
        d_data.data_ptr(), off.ctypes.data_as(_lib.U64P), cl.ctypes.data_as(_lib.U64P), cl.size,
        payload.data_ptr(), poff.ctypes.data_as(_lib.U64P), cap.ctypes.data_as(_lib.U64P), pay_len.data_ptr(),
        ib.data_ptr(), _stream_ptr(stream)))
    return payload, poff.astype(np.int64), pay_len, ib


def order2_decode(payload, pay_off, pay_len, first, chunk_lens, stream=None):
    import torch
    cl, off, _, _ = _layout(chunk_lens)
    po = np.ascontiguousarray(pay_off, dtype=np.uint64)
    pl = np.ascontiguousarray(pay_len, dtype=np.uint64)
    fb = np.ascontiguousarray(first, dtype=np.uint8)
    out = torch.empty(max(int(cl.sum()), 1), dtype=torch.uint8, device=payload.device)
    _lib.check(_lib.load().boa_order2_decode_dev(
        payload.data_ptr(), po.ctypes.data_as(_lib.U64P), pl.ctypes.data_as(_lib.U64P), fb.ctypes.data,
        off.ctypes.data_as(_lib.U64P), cl.ctypes.data_as(_lib.U64P), cl.size, out.data_ptr(), _stream_ptr(stream)))
    return out
