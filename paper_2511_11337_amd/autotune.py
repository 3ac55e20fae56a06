"""Autotuner for the launch shapes that do not change the arithmetic.

The encoder's time tile (rows per launch = lanes x tile) and the decoder's
kernel (fused persistent kernel with 1, 2, 4, 8 or 16 lanes per workgroup, or the
per-step kernel chain replayed as a hipGraph or launched plainly) only change
how work is split into launches; the per-element operation sequences are fixed by the
numerics contract, so any choice produces the same bitstream (checked by the
tile- and lane-independence tests).  The tuner times the candidates on a
prefix of the real chunks with the library's own HIP-event kernel timer off,
using wall time around device-level calls, and caches the winner per
(model shape, dtype, device, lane count) in a JSON file.  Shapes tuned ahead
of time for a device ship in tuned.json beside this module and are used
without a sweep (use_table=False sweeps anyway).
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

CACHE = os.path.join(os.path.expanduser("~"), ".cache", "boa_autotune.json")
TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")
TILES = (64, 128, 256, 512, 1024, 2048)
FUSED_LANES = (1, 2, 4, 8, 16)
MAX_TILE_ROWS = 1 << 21          # lanes x tile rows per encoder launch (~20 GiB of activations at d_model 256)


def _key(model, dtype, lanes):
    """Table / cache key: the device by ISA and compute-unit count (its
    marketing name depends on the host's id tables), the model shape, the
    dtype and the lane count rounded up to a power of two."""
    import torch
    p = torch.cuda.get_device_properties(0)
    dev = f"{getattr(p, 'gcnArchName', p.name).split(':')[0]}x{p.multi_processor_count}"
    c = model.cfg
    return f"v3|{dev}|d{c.d_model}|l{c.n_layers}|{dtype}|lanes{1 << max(0, int(lanes - 1).bit_length())}"


def in_table(model, dtype, lanes) -> bool:
    return _key(model, dtype, lanes) in _load(TABLE)


def _load(path=None):
    try:
        with open(path or CACHE) as f:
            return json.load(f)
    except Exception:
        return {}


def _save(d):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE, "w") as f:
            json.dump(d, f, indent=1)
    except OSError:
        pass


def tune(model, d_data, chunk_lens, dtype="f32", sample_bytes=2048, use_cache=True, verbose=False,
         use_table=True) -> dict:
    """Pick the encoder tile and the decoder kernel for this workload.  Returns
    {"tile_t", "decode_kernel", "fused_lanes", "use_graph"}."""
    import torch
    import paper_2511_11337_amd as boa
    lens = np.asarray(chunk_lens, dtype=np.int64)
    key = _key(model, dtype, len(lens))
    if use_table:
        table = _load(TABLE)
        if key in table:
            return dict(table[key])
    cache = _load() if use_cache else {}
    if key in cache:
        return cache[key]
    # prefix sample of every chunk, same lane count
    off = np.concatenate([[0], np.cumsum(lens)[:-1]])
    sub = np.minimum(lens, sample_bytes)
    host = d_data.cpu().numpy() if d_data.is_cuda else np.asarray(d_data)
    sample = np.concatenate([host[o:o + n] for o, n in zip(off, sub)])
    d_s = torch.from_numpy(sample).cuda()
    best_t, best_tile = None, 0
    for tile in TILES:
        if tile > sample_bytes or (tile > TILES[0] and tile * len(lens) > MAX_TILE_ROWS):
            break
        boa.encode_dev(model, d_s, sub, dtype=dtype, tile_t=tile, ideal=False)     # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        boa.encode_dev(model, d_s, sub, dtype=dtype, tile_t=tile, ideal=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if verbose:
            print(f"[autotune] encode tile {tile}: {dt * 1e3:.2f} ms")
        if best_t is None or dt < best_t:
            best_t, best_tile = dt, tile
    payload, poff, plen, _ = boa.encode_dev(model, d_s, sub, dtype=dtype, tile_t=best_tile, ideal=False)
    plen_h = plen.cpu().numpy().astype(np.uint32).astype(np.uint64)
    firsts = sample[np.concatenate([[0], np.cumsum(sub)[:-1]])]
    # decoder: the fused persistent kernel at each lanes-per-workgroup count,
    # and the per-step kernel chain replayed as a graph or launched plainly
    cands = [dict(decode_kernel="fused", fused_lanes=g, use_graph=True) for g in FUSED_LANES]
    cands += [dict(decode_kernel="steps", fused_lanes=0, use_graph=g) for g in (True, False)]
    best_c, best_dt = None, None
    for c in cands:
        try:
            boa.decode_dev(model, payload, poff, plen_h, firsts, sub, dtype=dtype, **c)
        except boa.BoaError:            # lanes per workgroup beyond the device's LDS
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        boa.decode_dev(model, payload, poff, plen_h, firsts, sub, dtype=dtype, **c)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if verbose:
            print(f"[autotune] decode {c}: {dt * 1e3:.2f} ms")
        if best_dt is None or dt < best_dt:
            best_c, best_dt = c, dt
    res = {"tile_t": int(best_tile), **best_c}
    cache[key] = res
    if use_cache:
        _save(cache)
    return res
