"""Autotuner for the filter-bank launch shape and the serving block length.

``tune_packing`` times every valid (filters_per_lane F, waves_per_group W)
candidate on the device for a bank shape, each also with the time split the
library's planner picks for it when that is a split (and, for banks too small
to fill the device, a few fixed splits), and keeps the fastest; results are
cached in a JSON file keyed by the GPU architecture and a signature of the
bank shape (filters per band, largest delay per band, templates, block).
``tune_block`` picks the shortest block length whose throughput reaches a
given fraction of the best candidate's (shorter blocks mean lower latency).

Results never depend on the choice beyond floating-point rounding of the sum
(each choice is tested against the FP64 oracle within the same tolerance).
"""
from __future__ import annotations

import hashlib
import json
import os
import time

DEFAULT_CANDIDATES = [(2, 4), (2, 8), (4, 4), (4, 8), (6, 4), (6, 8), (8, 4)]
# banks with fewer lanes than this cannot fill the device with filters alone;
# for them the tuner also tries splitting each block in time
SMALL_BANK_LANES = 65536
SMALL_BANK_CANDIDATES = [(1, 1, 1), (1, 2, 1), (4, 1, 1), (1, 1, 16), (1, 2, 32), (4, 1, 16),
                         (4, 1, 64), (1, 1, 64)]
CACHE_ENV = "SPIIR_TUNE_CACHE"


def _cache_path() -> str:
    return os.environ.get(CACHE_ENV, os.path.join(os.path.expanduser("~"), ".cache", "spiir",
                                                  "tune.json"))


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name)


def signature(tables, block: int) -> str:
    per_band = tables.n_filters.sum(axis=0).tolist()
    off = tables.offsets()
    dmax = []
    for h in range(tables.n_bands):
        ds = [tables.delay[off[t, h]:off[t, h] + tables.n_filters[t, h]] for t in range(tables.n_templates)]
        ds = [d for d in ds if len(d)]
        dmax.append(int(max(int(d.max()) for d in ds)) if ds else 0)
    key = json.dumps({"T": tables.n_templates, "per_band": per_band, "dmax": dmax, "block": block,
                      "segments": int((tables.n_filters > 0).sum())}, sort_keys=True)
    return hashlib.sha1(key.encode()).hexdigest()[:16]


def _load_cache() -> dict:
    try:
        with open(_cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(c: dict) -> None:
    path = _cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_bank(tables, block: int, steps: int = 3, warmup: int = 1, **bank_kw) -> float:
    """Milliseconds per block for a fresh bank on a white-noise stream."""
    import torch

    from . import spiir as S
    bank = S.Bank(tables, block, **bank_kw)
    x = torch.randn((warmup + steps) * block, dtype=torch.float32, device="cuda")
    z = torch.empty((tables.n_templates, block), dtype=torch.complex64, device="cuda")
    for i in range(warmup):
        bank.process_block(x[i * block:(i + 1) * block], z)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(warmup, warmup + steps):
        bank.process_block(x[i * block:(i + 1) * block], z)
    e1.record()
    torch.cuda.synchronize()
    bank.destroy()
    return e0.elapsed_time(e1) / steps


def tune_packing(tables, block: int, candidates=None, steps: int = 3, use_cache: bool = True,
                 **bank_kw) -> dict:
    """Fastest (filters_per_lane, waves_per_group) for this bank shape."""
    from . import spiir as S
    key = f"{_arch()}:{signature(tables, block)}:{bank_kw.get('precision', 'fp32')}"
    cache = _load_cache() if use_cache else {}
    if key in cache:
        return dict(cache[key], cached=True)
    results = []
    if candidates is None:
        candidates = list(DEFAULT_CANDIDATES)
        # each default shape also with the split the planner picks for it
        for F, Wv in DEFAULT_CANDIDATES:
            try:
                P = S.spiir_plan(tables, block, **dict(bank_kw, filters_per_lane=F, waves_per_group=Wv,
                                                       time_chunks=S.TIME_CHUNKS_AUTO))["time_chunks"]
            except S.SpiirError:
                continue
            if P > 1:
                candidates.append((F, Wv, P))
        if tables.total_filters / 4 < SMALL_BANK_LANES:
            candidates += [c for c in SMALL_BANK_CANDIDATES if c not in candidates]
    for cand in candidates:
        F, Wv = cand[0], cand[1]
        P = cand[2] if len(cand) > 2 else 1
        kw = dict(bank_kw, filters_per_lane=F, waves_per_group=Wv, time_chunks=P)
        try:
            S.spiir_plan(tables, block, **kw)
        except S.SpiirError:
            continue
        ms = time_bank(tables, block, steps=steps, **kw)
        results.append({"filters_per_lane": F, "waves_per_group": Wv, "time_chunks": P, "ms": ms})
    if not results:
        raise RuntimeError("no valid launch shape for this bank")
    best = min(results, key=lambda r: r["ms"])
    out = {"filters_per_lane": best["filters_per_lane"], "waves_per_group": best["waves_per_group"],
           "time_chunks": best["time_chunks"], "ms_per_block": best["ms"], "candidates": results,
           "tuned_at": time.time()}
    if use_cache:
        cache = _load_cache()
        cache[key] = out
        _store_cache(cache)
    return dict(out, cached=False)


def tune_block(tables, blocks=(256, 512, 1024, 2048, 4096), target: float = 0.9, steps: int = 3,
               **bank_kw) -> dict:
    """Shortest block length reaching `target` of the best filter-samples/s."""
    rates = []
    for n in blocks:
        if n % (1 << (tables.n_bands - 1)):
            continue
        ms = time_bank(tables, n, steps=steps, **bank_kw)
        rates.append({"block": n, "ms": ms,
                      "filter_samples_per_s": tables.filter_samples_per_block(n) / (ms * 1e-3)})
    best = max(r["filter_samples_per_s"] for r in rates)
    pick = min((r for r in rates if r["filter_samples_per_s"] >= target * best),
               key=lambda r: r["block"])
    return {"block": pick["block"], "target": target, "rates": rates}


def tuned_bank_kwargs(tables, block: int, **bank_kw) -> dict:
    """Bank keyword arguments with the tuned launch shape filled in."""
    t = tune_packing(tables, block, **bank_kw)
    return dict(bank_kw, filters_per_lane=t["filters_per_lane"], waves_per_group=t["waves_per_group"],
                time_chunks=t.get("time_chunks", 1))


__all__ = ["tune_packing", "tune_block", "tuned_bank_kwargs", "signature", "time_bank"]
