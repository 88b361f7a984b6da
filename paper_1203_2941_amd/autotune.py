"""Queue-depth and launch-shape autotuner for the wavefront transport.

A candidate is (queue_depth, walk_blocks_per_cu, blocks_per_cu): packets
per queue, 256-thread blocks per CU of the walk kernel, and blocks per CU of
the emission and interaction kernels. Deeper queues give each round more
flights per lane (shorter round tails) at the cost of memory. The tuner
times a packet subsample of the caller's models (one batch per candidate,
same seeds) and keeps the fastest. Results are cached per model signature
in a JSON file.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Dict, List, Sequence, Tuple

from .context import Context, run_batch

CANDIDATES: List[Tuple[int, int, int]] = [
    (1 << 22, 4, 2), (1 << 23, 4, 2), (1 << 24, 4, 2), (1 << 25, 4, 2), (1 << 25, 3, 2),
    (1 << 25, 4, 1), (1 << 26, 4, 2), (1 << 24, 4, 3), (1 << 25, 4, 3)]
CACHE = os.environ.get("MCRT_TUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "mcrt_autotune.json"))


def signature(contexts: Sequence[Context], mode: str) -> str:
    parts = [mode, str(len(contexts))]
    for c in contexts:
        parts.append(f"{c.nx}x{c.ny}x{c.nz}:{c.nl}:{c.ns}:{int(c.fp64)}")
    return hashlib.sha1("|".join(parts).encode()).hexdigest()[:16]


def _load() -> Dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: Dict) -> None:
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE, "w") as f:
            json.dump(d, f, indent=1)
    except OSError:
        pass


def tune(contexts: Sequence[Context], n_packets: Sequence[int], seeds: Sequence[int],
         sample_frac: float = 0.05, min_packets: int = 20000, candidates=None,
         use_cache: bool = True, **opts) -> Dict:
    """Best (queue_depth, walk_blocks_per_cu, blocks_per_cu) for a batch;
    returns a dict with the choice and the measured rates of every candidate."""
    mode = opts.get("mode", "bw_ticket")
    key = signature(contexts, str(mode))
    cache = _load() if use_cache else {}
    if use_cache and key in cache:
        return cache[key]
    cand = candidates or CANDIDATES
    sub = [max(min_packets, int(n * sample_frac)) for n in n_packets]
    rates = {}
    for qd, wb, bpc in cand:
        t0 = time.perf_counter()
        st = run_batch(contexts, sub, seeds, queue_depth=qd, walk_blocks_per_cu=wb,
                       blocks_per_cu=bpc, **opts)
        dt = time.perf_counter() - t0
        ms = st[0]["kernel_ms"] if st else dt * 1e3
        rates[f"{qd}x{wb}x{bpc}"] = sum(sub) / (ms / 1e3)
    best = max(rates, key=rates.get)
    qd, wb, bpc = (int(x) for x in best.split("x"))
    res = {"queue_depth": qd, "walk_blocks_per_cu": wb, "blocks_per_cu": bpc,
           "packets_per_s": rates[best], "rates": rates, "sample_packets": int(sum(sub))}
    if use_cache:
        cache[key] = res
        _store(cache)
    return res
