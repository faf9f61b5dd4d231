"""Autotuner for the batched path.

Times a few V-cycles of a sample batch for every candidate of (row tile =
segment length, coarse-workgroup node threshold, cycles per graph replay)
and keeps the fastest per (dimension, largest grid side, precision).  Results
are cached in a JSON file (BCMG_TUNING_CACHE, default ~/.cache/bcmg_tuning.json).
"""
from __future__ import annotations

import itertools
import json
import os
import time

import torch

from . import _native as N
from .batching import BatchConfig, BatchSolver

SEG_LENS = (64, 128)
COARSE_NODES = (300, 1200, 5000)
CYCLES_PER_STEP = (1, 2, 4)


def cache_path() -> str:
    p = os.environ.get("BCMG_TUNING_CACHE", os.path.expanduser("~/.cache/bcmg_tuning.json"))
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
    except OSError:
        p = "/tmp/bcmg_tuning.json"
    return p


def _key(d: int, max_side: int, precision: int) -> str:
    return f"d{d}_n{max_side}_p{precision}"


def load(d: int, max_side: int, precision: int):
    try:
        return json.load(open(cache_path())).get(_key(d, max_side, precision))
    except (OSError, ValueError):
        return None


def tune(sample_cases, precision: int = N.MIXED, cycles: int = 4, use_cache: bool = True) -> dict:
    """Return {'seg_len', 'coarse_nodes', 'cycles_per_step', 'table'} for the sample."""
    d = sample_cases[0].d
    max_side = max(c.N + 1 for c in sample_cases)
    if use_cache:
        hit = load(d, max_side, precision)
        if hit:
            return hit
    table = []
    for seg_len in SEG_LENS:
        cfg = BatchConfig(seg_len=seg_len, precision=precision, max_cycles=cycles)
        bs = BatchSolver(sample_cases, cfg)
        for cn, cps in itertools.product(COARSE_NODES, CYCLES_PER_STEP):
            bs.batch.set_param(N.PARAM_COARSE_NODES, cn)
            bs.cfg.cycles_per_step = cps
            bs.reset()
            bs.batch.step(cps)  # capture the graph outside the timing
            bs.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            done = 0
            while done < cycles:
                bs.batch.step(cps)
                done += cps
            torch.cuda.synchronize()
            table.append({"seg_len": seg_len, "coarse_nodes": cn, "cycles_per_step": cps,
                          "ms_per_cycle": (time.perf_counter() - t0) * 1e3 / done})
        bs.close()
    best = min(table, key=lambda r: r["ms_per_cycle"])
    res = {"seg_len": best["seg_len"], "coarse_nodes": best["coarse_nodes"],
           "cycles_per_step": best["cycles_per_step"], "table": table}
    try:
        p = cache_path()
        cur = json.load(open(p)) if os.path.exists(p) else {}
        cur[_key(d, max_side, precision)] = res
        json.dump(cur, open(p, "w"), indent=1)
    except (OSError, ValueError):
        pass
    return res
