"""Batched solves: many independent problems advanced by whole V-cycles.

A batch aligns every problem's levels at the coarsest grid, so one launch per
step of the cycle serves all problems that have that level, and the cycle
sequence is captured once in a hipGraph and replayed (bcmg_batch_*).  The
small coarse levels of each problem run in one workgroup per problem.
This module builds the problems of a batch from seeded cases and runs them,
with the row tile (segment length), the coarse-workgroup threshold and the
cycles per graph replay taken from the autotuner.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np
import torch

from . import _native as N
from . import workloads as W
from .solver import Batch, Problem


@dataclass
class BatchConfig:
    seg_len: int = 128
    coarse_nodes: int = 1200
    cycles_per_step: int = 2
    precision: int = N.MIXED
    tol: float = 1e-10
    max_cycles: int = 200


@dataclass
class BatchResult:
    problems: int
    unknowns: int
    elapsed_s: float
    cycles: list
    status: list
    alg_bytes: float

    @property
    def unknowns_per_s(self) -> float:
        return self.unknowns / self.elapsed_s


def make_problem(case: W.Case, cfg: BatchConfig, stream=None) -> tuple[Problem, torch.Tensor, int]:
    """Set up one case (device-side setup), its boundary data at the projections
    and its initial guess (0, g_B on eliminated nodes)."""
    G = Problem(case.d, case.N, case.phi, precision=cfg.precision, seg_len=cfg.seg_len,
                max_cycles=cfg.max_cycles, stream=stream)
    gi = G.ghost_info(0)
    gq = W.points_eval(case.g, gi["q"].cpu().numpy(), case.d)
    G.set_data(case.f, gq)
    u = G.initial_guess(torch.from_numpy(case.gB).cuda())
    info = G.level_info(0)
    return G, u, info["n_inside"] + info["n_ghost"]


def cycle_bytes(G: Problem, precision: int) -> float:
    """Algorithmic HBM bytes of one cycle, summed over levels: per level node
    of INSIDE/GHOST rows, nu1+nu2 red-black sweeps (read u of the other colour,
    read f, write u: 3 words), residual (read u, f, write r: 3), restriction
    (read r: 1 word per fine node, write coarse f), prolongation (read and
    write u: 2); the finest level adds the FP64 residual (read u, f, write r:
    24 B) and, in mixed precision, the update (read e, read and write u: 20 B)."""
    w = 4.0 if precision == N.MIXED else 8.0
    nu = G.opts.nu1 + G.opts.nu2
    tot = 0.0
    for l in range(G.levels):
        info = G.level_info(l)
        n = info["n_inside"] + info["n_ghost"]
        tot += n * w * (3 * nu + 3 + 1 + 2)
    n0 = G.level_info(0)
    n0 = n0["n_inside"] + n0["n_ghost"]
    tot += n0 * 24.0
    if precision == N.MIXED:
        tot += n0 * 20.0
    return tot


class BatchSolver:
    def __init__(self, cases: list[W.Case], cfg: BatchConfig):
        self.cfg = cfg
        self.items = [make_problem(c, cfg) for c in cases]
        self.cases = cases
        self.batch = Batch(len(cases))
        self.batch.set_param(N.PARAM_COARSE_NODES, cfg.coarse_nodes)
        self.slots = [self.batch.add(G, u, cfg.tol) for G, u, _ in self.items]
        self.unknowns = sum(n for _, _, n in self.items)
        self._bytes_per_cycle = [cycle_bytes(G, cfg.precision) for G, _, _ in self.items]

    def reset(self):
        for (G, u, _), c in zip(self.items, self.cases):
            u.zero_()
            G.fill_boundary(torch.from_numpy(c.gB).cuda(), u)
        torch.cuda.synchronize()
        self.batch.restart()

    def run(self) -> BatchResult:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = 0
        while True:
            act = self.batch.step(self.cfg.cycles_per_step)
            steps += 1
            if not act.any() or steps * self.cfg.cycles_per_step > self.cfg.max_cycles + 4:
                break
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        cyc, stat = [], []
        for s in self.slots:
            st, _ = self.batch.stats(s)
            cyc.append(st.cycles)
            stat.append(st.status)
        alg = sum(b * c for b, c in zip(self._bytes_per_cycle, cyc))
        return BatchResult(len(self.slots), self.unknowns, el, cyc, stat, alg)

    def close(self):
        self.batch.close()
        for G, _, _ in self.items:
            G.close()
