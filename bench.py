"""Benchmark: unknowns solved per second to a relative residual of 1e-10.

Default workload (one GPU): 3D Poisson on the flower domain
phi = r - (0.5 + 0.1 sin(3 theta) sin(4 varphi)) about (0.01, 0.01, 0.01) in
[-1,1]^3 with 513^3 nodes, exact solution exp(x+y+z) (f and the Dirichlet
data from it), V(2,1) red-black Gauss-Seidel cycles with distance-dependent
ghost relaxation down to a 5^3 grid, solved from u = 0 to
||r|| <= 1e-10 ||r0||, once in FP64 and once in mixed precision (FP32 cycle
on the correction, FP64 residual, update and coarse solve).  The headline
value is the mixed-precision rate; the FP64 rate is reported beside it.
Synthetic input generated on the host, copied to HBM before the timed
region; setup (classification, ghost geometry, extension band, coarse
inverse) is done once per problem and reported separately.
--workload flower257 runs the 257^3 FP64 solve alone.

A step is one full solve (V-cycles replayed from a captured hipGraph).  After
the timed steps, HIP events on the solver's stream time the finest-level
red-black sweep of the headline problem for the roofline line: around a
burst of 100 back-to-back red + black sweeps (the roofline figure), and
around every finest-level colour launch of solves run as direct launches
(events recorded inside a graph cannot be timed; reported beside it).  The
oracle (plain C, FP64, one thread) is timed on a bounded sample of the same
problem for the CPU baseline.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM traffic of the finest sweep per workload, from committed counter runs
TRAFFIC_FILES = {
    (512, "mixed"): os.path.join(ROOT, "profiles", "k_rb_sweep_flower513_mixed_traffic.json"),
    (256, "fp64"): os.path.join(ROOT, "profiles", "k_rb_sweep_flower257_fp64_traffic.json"),
}
KERNEL_SRC = [os.path.join(ROOT, "paper_2207_14208_amd", "csrc", f) for f in ("seg.h", "rb_sweep.h")]
METRIC = "unknowns solved/s to rel. residual 1e-10 (FP64 vs mixed); served p50/p99 ms"


def kernel_fingerprint(paths=KERNEL_SRC) -> str:
    """sha256 of the red-black sweep's source (the kernel and the segment
    helpers it uses) with comments and white space removed."""
    import hashlib
    import re
    src = ""
    for path in paths:
        with open(path) as fh:
            src += fh.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return hashlib.sha256(re.sub(r"\s+", "", src).encode()).hexdigest()


def stored_traffic(N: int, precision: str):
    """HBM bytes per finest-level red-black launch, from the committed
    FETCH_SIZE and WRITE_SIZE counter runs (scaled by the same counters on a
    plain copy kernel of known size); None when no record exists for the
    workload or the kernel source has changed since the counters were taken."""
    path = TRAFFIC_FILES.get((N, precision))
    if path is None:
        return None
    try:
        with open(path) as fh:
            rec = json.load(fh)
        fp = kernel_fingerprint()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_fingerprint") != fp or rec.get("N") != N or rec.get("precision") != precision:
        return None
    return rec["bytes_per_launch"]


# intervals per axis of the workloads that take --N, when it is not given
DEFAULT_N = {"flower513": 512, "flower257": 256, "probe513": 512, "cycle_options": 256, "neumann": 256}


def intervals(args) -> int:
    """--N, or the workload's default intervals per axis."""
    return args.N or DEFAULT_N[args.workload]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=0,
                    help="intervals per axis (default: 512 for flower513 and probe513, 256 for flower257, "
                         "cycle_options and neumann)")
    ap.add_argument("--max-cycles", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-cycles", type=int, default=0, help="oracle V-cycles in the CPU sample (default: 1 at "
                                                                "513^3, 2 below)")
    ap.add_argument("--workload", choices=["flower513", "flower257", "probe513", "cycle_options", "batched", "served",
                                           "rho_sweep", "neumann"],
                    default="flower513",
                    help="flower513: the 513^3 flower, FP64 against mixed precision (the headline); flower257: "
                         "the 257^3 FP64 solve; probe513: the finest red-black sweep on the full 513^3 box (the "
                         "roofline probe); cycle_options: the 257^3 flower with the V- and W-cycle and the "
                         "red-black and weighted-Jacobi smoothers; batched: 512 2D star problems; served: the "
                         "continuous-batching "
                         "request loop; rho_sweep: convergence factors of the paper's 2D tests, batched; neumann: "
                         "the 257^3 ellipsoid with Neumann rows and the reaction term against Dirichlet Poisson")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64", help="flower257: precision")
    ap.add_argument("--check-interval", type=int, default=16,
                    help="flower513, flower257: at most this many cycles per convergence check of the solve "
                         "(bcmg_options.check_interval; 1 checks after every cycle)")
    ap.add_argument("--problems", type=int, default=512, help="batched: number of problems")
    ap.add_argument("--tuned", default="",
                    help="batched: SEG_LEN,COARSE_NODES,CYCLES_PER_STEP instead of the autotuner's choice (for "
                         "counter runs, which need the same launches in every pass)")
    ap.add_argument("--no-one-by-one", action="store_true",
                    help="batched: skip the one-problem-at-a-time comparison solves (for counter runs)")
    ap.add_argument("--requests", type=int, default=400, help="served: measured requests")
    ap.add_argument("--served-dtau", choices=["exp", "poly"], default="exp",
                    help="served: the optimal dtau form (exponential, Remark exptheta2D; or polynomial, Prop. opt3D)")
    ap.add_argument("--prepare-workers", type=int, default=2,
                    help="served: host threads that sample and set up admitted requests")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the workload, copy a device buffer of this size once (a plain copy kernel of "
                         "known size, for scaling hardware traffic counters)")
    return ap.parse_args()


def copy_probe(mib):
    """One device-to-device copy of mib MiB before the workload: a plain copy
    kernel of known size, against which the traffic counters are scaled."""
    import torch
    src = torch.ones(mib << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def rho_last(hist):
    """Per-cycle residual ratio between the last two checked cycles (cycles
    without a check have NaN in the history)."""
    import numpy as np
    idx = np.flatnonzero(~np.isnan(hist))
    if len(idx) < 3:
        return None
    a, b = idx[-2], idx[-1]
    return float((hist[b] / hist[a]) ** (1.0 / (b - a)))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1 (sharding the grid "
                                   "across GPUs is not implemented)"}))
        sys.exit(2)
    if args.copy_probe_mib > 0:
        copy_probe(args.copy_probe_mib)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "rho_sweep":
        return bench_rho_sweep(args)
    if args.workload == "served":
        return bench_served(args)
    if args.workload == "neumann":
        return bench_neumann(args)
    if args.workload == "probe513":
        return bench_probe(args)
    if args.workload == "cycle_options":
        return bench_cycle_options(args)
    return bench_flower(args)


def bench_cycle_options(args):
    """The flower (257^3 by default), FP64 to 1e-10, with each cycle shape
    (V, W) and interior smoother (red-black Gauss-Seidel, weighted Jacobi):
    cycles and time per solve.  value: unknowns/s of the default V-cycle with
    red-black smoothing."""
    import numpy as np
    import torch

    from paper_2207_14208_amd import _native as NAT
    from paper_2207_14208_amd import workloads as W
    from paper_2207_14208_amd.solver import Problem
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    N = intervals(args)
    case = W.flower3d(N)
    phi = torch.from_numpy(case.phi).cuda()
    f = torch.from_numpy(case.f).cuda()
    res = {}
    for name, cyc, sm in (("V_rb", NAT.CYCLE_V, NAT.SMOOTH_RB), ("W_rb", NAT.CYCLE_W, NAT.SMOOTH_RB),
                          ("V_jacobi", NAT.CYCLE_V, NAT.SMOOTH_JACOBI), ("W_jacobi", NAT.CYCLE_W, NAT.SMOOTH_JACOBI)):
        G = Problem(3, N, phi, cycle=cyc, smoother=sm, max_cycles=args.max_cycles)
        q = G.ghost_info(0)["q"]
        G.set_data(f, torch.exp(q[:, 0] + q[:, 1] + q[:, 2]))
        info = G.level_info(0)
        u = torch.zeros(G.nodes, dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            u.zero_()
            G.solve(u, 1e-10)
        torch.cuda.synchronize()
        times = []
        for _ in range(args.steps):
            u.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, hist = G.solve(u, 1e-10)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        ms = float(np.median(times) * 1e3)
        res[name] = {"status": NAT.STATUS_NAMES.get(st.status), "cycles": st.cycles, "ms_per_solve": ms,
                     "us_per_cycle": ms * 1e3 / max(st.cycles, 1),
                     "unknowns_per_s": (info["n_inside"] + info["n_ghost"]) / (ms / 1e3)}
        G.close()
        del G, u
        torch.cuda.empty_cache()
    out = {"metric": METRIC, "value": res["V_rb"]["unknowns_per_s"], "unit": "unknowns/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["V_rb"]["ms_per_solve"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (analytic level set and manufactured solution)",
           "config": {"workload": f"3D flower, {N + 1}^3 nodes, FP64 to 1e-10: V/W cycle x red-black/weighted-Jacobi "
                                  f"smoothing (value: V, red-black)", "nodes_per_axis": N + 1},
           "variants": res}
    print(json.dumps(out))


def bench_probe(args):
    """Roofline probe: the red-black sweep of the finest level on the whole
    513^3 box (phi = -1 everywhere: 511^3 INSIDE nodes, rows of 511 nodes),
    timed by HIP events around 100 back-to-back red + black sweeps, for the
    FP32 sweep of a mixed-precision problem in the split and natural storage
    orders and for the FP64 sweep.  Algorithmic bytes per colour launch:
    1.5 esz per INSIDE node (f and the written u at the colour's nodes, u of
    the other colour), as for the solve's sweep."""
    import torch

    from paper_2207_14208_amd import _native as NAT
    from paper_2207_14208_amd.solver import Problem
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    N = intervals(args)
    phi = -torch.ones((N + 1) ** 3, dtype=torch.float64, device="cuda")
    reps = 100
    res = {}
    for name, prec, layout in (("fp32_split", NAT.MIXED, NAT.LAYOUT_SPLIT), ("fp32_natural", NAT.MIXED, NAT.LAYOUT_NATURAL),
                               ("fp64_natural", NAT.FP64, NAT.LAYOUT_NATURAL)):
        G = Problem(3, N, phi, precision=prec, layout=layout)
        info = G.level_info(0)
        u = torch.zeros(G.nodes, dtype=torch.float64, device="cuda")
        G.timing_sweeps(u, 5)
        ms = G.timing_sweeps(u, reps)
        avg_s = ms / (2 * reps) / 1e3
        esz = 4 if prec == NAT.MIXED else 8
        alg = 1.5 * esz * info["n_inside"]
        res[name] = {"avg_launch_us": avg_s * 1e6, "alg_bytes_per_launch": alg, "achieved_GBps": alg / avg_s / 1e9,
                     "frac": alg / avg_s / 1e9 / HBM_PEAK_GBS, "n_inside": info["n_inside"],
                     "n_segments": info["n_segments"]}
        G.close()
        del G, u
        torch.cuda.empty_cache()
    best = res["fp32_split"]
    out = {"metric": "finest red-black sweep bandwidth on the full 513^3 box (roofline probe)",
           "value": best["achieved_GBps"], "unit": "GB/s", "n_gpus": 1, "steps": reps, "warmup": 5,
           "ms_per_step": 2 * best["avg_launch_us"] / 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic (phi = -1 on the whole box)",
           "config": {"workload": f"roofline probe: red-black sweep of the full {N + 1}^3 box, FP32 split layout "
                                  f"(FP32 natural and FP64 beside it)", "nodes_per_axis": N + 1},
           "roofline": {"bound": "hbm", "kernel": "k_rb_sweep_split4<3> (split layout, one colour)",
                        "achieved": best["achieved_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": best["frac"], "traffic": None, "avg_launch_us": best["avg_launch_us"],
                        "alg_bytes_per_launch": best["alg_bytes_per_launch"]},
           "variants": res}
    print(json.dumps(out))


def bench_flower(args):
    """The flower solves: 513^3 FP64 against mixed precision (headline:
    mixed), or 257^3 in one precision."""
    import numpy as np
    import torch

    from paper_2207_14208_amd import _native as NAT
    from paper_2207_14208_amd import workloads as W
    from paper_2207_14208_amd.solver import Problem, timing_enable, timing_read

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)
    dev = "cuda"
    big = args.workload == "flower513"
    N = intervals(args)
    names = ["fp64", "mixed"] if big else [args.precision]
    head = names[-1]
    prec_of = {"fp64": NAT.FP64, "mixed": NAT.MIXED}

    case = W.flower3d(N)
    phi = torch.from_numpy(case.phi).to(dev)
    f = torch.from_numpy(case.f).to(dev)
    ue = torch.from_numpy(W.sample(3, N, case.u_exact)).to(dev)
    torch.cuda.synchronize()

    def make_problem(prec):
        G = Problem(3, N, phi, precision=prec, max_cycles=args.max_cycles, check_interval=args.check_interval)
        q = G.ghost_info(0)["q"]
        gq = torch.exp(q[:, 0] + q[:, 1] + q[:, 2])  # Dirichlet data g = exp(x+y+z) at the projections Q
        G.set_data(f, gq)
        return G

    res, sols = {}, {}
    G_head = u_head = None
    for name in names:
        prec = prec_of[name]
        # the first setup in a process also loads the kernels (the library's
        # and torch's): time a second one
        make_problem(prec).close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G = make_problem(prec)
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        info = G.level_info(0)
        unknowns = info["n_inside"] + info["n_ghost"]
        u = torch.zeros(G.nodes, dtype=torch.float64, device=dev)

        def step():
            u.zero_()
            return G.solve(u, 1e-10)

        for _ in range(args.warmup):
            st, hist = step()
        torch.cuda.synchronize()
        times = []
        t_all = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            st, hist = step()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - ts)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_all
        # a reduced --max-cycles (counter collection) may stop before the tolerance
        assert st.status == 0 or (st.status == NAT.ERR_NOT_CONVERGED and st.cycles == args.max_cycles), \
            f"{name} solve failed: {st}"
        cls = G.classes(0)
        inside = cls == NAT.INSIDE
        unk = inside | (cls == NAT.GHOST)
        res[name] = {
            "unknowns_per_s": unknowns * args.steps / elapsed, "ms_per_solve": elapsed * 1e3 / args.steps,
            "solve_ms_median": float(np.median(times) * 1e3), "solve_ms_device": st.solve_ms,
            "cycles": st.cycles, "rel_residual": st.r_final / st.r0,
            "rho_last": rho_last(hist),
            "checks": int(np.count_nonzero(~np.isnan(hist))) - 1,
            "setup_ms": setup_ms, "max_err_vs_exact": (u[inside] - ue[inside]).abs().max().item(),
            "unknowns": unknowns, "n_inside": info["n_inside"], "n_ghost": info["n_ghost"], "levels": G.levels,
        }
        sols[name] = u[unk].clone()
        if name == head:
            G_head, u_head = G, u
        else:
            G.close()
            del G
            torch.cuda.empty_cache()
    if big:
        res["mixed"]["max_rel_diff_vs_fp64"] = ((sols["mixed"] - sols["fp64"]).abs().max() /
                                                sols["fp64"].abs().max()).item()
    del sols

    # roofline of the headline problem's finest-level red-black sweep (one
    # colour).  HIP events on the solver's stream: (1) around a burst of
    # back-to-back sweeps (the kernel's own cadence, used for the roofline),
    # and (2) around every finest-level colour launch of full solves run as
    # direct launches (includes the launch gaps between the cycle's kernels)
    G, u = G_head, u_head
    timing_enable(True)
    for _ in range(max(2, min(args.steps, 5))):
        u.zero_()
        G.solve(u, 1e-10)
    torch.cuda.synchronize()
    launches, tot_ms, nodes = timing_read()
    timing_enable(False)
    in_solve_us = tot_ms / max(launches, 1) * 1e3
    esz = 8 if head == "fp64" else 4
    alg_bytes = 1.5 * esz * nodes  # per colour launch: read f and write u at its nodes, read u of the other colour
    reps = 100
    burst_ms = G.timing_sweeps(u, reps)
    avg_s = burst_ms / (2 * reps) / 1e3
    achieved = alg_bytes / avg_s / 1e9 if avg_s > 0 else 0.0
    r = res[head]
    out = {
        "metric": METRIC,
        "value": r["unknowns_per_s"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32+f64",
        "data": "synthetic (analytic level set and manufactured solution)",
        "config": {
            "workload": (f"3D flower, {N + 1}^3 nodes, u=exp(x+y+z), FP64 vs mixed-precision V(2,1) RB-GS to rel. "
                         f"residual 1e-10 (value: mixed)") if big else
                        f"3D flower, {N + 1}^3 nodes, u=exp(x+y+z), {head.upper()} V(2,1) RB-GS to rel. residual 1e-10",
            "nodes_per_axis": N + 1,
            "unknowns": r["unknowns"],
            "n_inside": r["n_inside"],
            "n_ghost": r["n_ghost"],
            "levels": r["levels"],
            "check_interval": args.check_interval,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("k_rb_sweep<3, double> (finest level, one colour)" if head == "fp64" else
                       "k_rb_sweep_split4<3> (finest level, split storage order, one colour)"),
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": stored_traffic(N, head),
            "avg_launch_us": avg_s * 1e6,
            "launches_timed": 2 * reps,
            "avg_launch_us_in_solve": in_solve_us,
            "alg_bytes_per_launch": alg_bytes,
        },
    }
    for name in names:
        out[name] = res[name]
    if big:
        out["speedup_mixed_vs_fp64"] = res["mixed"]["unknowns_per_s"] / res["fp64"]["unknowns_per_s"]
    G.close()
    del G, u
    torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        import oracle
        oracle.build()
        cpu_cycles = args.cpu_cycles or (1 if N >= 512 else 2)
        ref_cycles = res["fp64"]["cycles"] if "fp64" in res else r["cycles"]
        cpu_t0 = time.perf_counter()
        O = oracle.Problem(3, N, case.phi)
        og = O.ghosts(0)
        O.set_rhs(case.f, np.exp(og["q"][:, 0] + og["q"][:, 1] + og["q"][:, 2]))
        cpu_setup = time.perf_counter() - cpu_t0
        uo = np.zeros(O.nodes(0))
        r0 = O.norm(0, O.residual(0, uo))
        tc = time.perf_counter()
        for _ in range(cpu_cycles):
            O.vcycle(uo)
            O.norm(0, O.residual(0, uo))
        per_cycle = (time.perf_counter() - tc) / cpu_cycles
        cpu_solve = per_cycle * ref_cycles
        out["cpu_baseline"] = {
            "value": r["unknowns"] / cpu_solve,
            "unit": "unknowns/s",
            "cores": 1,
            "kind": "oracle",
            "sample": (f"oracle (plain C, FP64, 1 thread: it has no threading) on the same {N + 1}^3 problem: setup "
                       f"({cpu_setup:.1f} s, excluded like on the GPU) then {cpu_cycles} V-cycle(s) with residual "
                       f"norms ({per_cycle:.2f} s each), scaled to the {ref_cycles} cycles of the FP64 solve"),
            "r0": r0,
        }
    print(json.dumps(out))


def bench_neumann(args):
    """257^3 ellipsoid of Sec. 4.2, u = exp(x+y+z): the reaction-diffusion
    problem u - Laplace u = f with Neumann rows (g = grad u(Q) . n) on the
    whole boundary, against the Poisson problem with Dirichlet rows, both
    FP64 V(2,1) to ||r|| <= 1e-10 ||r0||."""
    import numpy as np
    import torch

    from paper_2207_14208_amd import _native as NAT
    from paper_2207_14208_amd import workloads as W
    from paper_2207_14208_amd.solver import Problem
    N = intervals(args)
    out = {"metric": METRIC,
           "unit": "unknowns/s", "n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "data": "synthetic (analytic level set and manufactured solution)", "steps": args.steps,
           "warmup": args.warmup, "dtype": "f64"}
    phi = torch.from_numpy(W.sample(3, N, W.phi_ellipsoid())).cuda()
    xs = [torch.from_numpy(np.ascontiguousarray(a)).cuda().ravel() for a in W.node_coords(3, N)]
    ue = torch.exp(xs[0] + xs[1] + xs[2])
    res = {}
    for name, bc, c in (("neumann", NAT.BC_NEUMANN, 1.0), ("dirichlet", NAT.BC_DIRICHLET, 0.0)):
        G = Problem(3, N, phi, bc=bc, reaction=c, max_cycles=args.max_cycles)
        gi = G.ghost_info(0)
        q, n = gi["q"], gi["n"]
        eq = torch.exp(q[:, 0] + q[:, 1] + q[:, 2])
        g = eq * (n[:, 0] + n[:, 1] + n[:, 2]) if bc == NAT.BC_NEUMANN else eq
        G.set_data(c * ue - 3.0 * ue, g)
        info = G.level_info(0)
        unknowns = info["n_inside"] + info["n_ghost"]
        u = torch.zeros(G.nodes, dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            u = G.initial_guess(ue)
            G.solve(u, 1e-10)
        torch.cuda.synchronize()
        el = 0.0
        for _ in range(args.steps):
            u = G.initial_guess(ue)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, hist = G.solve(u, 1e-10)
            torch.cuda.synchronize()
            el += time.perf_counter() - t0
        el /= args.steps
        cls = G.classes(0)
        m = cls == NAT.INSIDE
        h = np.asarray(hist, dtype=np.float64)
        res[name] = {"unknowns": unknowns, "n_ghost": info["n_ghost"], "unknowns_per_s": unknowns / el,
                     "ms_per_solve": el * 1e3, "cycles": st.cycles, "status": NAT.STATUS_NAMES.get(st.status),
                     "rho_last": float(h[-1] / h[-2]) if len(h) >= 2 and h[-2] > 0 else None,
                     "max_err_vs_exact": (u[m] - ue[m]).abs().max().item()}
        G.close()
        del G
        torch.cuda.empty_cache()
    out["config"] = {"workload": f"3D ellipsoid, {N + 1}^3 nodes, u=exp(x+y+z): u - Laplace u with Neumann rows "
                                 f"vs Poisson with Dirichlet rows, FP64 V(2,1) to 1e-10", "nodes_per_axis": N + 1}
    out["value"] = res["neumann"]["unknowns_per_s"]
    out["ms_per_step"] = res["neumann"]["ms_per_solve"]
    out["neumann"] = res["neumann"]
    out["dirichlet"] = res["dirichlet"]
    print(json.dumps(out))


def bench_rho_sweep(args):
    """Convergence factors (homogeneous problem, U(-1,1) start, mean of
    rho^(11..15)) of the paper's 2D tests, all in one batch: circle and
    flower for N = 64..1024 under the three Delta-tau modes, and the
    rectangle for theta = 0.1..0.9 against a constant Delta-tau scan.  The
    oracle runs the circle N = 256 spec (same protocol and cycle) as the CPU
    sample."""
    import torch

    from paper_2207_14208_amd import experiments as X
    specs = [X.Spec(dom, n, dt) for dom in ("circle", "flower") for n in (64, 128, 256, 512, 1024)
             for dt in ("opt_exp", "opt_poly", "const:1.75")]
    specs += [X.Spec("rectangle", 128, f"const:{dt}", theta=th) for th in (0.1, 0.3, 0.5, 0.7, 0.9)
              for dt in (0.5, 1.0, 1.5, 1.75, 2.0, 2.5)]
    X.rho_sweep(specs[:3])  # load the kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = X.rho_sweep(specs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    table = {}
    for r in res:
        s = r["spec"]
        key = f"{s['domain']}" + (f" theta={s['theta']}" if s["domain"] == "rectangle" else f" N={s['N']}")
        table.setdefault(key, {})[s["dtau"]] = round(r["rho"], 4)
    out = {"metric": "convergence-factor problems per second (16 V-cycles each, batched)", "value": len(specs) / el,
           "unit": "problems/s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": el * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (paper's 2D domains, homogeneous problem, seeded U(-1,1) start)",
           "config": {"workload": "rho sweep: circle and flower N=64..1024 x {opt_exp, opt_poly, const 1.75}, "
                                  "rectangle N=128 theta 0.1..0.9 x const dtau 0.5..2.5; V(2,1) red-black",
                      "problems": len(specs)},
           "rho": table}
    if not args.no_cpu_baseline:
        import numpy as np

        import oracle
        from paper_2207_14208_amd import workloads as W
        oracle.build()
        spec = X.Spec("circle", 256, "opt_exp")
        t1 = time.perf_counter()
        O = oracle.Problem(2, 256, W.sample(2, 256, X.DOMAINS["circle"][1](256, 0.5)), oracle.Options(max_cycles=16))
        O.set_rhs(np.zeros(O.nodes(0)), np.zeros(O.counts(0)[1]))
        u = X.initial_guess(O.classes(0), spec.seed)
        _, hist = O.solve(u, 0.0, 16)
        cpu_s = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": 1.0 / cpu_s, "unit": "problems/s", "cores": 1, "kind": "oracle",
                               "sample": f"oracle (plain C, FP64, 1 thread): the circle N=256 opt_exp spec, setup "
                                         f"and 16 V-cycles, {cpu_s:.2f} s; rho {X.rho_from_history(hist):.4f}"}
    print(json.dumps(out))


def bench_batched(args):
    """512 independent 2D star problems (sides 65..1025, seed 2207),
    mixed precision, solved together by the batched engine (hipGraph-replayed
    cycles, per-problem coarse workgroups, autotuned row tile, coarse
    threshold and cycles per replay), against the same problems solved one
    after another by the single-problem solver, in FP64 and in mixed
    precision."""
    import numpy as np
    import torch

    from paper_2207_14208_amd import _native as NAT
    from paper_2207_14208_amd import autotune
    from paper_2207_14208_amd import workloads as W
    from paper_2207_14208_amd.batching import BatchConfig, BatchSolver, make_problem

    t0 = time.perf_counter()
    sample = [W.star_case(i, *p) for i, p in enumerate(W.star_params(24, seed=1))]
    if args.tuned:
        seg, cn, cps = (int(v) for v in args.tuned.split(","))
        tuned = {"seg_len": seg, "coarse_nodes": cn, "cycles_per_step": cps}
    else:
        tuned = autotune.tune(sample, NAT.MIXED, cycles=4, use_cache=False)
    tune_s = time.perf_counter() - t0
    params = W.star_params(args.problems, seed=2207)
    cases = [W.star_case(i, *p) for i, p in enumerate(params)]
    cfg = BatchConfig(seg_len=tuned["seg_len"], coarse_nodes=tuned["coarse_nodes"],
                      cycles_per_step=tuned["cycles_per_step"], precision=NAT.MIXED, max_cycles=args.max_cycles)
    t1 = time.perf_counter()
    bs = BatchSolver(cases, cfg)
    setup_s = time.perf_counter() - t1
    print(f"batched: tuned {tuned['seg_len']}/{tuned['coarse_nodes']}/{tuned['cycles_per_step']} in {tune_s:.1f} s, "
          f"set up {len(cases)} problems in {setup_s:.1f} s", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        bs.reset()
        bs.run()
    times = []
    for _ in range(args.steps):
        bs.reset()
        r = bs.run()
        times.append(r.elapsed_s)
    el = float(np.median(times))
    ok = sum(1 for s in r.status if s == 0)
    print(f"batched: {el * 1e3:.1f} ms per batch solve; one-by-one solves next", file=sys.stderr, flush=True)
    # the single-problem solver, one problem after another (same problems,
    # same tolerance), in FP64 and in mixed precision: the first comparison
    # is batching and precision together, the second batching alone
    one_by_one = {"fp64": (float("nan"), [0]), "mixed": (float("nan"), [0])}
    for pname, prec in () if args.no_one_by_one else (("fp64", NAT.FP64), ("mixed", NAT.MIXED)):
        el1, cyc1 = 0.0, []
        for c in cases:
            G, u, _ = make_problem(c, BatchConfig(seg_len=128, precision=prec, max_cycles=args.max_cycles))
            torch.cuda.synchronize()
            ts = time.perf_counter()
            st, _ = G.solve(u, 1e-10)
            torch.cuda.synchronize()
            el1 += time.perf_counter() - ts
            cyc1.append(st.cycles)
            G.close()
        one_by_one[pname] = (el1, cyc1)
    plain_el, plain_cycles = one_by_one["fp64"]
    mixed_el, mixed_cycles = one_by_one["mixed"]
    out = {"metric": METRIC,
           "value": r.unknowns / el, "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": el * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32+f64", "data": "synthetic (seeded star domains and manufactured solution)",
           "config": {"workload": f"{args.problems} 2D star problems, sides 65..1025 (seed 2207), mixed precision, "
                                  "batched V(2,1) to rel. residual 1e-10",
                      "problems": args.problems, "unknowns": r.unknowns, "converged": ok,
                      "cycles_min_median_max": [int(np.min(r.cycles)), int(np.median(r.cycles)), int(np.max(r.cycles))],
                      "tuned": {k: tuned[k] for k in ("seg_len", "coarse_nodes", "cycles_per_step")},
                      "tune_s": tune_s, "setup_s": setup_s},
           "effective_hbm": {"alg_bytes": r.alg_bytes, "GBps": r.alg_bytes / el / 1e9,
                             "frac_of_8TBps": r.alg_bytes / el / 8e12},
           "plain_fp64_one_by_one": {"unknowns_per_s": r.unknowns / plain_el, "seconds": plain_el,
                                     "cycles_median": int(np.median(plain_cycles))},
           "mixed_one_by_one": {"unknowns_per_s": r.unknowns / mixed_el, "seconds": mixed_el,
                                "cycles_median": int(np.median(mixed_cycles))},
           "speedup_vs_plain": (r.unknowns / el) / (r.unknowns / plain_el),
           "speedup_of_batching": (r.unknowns / el) / (r.unknowns / mixed_el)}
    print(json.dumps(out))
    bs.close()


def bench_served(args):
    from paper_2207_14208_amd import serving
    print(json.dumps(serving.bench(args)))


if __name__ == "__main__":
    main()
