"""Benchmark: batched Newton power flow on one MI355X.

Workload (default): synthetic 118-bus meshed grid (tree + 60 extra branches,
53 PV, 64 PQ, slack bus 0), batch of 1024 load scenarios, tolerance 1e-8 pu,
flat start.  One step runs the whole path on the batch, inputs resident in
HBM: the plain FP64 Newton solve, the mixed-precision solve (FP32 LU
refactorisation and solves, FP64 mismatch / convergence / update and two
FP64-residual refinement steps), one differentiable-layer forward + backward
(mixed-precision solve keeping the factors + adjoint), the mixed-precision
solve with adaptive refinement and without refinement, one layer forward +
backward through both completion steps (Step-2 recovery of the generation
block and its backward term), one training step of the synthetic task and a
refresh of the exported operators.  Each part is timed with HIP events on
the stream the kernels run on; rates use the median over the timed steps.

``value`` is the mixed-precision solves/s; the other rates are reported
beside it.  The roofline entry covers the dominant kernel (the
mixed-precision Newton kernel): algorithmic bytes per launch (the model in
``algorithmic_bytes_per_solve``) over its median launch duration.

Legs on the other grids (``--legs``, default all three), each from its own
templates with 3 warm-up runs and the median of ``--repeats`` timed runs:
the 1354-bus batch of 4096 (FP64 and mixed-precision solves, the refinement
variants, and the layer), the 300-bus batch of 2048 (the differentiable
layer as its workload states it: FP64 template, tolerance 1e-10, forward +
backward), and the 9241-bus batch of 256 (FP64 and mixed-precision solves,
mixed-precision forward + FP32-factor adjoint in one autograd step, peak
device bytes and the LU fill ratio).  Each leg carries its own roofline.

``--phases`` loads the measurement build of the library
(libsablepf_phases.so) and reports the Newton kernel's per-phase time of
workgroup 0 on every grid (its timings carry the counters' overhead).
``cpu_baseline`` times the CPU oracle on a bounded sample.
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
KERNEL_SOURCES = ("paper_2606_07099_amd/csrc/pf_kernels.hip", "paper_2606_07099_amd/csrc/pf_kernels.h")

# HBM bytes per launch of the Newton kernel ("grid/precision" on the full
# batch), from rocprofv3 FETCH_SIZE and WRITE_SIZE passes (each scaled by the
# same counter on a 512 MiB device-to-device copy), keyed by the SHA-256 of
# the kernel sources they were taken on; a changed kernel reports null.
# Sources: profiles/*_hbm_counters.md
MEASURED_TRAFFIC = {
    "0e9949f99c6bfeb39010a3811daa701dedba881ec271c092c0951986c17ab1d1": {
        "c1/mixed": 7003853,
        "c1/fp64": 6899376,
        "c2/mixed": 43249094750,
        "c2/fp64": 46121311935,
        "c3/mixed": 2992607351,
        "c3/fp64": 3339025927,
        "c4/mixed": 37813363924,
        "c4/fp64": 39909501093,
    },
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--legs", default="c2,c3,c4",
                    help="comma-separated other grids to time after the main workload ('none' for none)")
    ap.add_argument("--repeats", type=int, default=10, help="timed runs per leg measurement (median)")
    ap.add_argument("--profile-solve", choices=("fp64", "mixed"), default=None,
                    help="only time this solve of the workload (one template, --steps launches after "
                         "--warmup), for profilers that attribute counters per kernel dispatch")
    ap.add_argument("--phases", action="store_true",
                    help="per-phase clocks of the Newton kernel (measurement build of the library)")
    ap.add_argument("--workload", default="c1", help="grid name in gen.grids.SPECS")
    ap.add_argument("--scenarios", default="lognormal", choices=("lognormal", "uniform10"),
                    help="load scenarios: lognormal scaling of each PQ load, or the paper's "
                         "independent uniform +-10%% perturbation of P and Q")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-reference-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first, as the known-size "
                         "reference for HBM byte counters")
    return ap.parse_args()


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def algorithmic_bytes_per_solve(n_bus, nnz_lu, iters, w, refine):
    """Streaming byte model of one solve from flat start: 5 FP64 boundary
    vectors, and per Newton iteration the LU values written once and read by
    (1 + R) forward+backward solve passes plus (10 + 4R) FP64 state vectors."""
    return 5 * n_bus * 8 + iters * (w * nnz_lu * (2 + refine) + (10 + 4 * refine) * n_bus * 8)


def _oracle_worker(args):
    name, batch, idx, mode = args
    from gen.grids import make_case
    from oracle.newton import newton
    from oracle.ybus import ybus_of
    spec, net, sc = make_case(name, batch=batch, scenario_mode=mode)
    Y = ybus_of(net)
    t0 = time.perf_counter()
    for b in idx:
        newton(Y, net.bus_type, sc.pd[b], sc.qd[b], sc.pg[b], sc.vset[b], tol=spec.tol)
    return len(idx), time.perf_counter() - t0


def cpu_baseline(name, batch, budget_s, mode="lognormal"):
    """The oracle (dense FP64 Newton, one scenario per task) on the host's
    cores, one BLAS thread per worker process."""
    import multiprocessing as mp
    import numpy as np
    cores = len(os.sched_getaffinity(0))
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    ctx = mp.get_context("spawn")
    # calibrate on a few scenarios, then size the sample to the time budget
    n0, t0 = _oracle_worker((name, batch, list(range(min(8, batch))), mode))
    per = t0 / max(n0, 1)
    # scenarios to fill the budget on every core: an even subsample of the
    # batch, or the whole batch repeated when it is shorter than the budget
    n = int(max(cores, budget_s * cores / max(per, 1e-6)))
    if n <= batch:
        idx = np.unique(np.linspace(0, batch - 1, n).astype(int)).tolist()
    else:
        idx = list(range(batch)) * min(64, -(-n // batch))
    chunks = [idx[i::cores] for i in range(cores) if idx[i::cores]]
    t = time.perf_counter()
    with ctx.Pool(len(chunks)) as pool:
        res = pool.map(_oracle_worker, [(name, batch, c, mode) for c in chunks])
    wall = time.perf_counter() - t
    solved = sum(r[0] for r in res)
    # the workers' set-up (grid generation, Y_bus) is inside the wall time;
    # report the solve-only rate from the workers' own clocks as well
    solve_rate = solved / max(max(r[1] for r in res), 1e-9)
    return {"value": solved / wall, "unit": "solves/s", "cores": len(chunks), "kind": "oracle",
            "sample": (f"{solved} scenario solves ({solved / batch:.2f} x the batch of {batch}, "
                       f"evenly spread), dense FP64 Newton + LAPACK, 1 BLAS thread per process"),
            "solve_only_value": solve_rate, "wall_s": wall}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def median_seconds(fn, warmup, repeats):
    """Median duration of fn() over `repeats` timed runs (HIP events on the
    current stream, where the library enqueues its kernels), after `warmup`
    untimed ones."""
    import numpy as np
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    marks = []
    for _ in range(repeats):
        a, b = _events(torch)
        a.record(stream)
        fn()
        b.record(stream)
        marks.append((a, b))
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in marks]) * 1e-3)


def roofline_entry(kernel, n_bus, nnz_lu, iters, w, refine, batch, seconds, grid, precision, regime):
    bytes_launch = batch * algorithmic_bytes_per_solve(n_bus, nnz_lu, iters, w, refine)
    achieved = bytes_launch / seconds / 1e9
    traffic = MEASURED_TRAFFIC.get(kernel_source_hash(), {}).get(f"{grid}/{precision}")
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_over_algorithmic": (traffic / bytes_launch) if traffic else None,
            "kernel_source_sha256": kernel_source_hash()[:16], "kernel": kernel,
            "bytes_per_launch": bytes_launch, "median_launch_ms": 1e3 * seconds,
            "mean_updates": iters, "regime": regime}


def _solve_stats(out):
    import numpy as np
    it, st, fn = (x.cpu().numpy() for x in out[2:])
    return {"iterations": np.bincount(it).tolist(), "converged": int((st == 0).sum()),
            "max_final_mismatch": float(np.nanmax(fn)), "mean_updates": float(it.mean())}


def solve_leg(name, args, scenario_mode="lognormal"):
    """FP64 and mixed-precision (2, adaptive and no refinement) solves and
    the layer (forward + adjoint) on the full batch of one grid."""
    import torch
    from gen.grids import make_case
    from paper_2606_07099_amd import PFLayer, PFTemplate
    spec, net, sc = make_case(name, scenario_mode=scenario_mode)
    B, dev = sc.batch, torch.device("cuda:0")
    d = {k: torch.as_tensor(getattr(sc, k), device=dev) for k in ("pd", "qd", "pg", "vset")}
    res = {"workload": f"{spec.n_bus}-bus synthetic meshed grid, batch {B}, tol {spec.tol:g}",
           "n_bus": spec.n_bus, "batch": B, "tol": spec.tol}
    outs = {}
    variants = (("fp64", dict(precision="fp64")), ("mixed", dict(precision="mixed")),
                ("mixed_adaptive", dict(precision="mixed", refine_adaptive=True)),
                ("mixed_unrefined", dict(precision="mixed", refine_steps=0)))
    infos = {}
    for key, kw in variants:
        t0 = time.perf_counter()
        tpl = PFTemplate.from_network(net, B, tol=spec.tol, keep_factors=False, **kw)
        build_s = time.perf_counter() - t0
        out = [torch.empty((B, net.n_bus), dtype=torch.float64, device=dev) for _ in range(2)] + \
            [torch.empty(B, dtype=torch.int32, device=dev) for _ in range(2)] + \
            [torch.empty(B, dtype=torch.float64, device=dev)]
        sec = median_seconds(lambda: tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"], out=out),
                             args.warmup, args.repeats)
        outs[key] = out
        infos[key] = tpl.info()
        res[key] = {"solves_per_s": B / sec, "ms": 1e3 * sec, "template_build_ms": 1e3 * build_s,
                    **_solve_stats(out)}
        del tpl
    # the adaptive variant runs a refinement solve only while the FP64 residual
    # of the correction is above the forcing term; count what it did
    res["mixed_adaptive"]["note"] = ("inexact-Newton forcing term; when no refinement solve runs it is "
                                     "the unrefined (R = 0) iteration")
    # the layer: mixed-precision template keeping its factors, forward + adjoint
    tpl = PFTemplate.from_network(net, B, tol=spec.tol, precision="mixed", keep_factors=True)
    layer = PFLayer(tpl)
    leaves = {k: d[k].clone().requires_grad_(True) for k in d}

    def step():
        for v in leaves.values():
            v.grad = None
        vm, va = layer(leaves["pd"], leaves["qd"], leaves["pg"], leaves["vset"])
        L = (torch.relu(vm - 1.05) ** 2).sum() + (torch.relu(0.95 - vm) ** 2).sum() + 0.1 * (va ** 2).sum()
        L.backward()
    sec = median_seconds(step, args.warmup, args.repeats)
    res["layer_mixed"] = {"fwd_bwd_samples_per_s": B / sec, "ms": 1e3 * sec}
    del layer, tpl
    res["fp64_over_mixed"] = res["fp64"]["ms"] / res["mixed"]["ms"]
    info = infos["mixed"]
    res["template"] = {k: info[k] for k in ("n_j", "nnz_j1", "nnzb_lu", "nnz_lu", "fill_ratio", "n_levels_l",
                                            "n_levels_u", "lds_resident", "block_threads", "lds_bytes",
                                            "slice_width", "workspace_bytes")}
    regime = ("HBM-resident slices of {} scenarios per workgroup: state and factors streamed from HBM"
              .format(info["slice_width"]) if not info["lds_resident"] else "cache-resident (LDS)")
    res["roofline"] = {
        "mixed": roofline_entry("k_newton<float> (mixed precision, 2 refinement steps)", net.n_bus,
                                info["nnz_lu"], res["mixed"]["mean_updates"], 4, 2, B,
                                res["mixed"]["ms"] * 1e-3, name, "mixed", regime),
        "fp64": roofline_entry("k_newton<double> (FP64)", net.n_bus, infos["fp64"]["nnz_lu"],
                               res["fp64"]["mean_updates"], 8, 0, B, res["fp64"]["ms"] * 1e-3, name, "fp64",
                               regime)}
    return res


def layer_leg_c3(args):
    """The differentiable-layer workload as stated for the 300-bus grid:
    FP64 template, forward Newton to 1e-10, adjoint reusing the factors, the
    voltage-band + angle loss; fwd+bwd samples/s."""
    import torch
    from gen.grids import make_case
    from paper_2606_07099_amd import PFLayer, PFTemplate
    spec, net, sc = make_case("c3")
    B, dev = sc.batch, torch.device("cuda:0")
    d = {k: torch.as_tensor(getattr(sc, k), device=dev) for k in ("pd", "qd", "pg", "vset")}
    tpl = PFTemplate.from_network(net, B, tol=spec.tol, precision="fp64", keep_factors=True)
    layer = PFLayer(tpl)
    leaves = {k: d[k].clone().requires_grad_(True) for k in d}
    state = {}

    def step():
        for v in leaves.values():
            v.grad = None
        vm, va = layer(leaves["pd"], leaves["qd"], leaves["pg"], leaves["vset"])
        L = (torch.relu(vm - 1.05) ** 2).sum() + (torch.relu(0.95 - vm) ** 2).sum() + 0.1 * (va ** 2).sum()
        L.backward()
        state["L"] = L
    sec = median_seconds(step, args.warmup, args.repeats)
    out = [torch.empty((B, net.n_bus), dtype=torch.float64, device=dev) for _ in range(2)] + \
        [torch.empty(B, dtype=torch.int32, device=dev) for _ in range(2)] + \
        [torch.empty(B, dtype=torch.float64, device=dev)]
    sec_fwd = median_seconds(lambda: tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"], out=out),
                             args.warmup, args.repeats)
    info = tpl.info()
    return {"workload": f"{spec.n_bus}-bus synthetic meshed grid, batch {B}, FP64, forward to {spec.tol:g}, "
                        "adjoint reusing the factors at the solution",
            "fwd_bwd_samples_per_s": B / sec, "fwd_bwd_ms": 1e3 * sec,
            "forward_with_refactor_solves_per_s": B / sec_fwd, "forward_ms": 1e3 * sec_fwd,
            "loss": float(state["L"]), **_solve_stats(out),
            "template": {k: info[k] for k in ("nnz_lu", "fill_ratio", "lds_resident", "slice_width",
                                              "workspace_bytes")}}


def layer_leg_c4(args):
    """The 9241-bus batch of 256: mixed-precision forward + FP32-factor
    adjoint in one autograd step (with the configured 2 FP64-residual
    refinement steps, and without refinement as the paper runs it), peak
    device bytes and the LU fill ratio."""
    import torch
    from gen.grids import make_case
    from paper_2606_07099_amd import PFLayer, PFTemplate
    spec, net, sc = make_case("c4")
    B, dev = sc.batch, torch.device("cuda:0")
    d = {k: torch.as_tensor(getattr(sc, k), device=dev) for k in ("pd", "qd", "pg", "vset")}
    res = {}
    for key, refine in (("mixed", 2), ("mixed_unrefined", 0)):
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        tpl = PFTemplate.from_network(net, B, tol=spec.tol, precision="mixed", refine_steps=refine,
                                      keep_factors=True)
        layer = PFLayer(tpl)
        leaves = {k: d[k].clone().requires_grad_(True) for k in d}

        def step():
            for v in leaves.values():
                v.grad = None
            vm, va = layer(leaves["pd"], leaves["qd"], leaves["pg"], leaves["vset"])
            L = (torch.relu(vm - 1.05) ** 2).sum() + (torch.relu(0.95 - vm) ** 2).sum() + 0.1 * (va ** 2).sum()
            L.backward()
        sec = median_seconds(step, args.warmup, args.repeats)
        info = tpl.info()
        res[key] = {"fwd_bwd_samples_per_s": B / sec, "fwd_bwd_ms": 1e3 * sec, "refine_steps": refine,
                    "peak_device_bytes": int(info["workspace_bytes"] + torch.cuda.max_memory_allocated()),
                    "template_workspace_bytes": int(info["workspace_bytes"]),
                    "fill_ratio": info["fill_ratio"], "nnz_lu": info["nnz_lu"], "nnz_j1": info["nnz_j1"]}
        del layer, tpl, leaves
    return res


PHASE_NAMES = ("setup", "mismatch", "fill", "factor_levels", "factor_tail", "bsolve_tail", "bsolve_levels",
               "refine_dv", "refine_residual", "refine_fsolve_levels", "refine_tail", "refine_bsolve_levels",
               "other", "keep_refactor", "output")


def phase_report(grids, args):
    """Per-launch time of each Newton phase (workgroup 0, wall clock), FP64
    and mixed precision (2 refinement steps), on each grid's full batch."""
    import ctypes
    import numpy as np
    import torch
    from gen.grids import make_case
    from paper_2606_07099_amd import PFTemplate
    from paper_2606_07099_amd._lib import check, lib
    L = lib()
    buf = (ctypes.c_uint64 * 32)()
    rate = ctypes.c_double(0.0)
    out = {}
    for name in grids:
        spec, net, sc = make_case(name)
        B, dev = sc.batch, torch.device("cuda:0")
        d = {k: torch.as_tensor(getattr(sc, k), device=dev) for k in ("pd", "qd", "pg", "vset")}
        out[name] = {}
        for prec in ("fp64", "mixed"):
            tpl = PFTemplate.from_network(net, B, tol=spec.tol, precision=prec, keep_factors=False)
            for _ in range(args.warmup):
                tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"])
            check(L.pf_debug_phase_clocks(buf, 32, 1, ctypes.byref(rate)))
            for _ in range(args.repeats):
                tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"])
            check(L.pf_debug_phase_clocks(buf, 32, 1, ctypes.byref(rate)))
            t = np.array(buf[:32], dtype=np.float64)
            launches = max(t[16], 1.0)
            us = 1e6 * t[:15] / rate.value / launches
            out[name][prec] = {"us_per_launch": {k: float(v) for k, v in zip(PHASE_NAMES, us)},
                               "total_us": float(us.sum()), "newton_steps_per_launch": float(t[17] / launches),
                               "refine_steps_per_launch": float(t[18] / launches),
                               "slice_width": tpl.info()["slice_width"]}
            del tpl
    return out


def profile_solve(args, name, spec, net, sc, d):
    """One solve variant of the workload, nothing else on the device: the
    known-size copy (if asked), then --warmup and --steps launches."""
    import torch
    from paper_2606_07099_amd import PFTemplate
    B = sc.batch
    tpl = PFTemplate.from_network(net, B, tol=spec.tol, precision=args.profile_solve, keep_factors=False)
    if args.copy_reference_mib:
        src = torch.ones(args.copy_reference_mib << 17, dtype=torch.float64, device="cuda:0")
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
        del src
    sec = median_seconds(lambda: tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"]), args.warmup, args.steps)
    out = tpl.solve(d["pd"], d["qd"], d["pg"], d["vset"])
    info = tpl.info()
    print(json.dumps({"workload": f"{spec.n_bus}-bus synthetic meshed grid, batch {B}, tol {spec.tol:g}",
                      "solve": args.profile_solve, "median_ms": 1e3 * sec, "solves_per_s": B / sec,
                      "nnz_lu": info["nnz_lu"], "slice_width": info["slice_width"],
                      **_solve_stats(out)}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not supported "
                                   "(scenarios are independent and would shard across GPUs with no exchange)"}))
        sys.exit(2)
    if args.phases:
        os.environ["SABLE_PHASE_CLOCKS"] = "1"   # before the library is loaded
    import numpy as np
    import torch
    from gen.grids import SPECS, make_case
    from paper_2606_07099_amd import PFTemplate, PFLayer
    from paper_2606_07099_amd.training import SyntheticDispatchTask

    name = args.workload
    spec, net, sc = make_case(name, scenario_mode=args.scenarios)
    B = sc.batch
    dev = torch.device("cuda:0")
    d = {k: torch.as_tensor(getattr(sc, k), device=dev) for k in ("pd", "qd", "pg", "vset")}
    if args.profile_solve:
        profile_solve(args, name, spec, net, sc, d)
        return
    t_build = time.perf_counter()
    tpl64 = PFTemplate.from_network(net, B, tol=spec.tol, precision="fp64", keep_factors=False)
    t_build = time.perf_counter() - t_build
    tplmp = PFTemplate.from_network(net, B, tol=spec.tol, precision="mixed", keep_factors=False)
    tpllay = PFTemplate.from_network(net, B, tol=spec.tol, precision="mixed", keep_factors=True)
    # variants reported beside the configured 2-step refinement: adaptive
    # refinement (at most 2 steps) and no refinement at all
    tplad = PFTemplate.from_network(net, B, tol=spec.tol, precision="mixed", keep_factors=False,
                                    refine_adaptive=True)
    tplr0 = PFTemplate.from_network(net, B, tol=spec.tol, precision="mixed", keep_factors=False,
                                    refine_steps=0)
    layer = PFLayer(tpllay)
    # synthetic end-to-end training: an MLP proposes the decision block, the
    # layer completes it (both steps), Adam updates the MLP
    task = SyntheticDispatchTask(net, sc, dev, precision="mixed", tol=spec.tol)
    train_losses = []
    # the four operators of the layer (J1, J1^T, J2^T, J3^T) refreshed in place
    # as batch-global CSR matrices at the mixed-precision solution
    from paper_2606_07099_amd.pf import PF_OP_J1, PF_OP_J1T, PF_OP_J2T, PF_OP_J3T
    op_ids = (PF_OP_J1, PF_OP_J1T, PF_OP_J2T, PF_OP_J3T)
    op_mats = {}

    def refresh_operators():
        for w in op_ids:
            op_mats[w] = tplmp.operator(w, outmp[0], outmp[1], out=op_mats.get(w))
    # both completion steps (Step 2 recovers the generation block) under a
    # loss that adds a generation cost and a reactive-reserve penalty
    layerc = PFLayer(tpllay, recover=True)
    slack_w = torch.as_tensor((net.bus_type == 2).astype(np.float64), device=dev)
    gen_w = torch.as_tensor((net.bus_type != 0).astype(np.float64), device=dev)
    info64, infomp = tpl64.info(), tplmp.info()

    out64 = [torch.empty((B, net.n_bus), dtype=torch.float64, device=dev) for _ in range(2)] + \
        [torch.empty(B, dtype=torch.int32, device=dev) for _ in range(2)] + \
        [torch.empty(B, dtype=torch.float64, device=dev)]
    outmp = [x.clone() for x in out64]
    outad = [x.clone() for x in out64]
    outr0 = [x.clone() for x in out64]
    leaves = {k: d[k].clone().requires_grad_(True) for k in d}

    def layer_step():
        for v in leaves.values():
            v.grad = None
        vm, va = layer(leaves["pd"], leaves["qd"], leaves["pg"], leaves["vset"])
        L = (torch.relu(vm - 1.05) ** 2).sum() + (torch.relu(0.95 - vm) ** 2).sum() + 0.1 * (va ** 2).sum()
        L.backward()

    def layer_completed_step():
        for v in leaves.values():
            v.grad = None
        vm, va, po, qo = layerc(leaves["pd"], leaves["qd"], leaves["pg"], leaves["vset"])
        L = ((torch.relu(vm - 1.05) ** 2).sum() + (torch.relu(0.95 - vm) ** 2).sum() + 0.1 * (va ** 2).sum()
             + ((po * slack_w) ** 2).sum() + 0.5 * ((qo * gen_w) ** 2).sum())
        L.backward()

    if args.copy_reference_mib:
        src = torch.ones(args.copy_reference_mib << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    stream = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    for _ in range(args.warmup):
        tpl64.solve(d["pd"], d["qd"], d["pg"], d["vset"], out=out64)
        tplmp.solve(d["pd"], d["qd"], d["pg"], d["vset"], out=outmp)
        tplad.solve(d["pd"], d["qd"], d["pg"], d["vset"], out=outad)
        tplr0.solve(d["pd"], d["qd"], d["pg"], d["vset"], out=outr0)
        layer_step()
        layer_completed_step()
        train_losses.append(task.step())
        refresh_operators()
    torch.cuda.synchronize()

    marks = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e = [ev() for _ in range(9)]
        e[0].record(stream)
        tpl64.solve(d["pd"], d["qd"], d["pg"], d["vset"], out=out64)
        e[1].record(stream)
        tplmp.solve(d["pd"], d["qd"], d["pg"], d["vset"], out=outmp)
        e[2].record(stream)
        layer_step()
        e[3].record(stream)
        tplad.solve(d["pd"], d["qd"], d["pg"], d["vset"], out=outad)
        e[4].record(stream)
        tplr0.solve(d["pd"], d["qd"], d["pg"], d["vset"], out=outr0)
        e[5].record(stream)
        layer_completed_step()
        e[6].record(stream)
        train_losses.append(task.step())
        e[7].record(stream)
        refresh_operators()
        e[8].record(stream)
        marks.append(e)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    def med(k):
        return float(np.median([m[k].elapsed_time(m[k + 1]) for m in marks]) * 1e-3)
    t64, tmp, tfb, tad, tr0, tfc, ttr, top = (med(k) for k in range(8))
    op_nnz = {int(w): int(op_mats[w].values().numel()) for w in op_ids}
    train_losses = [float(x) for x in train_losses]
    st = {k: _solve_stats(o) for k, o in (("fp64", out64), ("mixed", outmp), ("mixed_adaptive", outad),
                                          ("mixed_unrefined", outr0))}
    mp_rate = B / tmp
    cache_regime = ("cache-resident: state, factors and schedules live in LDS (the HBM counters read "
                    "7.0 MB per launch, the boundary I/O, against the streaming model's bytes), and the "
                    "SQ counters show the launch waiting on LDS results and barriers; frac is the "
                    "streaming model over the HBM peak, not an HBM efficiency"
                    if infomp["lds_resident"] else "HBM-resident slices")
    roof = roofline_entry("k_newton<float> (mixed-precision Newton, one launch per solve)", net.n_bus,
                          infomp["nnz_lu"], st["mixed"]["mean_updates"], 4, 2, B, tmp, name, "mixed",
                          cache_regime)
    if not (B == SPECS[name].batch and args.scenarios == "lognormal"):
        roof["traffic"] = roof["traffic_over_algorithmic"] = None

    res = {
        "metric": "PF solves/sec (FP32-LU+refine vs FP64) & PF-layer fwd+bwd samples/sec @1e-8pu",
        "value": mp_rate,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": ("synthetic (seeded meshed grid and lognormal load scenarios)" if args.scenarios == "lognormal"
                 else "synthetic (seeded meshed grid, uniform +-10% P and Q load perturbations)"),
        "config": {"workload": f"{spec.n_bus}-bus synthetic meshed grid, batch {B}, tol {spec.tol:g}",
                   "n_bus": spec.n_bus, "n_pv": spec.n_pv, "n_branch": spec.n_branch,
                   "batch": B, "tol": spec.tol, "refine_steps": 2, "scenarios": args.scenarios,
                   "parallelism": "single GPU"},
        "timing": f"median over {args.steps} steps of HIP events on the kernels' stream, after {args.warmup} "
                  "warm-up steps",
        "fp64_solves_per_s": B / t64,
        "mixed_solves_per_s": mp_rate,
        "layer_fwd_bwd_samples_per_s": B / tfb,
        "mixed_adaptive_solves_per_s": B / tad,
        "mixed_unrefined_solves_per_s": B / tr0,
        "layer_completed_fwd_bwd_samples_per_s": B / tfc,
        "train_samples_per_s": B / ttr,
        "operator_refresh": {"operators": "J1, J1^T, J2^T, J3^T (batch-global CSR, values in place)",
                             "values": sum(op_nnz.values()), "ms": 1e3 * top,
                             "values_per_s": sum(op_nnz.values()) / top},
        "train": {"task": "MLP (2 x 256 hidden) -> PV dispatch and |V| setpoints -> PF layer (both "
                          "completion steps, mixed precision) -> generation cost + voltage and "
                          "reactive penalties -> Adam",
                  "loss_first": train_losses[0], "loss_last": train_losses[-1],
                  "optimizer_steps": len(train_losses),
                  "peak_torch_bytes": int(torch.cuda.max_memory_allocated()),
                  "template_workspace_bytes": int(task.tpl.info()["workspace_bytes"])},
        "ms": {"fp64_solve": 1e3 * t64, "mixed_solve": 1e3 * tmp,
               "mixed_adaptive_solve": 1e3 * tad, "mixed_unrefined_solve": 1e3 * tr0,
               "layer_fwd_bwd": 1e3 * tfb, "layer_completed_fwd_bwd": 1e3 * tfc,
               "train_step": 1e3 * ttr, "template_build": 1e3 * t_build},
        "iterations": {k: v["iterations"] for k, v in st.items()},
        "converged": {k: v["converged"] for k, v in st.items()},
        "max_final_mismatch": {k: v["max_final_mismatch"] for k, v in st.items()},
        "device_memory": {"templates_workspace_bytes": int(sum(t.info()["workspace_bytes"] for t in
                                                              (tpl64, tplmp, tpllay, tplad, tplr0, task.tpl))),
                          "torch_peak_bytes": int(torch.cuda.max_memory_allocated()),
                          "per_template": {"fp64": int(info64["workspace_bytes"]),
                                           "mixed": int(infomp["workspace_bytes"]),
                                           "mixed_keep_factors": int(tpllay.info()["workspace_bytes"])}},
        "template": {k: infomp[k] for k in ("n_j", "nnz_j1", "nnzb_lu", "nnz_lu", "fill_ratio",
                                            "n_levels_l", "n_levels_u", "lds_resident",
                                            "block_threads", "lds_bytes", "slice_width", "workspace_bytes")},
        "roofline": roof,
        "phase_clocks_build": bool(args.phases),
    }
    del tpl64, tplmp, tpllay, tplad, tplr0, layer, layerc, task, op_mats
    torch.cuda.empty_cache()
    legs = [g for g in args.legs.split(",") if g and g != "none" and g != name]
    if legs:
        res["legs"] = {}
    for g in legs:
        if g == "c3":
            res["legs"]["c3_layer"] = layer_leg_c3(args)
        else:
            res["legs"][g] = solve_leg(g, args)
            if g == "c4":
                res["legs"][g]["layer_fwd_bwd"] = layer_leg_c4(args)
        torch.cuda.empty_cache()
    if args.phases:
        res["phases"] = phase_report([name] + [g for g in legs], args)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(name, B, args.cpu_seconds, args.scenarios)
        res["cpu_baseline"]["cpu_model"] = cpu_model()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
