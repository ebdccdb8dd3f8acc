"""Benchmark: batched Newton power flow on one MI355X.

Workload (default): synthetic 118-bus meshed grid (tree + 60 extra branches,
53 PV, 64 PQ, slack bus 0), batch of 1024 load scenarios, tolerance 1e-8 pu,
flat start.  One step runs the whole path on the batch, inputs resident in
HBM: the plain FP64 Newton solve, the mixed-precision solve (FP32 LU
refactorisation and solves, FP64 mismatch / convergence / update and two
FP64-residual refinement steps), one differentiable-layer forward + backward
(mixed-precision solve keeping the factors + adjoint), the mixed-precision
solve with adaptive refinement and without refinement, and one layer forward
+ backward through both completion steps (Step-2 recovery of the generation
block and its backward term).  Each part is timed with HIP events on the
stream the kernels run on.

``value`` is the mixed-precision solves/s; the other rates are reported
beside it.  The roofline entry covers the dominant kernel (the
mixed-precision Newton kernel): algorithmic bytes per launch (the model in
``algorithmic_bytes_per_solve``) over its measured average launch duration.
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

# HBM bytes per launch of the mixed-precision Newton kernel on the default
# workload, from rocprofv3 FETCH_SIZE and WRITE_SIZE passes (each scaled by
# the same counter on a 512 MiB device-to-device copy), keyed by the SHA-256
# of the kernel sources they were taken on; a changed kernel reports null.
# Sources: profiles/k_newton_118bus_b1024_hbm_counters.md,
# profiles/k_newton_1354bus_b4096_hbm_counters.md
MEASURED_TRAFFIC = {
    "54aa4290f59904b38a63c93c86efd80e2d2982242dc8796505c573aabb1edc36": {"c1": 6940356,
                                                                         "c2": 46518049629},
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
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


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not supported "
                                   "(scenarios are independent and would shard across GPUs with no exchange)"}))
        sys.exit(2)
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

    t64 = np.array([m[0].elapsed_time(m[1]) for m in marks]) * 1e-3
    tmp = np.array([m[1].elapsed_time(m[2]) for m in marks]) * 1e-3
    tfb = np.array([m[2].elapsed_time(m[3]) for m in marks]) * 1e-3
    tad = np.array([m[3].elapsed_time(m[4]) for m in marks]) * 1e-3
    tr0 = np.array([m[4].elapsed_time(m[5]) for m in marks]) * 1e-3
    tfc = np.array([m[5].elapsed_time(m[6]) for m in marks]) * 1e-3
    ttr = np.array([m[6].elapsed_time(m[7]) for m in marks]) * 1e-3
    top = np.array([m[7].elapsed_time(m[8]) for m in marks]) * 1e-3
    op_nnz = {int(w): int(op_mats[w].values().numel()) for w in op_ids}
    train_losses = [float(x) for x in train_losses]
    itad, stad, fnad = (x.cpu().numpy() for x in outad[2:])
    itr0, str0, fnr0 = (x.cpu().numpy() for x in outr0[2:])
    it64, st64, fn64 = (x.cpu().numpy() for x in out64[2:])
    itmp, stmp, fnmp = (x.cpu().numpy() for x in outmp[2:])
    mp_rate = B / tmp.mean()
    # dominant kernel: the mixed-precision Newton kernel, one launch per solve
    bytes_launch = B * algorithmic_bytes_per_solve(net.n_bus, infomp["nnz_lu"], float(itmp.mean()), 4, 2)
    achieved = bytes_launch / tmp.mean() / 1e9

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
        "fp64_solves_per_s": B / t64.mean(),
        "mixed_solves_per_s": mp_rate,
        "layer_fwd_bwd_samples_per_s": B / tfb.mean(),
        "mixed_adaptive_solves_per_s": B / tad.mean(),
        "mixed_unrefined_solves_per_s": B / tr0.mean(),
        "layer_completed_fwd_bwd_samples_per_s": B / tfc.mean(),
        "train_samples_per_s": B / ttr.mean(),
        "operator_refresh": {"operators": "J1, J1^T, J2^T, J3^T (batch-global CSR, values in place)",
                             "values": sum(op_nnz.values()), "ms": 1e3 * top.mean(),
                             "values_per_s": sum(op_nnz.values()) / top.mean()},
        "train": {"task": "MLP (2 x 256 hidden) -> PV dispatch and |V| setpoints -> PF layer (both "
                          "completion steps, mixed precision) -> generation cost + voltage and "
                          "reactive penalties -> Adam",
                  "loss_first": train_losses[0], "loss_last": train_losses[-1],
                  "optimizer_steps": len(train_losses),
                  "peak_torch_bytes": int(torch.cuda.max_memory_allocated()),
                  "template_workspace_bytes": int(task.tpl.info()["workspace_bytes"])},
        "ms": {"fp64_solve": 1e3 * t64.mean(), "mixed_solve": 1e3 * tmp.mean(),
               "mixed_adaptive_solve": 1e3 * tad.mean(), "mixed_unrefined_solve": 1e3 * tr0.mean(),
               "layer_fwd_bwd": 1e3 * tfb.mean(), "layer_completed_fwd_bwd": 1e3 * tfc.mean(),
               "train_step": 1e3 * ttr.mean(),
               "template_build": 1e3 * t_build},
        "iterations": {"fp64": np.bincount(it64).tolist(), "mixed": np.bincount(itmp).tolist(),
                       "mixed_adaptive": np.bincount(itad).tolist(),
                       "mixed_unrefined": np.bincount(itr0).tolist()},
        "converged": {"fp64": int((st64 == 0).sum()), "mixed": int((stmp == 0).sum()),
                      "mixed_adaptive": int((stad == 0).sum()), "mixed_unrefined": int((str0 == 0).sum())},
        "max_final_mismatch": {"fp64": float(fn64.max()), "mixed": float(fnmp.max()),
                               "mixed_adaptive": float(fnad.max()), "mixed_unrefined": float(fnr0.max())},
        "device_memory": {"templates_workspace_bytes": int(sum(t.info()["workspace_bytes"] for t in
                                                              (tpl64, tplmp, tpllay, tplad, tplr0, task.tpl))),
                          "torch_peak_bytes": int(torch.cuda.max_memory_allocated()),
                          "per_template": {"fp64": int(info64["workspace_bytes"]),
                                           "mixed": int(infomp["workspace_bytes"]),
                                           "mixed_keep_factors": int(tpllay.info()["workspace_bytes"])}},
        "template": {k: infomp[k] for k in ("n_j", "nnz_j1", "nnzb_lu", "nnz_lu", "fill_ratio",
                                            "n_levels_l", "n_levels_u", "lds_resident",
                                            "block_threads", "lds_bytes", "slice_width", "workspace_bytes")},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (MEASURED_TRAFFIC.get(kernel_source_hash(), {}).get(name)
                                 if B == SPECS[name].batch and args.scenarios == "lognormal" else None),
                     "kernel_source_sha256": kernel_source_hash()[:16],
                     "kernel": "k_newton<float> (mixed-precision Newton, one launch per solve)",
                     "bytes_per_launch": bytes_launch, "avg_launch_ms": 1e3 * tmp.mean()},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(name, B, args.cpu_seconds, args.scenarios)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
