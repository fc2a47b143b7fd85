#!/usr/bin/env python3
"""Throughput of the filtered SELBM time step on one MI355X.

Workload: the 3D Taylor-Green vortex, D3Q27, periodic [0, 2 pi]^3 split into
16^3 hexahedra of order N = 7 (4096 elements, 512 nodes each, 56.6 M
node-velocities), Re = 1600, Ma = 0.1, the paper's quadratic filter
(gamma = 0.1, k_c = 2), SSPRK3, inputs resident in HBM. The headline form is
FP32 deviation storage; the FP64, learned-closure and discontinuous forms are
timed beside it, and the other workload shapes (2D Taylor-Green, double shear
layer, curved channel, the paper's D3Q19 Taylor-Green runs at N = 8 and 12,
O-grid pipe at N = 7 and its N = 5 closure variant) get throughput lines of
their own.

Prints ONE JSON line. ``value`` is node-velocity updates per second (1e9,
local nodes E (N+1)^3 Q per step). ``roofline`` prices one later SSPRK stage
(its element kernel plus its shared-node assembly, average launch durations
measured here with HIP events on the library's stream) with the method's
algorithmic bytes per node-velocity for such a stage, s (3 + (d^2 + 1)/Q):
read the stage value and the post-collision state, write the result, read the
metric and mass weight once per node; ``step`` gives the whole step against
s (8 + 3 (d^2 + 1)/Q). ``cpu_baseline`` times the FP64 CPU oracle, built
with -O2 -march=native on this host, on whole-mesh steps of the same
workload, on all host threads and on one.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "node-velocity updates/sec (GLUPS) and % HBM roofline, FP64 vs FP32 vs closure"
PEAK_HBM_GBS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "tgv3d_n7_q27_fp32dev_hbm_counters.json")


def src_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2509_19171_amd", "csrc")
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def method_bytes(dim, Q, s):
    """The method's algorithmic bytes per node-velocity (collision recomputed
    in registers, filter fused, so no passes of their own): SSPRK3 makes 8
    state accesses per step (stage 1 reads f and writes f1; stages 2 and 3
    read f, the stage value and write the next), and every stage reads the
    metric and the mass weight (dim^2 + 1 values per node, shared by the Q
    velocities)."""
    geo = (dim * dim + 1) / Q
    return {"stage1": s * (2 + geo), "later_stage": s * (3 + geo), "step": s * (8 + 3 * geo)}


def algorithmic_bytes(info, Q, s):
    """Per step: the method's bytes (method_bytes) times the node-velocities.
    Per launch, this implementation's own count of what each kernel must move
    at least, every value once:
      stage1   read the operand and write the post-collision state at every
               unique node, write the density, write interior results and
               the boundary-node element contributions, read the metric;
      stage23  read the operand at every unique node, read the post-collision
               state and write the result at interior nodes, write the
               boundary-node contributions, read the metric, the interior
               inverse mass and density;
      assembly read the contributions, read two states and write one at every
               node group, read the group mass and density and the member
               lists (4-byte ints);
      filter   read and write every unique node."""
    E, npn, dim = info["E"], info["np"], info["dim"]
    nb = info["boundary_nodes_per_element"]
    ni = npn - nb
    G = info["unique_nodes"]
    ng = info["groups"]
    nv = E * npn * Q
    step = method_bytes(dim, Q, s)["step"] * nv
    per = {
        "stage1": s * (2 * Q * G + G + Q * E * ni + Q * E * nb + E * npn * dim * dim),
        "stage23": s * (Q * G + 2 * Q * E * ni + Q * E * nb + E * npn * dim * dim + 2 * E * ni),
        "assembly": s * (Q * E * nb + 3 * Q * ng + 2 * ng) + 4 * (E * nb + ng),
        "filter": s * 2 * Q * G,
        # closure: read the state at every unique node and the metric, write 6 features per node id
        "features": s * (Q * G + E * npn * dim * dim) + 8 * E * npn + 24 * G,
        # closure network: read 6 features, write one increment per node id
        "network": 28 * G,
    }
    return nv, step, per


MLP_FLOP_PER_ROW = 2 * (6 * 64 + 64 * 64 * 2 + 64)  # 17280: three hidden layers and the output
PEAK_FP32_MATRIX_TFLOPS = 157.3
# training: forward, back-propagated deltas and weight gradient, each a pass
# of the size of the forward
TRAIN_FLOP_PER_ROW = 3 * MLP_FLOP_PER_ROW


def time_form(case, precision, steps, warmup, torch, closure=None):
    from paper_2509_19171_amd import sel

    sim = sel.from_case(case, precision, closure=closure)
    info = sim.mesh.info()
    sim.step(warmup)
    sim.sync()
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    sim.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    # second timed window: HIP events around every launch for per-kernel durations
    kern = sim.step_timed(steps)
    sim.sync()
    out = dict(ms_total=ms, ms_per_step=ms / steps, kernels=kern, info=info)
    del sim
    torch.cuda.empty_cache()
    return out


def time_training(torch, steps=100, warmup=10, batch=4096, rows=1 << 20):
    """Adam steps of the closure network on seeded minibatches of a seeded
    feature set (the recipe of the closure training: minibatches of 4096)."""
    from paper_2509_19171_amd import inputs as I
    from paper_2509_19171_amd import sel

    g = torch.Generator(device="cpu").manual_seed(7)
    X = torch.randn((rows, 6), generator=g).cuda()
    y = torch.rand((rows,), generator=g).cuda()
    idx = [torch.randint(0, rows, (batch,), generator=g, dtype=torch.int32).cuda() for _ in range(8)]
    params = torch.tensor(I.closure_blob(0, mean=[0.0] * 6, std=[1.0] * 6), device="cuda")
    tr = sel.MLPTrainer(params)
    for k in range(warmup):
        tr.step(X, y, idx=idx[k % 8], want_loss=False)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for k in range(steps):
        tr.step(X, y, idx=idx[k % 8], want_loss=False)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    tflops = TRAIN_FLOP_PER_ROW * batch / (ms * 1e-3) / 1e12
    return {"minibatch": batch, "ms_per_adam_step": round(ms, 5), "samples_per_s": round(batch / (ms * 1e-3), 1),
            "bound": "mfma", "achieved_TFLOPs": round(tflops, 3), "peak_TFLOPs": PEAK_FP32_MATRIX_TFLOPS,
            "frac": round(tflops / PEAK_FP32_MATRIX_TFLOPS, 5), "flop_per_sample": TRAIN_FLOP_PER_ROW}


def form_summary(f, nv, Q, s):
    """Rate, step time and the step's algorithmic HBM fraction of one form
    (its own mesh information: the discontinuous form has more node ids); the
    closure form adds the bytes of its feature and network kernels."""
    info = f["info"]
    out = {"value": round(nv / (f["ms_per_step"] * 1e-3) / 1e9, 3), "ms_per_step": round(f["ms_per_step"], 5)}
    kern = f["kernels"]
    _, step_bytes, per = algorithmic_bytes(info, Q, s)
    if kern.get("network", (0, 0))[1]:
        step_bytes += per["features"] + per["network"]
    gbs = step_bytes / (f["ms_per_step"] * 1e-3) / 1e9
    out["step_hbm"] = {"algorithmic_bytes_per_step": int(step_bytes), "achieved": round(gbs, 1),
                       "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4)}
    if kern.get("network", (0, 0))[1]:
        fms, fn = kern["features"]
        mms, mn = kern["network"]
        G = info["unique_nodes"]
        out["closure_kernels"] = {
            "features": {"avg_ms": round(fms / fn, 5),
                         "algorithmic_GBs": round(per["features"] / (fms / fn * 1e-3) / 1e9, 1)},
            "network": {"avg_ms": round(mms / mn, 5), "bound": "mfma",
                        "achieved_TFLOPs": round(MLP_FLOP_PER_ROW * G / (mms / mn * 1e-3) / 1e12, 2),
                        "peak_TFLOPs": PEAK_FP32_MATRIX_TFLOPS, "dtype": "f32",
                        "frac": round(MLP_FLOP_PER_ROW * G / (mms / mn * 1e-3) / 1e12 / PEAK_FP32_MATRIX_TFLOPS, 4)},
            "share_of_step": round((fms / fn + mms / mn) / f["ms_per_step"], 4),
        }
    return out


def cpu_baseline(case, budget_s=12.0):
    """The FP64 oracle, built here with -O2 -march=native, on whole-mesh steps
    of the workload: on every thread OpenMP is given (the machine's CPU share),
    then on one thread. Each leg runs about budget_s seconds at most."""
    import shutil
    import tempfile

    import oracle

    tmpdir = tempfile.mkdtemp(prefix="sel_oracle_")
    try:
        oracle.use_library(oracle.build(native=True, path=os.path.join(tmpdir, "liboracle_native.so")))
        nproc = os.cpu_count()
        try:
            import subprocess

            nproc = int(subprocess.run(["nproc"], capture_output=True, text=True, check=True).stdout.strip())
        except Exception:
            pass
        threads = oracle.get_threads()
        legs = {}
        for name, nt in (("all_threads", threads), ("single_thread", 1)):
            oracle.set_threads(nt)
            o = oracle.from_case(case)
            t0 = time.perf_counter()
            o.step(1)
            t1 = time.perf_counter() - t0
            n = 1
            extra = int(max(0, min(8, budget_s / max(t1, 1e-3) - 1)))
            if extra:
                t0 = time.perf_counter()
                o.step(extra)
                t1 += time.perf_counter() - t0
                n += extra
            legs[name] = {"value": case.nv * n / t1 / 1e9, "threads": nt, "steps": n, "seconds": round(t1, 2)}
            del o
        oracle.set_threads(threads)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    a = legs["all_threads"]
    return {"value": a["value"], "unit": "GNVU/s", "cores": a["threads"], "kind": "oracle",
            "sample": f"{a['steps']} FP64 step(s) of the same 16^3 N=7 D3Q27 workload (whole mesh, "
                      f"{a['seconds']} s, {a['threads']} OpenMP threads; oracle built with -O2 -march=native)",
            "single_thread": {"value": legs["single_thread"]["value"], "unit": "GNVU/s",
                              "sample": f"{legs['single_thread']['steps']} whole-mesh step(s), "
                                        f"{legs['single_thread']['seconds']} s"},
            "nproc": nproc}


def time_config(name, case, precision, steps, warmup, torch, closure=None, hbm=True):
    """Throughput line of another workload shape (not the headline)."""
    f = time_form(case, precision, steps, warmup, torch, closure=closure)
    info = f["info"]
    s = 4 if precision.startswith("fp32") else 8
    nv, step_bytes, per = algorithmic_bytes(info, case.Q, s)
    if closure is not None:
        step_bytes += per["features"] + per["network"]
    out = {"workload": name, "precision": precision + ("+closure" if closure is not None else ""),
           "elements": info["E"], "order": info["N"], "Q": case.Q, "node_velocities": nv, "steps": steps,
           "value": round(nv / (f["ms_per_step"] * 1e-3) / 1e9, 3), "unit": "GNVU/s",
           "ms_per_step": round(f["ms_per_step"], 5)}
    if hbm:
        gbs = step_bytes / (f["ms_per_step"] * 1e-3) / 1e9
        out["step_hbm"] = {"algorithmic_bytes_per_step": int(step_bytes), "achieved": round(gbs, 1),
                           "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4)}
    else:
        out["step_hbm"] = None
        out["note"] = "working set fits in the 256 MB last-level cache: HBM fraction not meaningful"
    return out


def other_configs(torch, steps):
    """The other workload shapes, each at its configured size."""
    from paper_2509_19171_amd import inputs as I

    out = []
    k = max(20, steps // 5)
    for prec in ("fp64", "fp32dev"):
        out.append(time_config("2D Taylor-Green vortex, D2Q9, 8x8 quads, N=5", I.case_tgv2d(), prec, k, 10, torch,
                               hbm=False))
        out.append(time_config("2D double shear layer, D2Q9, 32x32 quads, N=7, exponential filter",
                               I.case_double_shear(), prec, k, 10, torch, hbm=False))
        out.append(time_config("2D curved Poiseuille channel, D2Q9, 16x8 quads, N=7, FBB walls",
                               I.case_poiseuille(curved=True), prec, k, 10, torch, hbm=False))
    # the paper's 3D Taylor-Green runs (Sec. 3.4): D3Q19, 16^3 hexes, N = 8 and
    # 12 (N = 12 takes the several-nodes-per-thread kernels)
    kt = max(10, steps // 20)
    for N in (8, 12):
        print(f"[bench] timing the Taylor-Green vortex at N = {N}", file=sys.stderr, flush=True)
        tgv = I.case_tgv3d(nel=16, N=N, Q=19, Re=1600.0, Ma=0.1 / math.sqrt(3.0), steps=0, filt="quad")
        for prec in ("fp32dev", "fp64"):
            out.append(time_config(f"3D Taylor-Green vortex, D3Q19, 16^3 hexes, N={N}, Re 1600", tgv, prec, kt, 3,
                                   torch))
        del tgv
        torch.cuda.empty_cache()
    print("[bench] timing the O-grid pipe", file=sys.stderr, flush=True)
    pipe = I.case_pipe()
    kp = max(10, steps // 10)
    for prec in ("fp32dev", "fp64"):
        out.append(time_config("turbulent pipe, D3Q27, O-grid of 20,480 curved hexes, N=7, FBB wall", pipe, prec,
                               kp, 5, torch))
    del pipe
    torch.cuda.empty_cache()
    coarse = I.case_pipe(N=5)
    blob = I.closure_blob(0, mean=[0.0] * 6, std=[1.0] * 6)
    out.append(time_config("turbulent pipe, coarse N=5 variant, plain", coarse, "fp32dev", kp, 5, torch))
    out.append(time_config("turbulent pipe, coarse N=5 variant, learned closure", coarse, "fp32dev", kp, 5, torch,
                           closure=blob))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", default="fp32dev", choices=["fp32dev", "fp64"])
    ap.add_argument("--nel", type=int, default=16)
    ap.add_argument("--order", type=int, default=7)
    ap.add_argument("--q", type=int, default=27, choices=[19, 27], help="lattice D3Q19 or D3Q27")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-form", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the step runs on one GPU; --gpus {args.gpus} is not supported "
              "(the element-partitioned multi-GPU step is designed, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2509_19171_amd import inputs as I
    from paper_2509_19171_amd import sel

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        dst.copy_(src)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "ms": ms,
                          "GBs_read_plus_write": 2 * nbytes / (ms * 1e-3) / 1e9}), flush=True)
        return
    sel.load()
    case = I.case_tgv3d(nel=args.nel, N=args.order, Q=args.q, steps=0)
    # the closure and the discontinuous coupling take one thread per element
    # node: not built for elements of more than 1024 nodes
    one_thread_per_node = (args.order + 1) ** 3 <= 1024
    forms = {}
    order = [args.precision] + ([] if args.no_other_form else [p for p in ("fp32dev", "fp64") if p != args.precision])
    for prec in order:
        k = args.steps if prec == args.precision else max(20, args.steps // 2)
        w = args.warmup if prec == args.precision else max(5, args.warmup // 2)
        print(f"[bench] timing {prec}: {w} warmup + {k} steps", file=sys.stderr, flush=True)
        forms[prec] = time_form(case, prec, k, w, torch)
    if not args.no_other_form and one_thread_per_node:
        # closure form: same workload, features and network inferred every step
        # (a seeded untrained network; the cost does not depend on the weights)
        blob = I.closure_blob(0, mean=[0.0] * 6, std=[1.0] * 6)
        k, w = max(20, args.steps // 2), max(5, args.warmup // 2)
        print(f"[bench] timing fp32dev+closure: {w} warmup + {k} steps", file=sys.stderr, flush=True)
        forms["fp32dev+closure"] = time_form(case, "fp32dev", k, w, torch, closure=blob)
        # discontinuous coupling on the same workload: every element keeps its
        # own face nodes and the elements couple through upwind face fluxes
        print(f"[bench] timing fp32dev+dg: {w} warmup + {k} steps", file=sys.stderr, flush=True)
        forms["fp32dev+dg"] = time_form(dataclasses.replace(case, coupling="dg"), "fp32dev", k, w, torch)
        print("[bench] timing closure training steps", file=sys.stderr, flush=True)
        training = time_training(torch)

    head = forms[args.precision]
    info = head["info"]
    s = 4 if args.precision == "fp32dev" else 8
    nv, step_bytes, per_kind = algorithmic_bytes(info, case.Q, s)
    value = nv / (head["ms_per_step"] * 1e-3) / 1e9
    kern = head["kernels"]
    avg = {k: v[0] / v[1] for k, v in kern.items() if v[1]}
    # roofline: one later SSPRK stage = its element kernel + its shared-node
    # assembly (the assembly runs once per stage with the same work), priced
    # with the method's bytes per node-velocity of such a stage
    stage_ms = avg["stage23"] + avg["assembly"]
    stage_bytes = method_bytes(info["dim"], case.Q, s)["later_stage"] * nv
    ach = stage_bytes / (stage_ms * 1e-3) / 1e9
    traffic = None
    counters = None
    if os.path.exists(COUNTERS):
        with open(COUNTERS) as fh:
            cnt = json.load(fh)
        if (cnt.get("src_hash") == src_hash() and cnt.get("precision") == args.precision
                and cnt.get("workload") == f"tgv3d {args.nel}^3 N={args.order} D3Q{args.q}"):
            counters = cnt.get("hbm_bytes_per_launch", {})
            if "stage23" in counters and "assembly" in counters:
                traffic = int(counters["stage23"] + counters["assembly"])
    roof = {"bound": "hbm",
            "kernel": "later SSPRK stage: element kernel (k_stage23_mf for FP32 3D order 7, else k_stage: "
                      "streaming, wall flux, interior update) + k_group_split shared-node assembly",
            "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": int(stage_bytes),
            "bytes_per_node_velocity": round(method_bytes(info["dim"], case.Q, s)["later_stage"], 4),
            "avg_launch_ms": round(stage_ms, 5),
            "avg_launch_ms_parts": {"element": round(avg["stage23"], 5), "assembly": round(avg["assembly"], 5)}}
    step_gbs = step_bytes / (head["ms_per_step"] * 1e-3) / 1e9
    result = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GNVU/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32dev" else "f64",
        "data": "synthetic",
        "config": {"workload": f"3D Taylor-Green vortex, D3Q{args.q}, periodic [0,2pi]^3, {args.nel}^3 hexes, "
                               f"N={args.order}, Re=1600, Ma=0.1, quadratic filter, SSPRK3",
                   "precision": args.precision, "elements": info["E"], "order": args.order, "Q": case.Q,
                   "local_nodes": info["E"] * info["np"], "unique_nodes": info["unique_nodes"],
                   "node_velocities": nv},
        "roofline": roof,
        # the same steps counted over unique nodes (each shared node once)
        "unique_node_rate": {"value": round(info["unique_nodes"] * case.Q / (head["ms_per_step"] * 1e-3) / 1e9, 3),
                             "unit": "GNVU/s"},
        "step": {"algorithmic_bytes_per_step": int(step_bytes), "achieved": round(step_gbs, 1),
                 "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(step_gbs / PEAK_HBM_GBS, 4)},
        "kernels": {k: {"ms_total": round(v[0], 4), "launches": v[1],
                        "avg_ms": round(v[0] / v[1], 5),
                        # this implementation's own per-launch count (algorithmic_bytes)
                        "design_bytes_per_launch": int(per_kind[k]),
                        "design_GBs": round(per_kind[k] / (v[0] / v[1] * 1e-3) / 1e9, 1),
                        "hbm_bytes_per_launch_counters": (counters or {}).get(k)}
                    for k, v in kern.items() if v[1]},
        "forms": {p: form_summary(f, nv, case.Q, 4 if p.startswith("fp32") else 8) for p, f in forms.items()},
        "src_hash": src_hash(),
    }
    if not args.no_other_form:
        if one_thread_per_node:
            result["closure_training"] = training
        print("[bench] timing the other workload shapes", file=sys.stderr, flush=True)
        result["other_configs"] = other_configs(torch, args.steps)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
