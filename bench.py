"""Benchmark of the time-reversible FDTD gradient on one MI355X.

One "step" is one full gradient evaluation: the forward pass over T time
steps with interface recording, then the time-reversed pass over T steps that
returns dL/deps.  Throughput is fwd+rev Mcell-steps/s = cells * T / time.

Default workload: the silicon-slab waveguide on 256 x 256 x 128 cells with a
12-cell CPML and 4000 time steps, FP32 fields, a Gaussian current sheet at a
30-cell wavelength, a 64 x 64 x 8 seeded-random design block on the slab and a
64 x 64 output plane; interface fields stored in FP32 at every step.  Its
working set (about 1.2 GB) is far larger than the 256 MB Infinity Cache, so
the sweeps stream from HBM.  The compressed recorders (FP8-E4M3 with
per-block scales at k = 16, 64x smaller, and BF16 at k = 4) are timed in the
same run, and the gradient errors of every storage setting are measured
against the FP64 oracle's exact gradient of the same recipe on a 128^3 crop.

Prints one JSON line (see the keys below).  Run with --gpus 1 only: one GPU
is measured.
"""

from __future__ import annotations

import os

# the host baseline (the NumPy oracle) is timed single-threaded: fix the BLAS/OpenMP
# pools before numpy is first imported
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import argparse
import hashlib
import json
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+rev Mcell-steps/s, boundary-store GB, grad rel-err vs FP64 oracle"
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    # name: (preset, preset kwargs, store dtype, k)
    "c2": ("c2", {}, "fp32", 1),
    "c4": ("c4", {}, "fp32", 1),
    "c4p": ("c4p", {}, "fp32", 1),            # c4 at the paper's ~136 steps per period
    "c4crop": ("c4crop", {}, "fp32", 1),      # the c4 recipe on 128^3, 2000 steps
    "c4pcrop": ("c4pcrop", {}, "fp32", 1),
    "c5": ("c5", {}, "fp32", 1),
    "c3p": ("c3p", {}, "fp32", 1),
    "c2pw": ("c2pw", {}, "fp32", 1),          # plane-wave source, z-flux objective
    "c5crop": ("c5crop", {}, "fp32", 1),      # the c5 recipe on 128^3, 2000 steps
}
# workload -> its 128^3 crop, whose exact gradient the FP64 oracle stores (tests/golden)
CROPS = {"c4": "c4crop", "c4p": "c4pcrop", "c5": "c5crop"}
# storage settings timed beside the plain FP32 one (the first is reported as "compressed")
# (storage type, k, interpolation in time: "linear" as in the paper, or the cubic option)
_FP8_BF16 = [("fp8_e4m3_scaled", 16, "linear"), ("fp8_e4m3_scaled", 16, "cubic"), ("bf16", 4, "linear")]
COMPRESSED = {"c4": _FP8_BF16, "c4p": _FP8_BF16, "c5": _FP8_BF16}
# workloads whose working set fits the 256 MB Infinity Cache: their sweeps are not HBM-bound
CACHE_RESIDENT = {"c2", "c3p", "c2pw", "c4crop", "c4pcrop", "c5crop"}
DEFAULT_WORKLOAD = "c4"
KERNEL_SOURCES = ["paper_2603_24027_amd/csrc/common.h", "paper_2603_24027_amd/csrc/march.h",
                  "paper_2603_24027_amd/csrc/forward.hip", "paper_2603_24027_amd/csrc/forward2.hip",
                  "paper_2603_24027_amd/csrc/reverse.hip", "paper_2603_24027_amd/csrc/reverse2.hip",
                  "paper_2603_24027_amd/csrc/api.hip"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(prob, design_cells: int):
    """Minimal HBM bytes per launch of each kernel (each value read once, written once).

    fwd_step and adj_step sweep every cell: 52 B (read the six field components
    and eps, write the six) plus 32 B per PML slab cell and axis (four auxiliaries
    read and written); the adjoint launch also writes the next step's interface
    shell (two components per face cell of the interior's six faces, each read
    from an FP32 store and written: 16 B per face cell).  prim_rev sweeps the
    interior: 52 B per interior cell plus the FP64 gradient (16 B
    read-modify-write) and the adjoint E it reads (12 B) per design cell.
    """
    P = prob.pml
    N = prob.nx * prob.ny * prob.nz
    NI = (prob.nx - 2 * P) * (prob.ny - 2 * P) * (prob.nz - 2 * P)
    NP = N - NI
    S = 2 * P * (prob.ny * prob.nz + prob.nx * prob.nz + prob.nx * prob.ny)
    mx, my, mz = prob.nx - 2 * P, prob.ny - 2 * P, prob.nz - 2 * P
    shell = 2 * (my * mz + mx * mz + mx * my) if P > 0 else 0
    return {
        "fwd_step": 52 * N + 32 * S,
        "prim_rev": 52 * NI + 28 * design_cells,
        "adj_step": 52 * N + 32 * S + 16 * shell,
        # single-sweep lower bound of one time step, fwd + rev (52 B forward; 100 B interior /
        # 52 B PML reverse; PML auxiliaries; FP64 gradient)
        "step_min": 52 * N + 100 * NI + 52 * NP + 64 * S + 16 * design_cells,
    }


def read_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary of this kernel and workload
    (FETCH_SIZE and WRITE_SIZE, each scaled by a plain copy's reading), or None when there is
    none or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "%s_%s_pmc.txt" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            if line.startswith("json: "):
                rec = json.loads(line[len("json: "):])
                if rec.get("kernel_source_hash") == kernel_source_hash():
                    return rec.get("hbm_bytes_per_launch")
    return None


def host_description():
    """CPU model, logical CPUs of the host, and the CPUs this process may run on."""
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return model, os.cpu_count(), usable


def cpu_sample_steps(cells: int) -> int:
    """Time steps of the oracle sample: about 2.5e7 cell-steps (10-30 s of one core)."""
    return max(1, int(round(2.5e7 / cells)))


def oracle_baseline(prob_fn, sample_steps: int):
    """Time the FP64 oracle (as it stands) on the first steps of the workload's grid, one thread."""
    from oracle import adjoint
    prob = prob_fn(steps=sample_steps)
    t0 = time.perf_counter()
    adjoint.grad_time_reversal(prob, "fp64", 1)
    dt = time.perf_counter() - t0
    return prob.cells * sample_steps / dt / 1e6, dt, prob


def cosine(a, b) -> float:
    """Eq. 2: cosine similarity of two gradients."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


def rel_l2(a, b) -> float:
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_gradient(name: str, seed: int):
    """The FP64 oracle's exact gradient of this problem, stored by tests/golden/make_oracle_grads.py
    (None if that file was not made)."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_grad_%s_seed%d.npy" % (name, seed))
    return np.load(path) if os.path.exists(path) else None


SWEEP_TYPES = ["fp32", "fp16", "bf16", "fp8_e4m3_scaled", "fp8_e4m3b11fnuz", "fp8_e5m2fnuz", "fp8_e4m3fnuz",
               "fp8_e4m3", "fp8_e3m4", "fp8_e4m3fn"]
SWEEP_K = [1, 2, 4, 8, 16, 32]


def run_sweep(args, w, pk, torch, dev):
    """Every storage type x k on seeded random designs: storage, gradient agreement (Eq. 2
    cosine and relative L2) with the FP64 oracle's exact gradient (where stored) and with the
    plain FP32 full-storage GPU gradient, and fwd+rev Mcell-steps/s; one JSON line each."""
    from dataclasses import replace
    preset, kw, _, _ = WORKLOADS[args.workload]
    A = float(args.amplitude)
    probs = [w.make(preset, seed=s, **kw) for s in range(args.sweep_seeds)]
    exact = [oracle_gradient(p.name, s) for s, p in enumerate(probs)]
    if A != 1.0:
        # every field is linear in the source and the loss quadratic in the fields (either
        # objective), so the exact gradient at amplitude A is A^2 times the stored one
        probs = [replace(p, src_wave=(p.src_wave.astype(np.float64) * A).astype(np.float32),
                         msrc_wave=(p.msrc_wave.astype(np.float64) * A).astype(np.float32)) for p in probs]
        exact = [None if e is None else e * A * A for e in exact]
    refs = []
    for p in probs:
        g = pk.Gradient(p, "fp32", 1, device=dev)
        g.forward(torch.from_numpy(p.eps).to(dev))
        refs.append(g.backward().cpu().numpy().copy())
    full = pk.store_config(pk.Problem(probs[0]), "fp32", 1).payload_bytes
    cell_steps = probs[0].cells * probs[0].steps
    types = args.sweep_types.split(",") if args.sweep_types else SWEEP_TYPES
    ks = [int(v) for v in args.sweep_k.split(",")] if args.sweep_k else SWEEP_K
    for dtype in types:
        for k in ks:
            row = {"cos_oracle": [], "rel_oracle": [], "cos_fp32": [], "rel_fp32": []}
            rate = None
            for s, (p, ref) in enumerate(zip(probs, refs)):
                g = pk.Gradient(p, dtype, k, device=dev, interp=args.interp)
                e = torch.from_numpy(p.eps).to(dev)
                reps = 2 if s == 0 else 1          # seed 0 runs twice: the second call is timed
                for r in range(reps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    g.forward(e)
                    gr = g.backward().cpu().numpy()
                    if r == 1:
                        rate = cell_steps / (time.perf_counter() - t0) / 1e6
                ok = bool(np.all(np.isfinite(gr)))
                row["cos_fp32"].append(cosine(gr, ref) if ok else float("nan"))
                row["rel_fp32"].append(rel_l2(gr, ref) if ok else float("nan"))
                if exact[s] is not None:
                    row["cos_oracle"].append(cosine(gr, exact[s]) if ok else float("nan"))
                    row["rel_oracle"].append(rel_l2(gr, exact[s]) if ok else float("nan"))
            info = pk.store_config(pk.Problem(probs[0]), dtype, k)
            line = {"sweep": probs[0].name, "amplitude": A, "store_dtype": dtype, "k": k, "interp": args.interp,
                    "compression": round(full / info.payload_bytes, 3), "storage_GB": info.payload_bytes / 1e9,
                    "cos_vs_fp32_mean": float(np.mean(row["cos_fp32"])),
                    "rel_l2_vs_fp32_mean": float(np.mean(row["rel_fp32"])),
                    "Mcell_steps_per_s": round(rate, 1), "seeds": len(probs)}
            if row["cos_oracle"]:
                line.update({"cos_vs_oracle_mean": float(np.mean(row["cos_oracle"])),
                             "cos_vs_oracle_min": float(np.min(row["cos_oracle"])),
                             "rel_l2_vs_oracle_mean": float(np.mean(row["rel_oracle"])),
                             "oracle_seeds": len(row["cos_oracle"])})
            print(json.dumps(line), flush=True)


DESIGN_CONFIGS = [("fp32", 1), ("fp8_e4m3_scaled", 4), ("fp8_e4m3_scaled", 8), ("fp8_e4m3_scaled", 16),
                  ("fp8_e4m3_scaled", 32), ("fp8_e4m3b11fnuz", 16)]


def run_design_loop(args, w, pk, torch, dev):
    """Objective trajectories of the inverse-design loop with full and compressed interface
    storage from the same seeded starts (Section 3, Fig. 4: beta = 1 for the first 40
    iterations, then the subpixel-smoothed projection at beta = infinity; NAdam with a linear
    warm-up); one JSON line per (storage, seed).  --amplitude scales the source (all
    objectives then scale by its square) so that the unscaled 8-bit type sees fields in its
    range."""
    from dataclasses import replace
    from paper_2603_24027_amd.optimize import DesignLoop
    preset, kw, _, _ = WORKLOADS[args.workload]
    A = float(args.amplitude)
    for seed in range(args.sweep_seeds):
        prob = w.make(preset, seed=seed, **kw)
        if A != 1.0:
            prob = replace(prob, src_wave=(prob.src_wave.astype(np.float64) * A).astype(np.float32),
                           msrc_wave=(prob.msrc_wave.astype(np.float64) * A).astype(np.float32))
        ref = None
        for dtype, k in DESIGN_CONFIGS:
            t0 = time.perf_counter()
            loop = DesignLoop(prob, dtype, k, sigma=3.0, beta=1.0, beta_after=float("inf"), switch_at=40,
                              lr=args.design_lr, warmup=20, seed=seed, device=dev,
                              eps_range=(float(prob.eps.min()), 12.25))
            hist = loop.run(args.design_loop)
            if ref is None:
                ref = hist
            h, r = np.array(hist), np.array(ref)
            print(json.dumps({"design_loop": prob.name, "store_dtype": dtype, "k": k, "seed": seed,
                              "amplitude": A, "iterations": len(hist), "objective_first": hist[0],
                              "objective_last": hist[-1], "objective_best": float(h.max()),
                              "gain": hist[-1] / hist[0], "final_vs_fp32": hist[-1] / ref[-1],
                              "max_rel_dev_from_fp32": float(np.max(np.abs(h - r) / np.abs(r))),
                              "history": [float("%.6e" % v) for v in hist],
                              "s": round(time.perf_counter() - t0, 2)}), flush=True)
            del loop


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed gradient evaluations")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compressed", action="store_true")
    ap.add_argument("--no-crop", action="store_true", help="skip the 128^3-crop gradient errors (c4, c4p, c5)")
    ap.add_argument("--cpu-sample-steps", type=int, default=0,
                    help="time steps of the host oracle sample (0: about 2.5e7 cell-steps)")
    ap.add_argument("--time-steps", type=int, default=0,
                    help="run the workload's grid for this many time steps instead of its own (for counter runs, "
                         "whose per-dispatch cost makes thousands of launches slow; per-launch figures do not depend on it)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (for counter scaling) and exit")
    ap.add_argument("--sweep", action="store_true",
                    help="storage type x k sweep of gradient agreement (Fig. 3 analogue) instead of the benchmark")
    ap.add_argument("--sweep-seeds", type=int, default=3)
    ap.add_argument("--sweep-types", default="", help="comma-separated storage types (default: all)")
    ap.add_argument("--sweep-k", default="", help="comma-separated subsampling factors (default: 1,2,4,8,16,32)")
    ap.add_argument("--interp", default="linear", choices=["linear", "cubic"],
                    help="interpolation in time of the skipped steps in --sweep runs")
    ap.add_argument("--amplitude", type=float, default=1.0,
                    help="scale of the source signal in --sweep runs (field units relative to the unscaled 8-bit ranges)")
    ap.add_argument("--design-lr", type=float, default=0.1)
    ap.add_argument("--design-loop", type=int, default=0, metavar="ITERS",
                    help="run the inverse-design loop for ITERS iterations with FP32 k=1 and FP8 k in "
                         "{4, 8, 16, 32} storage instead of the benchmark (Fig. 4 analogue)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported by this build "
              "(the multi-GPU decomposition is a design only)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as w
    import paper_2603_24027_amd as pk

    pk.load()                      # fails loudly without the HIP library
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)     # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": src.numel() * 4, "copies": 3}))
        return

    if args.sweep:
        run_sweep(args, w, pk, torch, dev)
        return
    if args.design_loop:
        run_design_loop(args, w, pk, torch, dev)
        return

    preset, kw, dtype, k = WORKLOADS[args.workload]
    prob_fn = lambda **extra: w.make(preset, **{**kw, **extra})
    prob = prob_fn(steps=args.time_steps) if args.time_steps else prob_fn()
    eps = torch.from_numpy(prob.eps).to(dev)
    T = prob.steps
    cells = prob.cells

    fwd_rev_ms = {}

    def timed_run(dtype_, k_, steps, warmup, interp_="linear"):
        gobj = pk.Gradient(prob, dtype_, k_, device=dev, interp=interp_)
        for _ in range(warmup):
            gobj.forward(eps)
            gobj.backward()
        stream = torch.cuda.current_stream(dev)
        marks = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
                  torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b, c in marks:           # events on the stream the library launches on
            a.record(stream)
            gobj.forward(eps)
            b.record(stream)
            gobj.backward()
            c.record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        fwd_rev_ms[(dtype_, k_, interp_)] = (float(np.mean([a.elapsed_time(b) for a, b, _ in marks])),
                                    float(np.mean([b.elapsed_time(c) for _, b, c in marks])))
        return (t1 - t0), gobj

    def kernel_times(gobj, steps):
        """Per-kernel HIP events (start/stop carried by each dispatch) over `steps` gradients."""
        pk.timing_enable(True)             # one pass to create the event pool
        gobj.forward(eps)
        gobj.backward()
        pk.timing_read()
        pk.timing_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            gobj.forward(eps)
            gobj.backward()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kt = pk.timing_read()
        pk.timing_enable(False)
        return kt, t1 - t0

    def progress(msg):
        print("[bench] %s" % msg, file=sys.stderr, flush=True)

    progress("%s: %d cells x %d steps, %s k=%d" % (prob.name, cells, T, dtype, k))
    elapsed, gobj = timed_run(dtype, k, args.steps, args.warmup)
    progress("timed region: %.3f s for %d gradients" % (elapsed, args.steps))
    ms_per_step = elapsed / args.steps * 1e3
    value = cells * T * args.steps / elapsed / 1e6
    kt_steps = min(args.steps, 3)
    ktimes, kt_elapsed = kernel_times(gobj, kt_steps)
    progress("per-kernel event pass: %.3f s" % kt_elapsed)

    design_cells = int(np.prod(prob.design_shape))
    ab = algorithmic_bytes(prob, design_cells)
    kernels = {}
    for name in ("fwd_step", "fwd2_step", "prim_rev", "prim_rev2", "adj_step"):
        if name not in ktimes or ktimes[name][0] == 0:
            continue
        launches, total_ms = ktimes[name]
        avg_s = total_ms / launches / 1e3
        # the two-step sweeps read and write every value once per launch (two steps)
        a = {"fwd2_step": ab["fwd_step"], "prim_rev2": ab["prim_rev"]}.get(name, ab.get(name))
        kernels[name] = {"launches": launches, "avg_us": avg_s * 1e6, "alg_bytes": a, "GBps": a / avg_s / 1e9}
        if name in ("fwd2_step", "prim_rev2"):
            kernels[name]["time_steps_per_launch"] = 2
    dominant = max(kernels, key=lambda n: kernels[n]["avg_us"] * kernels[n]["launches"])
    dk = kernels[dominant]
    traffic = read_traffic(dominant, prob.name)
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": round(dk["GBps"], 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(dk["GBps"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                "alg_bytes_per_launch": ab[dominant], "avg_launch_us": round(dk["avg_us"], 2)}
    if args.workload in CACHE_RESIDENT:
        roofline["note"] = ("working set below the 256 MB Infinity Cache: the sweeps are partly served from it, "
                            "so this fraction of the HBM peak is not an HBM-bound measurement")
    step_gbs = ab["step_min"] * T * args.steps / elapsed / 1e9

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "t_fwd_ms": round(fwd_rev_ms[(dtype, k, "linear")][0], 3),
        "t_rev_ms": round(fwd_rev_ms[(dtype, k, "linear")][1], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": prob.name, "grid": [prob.nx, prob.ny, prob.nz], "pml": prob.pml,
                   "time_steps": T, "store_dtype": dtype, "k": k, "design_cells": design_cells,
                   "wavelength_cells": prob.wavelength,
                   "forward_steps_per_sweep": 2 if "fwd2_step" in kernels else 1,
                   "reverse_steps_per_primal_sweep": 2 if "prim_rev2" in kernels else 1},
        "boundary_store_GB": gobj.info.payload_bytes / 1e9,
        "roofline": roofline,
        "whole_step": {"alg_bytes_per_time_step": ab["step_min"], "GBps": round(step_gbs, 1),
                       "frac_of_hbm_peak": round(step_gbs / HBM_PEAK_GBS, 4),
                       "note": "single-sweep minimum bytes (fwd 52 B/cell, rev 100 B interior / 52 B PML "
                               "+ PML auxiliaries) over the measured fwd+rev time"},
        "kernels": {n: {kk: (round(v, 2) if isinstance(v, float) else v) for kk, v in d.items()}
                    for n, d in kernels.items()},
        "kernel_timing_pass_ms_per_step": round(kt_elapsed / kt_steps * 1e3, 3),
        "other_kernels": {n: {"launches": l, "total_ms": round(t, 3)} for n, (l, t) in ktimes.items()
                          if n not in kernels},
    }

    c_obj = None
    if not args.no_compressed:
        for i, (cd, ck, ci) in enumerate(COMPRESSED.get(args.workload, [("fp8_e4m3_scaled", 16, "linear")])):
            # the same timed protocol on fewer gradients (the GPU time of the run stays bounded)
            c_steps, c_warm = min(args.steps, 5), min(args.warmup, 1)
            c_el, obj = timed_run(cd, ck, c_steps, c_warm, ci)
            progress("compressed timed region (%s k=%d %s): %.3f s for %d gradients" % (cd, ck, ci, c_el, c_steps))
            rec = {"store_dtype": cd, "k": ck, "interp": ci, "steps": c_steps, "warmup": c_warm,
                   "value": round(cells * T * c_steps / c_el / 1e6, 1),
                   "ms_per_step": round(c_el / c_steps * 1e3, 3),
                   "t_fwd_ms": round(fwd_rev_ms[(cd, ck, ci)][0], 3),
                   "t_rev_ms": round(fwd_rev_ms[(cd, ck, ci)][1], 3),
                   "boundary_store_GB": obj.info.payload_bytes / 1e9,
                   "storage_reduction": gobj.info.payload_bytes / obj.info.payload_bytes}
            g_ref = gobj.buf.grad.cpu().numpy()
            g_c = obj.buf.grad.cpu().numpy()
            rec["grad_vs_fp32_k1_same_size"] = {"cosine": cosine(g_c, g_ref), "rel_l2": rel_l2(g_c, g_ref)}
            if i == 0:
                out["compressed"] = rec
                c_obj = obj
            else:
                out.setdefault("compressed_more", []).append(rec)
            del obj

    if not args.no_cpu_baseline:
        steps_cpu = args.cpu_sample_steps or cpu_sample_steps(cells)
        progress("oracle baseline on the host, %d steps" % steps_cpu)
        mcs, dt_cpu, sprob = oracle_baseline(prob_fn, steps_cpu)
        model, ncpu, usable = host_description()
        out["cpu_baseline"] = {"value": round(mcs, 4), "unit": "Mcell-steps/s", "cores": 1, "kind": "oracle",
                               "sample": "FP64 NumPy oracle (single thread: OMP/OpenBLAS/MKL threads 1, elementwise "
                                         "NumPy), time-reversal gradient (forward + reverse) of the same %dx%dx%d grid "
                                         "truncated to %d time steps: %.1f s"
                                         % (prob.nx, prob.ny, prob.nz, steps_cpu, dt_cpu),
                               "cpu_model": model, "host_logical_cpus": ncpu, "usable_cpus": usable}
    def form_name(d, kk, ip):
        return "%s_k%d%s" % (d, kk, "" if ip == "linear" else "_" + ip)

    exact = oracle_gradient(prob.name, 0)
    if exact is not None:
        errs = {form_name(dtype, k, "linear"): gobj.buf.grad.cpu().numpy()}
        if c_obj is not None:
            errs[form_name(c_obj.dtype, c_obj.k, c_obj.interp)] = c_obj.buf.grad.cpu().numpy()
        out["grad_err_vs_fp64_oracle"] = {
            name: {"rel_l2": rel_l2(g, exact), "cosine": cosine(g, exact)} for name, g in errs.items()}
    if args.workload in CROPS and not args.no_crop:
        # gradient error of every storage setting on the 128^3 crop of this workload's recipe
        cprob = w.make(CROPS[args.workload], seed=0)
        cexact = oracle_gradient(cprob.name, 0)
        if cexact is not None:
            ce = torch.from_numpy(cprob.eps).to(dev)
            res = {"workload": cprob.name}
            for cd, ck, ci in [("fp32", 1, "linear")] + COMPRESSED.get(args.workload, []):
                obj = pk.Gradient(cprob, cd, ck, device=dev, interp=ci)
                obj.forward(ce)
                gr = obj.backward().cpu().numpy()
                res[form_name(cd, ck, ci)] = {"rel_l2": rel_l2(gr, cexact), "cosine": cosine(gr, cexact),
                                              "boundary_store_GB": obj.info.payload_bytes / 1e9}
                del obj
            out["crop_grad_err_vs_fp64_oracle"] = res
            if "grad_err_vs_fp64_oracle" not in out:
                # no oracle gradient exists at this size (hours of one core): the errors of the
                # same storage settings on the oracle-checked 128^3 crop of the recipe stand for it
                out["grad_err_vs_fp64_oracle"] = {"measured_on": cprob.name,
                                                  **{kk: v for kk, v in res.items() if kk != "workload"}}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
