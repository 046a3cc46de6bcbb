"""Benchmark: mesh-node updates per second of the ALE lattice-Boltzmann step.

One step = the whole hot path over every node and discrete velocity: metrics
and transformed velocities, departure points, element walk, P2 gather,
Grad missing populations, moments, both correction passes, collision; the
wall force integral is evaluated once per timed run.  Workload: the plunging
NACA0012 O-mesh (~200k P2 nodes, h = 0.2c, k = 1, Ma = 0.2, Re = 1e4),
FP32 populations and bulk arithmetic with FP64 geometry (the headline line),
plus the FP64 path on the same mesh.  Inputs are seeded and synthetic and
resident in HBM before timing starts.

Prints ONE JSON line.  Per-kernel durations come from HIP events recorded by
the library on the same stream around each kernel.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
KERNELS = ["k_stream", "k_wallbc", "k_grad1", "k_collide"]


def kernel_bytes(info: dict, s: int) -> dict:
    """Algorithmic bytes per launch of each kernel: every datum the kernel
    must touch, counted once (s = bytes per population scalar)."""
    N, E = info["nodes"], info["elems"]
    node = 16 + 4 + 1                # X (2 f64), owner, owner slot/shift
    elem_walk = 48 + 16 + 24         # geometry (v0, A), neighbours + shifts, 6 node ids
    elem_grad = 32 + 24              # A and node ids of the owner element
    return {
        # read 18 populations, write 18 streamed populations + 4 moments
        "k_stream": N * (node + 18 * s + 18 * s + 4 * s) + E * elem_walk,
        # wall nodes only: no per-node bytes worth pricing at the mesh scale
        "k_wallbc": 0,
        # read 4 moments, write W (2)
        "k_grad1": N * (node + 4 * s + 2 * s) + E * elem_grad,
        # read 18 streamed populations + W (2), write 18 populations + X (2)
        "k_collide": N * (node + 18 * s + 2 * s + 18 * s + 2 * s) + E * elem_grad,
    }


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("alelb_kernels.hip", "alelb_impl.h"):
        with open(os.path.join(ROOT, "paper_2002_04353_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    rec = d.get(workload, {}).get(kernel)
    if not rec or rec.get("src_sha") != source_hash():
        return None
    return rec.get("bytes_per_launch")


def time_solver(alelb, torch, case, precision, steps, warmup):
    s = alelb.Solver(case["mesh"].arrays(), case["params"], precision=precision,
                     stream=torch.cuda.current_stream().cuda_stream)
    s.init_fields(**case["init"])
    s.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    s.step(steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    forces = s.forces()
    kms = s.time_kernels(max(10, min(steps, 50)))
    info = s.info()
    s.close()
    return dict(ms_per_step=ms / steps, wall_s=wall, kernel_ms=kms.tolist(), info=info, forces=forces)


def cpu_baseline(case, steps):
    from oracle import oracle as O
    o = O.Oracle(case["mesh"].arrays(), case["params"])
    o.init_fields(**case["init"])
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    N = case["mesh"].n_nodes
    return dict(value=N * steps / dt, unit="node-updates/s", cores=O.threads(), kind="oracle",
                sample=f"{steps} FP64 steps of the same {N}-node plunging-airfoil workload, "
                       f"{dt:.1f} s of wall time on the host's cores")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-steps", type=int, default=1000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU decomposition is "
              "a design, not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2002_04353_amd import alelb, cases
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_mib:
        # plain copy kernel of known size: reads and writes copy_mib MiB each
        n = args.copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"# copy {args.copy_mib} MiB x 3 done", file=sys.stderr, flush=True)
        del a, b
    case = cases.plunge()
    N = case["mesh"].n_nodes
    print(f"# workload plunge: {N} nodes, {case['mesh'].n_elems} elements", file=sys.stderr, flush=True)
    r32 = time_solver(alelb, torch, case, "fp32", args.steps, args.warmup)
    print(f"# fp32 {r32['ms_per_step'] * 1e3:.2f} us/step, kernels {r32['kernel_ms']}", file=sys.stderr, flush=True)
    r64 = None
    if not args.no_fp64:
        r64 = time_solver(alelb, torch, case, "fp64", args.steps, args.warmup)
        print(f"# fp64 {r64['ms_per_step'] * 1e3:.2f} us/step, kernels {r64['kernel_ms']}", file=sys.stderr,
              flush=True)
    value = N / (r32["ms_per_step"] * 1e-3)
    kb = kernel_bytes(r32["info"], 4)
    km = dict(zip(KERNELS, r32["kernel_ms"][:4]))
    dom = max(KERNELS, key=lambda k: km[k])
    achieved = kb[dom] / (km[dom] * 1e-3) / 1e9
    traffic = measured_traffic(dom, "plunge_fp32")
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
            "algorithmic_bytes_per_launch": kb[dom], "launch_ms": round(km[dom], 5)}
    step_bytes = sum(kb.values())
    out = {
        "metric": "mesh-node updates/s (FP32-mixed; FP64 and per-kernel HBM GB/s alongside)",
        "value": round(value, 1),
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded NACA0012 O-mesh, impulsive start)",
        "config": {"workload": f"plunging NACA0012, {N} P2 nodes, h=0.2c, k=1, Ma=0.2, Re=1e4, "
                               "FP32 populations / FP64 geometry",
                   "nodes": N, "elements": case["mesh"].n_elems, "dt": case["params"]["dt"]},
        "roofline": roof,
        "kernels_ms": {k: round(v, 5) for k, v in km.items()},
        "step_effective_GBs": round(step_bytes / (r32["ms_per_step"] * 1e-3) / 1e9, 1),
        "cl_cd_after_run": [round(r32["forces"]["cl"], 6), round(r32["forces"]["cd"], 6)],
    }
    if r64:
        kb64 = kernel_bytes(r64["info"], 8)
        km64 = dict(zip(KERNELS, r64["kernel_ms"][:4]))
        out["fp64"] = {"value": round(N / (r64["ms_per_step"] * 1e-3), 1), "ms_per_step": round(r64["ms_per_step"], 5),
                       "kernels_ms": {k: round(v, 5) for k, v in km64.items()},
                       "k_stream_GBs": round(kb64["k_stream"] / (km64["k_stream"] * 1e-3) / 1e9, 1)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_steps)
        out["cpu_baseline"]["value"] = round(out["cpu_baseline"]["value"], 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
