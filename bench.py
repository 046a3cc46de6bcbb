"""Benchmark: mesh-node updates per second of the ALE lattice-Boltzmann step.

One step = the whole hot path over every node and discrete velocity of every
case: metrics and transformed velocities, departure points, element walk, P2
gather, Grad missing populations, moments, both correction passes, collision;
the wall force integral of every case is evaluated once after the timed run.

Headline workload: the batched ensemble of 64 independent pitch+plunge
NACA0012 cases on seeded O-meshes of 50k-300k P2 nodes each (about 12M nodes
in all), FP32 populations and bulk arithmetic with FP64 geometry, advanced by
one graph-captured launch sequence per pair of steps.  Alongside: the same
batch in FP64, the single plunging-airfoil mesh (~200k nodes) in FP32 and
FP64, and the plunging airfoil on 9-node quadrilaterals (~190k nodes) in FP32.  Inputs are seeded and synthetic and resident in HBM before timing
starts.

Prints ONE JSON line.  Step times come from HIP events recorded on the stream
the library launches on; per-kernel durations from events the library records
around each kernel on that same stream.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# VALU issue: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 VALU instruction per 4 cycles per SIMD
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4
# the four kernels of a step, in the order time_kernels() reports them
KERNELS_ONE_WAVE = ["k_stream", "k_wall", "k_grad1", "k_collide"]
KERNELS_TILE = ["k_tile", "k_wall", "k_grad1", "k_grad2"]

# The method's own byte count per node-update, each datum across HBM once:
# 18 populations read (the gather's source) and 18 written, the 4 moments
# written and read once, W written and read once, the node's coordinates and
# owner (20 B), and its share of the element data: 6 node ids, 3 neighbour ids
# and the affine inverse, 84 B per element.  With s = 4 (FP32) and E = N / 2
# this is 254 B per node, with s = 8 it is 446 B.
NODE_ALG = 20
ELEM_ALG = 84


def kernel_names(schedule: dict) -> list:
    return KERNELS_TILE if schedule["waves"] > 0 else KERNELS_ONE_WAVE


def alg_bytes(N: int, E: int, s: int, tile: bool) -> dict:
    """The algorithmic bytes of one step (s = bytes per population scalar),
    each item assigned to the kernel that moves it in the schedule's family;
    the streaming kernel takes the node and element data, which the node
    kernels read again by design."""
    pops, mac, w = 18 * s, 4 * s, 2 * s
    stream = N * (NODE_ALG + pops + mac) + E * ELEM_ALG  # populations read, moments written
    if tile:  # the tile kernel also writes the populations; X is the design's own
        return {"k_tile": stream + N * pops, "k_wall": 0, "k_grad1": N * (mac + w), "k_grad2": N * w}
    return {"k_stream": stream, "k_wall": 0, "k_grad1": N * (mac + w), "k_collide": N * (pops + w)}


def design_bytes(info: dict, s: int, tile: bool, elem: str = "p2") -> dict:
    """Bytes each kernel of this design must move per launch, every datum it
    touches counted once: the algorithmic bytes plus the design's own (the
    one-wave schedules' streamed copy f~ written and read back, X and the
    node kernels' rereads of node and element data)."""
    N, E = info["nodes"], info["elems"]
    node = 16 + 4 + 2                # X (2 f64), owner, owner slot/shift
    if elem == "p2":
        elem_walk = 48 + 16 + 24     # geometry (v0, A), neighbours + shifts, 6 node ids
        elem_grad = 32 + 24          # A and node ids of the owner element
    else:
        elem_walk = 64 + 16 + 4 + 8 + 36  # corners, neighbours, shift codes, 2 area, 9 node ids
        elem_grad = 64 + 36          # corners and node ids of the owner element
    grad1 = N * (node + 4 * s + 2 * s) + E * elem_grad  # read 4 moments, write W (2)
    if tile:
        return {
            # read 18 populations + X (2), write 18 populations + 4 moments
            "k_tile": N * (node + 18 * s + 2 * s + 18 * s + 4 * s) + E * elem_walk,
            "k_grad1": grad1,
            # read W (2), write X (2)
            "k_grad2": N * (node + 2 * s + 2 * s) + E * elem_grad,
        }
    return {
        # read 18 populations, write 18 streamed populations + 4 moments
        "k_stream": N * (node + 18 * s + 18 * s + 4 * s) + E * elem_walk,
        "k_grad1": grad1,
        # read 18 streamed populations + W (2), write 18 populations
        "k_collide": N * (node + 18 * s + 2 * s + 18 * s) + E * elem_grad,
    }


def source_hash(files=("alelb_kernels.hip", "alelb_impl.h")) -> str:
    """Hash of kernel code (by default the step kernels': their source and
    header) with line comments and blank lines dropped, so that comment edits
    keep it."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2002_04353_amd", "csrc", f)) as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


MLP_SOURCES = ("mlp_kernels.hip", "alelb_impl.h")


def _profiled(kernel: str, workload: str, field: str, files=None):
    """A per-launch figure from the committed rocprofv3 counter runs, if they
    were taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    rec = d.get(workload, {}).get(kernel)
    if not rec or rec.get("src_sha") != (source_hash(files) if files else source_hash()):
        return None
    return rec.get(field)


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)."""
    return _profiled(kernel, workload, "bytes_per_launch")


def valu_roofline(kernel: str, workload: str, launch_ms: float):
    """VALU issue rate of a kernel: its profiled wave-instruction count per
    launch over the launch time measured in this run."""
    n = _profiled(kernel, workload, "valu_insts_per_launch")
    if n is None:
        return None
    g = n / (launch_ms * 1e-3) / 1e9
    return {"bound": "alu", "achieved": round(g, 1), "peak": VALU_PEAK_GINST, "unit": "G VALU wave-instr/s",
            "frac": round(g / VALU_PEAK_GINST, 4), "insts_per_launch": n, "kernel": kernel}


def time_solver(alelb, torch, meshes, params, init, precision, steps, warmup, graph=True, kernel_steps=20,
                split=False):
    st = torch.cuda.current_stream()
    flags = (alelb.F_GRAPH if graph else 0) | (alelb.F_PIPELINE if split else 0)
    s = alelb.Solver(meshes, params, precision=precision, flags=flags, stream=st.cuda_stream)
    s.init_fields(**init)
    sched = s.autotune(reps=10)
    s.step(warmup)
    st.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    s.step(steps)
    e1.record(st)
    st.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    forces = s.forces_batch() if isinstance(meshes, list) else [s.forces()]
    # the force integral of every case, host call included (launch, reduction, copy back)
    t1 = time.perf_counter()
    for _ in range(20):
        s.forces_batch() if isinstance(meshes, list) else s.forces()
    forces_us = (time.perf_counter() - t1) / 20 * 1e6
    kms = s.time_kernels(kernel_steps)
    info = s.info()
    s.close()
    return dict(ms_per_step=ms / steps, wall_s=wall, kernel_ms=kms.tolist(), info=info, forces=forces,
                forces_us=forces_us, schedule=sched)


def force_series(alelb, mesh, params, init, steps, every, precision="fp32"):
    """Lift, drag and moment coefficients every `every` steps of a run from the
    initial state (outside any timed region): the time series the plunging
    airfoil is reported by."""
    s = alelb.Solver(mesh, params, precision=precision, flags=alelb.F_GRAPH)
    s.init_fields(**init)
    s.autotune(reps=3)
    out = []
    for _ in range(steps // every):
        s.step(every)
        f = s.forces()
        out.append([round(f["t"], 3), round(f["cl"], 6), round(f["cd"], 6), round(f["cm"], 6)])
    s.close()
    return out


def host_cpu() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def _oracle_rate(O, mesh, params, init, seconds):
    o = O.Oracle(mesh.arrays(), params)
    o.init_fields(**init)
    steps, t0 = 0, time.perf_counter()
    while True:
        o.step(2)
        steps += 2
        dt = time.perf_counter() - t0
        if dt >= seconds:
            break
    return mesh.n_nodes * steps / dt, steps, dt


def cpu_baseline(mesh, params, init, seconds, label):
    """The oracle (built -O3, OpenMP over nodes) on the host's cores, on a
    bounded sample: whole steps of one case until about `seconds` of wall
    time have passed, with all the threads OpenMP starts, then with one."""
    from oracle import oracle as O
    O.build()
    cores = O.threads()
    rate, steps, dt = _oracle_rate(O, mesh, params, init, seconds)
    O.set_threads(1)
    rate1, steps1, dt1 = _oracle_rate(O, mesh, params, init, seconds / 2)
    O.set_threads(cores)
    N = mesh.n_nodes
    return dict(value=round(rate, 1), unit="node-updates/s", cores=cores, kind="oracle",
                sample=f"{steps} FP64 steps of {label} ({N} nodes), {dt:.1f} s of wall time on {cores} threads; "
                       f"{steps1} steps on one thread, {dt1:.1f} s",
                value_1thread=round(rate1, 1), host=host_cpu(), build="gcc -O3 -ffp-contract=off -fopenmp")


def train_step_bytes(widths, batch):
    """HBM bytes one training step must move at least, with the network's
    storage: BF16 activations padded to 32 columns feed the products, FP32
    activations feed the tanh derivative and the loss, back-propagated errors
    are BF16, and the bias gradients come from column sums taken where the
    errors are made.  Weights and per-chunk sums are negligible beside them."""
    ld = [-(-w // 32) * 32 for w in widths]
    L, B = len(widths) - 1, batch
    fwd = sum(B * ld[l] * 2 + B * widths[l + 1] * 4 + (B * ld[l + 1] * 2 if l + 1 < L else 0) for l in range(L))
    loss = B * widths[L] * (4 + 4 + 2)  # output and target in, BF16 error out
    bwd = 0
    for l in range(L - 1, -1, -1):
        bwd += B * widths[l + 1] * 2 + B * ld[l] * 2  # dW operands
        if l > 0:
            bwd += B * widths[l + 1] * 2 + B * widths[l] * 4 + B * widths[l] * 2  # dZ, tanh', new dZ
    return fwd + loss + bwd


def copy_calibration(torch, mib):
    """A plain device copy of known size (reads and writes `mib` MiB each),
    which scales the profiler's HBM byte counters."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"# copy {mib} MiB x 3 done", file=sys.stderr, flush=True)


def train_step_timing(torch, batches=(4096, 65536), reps=20):
    """Matrix-core rate (forward 2, backward 4 flops per weight and row) and
    HBM rate of the surrogate's training step, at its fit's batch size and at
    one large enough to fill the GPU; inputs resident on the device."""
    from paper_2002_04353_amd import mlp
    from paper_2002_04353_amd import surrogate as S
    macs = sum(S.WIDTHS[l] * S.WIDTHS[l + 1] for l in range(len(S.WIDTHS) - 1))
    rng = np.random.default_rng(0)
    step_ms, step_tf, step_gbs = {}, {}, {}
    for nb in batches:
        xb = torch.from_numpy(rng.uniform(-1, 1, (nb, S.WIDTHS[0])).astype(np.float32)).cuda()
        yb = torch.from_numpy(rng.standard_normal((nb, S.WIDTHS[-1])).astype(np.float32)).cuda()
        net = mlp.MLP(S.WIDTHS, nb)
        net.set_params(S.glorot(S.WIDTHS, 1))
        torch.cuda.synchronize()
        net.train_steps(xb.data_ptr(), yb.data_ptr(), [1e-4] * 3, on_device=True, batch=nb)
        t0 = time.perf_counter()
        net.train_steps(xb.data_ptr(), yb.data_ptr(), [1e-4] * reps, on_device=True, batch=nb)
        t_step = (time.perf_counter() - t0) / reps
        step_ms[nb] = round(t_step * 1e3, 3)
        step_tf[nb] = round(6.0 * macs * nb / t_step / 1e12, 2)
        step_gbs[nb] = round(train_step_bytes(S.WIDTHS, nb) / t_step / 1e9, 1)
        net.close()
        del xb, yb
    return step_ms, step_tf, step_gbs


def surrogate_run(torch, ens, extra_batches=3, steps=4096, iters=3000, seed=41):
    """Train the surrogate on the ensemble's own load histories: its 64 cases
    as the headline runs them, plus `extra_batches` more batches of motion
    parameters drawn from the same ranges on the same 64 meshes; evaluate it
    on one held-out batch of new parameters on those meshes, beside the
    method's answers without the network (training mean, nearest training
    case, affine fit), and time it against the solver and the matrix cores."""
    from paper_2002_04353_amd import cases
    from paper_2002_04353_amd import surrogate as S
    meshes = ens["meshes"]
    n = len(meshes)
    rng = np.random.default_rng(seed)

    def draws():
        return np.stack([rng.uniform(*cases.ENSEMBLE_RANGES[k], size=n) for k in S.PARAMS], axis=1)

    train = np.concatenate([ens["motion"]] + [draws() for _ in range(extra_batches)])
    test = draws()
    Ytr, t_train = S.solver_histories(meshes * (1 + extra_batches), train, steps)
    Yte, t_test = S.solver_histories(meshes, test, steps)
    nodes = sum(m.n_nodes for m in meshes)
    print(f"# surrogate data: {len(train)} + {len(test)} solver runs of {steps} steps on the ensemble's "
          f"{n} meshes ({nodes} nodes per batch), {t_train + t_test:.1f} s", file=sys.stderr, flush=True)
    # cases the solver could not carry through are left out of training and evaluation
    ok_tr, ok_te = np.isfinite(Ytr).all(axis=1), np.isfinite(Yte).all(axis=1)
    diverged = [int((~ok_tr).sum()), int((~ok_te).sum())]
    train, Ytr, test, Yte = train[ok_tr], Ytr[ok_tr], test[ok_te], Yte[ok_te]
    mesh_te = [m for m, ok in zip(meshes, ok_te) if ok]
    sur = S.Surrogate(meshes[0], steps, max_batch=4096)
    Xtr, Xte = S.scale_params(train), S.scale_params(test)
    t0 = time.perf_counter()
    losses = sur.fit(Xtr, Ytr, iters=iters, batch=256)
    t_fit = time.perf_counter() - t0
    rms = sur.validate(test, Yte)
    base = {k: S.rms_cl_cm(v, Yte) for k, v in S.baselines(Xtr, Ytr, Xte).items()}
    sur.predict(Xte)
    t0 = time.perf_counter()
    for _ in range(10):
        sur.predict(Xte)
    t_pred = (time.perf_counter() - t0) / 10
    step_ms, step_tf, step_gbs = train_step_timing(torch)
    sur.close()
    return {"train_cases": int(ok_tr.sum()), "test_cases": int(ok_te.sum()), "diverged_train_test": diverged,
            "data": f"the {n} ensemble cases and {extra_batches * n} more parameter draws on the same meshes "
                    f"(train), {n} new draws on them (held out)",
            "steps_per_history": steps, "samples": S.SAMPLES, "mesh_nodes_per_batch": nodes,
            "held_out_mesh_nodes": int(sum(m.n_nodes for m in mesh_te)),
            "solver_s_train": round(t_train, 2), "solver_s_test": round(t_test, 3),
            "fit_s": round(t_fit, 2), "fit_iters": iters, "loss_first_last": [round(float(losses[0]), 4),
                                                                           round(float(losses[-1]), 5)],
            "heldout_rms_cl_cm": [round(rms[0], 4), round(rms[1], 4)],
            "baseline_rms_cl_cm": {k: [round(v[0], 4), round(v[1], 4)] for k, v in base.items()},
            "predict_ms_for_test_cases": round(t_pred * 1e3, 3),
            "speedup_vs_solver": round(t_test / t_pred, 1),
            "train_step_ms_batch4096": step_ms[4096], "train_step_TFLOPs": step_tf[4096],
            "train_step_ms_batch65536": step_ms[65536], "train_step_TFLOPs_batch65536": step_tf[65536],
            "mfma_bf16_peak_TFLOPs": 2500.0,
            "train_step_roofline_batch65536": {"bound": "hbm", "achieved": step_gbs[65536], "peak": 8000.0,
                                               "unit": "GB/s", "frac": round(step_gbs[65536] / 8000.0, 4),
                                               "traffic": _profiled("train_step", "surrogate_batch65536",
                                                                    "bytes_per_step", MLP_SOURCES),
                                               "algorithmic_bytes": train_step_bytes(S.WIDTHS, 65536)}}


def _schedule(r):
    d = r["schedule"]
    return {"waves": d["waves"], "rings": d["rings"], "node_block": d["node_block"], "groups": d["groups"],
            "global_tiles": d["global_tiles"]}


def rooflines(r, s_bytes, workload, elem="p2"):
    """The dominant kernel's HBM roofline by algorithmic bytes (its share of
    the step's), the step's, and the measured traffic beside them."""
    info = r["info"]
    N, E = info["nodes"], info["elems"]
    tile = r["schedule"]["waves"] > 0
    names = kernel_names(r["schedule"])
    km = dict(zip(names, r["kernel_ms"][:4]))
    alg = alg_bytes(N, E, s_bytes, tile)
    des = design_bytes(info, s_bytes, tile, elem)
    dom = max((k for k in names if k != "k_wall"), key=lambda k: km[k])
    achieved = alg[dom] / (km[dom] * 1e-3) / 1e9
    traffic = measured_traffic(dom, workload)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
            "alg_bytes_per_launch": alg[dom], "alg_bytes_per_node": round(alg[dom] / N, 1), "nodes": N,
            "launch_ms": round(km[dom], 5),
            "traffic_over_alg": round(traffic / alg[dom], 3) if traffic else None,
            "design_bytes_per_launch": des[dom],
            "design_GBs": round(des[dom] / (km[dom] * 1e-3) / 1e9, 1)}
    total = sum(alg.values())
    step_gbs = total / (r["ms_per_step"] * 1e-3) / 1e9
    traffics = [measured_traffic(k, workload) for k in names]
    step_traffic = sum(traffics) if all(t is not None for t in traffics) else None
    step = {"bound": "hbm", "achieved": round(step_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(step_gbs / HBM_PEAK_GBS, 4), "alg_bytes_per_step": total,
            "alg_bytes_per_node": round(total / N, 1), "traffic": step_traffic,
            "traffic_over_alg": round(step_traffic / total, 3) if step_traffic else None}
    return roof, step, km, dom


def _summary(r, s_bytes, N, workload, elem="p2"):
    roof, step, km, _ = rooflines(r, s_bytes, workload, elem)
    return {"value": round(N / (r["ms_per_step"] * 1e-3), 1), "ms_per_step": round(r["ms_per_step"], 5),
            "schedule": _schedule(r),
            "kernels_ms": {k: round(v, 5) for k, v in km.items()},
            "roofline": roof, "step_roofline": step,
            "forces_call_us": round(r["forces_us"], 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cases", type=int, default=64, help="cases in the batched ensemble")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-single", action="store_true", help="skip the single-mesh plunge runs")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate network's run")
    ap.add_argument("--no-q2", action="store_true", help="skip the single-mesh run on 9-node quadrilaterals")
    ap.add_argument("--train-step-only", action="store_true",
                    help="time only the surrogate's training step (for profiling); prints its own JSON line")
    ap.add_argument("--mesh-cache", default=None,
                    help="directory for the ensemble's meshes (.npz): reused when present, else written")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="processes building the ensemble's meshes (1 = in this process)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): it measures one GPU's share; "
              "the multi-GPU decomposition is described, not implemented", file=sys.stderr)
        sys.exit(2)
    if args.train_step_only:
        import torch
        from paper_2002_04353_amd import alelb, surrogate as S
        if not torch.cuda.is_available():
            print("bench.py needs a GPU", file=sys.stderr)
            sys.exit(1)
        torch.cuda.set_device(0)
        alelb.load()
        if args.copy_mib:
            copy_calibration(torch, args.copy_mib)
        ms, tf, gbs = train_step_timing(torch)
        print(json.dumps({"metric": "surrogate training step", "widths": list(S.WIDTHS), "ms": ms,
                          "TFLOPs": tf, "GBs": gbs,
                          "algorithmic_bytes": {b: train_step_bytes(S.WIDTHS, b) for b in ms}}), flush=True)
        return
    from paper_2002_04353_amd import cases
    # meshes are built in a process pool before anything touches the GPU
    t0 = time.perf_counter()
    ens = cases.ensemble(n_cases=args.cases, workers=args.workers, cache_dir=args.mesh_cache)
    ens_init = cases.concat_init(ens["inits"])
    Nb = sum(m.n_nodes for m in ens["meshes"])
    Eb = sum(m.n_elems for m in ens["meshes"])
    print(f"# ensemble: {args.cases} cases, {Nb} nodes, {Eb} elements, built in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    single = None if args.no_single else cases.plunge()
    single_q2 = None if args.no_q2 else cases.plunge(elem="q2")

    import torch
    from paper_2002_04353_amd import alelb
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_mib:
        copy_calibration(torch, args.copy_mib)
    stream = torch.cuda.Stream()
    meshes = [m.arrays() for m in ens["meshes"]]
    with torch.cuda.stream(stream):
        rb32g = time_solver(alelb, torch, meshes, ens["params"], ens_init, "fp32", args.steps, args.warmup)
        print(f"# batched fp32 (one stream, graphs) {rb32g['ms_per_step'] * 1e3:.1f} us/step, kernels "
              f"{rb32g['kernel_ms']}, schedule {rb32g['schedule']}", file=sys.stderr, flush=True)
        rb32s = time_solver(alelb, torch, meshes, ens["params"], ens_init, "fp32", args.steps, args.warmup,
                            split=True)
        print(f"# batched fp32 (halves on two streams) {rb32s['ms_per_step'] * 1e3:.1f} us/step",
              file=sys.stderr, flush=True)
        rb32 = min((rb32g, rb32s), key=lambda r: r["ms_per_step"])
        rb32["launch"] = "halves on two streams" if rb32 is rb32s else "one stream, graph-captured step pairs"
        rb64 = None
        if not args.no_fp64:
            rb64 = time_solver(alelb, torch, meshes, ens["params"], ens_init, "fp64", args.steps, args.warmup,
                               split=rb32["launch"] == "halves on two streams")
            print(f"# batched fp64 {rb64['ms_per_step'] * 1e3:.1f} us/step, kernels {rb64['kernel_ms']}",
                  file=sys.stderr, flush=True)
        rs32 = rs64 = None
        if single is not None:
            sm = single["mesh"].arrays()
            rs32 = time_solver(alelb, torch, sm, single["params"], single["init"], "fp32", 2 * args.steps,
                               args.warmup)
            print(f"# single fp32 {rs32['ms_per_step'] * 1e3:.2f} us/step, kernels {rs32['kernel_ms']}",
                  file=sys.stderr, flush=True)
            if not args.no_fp64:
                rs64 = time_solver(alelb, torch, sm, single["params"], single["init"], "fp64", 2 * args.steps,
                                   args.warmup)
                print(f"# single fp64 {rs64['ms_per_step'] * 1e3:.2f} us/step, kernels {rs64['kernel_ms']}",
                      file=sys.stderr, flush=True)
        rq32 = None
        if single_q2 is not None:
            rq32 = time_solver(alelb, torch, single_q2["mesh"].arrays(), single_q2["params"], single_q2["init"],
                               "fp32", 2 * args.steps, args.warmup)
            print(f"# single q2 fp32 {rq32['ms_per_step'] * 1e3:.2f} us/step, kernels {rq32['kernel_ms']}",
                  file=sys.stderr, flush=True)
    torch.cuda.synchronize()

    value = Nb / (rb32["ms_per_step"] * 1e-3)
    roof, step_roof, km, dom = rooflines(rb32, 4, "ensemble_fp32")
    cl = [f["cl"] for f in rb32["forces"]]
    out = {
        "metric": "mesh-node updates/s (batched FP32-mixed; FP64 and single-mesh alongside; HBM GB/s vs peak)",
        "value": round(value, 1),
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(rb32["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded NACA0012 O-meshes, seeded motion parameters, impulsive start)",
        "config": {"workload": f"batched ensemble: {args.cases} pitch+plunge NACA0012 cases, {Nb} P2 nodes "
                               f"(meshes of 50k-300k nodes), Ma~U(0.2,0.7), k~U(0.05,1), Re=1850, "
                               f"FP32 populations / FP64 geometry, {rb32['launch']}",
                   "cases": args.cases, "nodes": Nb, "elements": Eb},
        "ms_per_step_one_stream_graphs": round(rb32g["ms_per_step"], 5),
        "ms_per_step_two_streams": round(rb32s["ms_per_step"], 5),
        "roofline": roof,
        "step_roofline": step_roof,
        "roofline_valu": valu_roofline(dom, "ensemble_fp32", km[dom]),
        "schedule": _schedule(rb32),
        "kernels_ms": {k: round(v, 5) for k, v in km.items()},
        "cl_range_after_run": [round(min(cl), 5), round(max(cl), 5)],
        "forces_call_us": round(rb32["forces_us"], 1),
    }
    if rb64:
        out["batched_fp64"] = _summary(rb64, 8, Nb, "ensemble_fp64")
    if rs32:
        Ns = single["mesh"].n_nodes
        out["single_fp32"] = dict(_summary(rs32, 4, Ns, "plunge_fp32"),
                                  workload=f"plunging NACA0012, {Ns} P2 nodes, h=0.2c, k=1, Ma=0.2, Re=1e4")
        # c_L, c_D, c_m every 50 steps over the first 600 (before the trailing-edge cold spot of this Re)
        out["single_fp32"]["t_cl_cd_cm_series"] = force_series(alelb, single["mesh"].arrays(), single["params"],
                                                               single["init"], 600, 50)
        if rs64:
            out["single_fp64"] = _summary(rs64, 8, Ns, "plunge_fp64")
    if rq32:
        Nq = single_q2["mesh"].n_nodes
        out["single_q2_fp32"] = dict(_summary(rq32, 4, Nq, "plunge_q2_fp32", "q2"),
                                     workload=f"plunging NACA0012, {Nq} Q2 nodes (9-node quadrilaterals, "
                                              "structured near-wall layers), h=0.2c, k=1, Ma=0.2, Re=1e4")
    if not args.no_surrogate:
        try:
            out["surrogate"] = surrogate_run(torch, ens)
        except Exception as exc:  # the solver's line above stays valid
            out["surrogate"] = {"error": f"{type(exc).__name__}: {exc}"}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(ens["meshes"][0], ens["params"][0], ens["inits"][0], args.cpu_seconds,
                                           "case 0 of the same ensemble")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
