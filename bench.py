"""Benchmark: 3-way ACA build of Laplace-domain BEM tensors on one MI355X.

One step = the whole hot path on the 3072-triangle cube workload (collocation, L = 64,
s_l = 20 (1 + 0.95 e^{i 2 pi (l + 1/2)/64}), leaf 32, eta 1, eps 1e-6, FP64): the dense
near field and the 3D-ACA of every far block for the single layer AND the double layer,
plus one reordered product (eq. product, 2 right-hand sides per frequency) with each.
The two operators are built together (gaca_build_both: the far blocks of both share every
far-field launch).  The problem (mesh, tree, partition, device geometry) is created before
the timed region; the right-hand sides are resident in HBM.

Prints ONE JSON line.  value = kernel entries per second, where the entries are the
tensor entries the method needs: the dense near field (m n L per near block), the rows
and columns the face ACAs read (rho (m + n) per face) and the frequency fibres (r L).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
PHASES = ["face", "aca", "expand", "tail"]
KID = {"slp": 0, "dlp": 1}
# HBM traffic of the dominant kernel from hardware counters, taken with the kernel source
# whose SHA-256 is stored beside it; any later change of that source voids the figure
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "far_aca_large_cube3072_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2312_11219_amd", "csrc", "far_aca.hip")


def measured_traffic(kernel_name):
    """Bytes per launch of kernel_name from the stored counter runs, or None when there are
    none for it or its source has changed since."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
        with open(KERNEL_SOURCE, "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != sha or not kernel_name.startswith(rec.get("kernel", "\0")):
        return None
    return rec.get("traffic_bytes_per_launch")


def dominant_kernels(kernels, all_stats):
    """Per-kernel device time (mean over steps), launches and algorithmic flops of one step,
    keyed by the kernel's name as the profiler lists it (FP64 build).  The face-ACA classes
    0-2 share their stream with the Gram-row kernel, so only class 3 (one kernel per launch
    window) is listed as a single kernel.  A joint build of both operators reports its shared
    launches in the stats of each operator: they are counted once, as kernel id -1."""
    out = {}
    nsteps = len(all_stats)
    for stp in all_stats:
        joint = stp[0]["joint_build"] > 1
        for k, st in zip(kernels[:1] if joint else kernels, stp):
            kid = -1 if joint else KID[k]
            rows = [(f"far_face_kernel<{kid}, false, false>", st["ms_far_phase"][0],
                     st["launches_phase"][0], st["far_flops_phase"][0]),
                    ("far_expand_kernel<false>", st["ms_far_phase"][2], st["launches_phase"][2],
                     st["far_flops_phase"][2]),
                    (f"far_tail_kernel<{kid}, false, false>", st["ms_far_phase"][3],
                     st["launches_phase"][3], st["far_flops_phase"][3]),
                    ("far_aca_large_kernel<512, false, 106496, 1> (faces with a side above 128)",
                     st["ms_far_by_kind"][3], st["launches_by_kind"][3], st["far_flops_by_kind"][3])]
            for name, ms, nl, fl in rows:
                e = out.setdefault(name, {"ms": 0.0, "launches": 0, "flops": 0.0})
                e["ms"] += ms / nsteps
                e["launches"] += nl / nsteps
                e["flops"] += fl / nsteps
    for e in out.values():
        e["launches"] = int(round(e["launches"]))
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="C2")
    ap.add_argument("--nrhs", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    # counter calibration: one y = 1.0 * x pass over this many bytes of FP32 before the
    # warm-up (a kernel of known traffic for the FETCH_SIZE / WRITE_SIZE scale)
    ap.add_argument("--copy-calibration", type=int, default=0)
    return ap.parse_args()


def cpu_baseline(cfg, xyz, tri, s, budget_s):
    """The oracle timed on a bounded sample of the same workload: seeded random far blocks
    (dense assembly + serial 3D-ACA, as the oracle does it) and near blocks, until about
    budget_s seconds of CPU work; reported in the same unit (entries per second)."""
    import numpy as np
    from oracle.aca3d import aca3d
    from oracle.hmatrix import Problem

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    op = Problem(xyz, tri, s, cfg["leaf"], cfg["eta"])
    rng = np.random.default_rng(0)
    far_order = rng.permutation(len(op.far))
    near_order = rng.permutation(len(op.near))
    # the workload's mix: near entries vs far blocks in proportion to their counts
    entries = 0.0
    t0 = time.perf_counter()
    nf = nn = 0
    fi = ni = 0
    while time.perf_counter() - t0 < budget_s and (fi < len(far_order) or ni < len(near_order)):
        for kernel in cfg["kernels"]:
            if fi < len(far_order):
                blk = op.far[far_order[fi]]
                T = op.block_tensor(kernel, blk, True)
                res = aca3d(T, cfg["eps"], cfg["eps_aca"])
                m, n = blk[1], blk[3]
                entries += sum(c.U.shape[1] * (m + n) for c in res.crosses) + res.rank * op.L
                nf += 1
            if ni < len(near_order):
                blk = op.near[near_order[ni]]
                op.block_tensor(kernel, blk, False)
                entries += blk[1] * blk[3] * op.L
                nn += 1
        fi += 1
        ni += 1
    dt = time.perf_counter() - t0
    return {"value": entries / dt, "unit": "entries/s", "cores": threads, "kind": "oracle",
            "sample": f"{fi} far + {ni} near blocks per kernel ({','.join(cfg['kernels'])}), "
                      f"seeded random order, {dt:.1f} s, oracle dense block assembly "
                      f"(C, OpenMP over pairs) + serial numpy 3D-ACA"}


def apply_bench(args):
    """--config C5: the 81920-triangle icosphere, L = 256, eps 1e-6, mixed build, then the
    compressed operator applied to 256 right-hand sides (N(0,1) + i N(0,1), seeded, made on
    the GPU) in four calls of 64 on the matrix cores; one JSON line with the build time,
    storage, apply time / flop rate / operator bytes per second and the apply's relative
    difference from the FP64 apply of the same operator on 8 of the right-hand sides."""
    import torch

    import paper_2312_11219_amd as gaca
    from inputs import circle_frequencies, get_config, mesh_for_config

    cfg = get_config(args.config)
    xyz, tri = mesh_for_config(args.config)
    s = circle_frequencies(cfg["L"], cfg["c0"], cfg["rho"])
    M, L = tri.shape[0], cfg["L"]
    nrhs, chunk = cfg.get("nrhs", 256), 64
    ctx = gaca.Context(0)
    prob = gaca.Problem(ctx, xyz, tri, s, leaf_size=cfg["leaf"], eta=cfg["eta"], eps3d=cfg["eps"],
                        eps_aca=cfg["eps_aca"], precision="mixed", verbose=1,
                        batch_bytes=80 << 30)
    t0 = time.perf_counter()
    h = prob.build("slp")
    build_s = time.perf_counter() - t0
    st = h.stats()
    print(f"build {build_s:.1f} s", file=sys.stderr, flush=True)
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    X = torch.empty((L, M, chunk), dtype=torch.complex64, device="cuda")
    ms_dev = flops = 0.0
    part_ms, part_fl = [0.0] * 3, [0.0] * 3
    first = None
    for c in range(nrhs // chunk):
        # N(0,1) real and imaginary parts
        X.real.normal_(generator=g)
        X.imag.normal_(generator=g)
        Y = h.apply(X, mode="sum")
        torch.cuda.synchronize()
        a = h.stats()
        ms_dev += a["ms_apply"]
        flops += a["apply_flops"]
        for k in range(3):
            part_ms[k] += a["ms_apply_part"][k]
            part_fl[k] += a["apply_flops_part"][k]
        print(f"apply {c}: {a['ms_apply']:.1f} ms", file=sys.stderr, flush=True)
        if first is None:
            first = (X[:, :, :8].clone(), Y[:, :8].clone())
    # FP64 reference after the timed applies (its workspace would shrink their column chunks)
    del X, Y
    Y64 = h.apply(first[0].to(torch.complex128), mode="sum")
    torch.cuda.synchronize()
    diff = ((first[1].to(torch.complex128) - Y64).norm() / Y64.norm()).item()
    del Y64, first
    opb = a["apply_operator_bytes"]
    names = ["apply_far_t_kernel (T = F X)", "apply_far_z_kernel (Z = W T)",
             "apply_leaf_mfma_kernel (near N X + far U Z)"]
    dom = max(range(3), key=lambda k: part_ms[k])
    dom_tf = part_fl[dom] / max(part_ms[dom], 1e-9) / 1e9
    out = {"metric": "3-way ACA build s + kernel entries/s, FP64 vs mixed-prec at stated rel err",
           "value": (st["entries_near"] + st["entries_face"] + st["entries_fibre"]) / build_s,
           "unit": "entries/s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": build_s * 1e3 + ms_dev, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "mixed (f32 faces/factors, f64 fibres/norms)",
           "data": "synthetic",
           "config": {"workload": f"icosphere subdivision 6 ({M} triangles), collocation P0 single "
                                  f"layer, L={L} circle frequencies c0={cfg['c0']} rho={cfg['rho']}, "
                                  f"leaf {cfg['leaf']}, eta {cfg['eta']}, eps {cfg['eps']}, mixed build "
                                  f"+ apply to {nrhs} rhs (4 x 64) on the matrix cores",
                      "global_batch": nrhs, "parallelism": "single-gpu"},
           "build_s": build_s,
           "compression": st["compression"],
           "bytes_far": st["bytes_far"], "bytes_near": st["bytes_near"],
           "ranks": [st["rank_min"], st["rank_max"], round(st["rank_mean"], 2)],
           "face_rank_max": st["face_rank_max"],
           "far_phase_ms": dict(zip(PHASES, st["ms_far_phase"])),
           "apply": {"rhs": nrhs, "ms": ms_dev, "tflops": flops / ms_dev / 1e9,
                     "operator_GB_per_s": opb * (nrhs // chunk) / ms_dev / 1e6,
                     "rel_diff_vs_fp64_apply": diff},
           "apply_kernels": {names[k]: {"ms": part_ms[k], "tflops": part_fl[k] / max(part_ms[k], 1e-9) / 1e9}
                             for k in range(3)},
           "roofline": {"bound": "mfma", "kernel": names[dom] + " on v_mfma_f32_16x16x4f32",
                        "achieved": dom_tf, "peak": 157.3, "unit": "TFLOP/s",
                        "frac": dom_tf / 157.3, "traffic": None}}
    print(json.dumps(out), flush=True)


def build_all(prob, kernels):
    """The operators `kernels` of prob: both collocation operators in one joint build."""
    if sorted(kernels) == ["dlp", "slp"]:
        hs, hd = prob.build_both()
        return [hs, hd] if kernels[0] == "slp" else [hd, hs]
    return [prob.build(k) for k in kernels]


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the far blocks would shard by LPT across GPUs, see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.config == "C5":
        apply_bench(args)
        return

    import paper_2312_11219_amd as gaca
    from inputs import circle_frequencies, get_config, mesh_for_config, random_rhs

    cfg = get_config(args.config)
    xyz, tri = mesh_for_config(args.config)
    s = circle_frequencies(cfg["L"], cfg["c0"], cfg["rho"])
    M, L = tri.shape[0], cfg["L"]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    ctx = gaca.Context(0, stream=stream)
    kernels = cfg["kernels"]
    # one problem; with both operators they are built together (gaca_build_both: the blocks of
    # both share every far-field launch)
    t_setup = time.perf_counter()
    prob = gaca.Problem(ctx, xyz, tri, s, leaf_size=cfg["leaf"], eta=cfg["eta"],
                        eps3d=cfg["eps"], eps_aca=cfg["eps_aca"])
    t_setup = time.perf_counter() - t_setup
    X = torch.from_numpy(random_rhs(L, M, args.nrhs, seed=0)).to(dev)

    def step():
        hs = build_all(prob, kernels)
        for h in hs:
            h.apply(X, stream=stream)
        out = [h.stats() for h in hs]
        del hs
        return out

    if args.copy_calibration > 0:
        n = args.copy_calibration // 4
        xc = torch.ones(n, dtype=torch.float32, device=dev)
        yc = torch.empty_like(xc)
        torch.cuda.synchronize()
        torch.mul(xc, 1.0, out=yc)
        torch.cuda.synchronize()
        del xc, yc
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_stats = []
    for _ in range(args.steps):
        all_stats.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    last = all_stats[-1]
    entries_step = sum(st["entries_near"] + st["entries_face"] + st["entries_fibre"] for st in last)
    value = entries_step * args.steps / elapsed
    # dominant kernel: the far-field kernel with the largest device time over the step; each
    # launch is timed with HIP events on the stream it runs on
    kern = dominant_kernels(kernels, all_stats)
    dom_name = max(kern, key=lambda k: kern[k]["ms"])
    dom = kern[dom_name]
    far_ms = np.mean([sum(st["ms_far_kernel"] for st in stp) / stp[0]["joint_build"]
                      for stp in all_stats])
    near_ms = np.mean([sum(st["ms_near_kernel"] for st in stp) for stp in all_stats])
    achieved = dom["flops"] / (dom["ms"] * 1e-3) / 1e12
    phase_ms = np.mean([[sum(st["ms_far_phase"][k] for st in stp) / stp[0]["joint_build"]
                         for k in range(4)] for stp in all_stats], axis=0)
    out = {
        "metric": "3-way ACA build s + kernel entries/s, FP64 vs mixed-prec at stated rel err",
        "value": value,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"cube surface 16x16 squares per face ({M} triangles), "
                               f"collocation P0, single+double layer, L={L} circle frequencies "
                               f"c0={cfg['c0']} rho={cfg['rho']}, leaf {cfg['leaf']}, eta "
                               f"{cfg['eta']}, eps {cfg['eps']}, eps_aca {cfg['eps_aca']}, "
                               f"build + apply with {args.nrhs} rhs",
                   "global_batch": 1, "parallelism": "single-gpu"},
        "build_ms": {k: st["ms_total"] for k, st in zip(kernels, last)},
        "near_kernel_ms": near_ms,
        "far_kernel_ms": far_ms,
        "entries_per_step": entries_step,
        "ranks": {k: [st["rank_min"], st["rank_max"], round(st["rank_mean"], 2)]
                  for k, st in zip(kernels, last)},
        "compression": {k: st["compression"] for k, st in zip(kernels, last)},
        "setup_s": t_setup,
        "far_phase_ms": {name: float(phase_ms[k]) for k, name in enumerate(PHASES)},
        "far_kernels": {k: {"ms": round(v["ms"], 3), "launches": v["launches"],
                            "tflops": round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 3)}
                        for k, v in kern.items()},
        "far_iters": {k: st["far_iters"] for k, st in zip(kernels, last)},
        "aca_block_max_ms": {k: st["ms_far_aca_block_max"] for k, st in zip(kernels, last)},
        "roofline": {"bound": "alu", "kernel": dom_name,
                     "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS, "traffic": measured_traffic(dom_name),
                     "launches_per_step": dom["launches"],
                     "ms_per_launch": dom["ms"] / max(1, dom["launches"])},
    }
    if not args.no_mixed:
        # the FP64 apply of the same X as the mixed leg's reference, then the FP64 problem is
        # released (the mixed problem takes over its far-field streams)
        h64s = build_all(prob, kernels)
        y64s = [h.apply(X, stream=stream) for h in h64s]
        torch.cuda.synchronize()
        del h64s
        prob.close()
        out["mixed"] = mixed_leg(gaca, ctx, xyz, tri, s, cfg, X, kernels, stream, y64s, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, xyz, tri, s, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def mixed_leg(gaca, ctx, xyz, tri, s, cfg, X, kernels, stream, y64s, args):
    """The same step with the mixed-precision build (FP32 far-field faces and factors with
    the per-(block, frequency) scale, FP64 fibres/norms; near field stored FP32) and the
    relative difference of its apply from the FP64 build's apply of the same X (y64s)."""
    import numpy as np
    import torch
    pm = gaca.Problem(ctx, xyz, tri, s, leaf_size=cfg["leaf"], eta=cfg["eta"],
                      eps3d=cfg["eps"], eps_aca=cfg["eps_aca"], precision="mixed")
    X32 = X.to(torch.complex64)

    def step():
        hs = build_all(pm, kernels)
        out = [(h.stats(), h.apply(X32, stream=stream)) for h in hs]
        del hs
        return out

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step() for _ in range(max(1, args.steps))]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    last = runs[-1]
    entries = sum(st["entries_near"] + st["entries_face"] + st["entries_fibre"] for st, _ in last)
    errs = {}
    for k, (st, y), y64 in zip(kernels, last, y64s):
        d = (y.to(torch.complex128) - y64).norm().item() / y64.norm().item()
        errs[k] = d
    return {"value": entries * len(runs) / el, "unit": "entries/s",
            "ms_per_step": el / len(runs) * 1e3,
            "build_ms": {k: st["ms_total"] for k, (st, _) in zip(kernels, last)},
            "far_kernel_ms": float(np.mean([sum(st["ms_far_kernel"] for st, _ in r) / r[0][0]["joint_build"]
                                            for r in runs])),
            "far_phase_ms": [float(np.mean([sum(st["ms_far_phase"][k] for st, _ in r) / r[0][0]["joint_build"]
                                            for r in runs])) for k in range(4)],
            "apply_rel_diff_vs_fp64": errs,
            "ranks": {k: [st["rank_min"], st["rank_max"], round(st["rank_mean"], 2)]
                      for k, (st, _) in zip(kernels, last)},
            "far_iters": {k: st["far_iters"] for k, (st, _) in zip(kernels, last)}}


if __name__ == "__main__":
    main()
