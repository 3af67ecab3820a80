"""Benchmark: 3-way ACA build of Laplace-domain BEM tensors on one MI355X.

Default workload (--config C3): the unit ball as icosphere subdivision 5 (20480 triangles),
collocation P0 single layer, L = 128 frequencies s_l = 40 (1 + 0.95 e^{i 2 pi (l + 1/2)/128}),
leaf 32, eta 1, eps 1e-5 (face tolerance eps / 100).  One step = the whole hot path: the
dense near field and the 3D-ACA of every far block (Algorithm 1), then one reordered product
(eq. product, 2 right-hand sides per frequency).  The problem (mesh, tree, partition,
device geometry) is created before the timed region; the right-hand sides are resident in
HBM.  Two legs run one after the other: the FP64 build (value) and the mixed-precision
build (FP32 far-field faces and factors, FP64 fibres, norms and near-field quadrature).

Each leg states its relative Frobenius error against the FP64 oracle's dense tensor on a
seeded sample of far and near blocks; the oracle's dense blocks come from the cpu_baseline
leg, which times the oracle (dense assembly + serial 3D-ACA) on that sample.

Prints ONE JSON line.  value = kernel entries per second, where the entries are the
tensor entries the method evaluates: the near field (m n L per near block, of which the
conjugate mirror of the frequencies halves the evaluated part: both counts are stated), the
rows and columns the face ACAs read (rho (m + n) per face) and the frequency fibres (r L).
--config C2 runs the 3072-triangle cube (single and double layer built together), C5 the
81920-triangle icosphere build + apply of 256 right-hand sides.
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
FP32_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
PHASES = ["face", "aca", "expand", "tail"]
KID = {"slp": 0, "dlp": 1}
# HBM traffic per launch of the far-field kernels from hardware counters (rocprofv3
# FETCH_SIZE and WRITE_SIZE on this workload, scaled by a plain copy of known size), stored
# with the SHA-256 of the kernel sources; any later change of those sources voids the figures
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "far_traffic_icosphere20480.json")


TRAFFIC_SOURCES = ["paper_2312_11219_amd/csrc/far_aca.hip", "paper_2312_11219_amd/csrc/device_util.h",
                   "paper_2312_11219_amd/csrc/entries_dev.h", "paper_2312_11219_amd/csrc/fastmath_dev.h",
                   "paper_2312_11219_amd/csrc/galerkin_dev.h", "paper_2312_11219_amd/csrc/kernels.h",
                   "paper_2312_11219_amd/csrc/internal.h",
                   # the far-field driver: how many faces one launch covers (batches, classes)
                   "paper_2312_11219_amd/csrc/lib.cpp"]
COPY_KERNEL = "MulFunctor<float>"   # the torch y = 1.0 * x pass of --copy-calibration


def sources_sha256(paths):
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def write_traffic(fetch_db, write_db, copy_bytes, out_path):
    """Traffic record from two rocprofv3 --pmc result databases of this bench (one with
    FETCH_SIZE, one with WRITE_SIZE, both run with --copy-calibration copy_bytes): per far
    kernel the mean KiB per dispatch over the last build that launched it (a timed build:
    the first build of a problem sizes its batches from a generous guess and may cut them
    differently), scaled so that the calibration copy reads and writes copy_bytes, with the
    SHA-256 of the kernel and driver sources.  A build starts with its near-field kernels,
    so the near-field dispatches mark the build boundaries."""
    import re
    import sqlite3

    def per_kernel(db, counter):
        con = sqlite3.connect(db)
        rows = con.execute("select kernel_name, dispatch_id, sum(value), max(duration) from "
                           "counters_collection where counter_name = ? group by kernel_name, "
                           "dispatch_id order by dispatch_id", (counter,)).fetchall()
        con.close()
        disp, copy, starts = {}, None, []
        for name, did, v, dur in rows:
            if COPY_KERNEL in name and copy is None:
                copy = v
                continue
            short = re.sub(r"\(.*\)$", "", name).replace("void ", "").replace("gaca::", "")
            if short.startswith("near_"):
                starts.append(did)
            if not (short.startswith("far_") or short.startswith("near_")):
                continue
            disp.setdefault(short, []).append((did, v, dur))
        if copy is None:
            raise SystemExit(f"{db}: no calibration copy dispatch (run the bench with --copy-calibration)")
        out = {}
        for short, ds in disp.items():
            if not short.startswith("near_"):
                last = ds[-1][0]
                b = max([d for d in starts if d < last], default=-1)
                ds = [x for x in ds if x[0] > b]
            out[short] = [len(ds), sum(x[1] for x in ds), sum(x[2] for x in ds)]
        return out, copy

    fk, fcopy = per_kernel(fetch_db, "FETCH_SIZE")
    wk, wcopy = per_kernel(write_db, "WRITE_SIZE")
    ff, wf = copy_bytes / (fcopy * 1024.0), copy_bytes / (wcopy * 1024.0)
    kernels = {}
    for name, (n, v, dur) in fk.items():
        if name not in wk:
            continue
        wn, wv, _ = wk[name]
        fb, wb = v / n * 1024.0 * ff, wv / wn * 1024.0 * wf
        kernels[name] = {"dispatches": n, "fetch_kib_mean": v / n, "write_kib_mean": wv / wn,
                         "mean_duration_ms_under_counters": dur / n / 1e6,
                         "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                         "traffic_bytes_per_launch": fb + wb}
    rec = {"workload": "icosphere 20480 triangles, collocation P0 single layer, L = 128 (bench.py "
                       "default): FP64 and mixed legs; per kernel the dispatches of the last build "
                       "that launched it",
           "sources": TRAFFIC_SOURCES, "source_sha256": sources_sha256(TRAFFIC_SOURCES),
           "copy_kernel": f"y = 1.0 * x, FP32, {copy_bytes} bytes read + written "
                          f"(bench.py --copy-calibration {copy_bytes})",
           "copy_fetch_kib": fcopy, "copy_write_kib": wcopy, "fetch_factor": ff, "write_factor": wf,
           "kernels": kernels}
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(f"wrote {out_path}: {len(kernels)} kernels, fetch factor {ff:.4f}, write factor {wf:.4f}")


def measured_traffic(kernel_name):
    """HBM bytes per launch of kernel_name from the stored counter runs, or None when there
    are none for it or its sources have changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
        digest = sources_sha256(rec["sources"])
    except (OSError, ValueError, KeyError):
        return None
    k = rec.get("kernels", {}).get(kernel_name)
    if rec.get("source_sha256") != digest or k is None:
        return None
    return k.get("traffic_bytes_per_launch")


def roofline(name, d):
    """Roofline of one far-field kernel: the expand kernel streams the face pool (bound by
    HBM: algorithmic bytes per launch over the launch time), the others by FP64 VALU work
    (algorithmic flops over the launch time)."""
    ms = d["ms"] / max(1, d["launches"])
    if name.startswith("far_expand_kernel") and d.get("bytes", 0) > 0:
        ach = d["bytes"] / max(1, d["launches"]) / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "kernel": name, "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic(name),
                "launches_per_step": d["launches"], "ms_per_launch": ms}
    ach = d["flops"] / (d["ms"] * 1e-3) / 1e12
    return {"bound": "alu", "kernel": name, "achieved": ach, "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS, "traffic": measured_traffic(name),
            "launches_per_step": d["launches"], "ms_per_launch": ms}


def large_kernel_name(threads, mixed, path):
    """Instantiation of far_aca_large_kernel<threads, mixed, LDS history bytes, path> that the
    library launches for the faces with a side above 128 (the name rocprofv3 lists)."""
    mx = "true" if mixed else "false"
    if path == 2:
        return f"far_aca_large_kernel<512, {mx}, 106496, 2>"
    hb = {1024: 90112, 512: 106496}.get(threads, 60800 if path == 1 else 32768)
    return f"far_aca_large_kernel<{threads}, {mx}, {hb}, {path}>"


def far_kernels(kernels, all_stats, mixed=False):
    """Per-kernel device time (mean over steps), launches and algorithmic flops of one step,
    keyed by the kernel's name as the profiler lists it.  The face-ACA classes 0-2 share their
    stream with the Gram-row kernel and are not listed; class 3 is listed per kernel path.  A
    joint build of both operators reports its shared launches in the stats of each operator:
    they are counted once, as kernel id -1."""
    out = {}
    nsteps = len(all_stats)
    mx = "true" if mixed else "false"
    for stp in all_stats:
        joint = stp[0]["joint_build"] > 1
        for k, st in zip(kernels[:1] if joint else kernels, stp):
            kid = -1 if joint else KID[k]
            rows = [(f"far_face_kernel<{kid}, false, {mx}>", st["ms_far_phase"][0],
                     st["launches_phase"][0], st["far_flops_phase"][0], st["far_bytes_phase"][0]),
                    (f"far_expand_kernel<{mx}>", st["ms_far_phase"][2], st["launches_phase"][2],
                     st["far_flops_phase"][2], st["far_bytes_phase"][2]),
                    (f"far_tail_kernel<{kid}, false, {mx}>", st["ms_far_phase"][3],
                     st["launches_phase"][3], st["far_flops_phase"][3], 0.0)]
            for path in range(3):
                rows.append((large_kernel_name(st["threads_large_used"], mixed, path),
                             st["ms_far_large_path"][path], st["launches_large_path"][path],
                             st["far_flops_large_path"][path], 0.0))
            for name, ms, nl, fl, by in rows:
                if nl == 0:
                    continue
                e = out.setdefault(name, {"ms": 0.0, "launches": 0, "flops": 0.0, "bytes": 0.0})
                e["ms"] += ms / nsteps
                e["launches"] += nl / nsteps
                e["flops"] += fl / nsteps
                e["bytes"] += by / nsteps
    for e in out.values():
        e["launches"] = int(round(e["launches"]))
    return out


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="C3")
    ap.add_argument("--nrhs", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--far-sample", type=int, default=256)
    ap.add_argument("--large-sample", type=int, default=8)
    ap.add_argument("--leaf-rows", type=int, default=32)
    # counter calibration: one y = 1.0 * x pass over this many bytes of FP32 before the
    # warm-up (a kernel of known traffic for the FETCH_SIZE / WRITE_SIZE scale)
    ap.add_argument("--copy-calibration", type=int, default=0)
    # no run: the traffic record from the FETCH_SIZE and WRITE_SIZE result databases of two
    # counter runs of this bench with --copy-calibration (written to --traffic-out)
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DB", "WRITE_DB"))
    ap.add_argument("--traffic-out", default=TRAFFIC_FILE)
    return ap.parse_args()


def cpu_baseline(cfg, xyz, tri, s, args):
    """The oracle timed on a bounded, seeded sample of the same workload: far blocks (dense
    assembly + serial 3D-ACA, as the oracle does it) and the near blocks of a few leaf rows
    (dense assembly).  Returns the baseline record and the sample's dense oracle tensors,
    against which both GPU legs state their errors.

    Sample: --far-sample far blocks drawn uniformly among those with sides <= 256, plus
    --large-sample among those with a side above 256 (seed 0), and every near block of
    --leaf-rows leaf rows (seed 1)."""
    import numpy as np
    from oracle.aca3d import aca3d
    from oracle.hmatrix import Problem

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    op = Problem(xyz, tri, s, cfg["leaf"], cfg["eta"],
                 scheme=cfg.get("scheme", "collocation"))
    far = np.array(op.far, dtype=np.int64)
    near = np.array(op.near, dtype=np.int64)
    rng = np.random.default_rng(0)
    side = np.maximum(far[:, 1], far[:, 3])
    small = np.nonzero(side <= 256)[0]
    large = np.nonzero(side > 256)[0]
    fpick = sorted(rng.choice(small, min(args.far_sample, small.size), replace=False).tolist()
                   + rng.choice(large, min(args.large_sample, large.size), replace=False).tolist())
    rows = np.unique(near[:, 0])
    rsel = np.random.default_rng(1).choice(rows, min(args.leaf_rows, rows.size), replace=False)
    npick = np.nonzero(np.isin(near[:, 0], rsel))[0].tolist()
    L = op.L
    sample = {"far": {}, "near": {}}
    ent_alg = ent_eval = 0.0
    t0 = time.perf_counter()
    for kernel in cfg["kernels"]:
        for b in fpick:
            blk = tuple(int(v) for v in far[b])
            T = op.block_tensor(kernel, blk, True)
            res = aca3d(T, cfg["eps"], cfg["eps_aca"])
            m, n = blk[1], blk[3]
            ent_alg += sum(c.U.shape[1] * (m + n) for c in res.crosses) + res.rank * L
            ent_eval += m * n * L
            sample["far"][(kernel, blk)] = T
        for b in npick:
            blk = tuple(int(v) for v in near[b])
            N = op.block_tensor(kernel, blk, False)
            ent_alg += blk[1] * blk[3] * L
            ent_eval += blk[1] * blk[3] * L
            sample["near"][(kernel, blk)] = N
    dt = time.perf_counter() - t0
    desc = (f"{len(fpick)} far blocks ({len(fpick) - min(args.large_sample, large.size)} of "
            f"the {small.size} with sides <= 256, {min(args.large_sample, large.size)} of the "
            f"{large.size} above; seed 0) and the {len(npick)} near blocks of {len(rsel)} leaf "
            f"rows (seed 1), per operator ({','.join(cfg['kernels'])})")
    rec = {"value": ent_alg / dt, "unit": "entries/s", "cores": threads, "kind": "oracle",
           "sample": f"{desc}; {dt:.1f} s of oracle dense block assembly (C, OpenMP over "
                     f"pairs) + serial numpy 3D-ACA per far block",
           "count": "algorithmic-equivalent: near m n L + far sum rho (m + n) + r L, the "
                    "entries the GPU count charges for the same blocks",
           "evaluated_entries_per_s": ent_eval / dt}
    return rec, sample, desc


def sample_errors(hs, kernels, prob, sample):
    """Relative Frobenius errors of the operators hs against the oracle's dense tensors of the
    sample: far blocks reconstructed from their exported factors, near blocks exported."""
    import numpy as np
    far, near = prob.blocks()
    fidx = {tuple(int(v) for v in b): i for i, b in enumerate(far)}
    nidx = {tuple(int(v) for v in b): i for i, b in enumerate(near)}
    out = {}
    for k, h in zip(kernels, hs):
        fn = fd = nn_ = nd = 0.0
        for (kern, blk), T in sample["far"].items():
            if kern != k:
                continue
            e = h.export_block(fidx[blk])
            C = np.zeros_like(T)
            for c in e["crosses"]:
                C += (c["U"] @ c["W"].T)[:, :, None] * c["f"][None, None, :]
            fn += np.linalg.norm(C - T) ** 2
            fd += np.linalg.norm(T) ** 2
        for (kern, blk), N in sample["near"].items():
            if kern != k:
                continue
            G = h.near_block(nidx[blk], blk[1], blk[3])
            nn_ += np.linalg.norm(G - np.transpose(N, (0, 2, 1))) ** 2
            nd += np.linalg.norm(N) ** 2
        out[k] = {"far": float(np.sqrt(fn / fd)), "near": float(np.sqrt(nn_ / nd)),
                  "all": float(np.sqrt((fn + nn_) / (fd + nd)))}
    return out


def build_all(prob, kernels):
    """The operators `kernels` of prob: both collocation operators in one joint build."""
    if sorted(kernels) == ["dlp", "slp"]:
        hs, hd = prob.build_both()
        return [hs, hd] if kernels[0] == "slp" else [hd, hs]
    return [prob.build(k) for k in kernels]


def run_leg(gaca, ctx, xyz, tri, s, cfg, X, stream, args, precision, sample):
    """Warm-up, then args.steps timed steps (build of every operator + one apply each) with
    the given precision; the last step's operators give the errors against the sample and
    the apply results."""
    import numpy as np
    import torch
    kernels = cfg["kernels"]
    t_setup = time.perf_counter()
    # face-ACA workgroup sizes chosen by the library's autotuner during the warm-up build
    # (a fresh cache file per run, so the choice is measured on this device)
    import tempfile
    cache = os.path.join(tempfile.mkdtemp(prefix="gaca_bench_"), "autotune.txt")
    prob = gaca.Problem(ctx, xyz, tri, s, scheme=cfg.get("scheme", "collocation"),
                        leaf_size=cfg["leaf"], eta=cfg["eta"], eps3d=cfg["eps"],
                        eps_aca=cfg["eps_aca"], precision=precision, autotune_cache=cache)
    t_setup = time.perf_counter() - t_setup
    Xp = X if precision == "fp64" else X.to(torch.complex64)

    def step(keep=False):
        hs = build_all(prob, kernels)
        ys = [h.apply(Xp, stream=stream) for h in hs]
        st = [h.stats() for h in hs]
        if keep:
            return st, hs, ys
        del hs
        return st

    step()   # the autotuner's build (one build per candidate), never timed
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_stats = [step() for _ in range(args.steps - 1)]
    last, hs, ys = step(keep=True)
    all_stats.append(last)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    entries = sum(st["entries_near"] + st["entries_face"] + st["entries_fibre"] for st in last)
    kern = far_kernels(kernels, all_stats, mixed=precision != "fp64")
    dom_name = max(kern, key=lambda k: kern[k]["ms"])
    dom = kern[dom_name]
    joint = last[0]["joint_build"]
    leg = {
        "value": entries * args.steps / elapsed,
        "ms_per_step": elapsed / args.steps * 1e3,
        "build_ms": {k: st["ms_total"] for k, st in zip(kernels, last)},
        "near_kernel_ms": float(np.mean([sum(st["ms_near_kernel"] for st in stp) for stp in all_stats])),
        "far_kernel_ms": float(np.mean([sum(st["ms_far_kernel"] for st in stp) / joint for stp in all_stats])),
        "entries_per_step": entries,
        "entries_near_evaluated": sum(st["entries_near"] for st in last),
        "entries_near_mirrored": sum(st["entries_near_mirrored"] for st in last),
        "ranks": {k: [st["rank_min"], st["rank_max"], round(st["rank_mean"], 2)] for k, st in zip(kernels, last)},
        "face_rank_max": {k: st["face_rank_max"] for k, st in zip(kernels, last)},
        "compression": {k: st["compression"] for k, st in zip(kernels, last)},
        "far_iters": {k: st["far_iters"] for k, st in zip(kernels, last)},
        "far_launches": {k: st["n_far_launches"] for k, st in zip(kernels, last)},
        "autotuned_workgroups": {"threads_large": last[0]["threads_large_used"],
                                 "threads_small": last[0]["threads_small_used"],
                                 "state": ["options", "measured", "cache"][last[0]["autotune_state"]]},
        "setup_s": t_setup,
        "far_phase_ms": {name: float(np.mean([sum(st["ms_far_phase"][i] for st in stp) / joint
                                              for stp in all_stats])) for i, name in enumerate(PHASES)},
        "far_kernels": {k: {"ms": round(v["ms"], 3), "launches": v["launches"],
                            "tflops": round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 3),
                            "gbs": round(v["bytes"] / max(v["ms"], 1e-9) / 1e6, 1)}
                        for k, v in kern.items()},
        # every listed far-field kernel against its roofline (same model as "roofline")
        "far_rooflines": {k: {f: r[f] for f in ("bound", "achieved", "unit", "frac")}
                          for k, r in ((k, roofline(k, v)) for k, v in kern.items())},
        "dominant": (dom_name, dom),
    }
    if sample is not None:
        leg["errors_vs_oracle"] = sample_errors(hs, kernels, prob, sample)
    ys = [y.to(torch.complex128) for y in ys]
    torch.cuda.synchronize()
    del hs
    prob.close()
    return leg, ys


def main():
    args = parse()
    if args.write_traffic:
        write_traffic(args.write_traffic[0], args.write_traffic[1], args.copy_calibration or (1 << 30),
                      args.traffic_out)
        return
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the far blocks would be dealt to the GPUs longest estimated work first, each GPU "
              "building and applying its share, with X gathered on every GPU)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    if args.config == "C5":
        apply_bench(args)
        return

    import paper_2312_11219_amd as gaca
    from inputs import circle_frequencies, get_config, mesh_for_config, random_rhs

    cfg = get_config(args.config)
    xyz, tri = mesh_for_config(args.config)
    s = circle_frequencies(cfg["L"], cfg["c0"], cfg["rho"])
    p1 = cfg.get("scheme") == "p1"
    # operator size: elements, or vertices for the P1 double layer (which has no mixed path)
    M, L = (xyz.shape[0] if p1 else tri.shape[0]), cfg["L"]
    if p1:
        args.no_mixed = True
    kernels = cfg["kernels"]
    sample = desc = cpu = None
    if not args.no_cpu_baseline:
        print("cpu baseline: oracle on the seeded sample", file=sys.stderr, flush=True)
        cpu, sample, desc = cpu_baseline(cfg, xyz, tri, s, args)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    ctx = gaca.Context(0, stream=stream)
    X = torch.from_numpy(random_rhs(L, M, args.nrhs, seed=0)).to(dev)
    if args.copy_calibration > 0:
        n = args.copy_calibration // 4
        xc = torch.ones(n, dtype=torch.float32, device=dev)
        yc = torch.empty_like(xc)
        torch.cuda.synchronize()
        torch.mul(xc, 1.0, out=yc)
        torch.cuda.synchronize()
        del xc, yc
    print("fp64 leg", file=sys.stderr, flush=True)
    leg64, y64 = run_leg(gaca, ctx, xyz, tri, s, cfg, X, stream, args, "fp64", sample)
    dom_name, dom = leg64.pop("dominant")
    ops = "+".join(kernels)
    out = {
        "metric": "3-way ACA build s + kernel entries/s, FP64 vs mixed-prec at stated rel err",
        "value": leg64["value"],
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": leg64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{cfg['name']}: {cfg['mesh'][0]} mesh ({tri.shape[0]} triangles"
                               + (f", {M} vertices), collocation at the vertices, P1 {ops}" if p1 else
                                  f"), {cfg.get('scheme', 'collocation')} P0 {ops}")
                               + f", L={L} circle "
                               f"frequencies c0={cfg['c0']} rho={cfg['rho']}, leaf {cfg['leaf']}, "
                               f"eta {cfg['eta']}, eps {cfg['eps']}, eps_aca {cfg['eps_aca']}, "
                               f"FP64 build + apply with {args.nrhs} rhs per step",
                   "global_batch": 1, "parallelism": "single-gpu"},
        "build_s": {k: v / 1e3 for k, v in leg64["build_ms"].items()},
        "near_mirrored": bool(leg64["entries_near_mirrored"] > 0),
        "roofline": roofline(dom_name, dom),
        "fp64": leg64,
    }
    if not args.no_mixed:
        print("mixed leg", file=sys.stderr, flush=True)
        legmx, ymx = run_leg(gaca, ctx, xyz, tri, s, cfg, X, stream, args, "mixed", sample)
        dname, d = legmx.pop("dominant")
        legmx["dominant_kernel"] = {"kernel": dname, "ms_per_launch": d["ms"] / max(1, d["launches"]),
                                    "tflops": d["flops"] / max(d["ms"], 1e-9) / 1e9}
        legmx["apply_rel_diff_vs_fp64_apply"] = {
            k: float((a - b).norm().item() / b.norm().item()) for k, a, b in zip(kernels, ymx, y64)}
        legmx["speedup_vs_fp64"] = leg64["ms_per_step"] / legmx["ms_per_step"]
        out["mixed"] = legmx
    if sample is not None:
        err = {"sample": desc, "fp64": leg64["errors_vs_oracle"]}
        if "mixed" in out:
            err["mixed"] = out["mixed"]["errors_vs_oracle"]
            err["abs_diff_mixed_minus_fp64"] = {
                k: abs(err["mixed"][k]["all"] - err["fp64"][k]["all"]) for k in kernels}
        out["errors_vs_fp64_oracle"] = err
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


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



if __name__ == "__main__":
    main()
