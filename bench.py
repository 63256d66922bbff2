"""Benchmark of the MGPBD global iteration on one MI355X.

One step = one frame of Algorithm 1 (predict, 20 global iterations of
assemble -> lazy AMG setup -> Galerkin -> MGPCG -> update, velocity). The
default workload is the ellipsoid muscle (64x64x128 grid clipped to an
ellipsoid: 290,757 vertices, 1,646,400 tets, 3,615,756 edge and volume rows,
328,877,342 entries of A), the largest workload one GPU holds as a single
body, with the FP32 V-cycle / FP64 PCG precision form, lazy setup every 20
frames. Its solves need tens of thousands of PCG iterations to reach 1e-6
(the log-uniform compliances spread the small eigenvalues of A over four
decades), so every solve runs to 1e-6 or to a budget of 500 PCG iterations,
whichever comes first, and the line reports the relative residual reached.
Prints one JSON line.

value = PCG throughput: sum over solves of (rows x PCG iterations) divided by
the time spent in the PCG loops (V-cycles included; assembly, Galerkin and
setup excluded). ms_per_step = wall time per frame.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("ms/frame and PCG constraint-DOF·iters/s at 1e-6 rel residual; "
          "SpMV HBM GB/s")
PEAK_HBM_GBS = 8000.0


def batch_groups(sizes, limit: int = 2**31 - 1):
    """Indices of consecutive bodies grouped so that each group's entries of A
    (sizes[k] per body) sum to less than limit, the most a batch holds (its
    entry indices are 32-bit); a body at or above limit alone forms a group
    (the library then rejects it)."""
    groups, cur, tot = [], [], 0
    for k, n in enumerate(sizes):
        if cur and tot + n >= limit:
            groups.append(cur)
            cur, tot = [], 0
        cur.append(k)
        tot += n
    if cur:
        groups.append(cur)
    return groups


def spmv_bytes(m: int, nnz: int) -> int:
    """Algorithmic bytes of one fine-level A p product (FP64 CSR, int32
    columns, int64 row pointers): values + columns + row pointers + one read
    of p + one write of q."""
    return 12 * nnz + 8 * (m + 1) + 8 * m + 8 * m


def mf_bytes(m: int, nv: int, n_inc: int, n_edges: int, n_vols: int, n_arap: int = 0):
    """Algorithmic bytes of the two kernels of one matrix-free fine-level A p
    product (every array counted once). The vertex gather reads the incidence
    pointers, rows and gradients, the inverse masses and p, and writes u (4
    values per vertex); the row pass reads the row vertex ids, the positions
    (edge and volume gradients are recomputed from them), the row kinds and
    the stored gradients of ARAP rows (when there are any), u, alpha~ and p,
    and writes q."""
    gather = 8 * (nv + 1) + 4 * n_inc + 24 * n_inc + 8 * nv + 8 * m + 32 * nv
    rows = 16 * m + 32 * nv + 8 * m + 8 * m + 8 * m
    if n_edges + n_vols:
        rows += 32 * nv
    if n_arap:
        rows += m + 96 * n_arap
    return gather, rows


def measured_traffic(name: str, sources):
    """HBM bytes per launch from a committed counter summary (profiles/), or
    None when the kernel sources changed after the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for src in sources:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("sources_sha256") != h.hexdigest():
        return None
    try:
        return int(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# every file the matrix-free kernels are compiled from
MF_SOURCES = tuple("paper_2505_13390_amd/csrc/" + f for f in (
    "k_mfree.hip", "mfree.hpp", "rowops.hpp", "grad.hpp", "kernels.hpp", "devutil.hpp",
    "common.hpp")) + ("include/mgpbd.h",)


def host_cpu():
    """CPU model, logical CPUs of the host and CPUs this process may run on."""
    model = "unknown"
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
    except AttributeError:
        usable = os.cpu_count()
    return model, os.cpu_count(), usable


# oracle MGPCG iterations timed per workload (about 10-20 s on one core)
ORACLE_ITERS = {"C0": 200, "C1": 50, "C2": 24, "A0": 200, "A1": 100}


def cpu_baseline(w, lmax_scale: float, iters: int):
    """The FP64 oracle on the same workload: frame 0, global iteration 0,
    a fixed number of preconditioned CG iterations (setup not timed).
    Returns the baseline record and the oracle's dlambda of that solve."""
    import numpy as np

    from oracle import oracle as O
    oo = O.default_opts(lmax_scale=lmax_scale)
    sim = O.Sim(w, oo)
    pos, vel = O.positions(w)
    # semi-implicit Euler predict of frame 0 (what the first global iteration sees)
    free = w.inv_mass > 0
    g = np.asarray(w.gravity)
    vel[free] += w.dt * g
    pos[free] += w.dt * vel[free]
    val, b = sim.assemble(pos)
    rp, col = sim.pattern()
    del sim
    h = O.Hier.build(rp, col, val, oo)
    del val
    t0 = time.perf_counter()
    x, st = h.pcg(b, 1e-6, 1000, force_iters=iters)
    dt = time.perf_counter() - t0
    model, ncpu, usable = host_cpu()
    rec = {"value": w.n_rows * st["iters"] / dt, "unit": "constraint-DOF*iters/s", "cores": 1,
           "kind": "oracle", "host_cpu": model, "host_nproc": ncpu, "process_cpus": usable,
           "sample": "%s, frame 0 global iteration 0: %d MGPCG iterations of the single-thread "
                     "FP64 oracle (%.1f s; setup and assembly untimed)"
                     % (w.name, st["iters"], dt)}
    return rec, x


def oracle_parity(w, opt, iters, x_ref):
    """A fresh GPU body with the timed run's options, frame 0, global
    iteration 0 with the oracle's forced PCG count: the error of its dlambda
    (= lambda after the first iteration) against the oracle's."""
    import numpy as np

    from paper_2505_13390_amd import binding as B
    body = B.Body(w, opt)
    B.mgpbd_force_pcg_iters(body.ctx, [iters])
    body.step(1)
    lam = B.mgpbd_get_lambda(body.ctx, body.m)
    body.close()
    err = float(np.abs(lam - x_ref).max() / np.abs(x_ref).max())
    return {"forced_pcg_iters": iters, "lambda_max_rel_err": err,
            "compare": "GPU dlambda vs FP64 oracle dlambda, element-wise, "
                       "max |d| / max |ref|"}


def bench_batch(args, B, W):
    """The 64 beams of the batch workload, stepped together as one
    block-diagonal system (default) or one after another (--sequential)."""
    import numpy as np
    import torch
    ws = W.batch_c3() if args.config == "C3" else W.stiff_c4(copies=args.copies)
    n_iters = args.iters or ws[0].iters
    prec = B.PREC_MIXED if args.precision == "mixed" else B.PREC_FP64
    opt = B.mgpbd_default_options(precision=prec, reuse_interval=args.reuse,
                                  matrix_free={"mf": 1, "csr": 0, "auto": 2}[args.fine],
                                  lmax_scale=args.lmax_scale or (1.5 if args.config == "C4"
                                                                 else 1.05),
                                  smoother={"jacobi": 0, "chebyshev": 1, "gs": 2}[args.smoother])
    if args.max_pcg:
        opt.max_pcg = args.max_pcg
    if args.vcycle_tail is not None:
        opt.vcycle_tail = args.vcycle_tail
    if args.fuse_transfers is not None:
        opt.fuse_transfers = args.fuse_transfers
    rows = [w.n_rows for w in ws]
    t0 = time.perf_counter()
    bodies = [B.Body(w, opt) for w in ws]
    if args.sequential:
        groups = [[b] for b in bodies]
        step = lambda: [b.step(n_iters) for b in bodies]
    else:
        # one system holds fewer than 2^31 entries of A: larger sets of bodies
        # (the eight stiff ellipsoid copies, 2.63e9 entries) run as the fewest
        # batches below that, one after another within each frame
        groups = [[bodies[k] for k in g] for g in batch_groups([b.nnz for b in bodies])]
        handles = [B.mgpbd_batch_create([b.ctx for b in g]) for g in groups]

        def step():
            out = []
            for h, g in zip(handles, groups):
                out.extend(B.mgpbd_batch_step(h, [b.x for b in g], [b.v for b in g], n_iters))
            return out
    print("created %d bodies (%d rows, %d entries) as %d system(s) in %.1f s"
          % (len(ws), sum(rows), sum(b.nnz for b in bodies), len(groups),
             time.perf_counter() - t0), file=sys.stderr, flush=True)
    # frame and PCG time of one frame: the systems run one after another
    first = [0]
    for g in groups[:-1]:
        first.append(first[-1] + len(g))

    def frame_ms(r, key):
        if args.sequential:
            return sum(x[key] for x in r)
        return sum(r[k][key] for k in first)
    for f in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for f in range(args.steps):
        r = step()
        res.append(r)
        ms = frame_ms(r, "ms_total")
        its = [int(x["pcg_iters"].sum()) for x in r]
        print("frame %d: %.1f ms, pcg iterations per body (sum over the frame) min %d max %d"
              % (args.warmup + f, ms, min(its), max(its)), file=sys.stderr, flush=True)
        if len(r) <= 8:
            for k, x in enumerate(r):
                print("  body %d: pcg iters %s, last ratio %.2e"
                      % (k, x["pcg_iters"].tolist(), float(x["pcg_ratio"][-1])),
                      file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dof_iters = sum(float(m) * float(x["pcg_iters"].sum()) for r in res for m, x in zip(rows, r))
    pcg_s = sum(frame_ms(r, "ms_pcg") for r in res) / 1e3
    ratios = np.concatenate([x["pcg_ratio"] for r in res for x in r])
    out = {
        "metric": METRIC, "value": dof_iters / pcg_s, "unit": "constraint-DOF*iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == B.PREC_FP64 else "f32 V-cycle / f64 PCG", "data": "synthetic",
        "config": {"workload": ("batch_64_beams_n4-24" if args.config == "C3"
                                else "stiff_ellipsoid_x%d" % len(ws)),
                   "lmax_scale": opt.lmax_scale,
                   "bodies": len(ws), "rows": sum(rows),
                   "mode": ("sequential contexts" if args.sequential else
                            "%d batch(es) of %s bodies" % (len(groups),
                                                           "/".join(str(len(g)) for g in groups))),
                   "iters_per_frame": n_iters, "precision": args.precision,
                   "fine_operator": {"mf": "matrix-free", "csr": "csr",
                                     "auto": "timed choice"}[args.fine],
                   "smoother": args.smoother,
                   "pcg_budget_per_solve": int(opt.max_pcg),
                   "solves_at_tol": int((ratios <= 1e-6).sum()), "solves": int(ratios.size),
                   "residual_reached": {"median": float(np.median(ratios)),
                                        "max": float(ratios.max())},
                   "ms_pcg_per_frame": 1e3 * pcg_s / args.steps},
    }
    if args.config == "C4":
        # |b| of every global iteration of body 0 in the first timed frame
        out["bnorm_history_body0"] = [float(v) for v in res[0][0]["bnorm"]]
        out["context"] = ("paper: 40.6 s/frame (20 iterations per frame) for its 1,667K-tet, "
                          "526K-vertex human muscle with ARAP rows (Fig. 1, Table 1, Sec. 5.4) on "
                          "an RTX 4090 with a Ryzen 9 7950X host (Sec. 5.2); another mesh, "
                          "constraint set and machine, not a target")
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--copies", type=int, default=8,
                    help="C4: copies of the stiff ellipsoid stepped as one batch")
    ap.add_argument("--config", default="C2", choices=["C0", "C1", "C2", "C3", "C4", "A0", "A1"],
                    help="C2 (default): the ellipsoid muscle; C1: the 32x32x128 beam; C3: the "
                         "64-beam batch; C4: the stiff ellipsoid copies; A0/A1: the ARAP beams")
    ap.add_argument("--lmax-scale", type=float, default=None,
                    help="margin on the power-method lambda_max (default 1.05; 1.5 for the "
                         "ARAP beams and the stiff copies, whose matrices drift further between "
                         "lazy setups)")
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="default: mixed for C2, C3 and C4, fp64 otherwise")
    ap.add_argument("--sequential", action="store_true",
                    help="C3: step the bodies one after another, each as its own context")
    ap.add_argument("--reuse", type=int, default=20)
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--max-pcg", type=int, default=None,
                    help="PCG iteration budget per solve (default 500 for C2 and C4, whose "
                         "solves cannot reach 1e-6 in a benchmark's time; 5000 otherwise)")
    ap.add_argument("--fine", default="mf", choices=["mf", "csr", "auto"],
                    help="fine-level products: matrix-free (default), assembled CSR, or the "
                         "faster of the two timed at the first setup")
    ap.add_argument("--smoother", default="jacobi", choices=["jacobi", "chebyshev", "gs"],
                    help="V-cycle smoother (Sec. 4.5): omega-Jacobi (default), Chebyshev or "
                         "multicolour Gauss-Seidel")
    ap.add_argument("--candidate", default="smoothed", choices=["smoothed", "ones"],
                    help="near-kernel candidate: Gauss-Seidel-smoothed random vectors (Sec. 4.3, "
                         "the default) or the all-ones vector (piecewise-constant P)")
    ap.add_argument("--candidates", type=int, default=1,
                    help="near-kernel candidates per level (Sec. 4.3 generates six); 1 is the "
                         "one-candidate hierarchy of the headline line")
    ap.add_argument("--vcycle-tail", type=int, default=None,
                    help="rows per body at or below which the coarse V-cycle levels run as one "
                         "fused launch (default 0 = one launch per pass)")
    ap.add_argument("--fuse-transfers", type=int, default=None, choices=[0, 1],
                    help="1: residual + restriction in one pass and the prolongation folded into "
                         "the first post-sweep; 0 (default): separate transfer kernels")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-frames", action="store_true",
                    help="time each kernel of every PCG product inside the timed frames with HIP "
                         "events (launches kernels directly instead of replaying the graph, "
                         "which slows the frames by a few percent)")
    ap.add_argument("--no-profile", action="store_true", help="(accepted; the default)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed frames, copy a 1 GiB buffer 3 times (reference "
                         "kernel of known size for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the multi-GPU layout of this solver is a design "
              "note (instances or slabs per GPU), no figure at several GPUs is produced.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2505_13390_amd import binding as B
    from paper_2505_13390_amd import workloads as W

    torch.cuda.set_device(0)
    if args.precision is None:
        args.precision = "mixed" if args.config in ("C2", "C3", "C4") else "fp64"
    if args.max_pcg is None and args.config in ("C2", "C4"):
        args.max_pcg = 500
    if args.config in ("C3", "C4"):
        bench_batch(args, B, W)
        return
    w = W.CONFIGS[args.config]()
    n_iters = args.iters or w.iters
    prec = B.PREC_MIXED if args.precision == "mixed" else B.PREC_FP64
    if args.lmax_scale is None:
        args.lmax_scale = 1.5 if args.config.startswith("A") else 1.05
    opt = B.mgpbd_default_options(precision=prec, reuse_interval=args.reuse,
                                  lmax_scale=args.lmax_scale, n_cand=args.candidates,
                                  b_mode=1 if args.candidate == "ones" else 0,
                                  profile_spmv=1 if args.profile_frames else 0,
                                  matrix_free={"mf": 1, "csr": 0, "auto": 2}[args.fine],
                                  smoother={"jacobi": 0, "chebyshev": 1, "gs": 2}[args.smoother])
    if args.max_pcg:
        opt.max_pcg = args.max_pcg
    if args.vcycle_tail is not None:
        opt.vcycle_tail = args.vcycle_tail
    if args.fuse_transfers is not None:
        opt.fuse_transfers = args.fuse_transfers
    t0 = time.perf_counter()
    body = B.Body(w, opt)
    print("created %s: %d rows, %d entries in %.1f s" % (w.name, body.m, body.nnz,
                                                         time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    for f in range(args.warmup):
        r = body.step(n_iters)
        print("warmup frame %d: %.1f ms, pcg iters %s" % (f, r["ms_total"], r["pcg_iters"].tolist()),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for f in range(args.steps):
        res.append(body.step(n_iters))
        print("frame %d: %.1f ms, setup %.1f ms, pcg %.1f ms, iters %s"
              % (args.warmup + f, res[-1]["ms_total"], res[-1]["ms_setup"], res[-1]["ms_pcg"],
                 res[-1]["pcg_iters"].tolist()), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_frame = 1e3 * wall / args.steps
    dof_iters = sum(float(body.m) * float(r["pcg_iters"].sum()) for r in res)
    pcg_s = sum(r["ms_pcg"] for r in res) / 1e3
    value = dof_iters / pcg_s
    spmv_calls = sum(r["spmv_calls"] for r in res)
    spmv_ms = sum(r["spmv_ms"] for r in res)
    # the fine-level product of PCG (same context, same kernels) 200 times back
    # to back on the context's stream, a torch stream of default priority so
    # that torch's events see the launches
    reps = 200
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    B.mgpbd_set_stream(body.ctx, stream.cuda_stream)
    xp = torch.randn(body.m, dtype=torch.float64, device="cuda")
    yp = torch.empty_like(xp)
    torch.cuda.synchronize()
    for _ in range(5):
        B.mgpbd_apply(body.ctx, xp, yp)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        B.mgpbd_apply(body.ctx, xp, yp)
    e1.record(stream)
    torch.cuda.synchronize()
    avg_ms = e0.elapsed_time(e1) / reps
    B.mgpbd_set_stream(body.ctx, 0)
    del xp, yp
    traffic = None
    is_mf = B.mgpbd_get_fine_operator(body.ctx) == 1
    if is_mf:
        ne, nvol = int(w.edges.shape[0]), int(w.vol_tet.shape[0])
        nar = int(w.arap_tet.shape[0])
        gb, rb = mf_bytes(body.m, int(w.n_verts), 2 * ne + 4 * nvol + 4 * nar, ne, nvol, nar)
        nbytes = gb + rb
        kname = ("fine-level A p, matrix-free: k_mf_gather + k_mf_rows<OpPcgDot> "
                 "(one launch each)")
        counters = {"C1": "k_mf_apply_beam32x32x128_counters.txt",
                    "C2": "k_mf_apply_ellipsoid64x64x128_counters.txt",
                    "A1": "k_mf_apply_arap32x32x128_counters.txt"}.get(args.config)
        if counters:
            # the product timed here is the FP64 PCG product in either precision
            traffic = measured_traffic(counters, MF_SOURCES)
    else:
        gb = rb = None
        nbytes = spmv_bytes(body.m, body.nnz)
        kname = "fine-level A p, CSR: k_rows/k_stream<OpPcgDot>"
    ach = nbytes / (avg_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": traffic,
            "kernel": kname, "bytes_per_launch": nbytes, "avg_launch_ms": round(avg_ms, 5),
            "timing": "%d back-to-back products after the timed frames, HIP events on "
                      "their stream" % reps}
    if gb is not None:
        roof["bytes_parts"] = {"k_mf_gather": gb, "k_mf_rows<OpPcgDot>": rb}
    if spmv_calls:
        # --profile-frames: HIP events around each kernel of every PCG product of
        # the timed frames (kernels launched directly, not from the graph)
        loop_ms = spmv_ms / spmv_calls
        first_ms = sum(r["spmv_first_ms"] for r in res) / spmv_calls
        roof["timed_region"] = {"products": int(spmv_calls), "avg_ms": round(loop_ms, 5),
                                "GB/s": round(nbytes / (loop_ms * 1e-3) / 1e9, 1),
                                "timing": "HIP events around each kernel of every PCG product"}
        if gb is not None:
            roof["timed_region"]["parts"] = {
                "k_mf_gather": {"bytes": gb, "avg_ms": round(first_ms, 5),
                                "GB/s": round(gb / (first_ms * 1e-3) / 1e9, 1)},
                "k_mf_rows<OpPcgDot>": {"bytes": rb, "avg_ms": round(loop_ms - first_ms, 5),
                                        "GB/s": round(rb / ((loop_ms - first_ms) * 1e-3) / 1e9,
                                                      1)}}
    nl = B.mgpbd_num_levels(body.ctx)
    lv = [B.mgpbd_get_level(body.ctx, l) for l in range(nl)]
    if spmv_calls:
        # each level's own V-cycle passes per V-cycle (levels inside the fused
        # tail are timed on its first level)
        ncyc = sum(r["vcycles"] for r in res)
        roof["timed_region"]["vcycle_level_us"] = [
            round(1e3 * sum(r["ms_level"][l] for r in res) / max(ncyc, 1), 2) for l in range(nl)]
    out = {
        "metric": METRIC, "value": value, "unit": "constraint-DOF*iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_frame,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == B.PREC_FP64 else "f32 V-cycle / f64 PCG",
        "data": "synthetic",
        "config": {"workload": w.name, "rows": body.m, "nnz": body.nnz,
                   "iters_per_frame": n_iters, "precision": args.precision,
                   "fine_operator": ("matrix-free" if is_mf else "csr") +
                                    (" (timed choice)" if args.fine == "auto" else ""),
                   "smoother": args.smoother, "reuse_interval": args.reuse, "tol": 1e-6,
                   "lmax_scale": args.lmax_scale, "candidates": args.candidates,
                   "candidate": args.candidate,
                   "pcg_iters_per_solve": float(np.mean([r["pcg_iters"].mean() for r in res])),
                   "pcg_budget_per_solve": int(opt.max_pcg),
                   "solves_at_tol": int(sum((r["pcg_ratio"] <= 1e-6).sum() for r in res)),
                   "solves": int(sum(r["pcg_ratio"].size for r in res)),
                   "residual_reached": {
                       "median": float(np.median(np.concatenate([r["pcg_ratio"] for r in res]))),
                       "max": float(max(r["pcg_ratio"].max() for r in res))},
                   "ms_pcg_per_frame": 1e3 * pcg_s / args.steps,
                   "ms_setup_per_frame": sum(r["ms_setup"] for r in res) / args.steps,
                   "ms_galerkin_per_frame": sum(r["ms_galerkin"] for r in res) / args.steps,
                   "ms_assembly_per_frame": sum(r["ms_assembly"] for r in res) / args.steps,
                   "ms_update_per_frame": sum(r["ms_update"] for r in res) / args.steps,
                   "vcycle_tail": int(opt.vcycle_tail),
                   "fuse_transfers": int(opt.fuse_transfers),
                   "levels": [x["n"] for x in lv],
                   "operator_complexity": round(sum(x["nnz"] for x in lv) / lv[0]["nnz"], 4)},
        "roofline": roof,
    }
    if args.config in ("C2", "C4"):
        out["context"] = ("paper: 40.6 s/frame (20 iterations per frame) for its 1,667K-tet, "
                          "526K-vertex human muscle with ARAP rows (Fig. 1, Table 1, Sec. 5.4) on "
                          "an RTX 4090 with a Ryzen 9 7950X host (Sec. 5.2); another mesh, "
                          "constraint set and machine, not a target")
    body.close()
    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes_read"] = src.numel() * 8
        del src, dst
    if roof is not None:
        # what a plain device copy reaches on this GPU (1 GiB read + 1 GiB
        # written per copy, far beyond the 256 MB Infinity Cache)
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        roof["copy_GBps"] = round(2 * src.numel() * 8 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
        del src, dst
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        n_or = ORACLE_ITERS.get(args.config, 50)
        out["cpu_baseline"], x_ref = cpu_baseline(w, args.lmax_scale, n_or)
        print("cpu baseline took %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
        out["oracle_parity"] = oracle_parity(w, opt, n_or, x_ref)
        print("oracle parity: %s" % out["oracle_parity"], file=sys.stderr, flush=True)
        del x_ref
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
