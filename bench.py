#!/usr/bin/env python3
"""Benchmark of compressed patch-based relaxation on one MI355X.

Default workload (nedelec_hex): curl curl u + 1e-3 u on the unit cube,
lowest-order hexahedral edge elements on 64^3 cells (811,200 dofs, 262,144
twelve-dof cell patches), four seeded Voronoi materials with coefficients
{1, 10, 100, 1000}; b ~ N(0, 1).  Other workloads (--workload):
  stokes_batch      independent Taylor-Hood Stokes systems of seeded uneven
                    sizes (--nsys, meshes n x n with n in [16, 128]), solved
                    system by system in shared launches; FP32 apply of every
                    patch's inverse, autotuned launch shape;
  q2_hex_lognormal  Q2 diffusion on 32^3 hexes with a lognormal coefficient;
                    every patch differs, so Algorithm 1 runs at eps 0.55 (4.8 %
                    of the patches become entries); --mlp adds the learned
                    predictor, --kmeans uses spectral k-means with 5 % instead.

One step is the whole hot path on resident device data: setup (validation,
cover counts and W, patch extraction, the database, FP64 inverses, grouping,
conversion to the apply precision) followed by a right-preconditioned
GMRES(30) solve to relative residual 1e-8, capped at --iters outer
iterations.  The same step is timed for the full-patch FP64 path (every
patch factored, FP64 apply).

Printed: one JSON line.  value = n * (preconditioner applications) / (step
wall time), in GDoF/s, for the compressed path.  roofline: the patch apply
(one application = the patch kernel and, in deterministic mode, the slot
sum), algorithmic bytes per application over its average duration from HIP
events recorded on the solve's stream inside the timed steps (around the
kernels of every 7th Arnoldi step: an event adds a gap of a few
microseconds between kernels, so bracketing every step would slow the
step measured for value); traffic from
the committed hardware-counter summary when the apply's source is unchanged.
cpu_baseline: the oracle on a bounded sample of the same workload (one
thread), with the rate of its apply alone beside the whole-path rate.

Beside the headline line's throughput:
  converged / fixed_iterations: whether each path reached the tolerance; when
      either stops at the iteration cap, the speedups compare equal iteration
      counts, not equal accuracy;
  equal_tol: Q2 diffusion on 32^3 hexes with the lognormal coefficient, where
      both paths converge, with the two-level combination of Eq.(2) and
      without it: iterations to the tolerance, their ratio against the 1.10
      bar, setup + solve time of each path, and the final error
      ||x - x_o|| / ||x_o|| against the oracle's FP64 all-patch solution x_o
      (computed on the host, outside every timed region);
  apply_protocol: the preconditioner application alone, 5 warm-ups and 50
      repetitions, median, cold (a 512 MiB write between applications) and
      warm (a HIP graph of 100 back-to-back applications on distinct r, z);
  hbm_copy_probe: a 1 GiB device copy timed with events (read + write bytes);
  reuse: database reuse along a sequence of systems (Algorithm 1 seeded with
      the previous database, k-means warm-started from the previous
      assignment) against setups from scratch.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "patch-relax GDoF/s + setup s, compressed BF16 vs full FP64, equal-iter tol"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_TFLOPS = 78.6
TIMING_STRIDE = 7
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "apply_traffic_nedelec_hex_64.md")
APPLY_SRC = os.path.join(ROOT, "paper_2306_10025_amd", "csrc", "k_apply.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="nedelec_hex",
                    choices=["nedelec_hex", "stokes_batch", "q2_hex_lognormal", "stokes_2d", "q5_hex"])
    ap.add_argument("--size", type=int, default=None, help="cells per direction")
    ap.add_argument("--nsys", type=int, default=256, help="systems of the stokes_batch workload")
    ap.add_argument("--iters", type=int, default=300, help="GMRES iteration cap per step")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--eps", type=float, default=None,
                    help="Algorithm 1 tolerance (default 1e-8; 0.55 for q2_hex_lognormal, whose "
                         "patches all differ: 4.8 %% of them become entries)")
    ap.add_argument("--kmeans", action="store_true",
                    help="q2_hex_lognormal: spectral k-means with 5 %% of the patches instead of Algorithm 1")
    ap.add_argument("--precision", default=None, help="apply precision of the compressed path")
    ap.add_argument("--scatter", default="two-stage", choices=["atomic", "two-stage"],
                    help="FP64 atomics or the deterministic two-stage slot sum")
    ap.add_argument("--mlp", action="store_true", help="Algorithm 1 with the learned predictor")
    ap.add_argument("--graph", action="store_true", help="replay restart cycles from a HIP graph")
    ap.add_argument("--autotune", action="store_true", help="tune the apply launch shape (default: stokes_batch only)")
    ap.add_argument("--no-autotune", action="store_true", help="default apply launch shapes")
    ap.add_argument("--no-full", action="store_true", help="skip the full FP64 comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-size", type=int, default=12, help="cells per direction of the CPU sample")
    ap.add_argument("--no-equal-tol", action="store_true", help="skip the equal-tolerance block")
    ap.add_argument("--sweep", action="store_true",
                    help="print the compressibility curve instead of the headline line: Algorithm 1 "
                         "(first and closest matching) over a range of eps on nedelec_hex and q2_hex_lognormal")
    ap.add_argument("--twolevel", action="store_true",
                    help="q2_hex_lognormal: add the coarse term of Eq.(2) to both paths")
    ap.add_argument("--tol-size", type=int, default=32, help="cells per direction of the equal-tolerance workload")
    ap.add_argument("--tol-max-iters", type=int, default=3000)
    ap.add_argument("--oracle-tol", type=float, default=1e-10,
                    help="tolerance of the oracle's all-patch FP64 solve that the final error is measured against")
    ap.add_argument("--no-protocol", action="store_true", help="skip the cold/warm apply protocol")
    ap.add_argument("--orth", default="delayed", choices=["delayed", "selective"],
                    help="Gram-Schmidt form of GMRES: delayed reorthogonalisation (two passes per step) or "
                         "selective reorthogonalisation (three passes when the second projection runs)")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="after the steps, copy this many MiB on the device (hardware-counter calibration)")
    a = ap.parse_args()
    if a.twolevel and a.workload not in ("q2_hex_lognormal", "q5_hex"):
        ap.error("--twolevel needs --workload q2_hex_lognormal or q5_hex (meshes with a coarse interpolation)")
    if a.size is None:
        a.size = {"nedelec_hex": 64, "stokes_batch": 128, "q2_hex_lognormal": 32, "stokes_2d": 64,
                  "q5_hex": 20}[a.workload]
    if a.precision is None:
        a.precision = {"stokes_batch": "fp32", "q5_hex": "fp64"}.get(a.workload, "bf16x3")
    if a.eps is None:
        a.eps = {"q2_hex_lognormal": 0.55, "q5_hex": 1e-7}.get(a.workload, 1e-8)
    return a


def make_workload(args):
    import gen
    if args.workload == "nedelec_hex":
        P = gen.nedelec_hex(args.size)
        name = f"nedelec_hex_{args.size}"
    elif args.workload == "stokes_batch":
        P = gen.uneven_stokes_batch(n_sys=args.nsys, nmin=min(16, args.size), nmax=args.size)
        name = f"stokes_batch_{args.nsys}x[16..{args.size}]"
    elif args.workload == "stokes_2d":
        P = gen.taylor_hood_stokes_2d(args.size)
        name = f"taylor_hood_stokes_{args.size}x{args.size}"
    elif args.workload == "q5_hex":
        # Experiment 3: degree-5 hexahedra, k = 1, one 216-dof patch per cell
        P = gen.qp_hex_diffusion(args.size, 5)
        name = f"q5_hex_{args.size}"
    else:
        P = gen.q2_hex_diffusion(args.size)
        name = f"q2_hex_lognormal_{args.size}"
    return P, name


def path_params(args, P, compressed):
    """Setup parameters of the two paths."""
    det = args.scatter == "two-stage"
    # kernels of every 7th Arnoldi step are bracketed by events (7 and the
    # restart length 30 are coprime, so the sample covers every basis size)
    # the uneven batch tunes the apply's launch shape (both paths; the
    # library keeps the choice per process and shape, so the warm-up step
    # pays for the timing); on the uniform workloads the tuned shapes are
    # within timing noise of the default, which the counter runs also use
    tune = args.autotune or args.workload == "stokes_batch"
    common = dict(restart=30, max_iters=args.iters, deterministic=det, timing=0 if args.graph else TIMING_STRIDE,
                  graph=args.graph, autotune=tune and not args.no_autotune, orth=args.orth)
    if not compressed:
        return dict(algo="full", precision="fp64", **common)
    if args.workload == "stokes_batch":
        return dict(algo="full", precision=args.precision, **common)
    if args.workload == "q2_hex_lognormal" and args.kmeans:
        return dict(algo="kmeans_spectral", m_target=max(1, int(0.05 * P.n_p)), precision=args.precision,
                    **common)
    if args.workload == "q5_hex":
        # Experiment 3's database: Algorithm 1 with the l1 criterion
        return dict(algo="tolerance", criterion="l1", eps=args.eps, precision=args.precision, **common)
    return dict(algo="tolerance", criterion="spectral", eps=args.eps, precision=args.precision,
                mlp=args.mlp, **common)


def algorithmic_bytes(P, m_p, precision, n_items, n_p_entries, st=None):
    """Bytes one preconditioner application and one Krylov product must move
    at minimum (HBM model; each array read or written once).  The product
    reads every matrix value (8 B) and the index data of the stored form: 4 B
    per column offset of a diagonal-form slice, 4 B per entry of a
    column-form slice (CSR's 4 B per entry when the statistics are absent),
    the slice offsets, x and y."""
    import numpy as np
    n, n_p = P.n, P.n_p
    sum_ps = int(P.ptr[-1])
    ps = np.diff(P.ptr)
    x_bytes = {"fp64": 8, "fp32": 4, "bf16": 2, "fp16": 2, "bf16x3": 4}[precision]
    db = int(np.sum(ps ** 2)) * x_bytes if m_p >= n_p else int(np.max(ps)) ** 2 * m_p * x_bytes
    apply = (4 * sum_ps          # patch dof lists
             + 8 * n             # r
             + 8 * n             # W
             + 8 * n             # z (one write)
             + 4 * n_p           # entry of each patch
             + 16 * n_items      # work items (the item form only: fixed tiles read none)
             + db)               # database inverses
    if st is not None and (st.get("sell_slots", 0) > 0 or st.get("sell_csr_slices", 0) > 0):
        # diagonal-form offsets, column-form columns, and for slices read from
        # the CSR copy their columns and row pointers
        index = (4 * (st["sell_diag_offsets"] + st["sell_col_entries"] + st.get("sell_csr_entries", 0))
                 + 8 * 64 * st.get("sell_csr_slices", 0) + 8 * ((n + 63) // 64 + 1))
    else:
        index = 4 * P.A.nnz + 8 * (n + 1)
    spmv = 8 * P.A.nnz + index + 8 * n + 8 * n
    return apply, spmv


def orth_bytes(n, m=30, form="delayed"):
    """Average HBM bytes of the Gram-Schmidt work of one Arnoldi step over a
    GMRES(m) cycle (j = 0 .. m-1).  Delayed reorthogonalisation: the dot pass
    reads the j+1 vectors [Q, u] and w, the update pass reads the j vectors
    of Q, u and w and writes v_j and the next vector (2j + 6 vectors).
    Selective: three passes over the j+1 basis vectors (two reads, one read
    plus the update), reads and writes of w, the new basis vector."""
    j_avg = (m - 1) / 2.0
    if form == "delayed":
        return 8 * n * (2 * j_avg + 6)
    return 8 * n * (3 * (j_avg + 1) + 2 * 3 + 2)


def traffic_from_profile():
    """HBM bytes per application of the apply from the committed counter
    summary, or None when the apply's source changed since it was taken."""
    try:
        txt = open(TRAFFIC_FILE).read()
        m = re.search(r"```json\n(.*?)\n```", txt, flags=re.S)
        rec = json.loads(m.group(1))
        sha = hashlib.sha1(open(APPLY_SRC, "rb").read()).hexdigest()
        if rec.get("source_sha1") != sha:
            return None
        return int(rec["hbm_bytes_per_apply"])
    except Exception:
        return None


def run_gpu(args, P, b_np):
    import numpy as np
    import torch

    import paper_2306_10025_amd as pr

    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dtype=dt)
    row_ptr = t(P.A.indptr.astype(np.int64), torch.int64)
    col = t(P.A.indices.astype(np.int32), torch.int32)
    val = t(P.A.data, torch.float64)
    ptr = t(P.ptr.astype(np.int64), torch.int64)
    dofs = t(P.dofs.astype(np.int32), torch.int32)
    b = t(b_np, torch.float64)
    x = torch.zeros_like(b)
    stream = pr._stream()
    sptr = P.meta.get("system_ptr") if args.workload == "stokes_batch" else None

    p0 = None
    if args.twolevel:
        P0 = P.meta["P0"]
        p0 = (t(P0.indptr.astype(np.int64), torch.int64), t(P0.indices.astype(np.int32), torch.int32),
              t(P0.data, torch.float64), P.n, P0.shape[1])

    def step(params):
        h = pr.pr_setup(row_ptr, col, val, ptr, dofs, P.n, params)
        try:
            if sptr is not None:
                pr.pr_set_systems(h, sptr)
            if p0 is not None:
                pr.pr_set_coarse(h, *p0)
            pr.pr_solve(h, b, x, args.tol)
            return pr.pr_get_solve_info(h), pr.pr_get_stats(h)
        finally:
            pr.pr_destroy(h)

    def timed(params, label, steps, warmup):
        for i in range(warmup):
            info, st = step(params)
            log(f"[{label}] warmup {i}: setup {st['t_total']:.3f}s iters {info['iters']} "
                f"relres {info['relres']:.3e} m_p {st['m_p']}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rec = []
        for i in range(steps):
            ts = time.perf_counter()
            info, st = step(params)       # setup and solve synchronise; destroy waits for the stream
            info["wall_s"] = time.perf_counter() - ts
            rec.append((info, st))
            log(f"[{label}] step {i}: setup {st['t_total']:.3f}s solve {info['seconds']:.3f}s "
                f"iters {info['iters']} relres {info['relres']:.3e} reorth {info['reorth']}")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return (t1 - t0) / steps, rec

    comp = pr.make_params(stream=stream, **path_params(args, P, True))
    sec_c, rec_c = timed(comp, "compressed " + args.precision, args.steps, args.warmup)
    out = dict(sec=sec_c, rec=rec_c)
    if not args.no_full:
        full = pr.make_params(stream=stream, **path_params(args, P, False))
        sec_f, rec_f = timed(full, "full fp64", args.steps, args.warmup)
        out.update(sec_full=sec_f, rec_full=rec_f)
    if not args.no_protocol:
        out["protocol"] = {"compressed": apply_protocol(P, comp, row_ptr, col, val, ptr, dofs)}
        if not args.no_full:
            out["protocol"]["full_fp64"] = apply_protocol(P, full, row_ptr, col, val, ptr, dofs)
        out["copy_probe"] = copy_probe()
    if args.copy_calib > 0:
        # a plain device copy of known size, for scaling the HBM byte counters
        nb = args.copy_calib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {args.copy_calib} MiB")
    return out


def apply_protocol(P, params, row_ptr, col, val, ptr, dofs, reps=50, warm=5, chain=100):
    """The preconditioner application alone on one handle (median over
    `reps` after `warm` warm-ups).  cold: a 512 MiB device write between
    applications evicts the caches, and events bracket pr_apply alone.  warm:
    a HIP graph of `chain` back-to-back applications on distinct r and z
    (the in-solve pattern without the Krylov kernels in between), timed per
    replay and divided by `chain`."""
    import numpy as np
    import torch

    import paper_2306_10025_amd as pr

    n = P.n
    side = torch.cuda.Stream()
    h = pr.pr_setup(row_ptr, col, val, ptr, dofs, n, params)
    try:
        pr.pr_set_stream(h, side)
        gen_ = torch.Generator(device="cuda")
        gen_.manual_seed(0)
        r = torch.randn(n, dtype=torch.float64, device="cuda", generator=gen_)
        z = torch.empty_like(r)
        flush = torch.empty(64 << 20, dtype=torch.float64, device="cuda")   # 512 MiB
        cold = []
        with torch.cuda.stream(side):
            for k in range(warm + reps):
                flush.fill_(float(k))
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(side)
                pr.pr_apply(h, r, z)
                e1.record(side)
                e1.synchronize()
                if k >= warm:
                    cold.append(e0.elapsed_time(e1) * 1000.0)
        del flush
        R = torch.randn(chain, n, dtype=torch.float64, device="cuda", generator=gen_)
        Z = torch.empty_like(R)
        with torch.cuda.stream(side):
            for k in range(3):
                pr.pr_apply(h, R[k], Z[k])
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            for k in range(chain):
                pr.pr_apply(h, R[k], Z[k])
        warm_us = []
        for k in range(warm + reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            g.replay()
            e1.record()
            e1.synchronize()
            if k >= warm:
                warm_us.append(e0.elapsed_time(e1) * 1000.0 / chain)
        # the graph's last product against an eager application on the same input
        ref = torch.empty_like(r)
        with torch.cuda.stream(side):
            pr.pr_apply(h, R[chain - 1], ref)
        torch.cuda.synchronize()
        same = bool(torch.equal(ref, Z[chain - 1]))
        del g, R, Z
        st = pr.pr_get_stats(h)
    finally:
        pr.pr_destroy(h)
    return {"cold_median_us": round(float(np.median(cold)), 3), "cold_min_us": round(float(np.min(cold)), 3),
            "warm_median_us": round(float(np.median(warm_us)), 3), "reps": reps, "warmups": warm,
            "graph_chain": chain, "graph_matches_eager": same, "m_p": int(st["m_p"]),
            "n_items": int(st["n_items"]), "apply_tile_p": int(st["apply_tile_p"])}


def copy_probe(mib=1024, reps=10):
    """Device-to-device copy of `mib` MiB timed with events: the bandwidth
    a plain streaming kernel reaches (read + write bytes)."""
    import numpy as np
    import torch
    src = torch.ones((mib << 20) // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    us = []
    for k in range(reps + 2):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        if k >= 2:
            us.append(e0.elapsed_time(e1) * 1000.0)
    t = float(np.median(us))
    return {"bytes": 2 * (mib << 20), "median_us": round(t, 2),
            "gbs": round(2 * (mib << 20) / (t * 1e-6) / 1e9, 1), "kernel": "torch copy_ (float64)"}


def oracle_solution(P, b, tol):
    """The oracle's FP64 solution of A x = b: GMRES(30) to `tol` with every
    patch factored and the two-level combination of Eq.(2) (host)."""
    import numpy as np

    import oracle as O
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles_csr(P.A, P.ptr, P.dofs)
    X = O.batch_inverse(tiles)
    prec = O.combo_preconditioner(P.A, P.ptr, P.dofs, W, X, np.arange(P.n_p), P.meta["P0"])
    return O.gmres(lambda v: P.A @ v, prec, b, tol=tol, restart=30, max_iters=2000)


def equal_tol_block(args):
    """Both paths to the tolerance (flexible GMRES(30)) on Q2 diffusion, 32^3
    hexes, lognormal coefficient: compressed (Algorithm 1, eps 0.55, 4.8 % of the patches
    factored; BF16X3 and plain BF16 applies; first and closest matching)
    against the all-patch FP64 path, each with the two-level combination of
    Eq.(2) and, for context, without it.  Per path: iterations, their ratio
    to the full path of the same level, setup (pr_setup plus pr_set_coarse)
    and solve time, end-to-end wall time (median of the timed steps), and the
    final error against the oracle's FP64 solution, which is computed
    afterwards on the host."""
    import numpy as np
    import torch

    import gen
    import paper_2306_10025_amd as pr

    P = gen.q2_hex_diffusion(args.tol_size)
    b_np = gen.rhs(P.n)
    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dtype=dt)
    row_ptr = t(P.A.indptr.astype(np.int64), torch.int64)
    col = t(P.A.indices.astype(np.int32), torch.int32)
    val = t(P.A.data, torch.float64)
    ptr = t(P.ptr.astype(np.int64), torch.int64)
    dofs = t(P.dofs.astype(np.int32), torch.int32)
    P0 = P.meta["P0"]
    p0 = (t(P0.indptr.astype(np.int64), torch.int64), t(P0.indices.astype(np.int32), torch.int32),
          t(P0.data, torch.float64))
    b = t(b_np, torch.float64)
    stream = pr._stream()
    common = dict(restart=30, max_iters=args.tol_max_iters, deterministic=True, stream=stream, flexible=True)
    comp = dict(algo="tolerance", eps=0.55, **common)
    legs = {
        "full_fp64": (dict(algo="full", precision="fp64", **common), True),
        "compressed_bf16x3": (dict(precision="bf16x3", **comp), True),
        "compressed_bf16": (dict(precision="bf16", **comp), True),
        "compressed_bf16x3_closest": (dict(precision="bf16x3", alg1_match="closest", **comp), True),
        "full_fp64_one_level": (dict(algo="full", precision="fp64", **common), False),
        "compressed_bf16x3_one_level": (dict(precision="bf16x3", **comp), False),
    }
    out = {}
    xs = {}
    for name, (kw, two) in legs.items():
        params = pr.make_params(**kw)
        walls, setups, coarse, solves, last = [], [], [], [], None
        for i in range(args.warmup + args.steps):
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            h = pr.pr_setup(row_ptr, col, val, ptr, dofs, P.n, params)
            try:
                if two:
                    pr.pr_set_coarse(h, *p0, P.n, P0.shape[1])
                rc = pr.pr_solve(h, b, x, args.tol)
                info, st = pr.pr_get_solve_info(h), pr.pr_get_stats(h)
            finally:
                pr.pr_destroy(h)
            torch.cuda.synchronize()
            wall = time.perf_counter() - ts
            if i >= args.warmup:
                walls.append(wall)
                setups.append(st["t_total"])
                coarse.append(st["t_coarse"])
                solves.append(info["seconds"])
            last = (rc, info, st)
        rc, info, st = last
        xs[name] = x.cpu().numpy()
        out[name] = {"two_level": two, "iters": int(info["iters"]), "converged": rc == pr.PR_OK,
                     "relres": info["relres"], "m_p": int(st["m_p"]),
                     "setup_s": round(float(np.median(setups)), 5),
                     "coarse_setup_s": round(float(np.median(coarse)), 5),
                     "solve_s": round(float(np.median(solves)), 5),
                     "e2e_s": round(float(np.median(walls)), 5)}
        if two:
            out[name]["coarse"] = {"n0": int(st["n_coarse"]), "nnz": int(st["coarse_nnz"]),
                                   "bandwidth": int(st["coarse_bandwidth"]), "block": int(st["coarse_block"]),
                                   "blocks": int(st["coarse_blocks"])}
        log(f"[equal tol {name}] iters {info['iters']} relres {info['relres']:.3e} "
            f"setup {out[name]['setup_s']:.4f}s (+ coarse {out[name]['coarse_setup_s']:.4f}s) "
            f"solve {out[name]['solve_s']:.4f}s")
    t0 = time.perf_counter()
    log("equal tol: oracle FP64 solution on the host ...")
    x_o, oinfo = oracle_solution(P, b_np, args.oracle_tol)
    t_oracle = time.perf_counter() - t0
    nx = float(np.linalg.norm(x_o))
    for name in out:
        out[name]["rel_err_vs_oracle"] = float(np.linalg.norm(xs[name] - x_o) / nx)
    for name, rec in out.items():
        if name.startswith("full"):
            continue
        full = out["full_fp64" if rec["two_level"] else "full_fp64_one_level"]
        rec["iter_ratio"] = round(rec["iters"] / max(full["iters"], 1), 4)
        rec["meets_iter_bar_1.10"] = bool(rec["converged"] and full["converged"] and rec["iter_ratio"] <= 1.10)
        rec["e2e_speedup_vs_full"] = round(full["e2e_s"] / rec["e2e_s"], 4)
    return {"workload": f"q2_hex_lognormal_{args.tol_size}", "n": P.n, "n_p": P.n_p, "tol": args.tol,
            "database": "algorithm 1, spectral criterion, eps=0.55",
            "two_level": "Eq.(2): P0 linear interpolation from the interior mesh vertices, A0 = P0^T A P0 "
                         "solved directly (block LU over its band)",
            "paths": out,
            "krylov": "flexible GMRES(30), FP64",
            "oracle": {"solver": "all-patch FP64 GMRES(30) with the two-level combination, MGS",
                       "tol": args.oracle_tol, "iters": int(oinfo["iters"]), "relres": oinfo["relres"],
                       "seconds": round(t_oracle, 2)}}


def reuse_block(args):
    """Database reuse along a sequence of linear systems (the closing remarks
    of the third numerical experiment; Section 3.2 on problem sequences): the
    lognormal coefficient of Q2 32^3 drifts by a seeded factor exp(0.05 g)
    from system 0 to system 1.  Algorithm 1 (eps 0.55) on system 1 from
    scratch against pr_setup_reuse with system 0's database; spectral k-means
    (5 % of the patches) on the 16^3 problem cold against warm-started.
    Setup time is the median of three setups; iterations are those of the
    compressed BF16X3 apply with the two-level combination (flexible
    GMRES(30), tolerance 1e-8)."""
    import numpy as np
    import torch

    import gen
    import paper_2306_10025_amd as pr

    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dtype=dt)
    stream = pr._stream()

    def system(nc, step):
        P = gen.q2_hex_diffusion(nc)
        if step == 0:
            return P
        k = P.meta["k"] * np.exp(0.05 * np.random.default_rng(11).standard_normal(nc ** 3))
        return gen.q2_hex_diffusion(nc, kfield=k)

    def arrays(P):
        P0 = P.meta["P0"]
        return (t(P.A.indptr.astype(np.int64), torch.int64), t(P.A.indices.astype(np.int32), torch.int32),
                t(P.A.data, torch.float64), t(P.ptr.astype(np.int64), torch.int64),
                t(P.dofs.astype(np.int32), torch.int32),
                (t(P0.indptr.astype(np.int64), torch.int64), t(P0.indices.astype(np.int32), torch.int32),
                 t(P0.data, torch.float64), P.n, P0.shape[1]), t(gen.rhs(P.n), torch.float64))

    def setup(P, arr, kw, blob=None, solve=False):
        rp, ci, va, pt, dd, p0, b = arr
        params = pr.make_params(restart=30, max_iters=2000, deterministic=True, stream=stream, flexible=True,
                                precision="bf16x3", **kw)
        times, st, info = [], None, None
        for rep in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = (pr.pr_setup(rp, ci, va, pt, dd, P.n, params) if blob is None
                 else pr.pr_setup_reuse(rp, ci, va, pt, dd, P.n, params, blob))
            times.append(time.perf_counter() - t0)
            try:
                st = pr.pr_get_stats(h)
                out_blob = pr.pr_export_database(h)
                if solve and rep == 0:
                    pr.pr_set_coarse(h, *p0)
                    x = torch.zeros_like(b)
                    pr.pr_solve(h, b, x, args.tol)
                    info = pr.pr_get_solve_info(h)
            finally:
                pr.pr_destroy(h)
        rec = {"setup_s": round(float(np.median(times)), 5), "m_p": int(st["m_p"]),
               "crit_evals": int(st["crit_evals"])}
        if info is not None:
            rec["iters"] = int(info["iters"])
        return rec, st, out_blob

    out = {}
    S0, S1 = system(32, 0), system(32, 1)
    A0, A1 = arrays(S0), arrays(S1)
    kw = dict(algo="tolerance", eps=0.55)
    _, _, blob = setup(S0, A0, kw)
    fresh, _, _ = setup(S1, A1, kw, solve=True)
    reuse, st, _ = setup(S1, A1, kw, blob=blob, solve=True)
    reuse.update(kept=int(st["reuse_kept"]), rescanned=int(st["reuse_rescanned"]),
                 appended=int(st["reuse_appended"]))
    out["algorithm_1_q2_hex_lognormal_32"] = {"fresh": fresh, "reuse": reuse,
                                              "setup_speedup": round(fresh["setup_s"] / reuse["setup_s"], 3)}
    log(f"[reuse] Algorithm 1: fresh {fresh} reuse {reuse}")
    K0, K1 = system(16, 0), system(16, 1)
    B0, B1 = arrays(K0), arrays(K1)
    kw = dict(algo="kmeans_spectral", m_target=int(0.05 * K0.n_p))
    _, _, kblob = setup(K0, B0, kw)
    cold, cst, _ = setup(K1, B1, kw, solve=True)
    warm, wst, _ = setup(K1, B1, kw, blob=kblob, solve=True)
    cold["passes"] = int(cst["kmeans_iters"])
    warm["passes"] = int(wst["kmeans_iters"])
    out["kmeans_spectral_q2_hex_lognormal_16"] = {"cold": cold, "warm": warm,
                                                  "setup_speedup": round(cold["setup_s"] / warm["setup_s"], 3)}
    log(f"[reuse] k-means: cold {cold} warm {warm}")
    out["sequence"] = "system 1 = system 0 with the coefficient times exp(0.05 g), g ~ N(0, 1) per cell (seed 11)"
    return out


def launches_per_solve(info):
    """Launches of each class in one solve: an apply and an SpMV per Arnoldi
    step and per restart cycle end, one orthogonalisation per step."""
    return {"apply": info["iters"] + info["cycles"], "spmv": info["iters"] + info["cycles"],
            "orth": info["iters"]}


def items_read(st):
    """Work items the apply reads: none when it runs over fixed tiles."""
    return 0 if int(st.get("apply_tile_p", 0)) > 0 else int(st["n_items"])


def summarize_classes(P, rec, precision, m_p, n_items, orth="delayed"):
    """Average duration of one launch of each kernel class, from the events
    recorded inside the timed steps (a sample of the Arnoldi steps), and the
    device time per step it implies."""
    apply_b, spmv_b = algorithmic_bytes(P, m_p, precision, n_items, m_p, rec[0][1] if rec else None)
    tot = {"apply": [0.0, 0, 0], "spmv": [0.0, 0, 0], "orth": [0.0, 0, 0]}
    for info, st in rec:
        lps = launches_per_solve(info)
        for k in tot:
            tot[k][0] += info[k + "_ms"]
            tot[k][1] += info["n_" + k]
            tot[k][2] += lps[k]
    res = {}
    for k, (ms, cnt, launches) in tot.items():
        avg_us = 1000.0 * ms / max(cnt, 1)
        steps = max(len(rec), 1)
        res[k] = dict(total_ms=avg_us * launches / steps / 1000.0, launches=launches / steps,
                      timed_launches=cnt / steps, avg_us=avg_us)
    res["apply"]["bytes"] = apply_b
    res["spmv"]["bytes"] = spmv_b
    res["orth"]["bytes"] = orth_bytes(P.n, form=orth)
    return res


def apply_flops(P, m_p):
    """Useful flops of one patch apply: 2 p^2 per patch."""
    import numpy as np
    return 2 * int(np.sum(np.diff(P.ptr) ** 2))


def roofline_mfma(name, flops, avg_us, bytes_per_launch):
    """Roofline of a kernel bound by the FP64 matrix cores (78.6 TFLOP/s)."""
    achieved = flops / (avg_us * 1e-6) / 1e12 if avg_us > 0 else 0.0
    return {"kernel": name, "bound": "mfma", "achieved": round(achieved, 2), "peak": FP64_MFMA_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / FP64_MFMA_TFLOPS, 4), "traffic": None,
            "flops_per_launch": int(flops), "bytes_per_launch": int(bytes_per_launch),
            "hbm_frac": round(bytes_per_launch / (avg_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4) if avg_us > 0 else 0.0,
            "avg_us": round(avg_us, 3)}


def roofline(name, bytes_per_launch, avg_us, traffic=None):
    achieved = bytes_per_launch / (avg_us * 1e-6) / 1e9 if avg_us > 0 else 0.0
    return {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "bytes_per_launch": int(bytes_per_launch), "avg_us": round(avg_us, 3)}


def cpu_baseline(args):
    """The oracle (unchanged) on a bounded sample of the same workload: cover
    counts, tiles, Algorithm 1 and FP64 GMRES(30) capped at 60 iterations;
    rate = n * applies / wall time."""
    import gen
    import oracle as O
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        return _cpu_baseline(args, gen, O)


def _cpu_baseline(args, gen, O):
    import numpy as np
    if args.workload == "nedelec_hex":
        P = gen.nedelec_hex(args.cpu_size)
        name, eps = f"nedelec_hex_{args.cpu_size}", args.eps
    elif args.workload == "stokes_batch":
        P = gen.uneven_stokes_batch(n_sys=4, nmin=8, nmax=24)
        name, eps = "stokes_batch_4x[8..24]", 1e-8
    elif args.workload == "stokes_2d":
        P = gen.taylor_hood_stokes_2d(16)
        name, eps = "taylor_hood_stokes_16x16", 1e-8
    elif args.workload == "q5_hex":
        P = gen.qp_hex_diffusion(10, 5)
        name, eps = "q5_hex_10", args.eps
    else:
        P = gen.q2_hex_diffusion(8)
        name, eps = "q2_hex_lognormal_8", 0.99
    crit = "l1" if args.workload == "q5_hex" else "spectral"
    b = gen.rhs(P.n)
    t0 = time.perf_counter()
    cnt, W = O.cover_weights(P.n, P.ptr, P.dofs)
    tiles = O.patch_tiles(P.A, P.ptr, P.dofs)
    res = O.alg1_tolerance(tiles, eps, crit)
    t_setup = time.perf_counter() - t0
    napply = [0]
    t_apply = [0.0]
    base = O.make_preconditioner(P.A, P.ptr, P.dofs, W, res["X"], res["phi"])

    def prec(v):
        napply[0] += 1
        ta = time.perf_counter()
        out = base(v)
        t_apply[0] += time.perf_counter() - ta
        return out
    x, info = O.gmres(lambda v: P.A @ v, prec, b, tol=args.tol, restart=30, max_iters=60)
    t_all = time.perf_counter() - t0
    rate = P.n * napply[0] / t_all / 1e9
    return {"value": rate, "unit": "GDoF/s", "cores": 1, "kind": "oracle",
            "apply_only_value": P.n * napply[0] / t_apply[0] / 1e9,
            "sample": (f"{name} (n={P.n}, n_p={P.n_p}, m_p={len(res['reps'])}): "
                       f"oracle setup (Algorithm 1, {crit}, eps={eps}) {t_setup:.2f}s + GMRES(30) {info['iters']} "
                       f"iters, {napply[0]} FP64 applies ({t_apply[0]:.3f}s of apply alone), {t_all:.2f}s "
                       f"wall; one thread (BLAS pool limited to 1; host cpu_count {os.cpu_count()})")}


SWEEP_EPS = {
    "nedelec_hex_64": [1e-8, 1e-6, 1e-4, 1e-3, 1e-2, 0.05, 0.1, 0.3],
    "q2_hex_lognormal_32": [0.05, 0.1, 0.15, 0.2, 0.3, 0.4, 0.55, 0.7],
}


def sweep(args):
    """Compressibility curve (the fourth numerical experiment's measure,
    (n_p - m_p) / n_p, against eps) of Algorithm 1 with first and closest
    matching, with the iterations each database costs: on Nedelec 64^3 at a
    300-iteration cap (the one-level method does not reach 1e-8 there, so
    the relative residual at the cap is reported), and on Q2 32^3 to 1e-8
    without and with the two-level combination of Eq.(2), each ratio taken
    against the all-patch path of the same level.  One JSON line."""
    import numpy as np
    import torch

    import gen
    import paper_2306_10025_amd as pr

    dev = torch.device("cuda:0")
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dtype=dt)
    stream = pr._stream()
    curves = {}
    for wname, make, levels in (("nedelec_hex_64", lambda: gen.nedelec_hex(64), (False,)),
                                ("q2_hex_lognormal_32", lambda: gen.q2_hex_diffusion(32), (False, True))):
        P = make()
        log(f"sweep {wname}: n={P.n} n_p={P.n_p}")
        row_ptr = t(P.A.indptr.astype(np.int64), torch.int64)
        col = t(P.A.indices.astype(np.int32), torch.int32)
        val = t(P.A.data, torch.float64)
        ptr = t(P.ptr.astype(np.int64), torch.int64)
        dofs = t(P.dofs.astype(np.int32), torch.int32)
        b = t(gen.rhs(P.n), torch.float64)
        p0 = None
        if "P0" in P.meta:
            P0 = P.meta["P0"]
            p0 = (t(P0.indptr.astype(np.int64), torch.int64), t(P0.indices.astype(np.int32), torch.int32),
                  t(P0.data, torch.float64), P.n, P0.shape[1])
        cap = 300 if wname.startswith("nedelec") else 3000

        def run(two, **kw):
            params = pr.make_params(restart=30, max_iters=cap, deterministic=True, stream=stream,
                                    flexible=True, **kw)
            x = torch.zeros_like(b)
            h = pr.pr_setup(row_ptr, col, val, ptr, dofs, P.n, params)
            try:
                if two:
                    pr.pr_set_coarse(h, *p0)
                rc = pr.pr_solve(h, b, x, args.tol)
                info, st = pr.pr_get_solve_info(h), pr.pr_get_stats(h)
            finally:
                pr.pr_destroy(h)
            return {"m_p": int(st["m_p"]), "iters": int(info["iters"]), "relres": info["relres"],
                    "converged": rc == pr.PR_OK, "setup_s": round(st["t_total"], 5),
                    "solve_s": round(info["seconds"], 5)}

        rec = {"n_p": P.n_p, "tol": args.tol, "max_iters": cap, "levels": {}}
        for two in levels:
            lev = "two_level" if two else "one_level"
            full = run(two, algo="full", precision="fp64")
            pts = []
            for eps in SWEEP_EPS[wname]:
                for match in ("first", "closest"):
                    r = run(two, algo="tolerance", eps=eps, precision=args.precision, alg1_match=match)
                    r.update(eps=eps, match=match,
                             compression=round((P.n_p - r["m_p"]) / P.n_p, 5),
                             iter_ratio=round(r["iters"] / max(full["iters"], 1), 4))
                    r["meets_iter_bar_1.10"] = bool(r["converged"] and full["converged"] and r["iter_ratio"] <= 1.10)
                    log(f"  {lev} eps {eps:g} {match}: m_p {r['m_p']} ({100 * r['m_p'] / P.n_p:.2f} %) "
                        f"iters {r['iters']} (full {full['iters']}) relres {r['relres']:.2e}")
                    pts.append(r)
            ok = [p for p in pts if p["meets_iter_bar_1.10"]]
            best = min(ok, key=lambda p: p["m_p"]) if ok else None
            rec["levels"][lev] = {"full_fp64": full, "points": pts,
                                  "smallest_database_meeting_1.10": (
                                      {k: best[k] for k in ("eps", "match", "m_p", "compression", "iters")}
                                      if best else None)}
        curves[wname] = rec
    print(json.dumps({"metric": "compressibility curve (n_p - m_p)/n_p and iteration ratio vs eps",
                      "apply_precision": args.precision, "criterion": "spectral", "data": "synthetic",
                      "curves": curves}), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU design is described but not built.", file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        sweep(args)
        return
    import numpy as np

    import gen
    t0 = time.perf_counter()
    P, wname = make_workload(args)
    b = gen.rhs(P.n)
    log(f"workload {wname}: n={P.n} nnz={P.A.nnz} n_p={P.n_p} "
        f"(generated in {time.perf_counter() - t0:.1f}s)")
    g = run_gpu(args, P, b)
    info, st = g["rec"][-1]
    m_p, n_items = st["m_p"], items_read(st)
    applies = np.mean([launches_per_solve(i)["apply"] for i, _ in g["rec"]])
    value = P.n * applies / g["sec"] / 1e9
    cls = summarize_classes(P, g["rec"], args.precision, m_p, n_items, args.orth)
    dom = max(("apply", "spmv", "orth"), key=lambda k: cls[k]["total_ms"])
    traffic = traffic_from_profile() if (wname == "nedelec_hex_64" and args.precision == "bf16x3"
                                         and args.scatter == "two-stage") else None
    kname = "patch apply (" + args.precision + ("" if args.scatter == "atomic" else ", two-stage") + ")"
    rl_apply = roofline(kname, cls["apply"]["bytes"], cls["apply"]["avg_us"], traffic)
    if args.workload == "q5_hex":
        # 216-dof patches stacked 16 per entry: 2 p^2 flops per patch against
        # 8 B of residual and slot per dof; the FP64 matrix cores bound it
        rl_apply = roofline_mfma("patch apply (fp64 matrix cores, grouped, two-stage)",
                                 apply_flops(P, m_p), cls["apply"]["avg_us"], cls["apply"]["bytes"])
    rl_spmv = roofline("hybrid sliced-ELL spmv (fp64)", cls["spmv"]["bytes"], cls["spmv"]["avg_us"])
    rl_orth = roofline("gram-schmidt per arnoldi step (fp64)", cls["orth"]["bytes"], cls["orth"]["avg_us"])
    database = {"tolerance": f"algorithm 1, spectral criterion, eps={args.eps}" + (" with the learned predictor" if args.mlp else ""),
                "kmeans_spectral": "algorithm 2 spectral k-means, m_p = 5 % of n_p",
                "tolerance_l1": f"algorithm 1, l1 criterion, eps={args.eps}",
                "full": "every patch (FP32 inverses)"}[path_params(args, P, True)["algo"]
                                                        + ("_l1" if args.workload == "q5_hex" else "")]
    if args.workload == "stokes_2d":
        database = f"algorithm 1, spectral criterion, eps={args.eps}"
    if args.twolevel:
        database += "; two-level combination of Eq.(2) (direct coarse solve)"
    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(g["sec"] * 1000.0, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {
            "workload": wname,
            "n": P.n, "nnz": int(P.A.nnz), "n_p": P.n_p, "p_s": int(np.max(np.diff(P.ptr))), "m_p": m_p,
            "database": database,
            "apply_precision": args.precision, "setup_precision": "f64",
            "krylov": "f64 GMRES(30), " + ("delayed" if args.orth == "delayed" else "selective") + " reorthogonalisation",
            "scatter": args.scatter, "graph": args.graph,
            "krylov_matrix": (f"hybrid sliced ELL, {st['sell_diag_slices']} of {(P.n + 63) // 64} slices "
                              f"in diagonal form, {st.get('sell_csr_slices', 0)} read from the CSR copy, "
                              f"{st['sell_slots']} stored values"),
            "tol": args.tol, "max_iters": args.iters, "parallelism": "single GPU",
        },
        "setup_s": round(float(np.mean([s["t_total"] + s["t_coarse"] for _, s in g["rec"]])), 4),
        "solve_s": round(float(np.mean([i["seconds"] for i, _ in g["rec"]])), 4),
        "median_ms_per_step": round(1000.0 * float(np.median([i["wall_s"] for i, _ in g["rec"]])), 3),
        "iters": int(info["iters"]),
        "converged": bool(info["relres"] <= args.tol),
        "reorth_steps": int(info["reorth"]),
        "relres": info["relres"],
        "applies_per_step": float(applies),
        "setup_detail": {k: (round(st[k], 5) if isinstance(st[k], float) else int(st[k]))
                         for k in ("t_validate", "t_extract", "t_database", "t_factor", "t_group",
                                   "t_autotune", "t_mlp_train", "crit_evals", "crit_pruned",
                                   "crit_refined", "crit_exact", "mlp_accepted", "mlp_fallback",
                                   "alg1_rounds", "alg1_batch_inverted")},
        "apply_gdofs": round(P.n / (cls["apply"]["avg_us"] * 1e-6) / 1e9, 3) if cls["apply"]["avg_us"] else None,
        "kernel_ms_per_step": {k: round(cls[k]["total_ms"], 3) for k in ("apply", "spmv", "orth")},
        "dominant_by_time": dom,
        "roofline": rl_apply,
        "roofline_spmv": rl_spmv,
        "roofline_orth": rl_orth,
    }
    if st.get("tune_threads"):
        line["config"]["apply_shape"] = {"threads": st["tune_threads"], "block_cap": st["tune_cap"],
                                         "slot_threads": st["tune_slot"],
                                         "tiles_per_wave": st["tune_tiles_per_wave"],
                                         "xcd_remap": st["tune_xcd_remap"]}
    if "rec_full" in g:
        fi, fs = g["rec_full"][-1]
        fcls = summarize_classes(P, g["rec_full"], "fp64", P.n_p, items_read(fs), args.orth)
        f_applies = np.mean([launches_per_solve(i)["apply"] for i, _ in g["rec_full"]])
        line["full_fp64"] = {
            "ms_per_step": round(g["sec_full"] * 1000.0, 3),
            "gdofs": round(P.n * f_applies / g["sec_full"] / 1e9, 4),
            "setup_s": round(float(np.mean([s["t_total"] + s["t_coarse"] for _, s in g["rec_full"]])), 4),
            "solve_s": round(float(np.mean([i["seconds"] for i, _ in g["rec_full"]])), 4),
            "median_ms_per_step": round(1000.0 * float(np.median([i["wall_s"] for i, _ in g["rec_full"]])), 3),
            "iters": int(fi["iters"]), "relres": fi["relres"], "converged": bool(fi["relres"] <= args.tol),
            "kernel_ms_per_step": {k: round(fcls[k]["total_ms"], 3) for k in ("apply", "spmv", "orth")},
            "roofline_apply": roofline("patch apply (fp64, all patches)", fcls["apply"]["bytes"],
                                       fcls["apply"]["avg_us"]),
        }
        line["e2e_speedup_vs_full"] = round(g["sec_full"] / g["sec"], 3)
        fixed = not (line["converged"] and line["full_fp64"]["converged"])
        line["fixed_iterations"] = fixed
        if fixed:
            line["note"] = (f"not converged at the {args.iters}-iteration cap (relres {info['relres']:.4g} "
                            f"compressed, {fi['relres']:.4g} full): value and the speedups compare equal "
                            "iteration counts, not equal accuracy; equal_tol compares at the tolerance")
        line["setup_speedup_vs_full"] = round(line["full_fp64"]["setup_s"] / max(line["setup_s"], 1e-9), 3)
        if cls["apply"]["avg_us"] and fcls["apply"]["avg_us"]:
            line["apply_speedup_vs_full"] = round(fcls["apply"]["avg_us"] / cls["apply"]["avg_us"], 3)
    if "protocol" in g:
        proto = {}
        for path, rec in g["protocol"].items():
            prec = args.precision if path == "compressed" else "fp64"
            mp = rec["m_p"] if path == "compressed" else P.n_p
            bpl, _ = algorithmic_bytes(P, mp, prec, items_read(rec), mp, st)
            rec = dict(rec, bytes_per_launch=int(bpl))
            for k in ("cold", "warm"):
                us = rec[f"{k}_median_us"]
                rec[f"{k}_frac"] = round(bpl / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
            proto[path] = rec
        line["apply_protocol"] = proto
        line["hbm_copy_probe"] = g["copy_probe"]
    if not args.no_equal_tol and args.workload == "nedelec_hex":
        log("equal-tolerance block (q2 hex lognormal) ...")
        line["equal_tol"] = equal_tol_block(args)
        log("reuse block (sequence of q2 hex lognormal systems) ...")
        line["reuse"] = reuse_block(args)
    if not args.no_cpu:
        log("cpu baseline (oracle on a bounded sample) ...")
        line["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
