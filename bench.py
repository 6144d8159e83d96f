"""Benchmark of the vertex-patch smoother on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one forward multiplicative sweep (all 2^d colours; per patch:
gather, evaluate, one local p-multigrid V-cycle, FP64 scatter-add) over the
3D 16^3 Q4 mesh perturbed by 0.2 h (3,375 patches, local levels 4 -> 2 -> 1,
Chebyshev degree 3) with inputs resident in HBM.  The headline value is the
smoother throughput in DoF/s (interior DoFs of the mesh x sweeps / time) of
the FP32 local solver whose Chebyshev intervals come from the learned bound
network (trained first, on the GPU, on Lanczos labels of random patches of
the same distribution); the plain FP64 local solver with per-patch Lanczos
bounds is timed beside it.  The comparison holds only if the outer GMG-CG
iteration count of the FP32+learned solver stays within one of the FP64
one; both counts are reported.  One JSON line is printed; the default run
adds the same record for the 32^3 Q7 jump workload (the matrix cores on the
hot path) under "secondary".  Each record carries the roofline of the FP32
smoothing kernel (against the 157.3 TFLOP/s FP32 peak, with the fraction of
what unpacked vector instructions can issue beside it) and the oracle's
sweep timed on the host, on all usable cores (up to 16 worker processes)
and on one, in processes forked before the GPU is used.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Peak figures of MI355X used for the roofline fraction.
HBM_PEAK_GBS = 8000.0
# FP32: 157.3 TFLOP/s on the vector ALUs (256 CUs x 4 SIMDs x 16 lanes x 2
# FP32 per lane with packed instructions x 2 flop x 2.4 GHz) and on the
# matrix cores alike; FP64: 78.6 TFLOP/s (no packed form).
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
# What the FP32 kernels here can issue on the vector ALUs: packed FP32 is
# disabled in them, so one FP32 FMA per lane and cycle (78.6 TFLOP/s).
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Dense FP32 matrix-core peak (v_mfma_f32_16x16x4_f32).
MFMA_FP32_PEAK_TFLOPS = 157.3


def mfma_flops_per_patch(dim, levels, k):
    """Algorithmic flops of one patch update that the FP32 kernels run on the
    matrix cores: the top level's 1D interpolation contractions when the top
    degree is 6 or 7 in 3D (slab-form top level).  Of the 2^d 8 d n^{d+1}
    contraction flops of f(q), half are interpolations (d forward, d
    transposed) and half collocation derivatives, which stay on the vector
    ALUs; counted 1 + 2k times.  Everything else is vector ALU."""
    if dim != 3 or levels[0] not in (6, 7):
        return 0
    n = levels[0] + 1
    return 2 ** dim * 4 * dim * n ** (dim + 1) * (1 + 2 * k)


def mixed_peak(share):
    """Peak of a kernel whose flops run a fraction `share` on the FP32 matrix
    cores and the rest on the vector ALUs, each at its own peak: the time
    the ideal kernel needs, inverted."""
    return 1.0 / (share / MFMA_FP32_PEAK_TFLOPS + (1.0 - share) / VALU_PEAK_TFLOPS)


def algorithmic_per_patch(dim, levels, k, tsize):
    """Algorithmic flops and HBM bytes of one interior patch update
    (N_MG = 1): sum-factorised applies f(q) = 2^d [8 d n^{d+1} + 2 d^2 n^d]
    (n = q+1) counted (1 + 2k) times at the top level and 2k times on the other
    smoothed levels, d 1D contractions per transfer each way, 6 vector flops
    per entry per Chebyshev step; bytes: FP64 gather of the closure and of the
    interior right-hand side, FP64 read+write of the interior on scatter,
    3^d vertices, 2^d coefficients and the stored inverse diagonals."""
    def f(q):
        n = q + 1
        return 2 ** dim * (8 * dim * n ** (dim + 1) + 2 * dim * dim * n ** dim)
    p = levels[0]
    F = f(p) * (1 + 2 * k)
    for q in levels[1:-1]:
        F += 2 * k * f(q)
    for qf, qc in zip(levels[:-1], levels[1:]):
        mf, mc = 2 * qf - 1, 2 * qc - 1
        if dim == 3:
            F += 2 * 2 * (mf * mf * mc * mf + mf * mc * mc * mf + mc ** 3 * mf)
        else:
            F += 2 * 2 * (mf * mc * mf + mc * mc * mf)
    for q in levels[:-1]:
        F += 6 * (2 * q - 1) ** dim * 2 * k
    B = 8 * ((2 * p + 1) ** dim + 3 * (2 * p - 1) ** dim) + 8 * dim * 3 ** dim + 8 * 2 ** dim
    B += tsize * sum((2 * q - 1) ** dim for q in levels[:-1])
    return F, B


def kernel_source_digest():
    """sha256 prefix of the patch-kernel sources: patch_kernels.hpp, then
    patch_kernels.hip and the patch_variants_*.hip files in name order."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2510_17785_amd", "csrc")
    names = ["patch_kernels.hpp"] + sorted(f for f in os.listdir(csrc)
                                           if f.startswith("patch_") and f.endswith(".hip"))
    h = hashlib.sha256()
    for f in names:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel="patch_kernel_fp32"):
    """HBM bytes per launch of the patch kernel from the committed rocprofv3
    counter summary profiles/<kernel>_<workload>.md, or None when the kernel
    source has changed since the counters were taken."""
    prof = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md")
    if not os.path.exists(prof):
        return None
    text = open(prof).read()
    if f"`{kernel_source_digest()}`" not in text:
        return None
    for line in text.splitlines():
        if line.startswith("TRAFFIC_BYTES_PER_LAUNCH"):
            return float(line.split("=")[1])
    return None


def has_bf16(w):
    """The BF16-input variants exist for 3D top degrees 6 and 7."""
    return w.dim == 3 and w.levels[0] in (6, 7)


def time_sweeps(S, u, b, steps, warmup, torch):
    """`steps` forward sweeps timed with two events on the stream the kernels
    run on, around all of them (an event between the colour launches would
    add a gap of its own to every launch).  Per launch: the sweep time over
    the colour count, which includes the short gaps between the dependent
    launches (so it bounds the kernel's own duration from above)."""
    for _ in range(warmup):
        S.smooth(u, b, +1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        S.smooth(u, b, +1)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sweep_ms = e0.elapsed_time(e1) / steps
    nc = S.n_colors
    per_launch = [sweep_ms / nc] * (steps * nc)
    return sweep_ms, per_launch, wall


def host_info():
    """Host cores this process may use and the CPU model."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return cores, model


def _oracle_sweep_worker(job):
    """One worker of the multi-core oracle baseline: the oracle's sweep over a
    set of patches of one colour (independent updates), repeated for the
    budget; returns (patch updates, seconds).  Setup untimed."""
    dim, n, p, levels, X, mu, b, verts, budget_s = job
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import fem
    from oracle.smoother import PatchSmoother
    with threadpool_limits(limits=1):
        S = PatchSmoother(fem.Mesh(dim, n, X, mu), p, levels, keep_closure=True, vertices=verts)
        u = np.zeros_like(b)

        def updates():
            # the oracle sweep's steps per patch (local residual, V-cycle,
            # scatter) on one vector: the sweep's copy of the whole vector is
            # paid once per sweep, not once per sampled patch
            for v in S.order:
                u[S.idx[v][1]] += S.solvers[v].solve(S.local_residual(v, u, b))

        updates()
        reps, t0 = 0, time.perf_counter()
        while True:
            updates()
            reps += 1
            if time.perf_counter() - t0 >= budget_s:
                break
        return reps * len(verts), time.perf_counter() - t0


def cpu_baseline(w, X, mu, b, budget_s=8.0, max_workers=16):
    """The oracle's sweep (FP64 dense level matrices, setup untimed) timed on
    the host: on all usable cores (a process pool, each worker updating its
    own patches of one colour, which are independent) and on one core; the
    rate of patch updates is extrapolated to a full sweep.  Runs in worker
    processes forked before the GPU is touched."""
    import multiprocessing as mp

    import numpy as np

    from oracle.smoother import patch_order, vertex_color

    cores, model = host_info()
    workers = max(1, min(cores, max_workers))
    order = patch_order(w.dim, w.n)
    colour0 = [v for v in order if vertex_color(v) == 0]
    rng = np.random.default_rng(0)
    per = 12 if w.p <= 4 else 2         # the oracle assembles dense patch matrices
    pick = [colour0[i] for i in rng.choice(len(colour0), min(len(colour0), per * workers), replace=False)]
    chunks = [pick[k::workers] for k in range(workers)]
    jobs = [(w.dim, w.n, w.p, w.levels, X, mu, b, c, budget_s) for c in chunks if c]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(len(jobs)) as pool:
        res = pool.map(_oracle_sweep_worker, jobs)
    wall = time.perf_counter() - t0
    rate_all = sum(r[0] / r[1] for r in res)          # concurrent workers: rates add
    one = _oracle_sweep_worker((w.dim, w.n, w.p, w.levels, X, mu, b, pick[:per], budget_s))
    rate_one = one[0] / one[1]
    n_patch = len(order)
    return {
        "value": w.n_interior_dofs * rate_all / n_patch,
        "unit": "DoF/s",
        "cores": len(jobs),
        "kind": "oracle",
        "sample": f"{len(pick)} patches of colour 0 of the same mesh in {len(jobs)} worker processes "
                  f"(one core each), {sum(r[0] for r in res)} patch updates in {budget_s:.0f} s "
                  f"each ({wall:.1f} s with setup); extrapolated to all {n_patch} patches of a sweep",
        "one_core": {"value": w.n_interior_dofs * rate_one / n_patch, "unit": "DoF/s", "cores": 1,
                     "sample": f"{per} patches, {one[0]} patch updates in {one[1]:.1f} s"},
        "host": {"nproc": os.cpu_count(), "usable_cores": cores, "cpu_model": model},
    }


def bench_batch(args, w):
    """The mixed-degree batch: four independent 24^3 meshes (0.2 h, mu = 1,
    boundary-vertex patches included) at degrees 2, 4, 6, 8 with default level
    lists, FP32 local solvers with Lanczos bounds, smoothed together; a step is
    one forward sweep of all four, enqueued directly with one workgroup per
    patch (graph sweeps and the batch launch-shape tuner are switched off in
    the library)."""
    import numpy as np
    import torch

    import synth
    from paper_2510_17785_amd import SmootherBatch

    ps = (2, 4, 6, 8)
    n = w.n
    X = [synth.make_vertices(3, n, w.alpha, w.mesh_seed + k) for k in range(4)]
    mu = [np.ones(n ** 3) for _ in ps]
    bh = [synth.make_rhs(3, n, p, w.rhs_seed + k) for k, p in enumerate(ps)]
    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    B = SmootherBatch(3, [n] * 4, ps, X, mu, precision="fp32", with_boundary=True)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    bd = [torch.tensor(b, device=dev) for b in bh]
    us = [torch.zeros_like(b) for b in bd]
    local = sum(S.local_dofs for S in B.instances)

    for _ in range(args.warmup):
        B.smooth(us, bd, +1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        B.smooth(us, bd, +1)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    print(f"# batch: {ms:.3f} ms per sweep; launch shapes {[S.launch for S in B.instances]}",
          file=sys.stderr, flush=True)
    levels = {2: (2, 1), 4: (4, 2, 1), 6: (6, 3, 1), 8: (8, 4, 2, 1)}
    F = sum(algorithmic_per_patch(3, levels[p], 3, 4)[0] for p in ps) * n ** 3
    achieved = F / (ms / 1e3) / 1e12
    out = {
        "metric": "batch patch-DoF/s (mixed degrees, instances concurrent per colour)",
        "value": local / (ms / 1e3),
        "unit": "patch-DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: four independent 3D {n}^3 meshes perturbed by {w.alpha} h, mu=1, "
                        f"degrees {ps} (levels {[levels[p] for p in ps]}), all vertex patches "
                        f"including boundary-cut ones, FP32 local solvers, Lanczos bounds",
            "patches": sum(S.n_patches for S in B.instances),
            "local_dofs_per_sweep": local,
        },
        "launch_shapes": {str(p): list(S.launch) for p, S in zip(ps, B.instances)},
        "setup_s": setup_s,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS,
            "valu_issue_frac": achieved / VALU_PEAK_TFLOPS,
            "traffic": None,
            "kernel": "patch_kernel<float,3,Levels<p...>,smooth> for p = 2, 4, 6, 8",
            "algorithmic_flops_per_sweep": F,
            "note": "algorithmic count of N^3 interior-patch equivalents per degree "
                    "(cut patches cost their share of cells)",
        },
    }
    B.close()
    if not args.no_cg:
        # each instance's own outer CG at its full size (GMG with boundary
        # patches on 24^3, 12^3, 6^3 and the dense coarse solve on 3^3):
        # FP32 local solver against FP64, the +1 iteration rule
        from paper_2510_17785_amd import GMGSolver
        cg = {}
        for k, p in enumerate(ps):
            row = {}
            for prec in ("fp64", "fp32"):
                t0 = time.perf_counter()
                G = GMGSolver(3, n, p, X[k], mu[k], precision=prec, with_boundary=True)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                _, it, rel = G.cg(bd[k], rtol=1e-8)
                t2 = time.perf_counter()
                G.close()
                row[prec] = {"iterations": it, "relres": rel, "setup_s": t1 - t0, "solve_s": t2 - t1}
            row["fp32_within_one"] = row["fp32"]["iterations"] <= row["fp64"]["iterations"] + 1
            cg[str(p)] = row
            print(f"# batch instance p={p} outer CG on {n}^3: FP64 {row['fp64']['iterations']}, "
                  f"FP32 {row['fp32']['iterations']} iterations (setup {row['fp64']['setup_s']:.1f} s / "
                  f"{row['fp32']['setup_s']:.1f} s)", file=sys.stderr, flush=True)
        out["outer_cg"] = cg
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_batch(w, ps, levels, X, mu, bh, local)
    print(json.dumps(out))
    return 0


def cpu_baseline_batch(w, ps, levels, X, mu, bh, local, budget_s=12.0):
    """The oracle's sweep on a bounded sample of patches of each instance
    (setup untimed), extrapolated to all patches of all instances."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import fem
    from oracle.smoother import PatchSmoother, patch_order

    total = 0.0
    desc = []
    with threadpool_limits(limits=1):
        for k, p in enumerate(ps):
            order = patch_order(3, w.n, with_boundary=True)
            rng = np.random.default_rng(k)
            ns = 4 if p <= 4 else 2
            pick = [order[i] for i in sorted(rng.choice(len(order), ns, replace=False))]
            S = PatchSmoother(fem.Mesh(3, w.n, X[k], mu[k]), p, levels[p], keep_closure=True,
                              vertices=pick, with_boundary=True)
            u = np.zeros_like(bh[k])
            reps, t0 = 0, time.perf_counter()
            while True:
                u = S.sweep(u, bh[k], +1)
                reps += 1
                if time.perf_counter() - t0 >= budget_s / len(ps):
                    break
            t = time.perf_counter() - t0
            total += t / reps * len(order) / ns
            desc.append(f"p={p}: {ns} patches x {reps} sweeps in {t:.1f} s")
    return {"value": local / total, "unit": "patch-DoF/s", "cores": 1, "kind": "oracle",
            "sample": "; ".join(desc) + " (oracle sweeps, setup untimed), extrapolated to all "
                      "patches of all four instances"}


DEFAULT_WORKLOAD = "3d-n16-q4"
SECOND_WORKLOAD = "3d-n32-q7-jump"

# Batched patch CG: independent 3D Q7 patches drawn like the patches of the
# 32^3 Q7 jump mesh (perturbation 0.25 h, cell coefficients 10^U(-4, 4)), as
# many as that mesh has interior vertices; FP64 local solver, Lanczos bounds.
PCG_WORKLOAD = "3d-q7-jump-local-pcg"
PCG_PATCHES, PCG_P, PCG_LEVELS, PCG_ALPHA, PCG_MU = 29791, 7, (7, 3, 1), 0.25, (-4.0, 4.0)
PCG_RTOL, PCG_MAXIT, PCG_SEED = 1e-8, 200, 6000


def bench_pcg(args):
    """CG on every patch problem A_{j,p} x = b_j, preconditioned by one local
    V-cycle (the measure of the local solver in Section 3.2), all patches in
    one call of pmg_patch_pcg; a step is one such call on the whole batch.
    Value: V-cycles per second (one V-cycle and one top-level apply per CG
    iteration of each patch)."""
    import numpy as np
    import torch

    import synth
    from paper_2510_17785_amd import PatchBatch

    X, mu = synth.make_random_patches(3, PCG_PATCHES, PCG_ALPHA, PCG_MU, PCG_SEED)
    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    B = PatchBatch(3, PCG_P, X, mu, levels=PCG_LEVELS, precision="fp64")
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    N = B.level_sizes[0]
    bh = np.random.default_rng(PCG_SEED + 1).standard_normal((PCG_PATCHES, N))
    b = torch.tensor(bh, device=dev)
    for _ in range(args.warmup):
        B.pcg(b, PCG_RTOL, PCG_MAXIT)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record()
    for s in range(args.steps):
        x, it, rel = B.pcg(b, PCG_RTOL, PCG_MAXIT)
        ev[s + 1].record()
    torch.cuda.synchronize()
    call_ms = [ev[s].elapsed_time(ev[s + 1]) for s in range(args.steps)]
    ms = sum(call_ms) / args.steps
    its = it.cpu().numpy()
    rels = rel.cpu().numpy()
    vcycles = int(its.sum())
    F, _ = algorithmic_per_patch(3, PCG_LEVELS, 3, 8)
    # per CG iteration: one V-cycle and one top-level apply (the F of a patch
    # update, whose evaluate apply becomes the CG operator apply), two dot
    # products and three vector updates (10 flops per entry)
    F_iter = F + 10 * N
    achieved = vcycles * F_iter / (ms / 1e3) / 1e12
    print(f"# patch CG: {ms:.2f} ms per batch, iterations min {its.min()} median "
          f"{int(np.median(its))} max {its.max()}, max relres {rels.max():.2e}", file=sys.stderr, flush=True)
    out = {
        "metric": "batched patch-CG V-cycles/s (CG preconditioned by the local V-cycle, FP64)",
        "value": vcycles / (ms / 1e3),
        "unit": "V-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{PCG_WORKLOAD}: {PCG_PATCHES} independent 3D Q{PCG_P} vertex patches "
                        f"perturbed by {PCG_ALPHA} h, cell mu=10^U{PCG_MU}, local levels "
                        f"{'->'.join(map(str, PCG_LEVELS))}, Chebyshev degree 3, Lanczos bounds, "
                        f"CG to {PCG_RTOL} relative residual (at most {PCG_MAXIT} iterations), "
                        f"b ~ N(0,1)",
            "patch_dofs": N,
        },
        "solves_per_s": PCG_PATCHES / (ms / 1e3),
        "patch_dofs_per_s": PCG_PATCHES * N / (ms / 1e3),
        "iterations": {"min": int(its.min()), "median": float(np.median(its)), "max": int(its.max()),
                       "mean": float(its.mean())},
        "max_relres": float(rels.max()),
        "setup_s": setup_s,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": measured_traffic(PCG_WORKLOAD, "patch_kernel_fp64"),
            "kernel": f"patch_kernel<double,3,Levels<{','.join(map(str, PCG_LEVELS))}>,pcg>",
            "algorithmic_flops_per_iteration": F_iter,
            "v_cycles_per_launch": vcycles,
            "avg_launch_ms": ms,
        },
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_pcg(X, mu, bh)
    B.close()
    print(json.dumps(out))
    return 0


def cpu_baseline_pcg(X, mu, bh, budget_s=12.0):
    """The oracle's patch CG on a bounded sample of the batch's patches
    (patch matrices and Lanczos bounds untimed), in V-cycles per second."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import fem, lanczos, pmg

    sample = [int(j) for j in np.random.default_rng(0).choice(len(X), 8, replace=False)]
    with threadpool_limits(limits=1):
        solvers = []
        for j in sample:
            s = pmg.LocalSolver(fem.PatchGeometry(X[j], mu[j]), PCG_LEVELS)
            s.set_bounds([lanczos.bounds(s.A[l], s.dinv[l], 12, 0, j, l)
                          for l in range(len(PCG_LEVELS) - 1)])
            solvers.append(s)
        vc, solves, t0 = 0, 0, time.perf_counter()
        while True:
            for s, j in zip(solvers, sample):
                vc += s.pcg(bh[j], PCG_RTOL, PCG_MAXIT)[1]
                solves += 1
            if time.perf_counter() - t0 >= budget_s:
                break
        t = time.perf_counter() - t0
    return {"value": vc / t, "unit": "V-cycles/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(sample)} of {len(X)} patches, {solves} oracle CG solves ({vc} V-cycles) "
                      f"in {t:.1f} s (FP64 dense level matrices, setup untimed)"}


STUDY_WORKLOAD = "local-solver-study"


def bench_study(args):
    """The single-patch study of Section 3.2 on the GPU (batched patch CG,
    omega = 1/2 Jacobi V-cycle, levels from 1, 3, 7, CG to 1e-8 within 100
    iterations): distortion 0..0.35 (2D) / 0..0.28 (3D), 20 patches per
    value; a jump of 1..1e8 in one cell of an undeformed patch; a jump of
    1e4 under distortion; p = 3, 7, 15 in 2D and 3, 7 in 3D; each with the
    damped Jacobi and with the Cartesian-reinforced smoother (omega = 1/2).
    A step is the ten studies, one pmg_patch_pcg call each (the median call
    time of up to five steps is used).  Value: V-cycles per second over all of them (small
    batches: the GPU is far from full)."""
    import numpy as np

    from paper_2510_17785_amd.study import run_study

    cases = [(2, 3), (2, 7), (2, 15), (3, 3), (3, 7)]
    dists = {2: (0.0, 0.05, 0.1, 0.15, 0.2, 0.25, 0.3, 0.35), 3: (0.0, 0.05, 0.1, 0.15, 0.2, 0.25, 0.28)}
    for _ in range(args.warmup):
        run_study(3, 7, distortions=(0.1,), jumps=(1.0,), realizations=4)
    tables, total_s, total_vc, flops = {}, 0.0, 0, 0.0
    res = {}
    steps = min(max(args.steps, 1), 5)   # each pass sets up ten batches: at most five passes
    for dim, p in cases:
        for sm in ("jacobi", "cartesian"):
            secs = []
            for _ in range(steps):
                r = run_study(dim, p, distortions=dists[dim], smoother=sm)
                secs.append(r["seconds"])
            r["seconds"] = float(np.median(secs))
            if sm == "jacobi":
                res[(dim, p)] = r
            total_s += r["seconds"]
            total_vc += r["v_cycles"]
            F, _ = algorithmic_per_patch(dim, r["levels"], 1, 8)
            flops += r["v_cycles"] * (F + 10 * r["patch_dofs"])
            tables[f"{dim}d-p{p}-{sm}"] = [{k: v for k, v in row.items()} for row in r["rows"]]
            print(f"# study {dim}D p={p} {sm}: {len(r['X'])} patches, {r['seconds'] * 1e3:.2f} ms, "
                  + "; ".join(f"{row['sweep']} {row['value']:g}: "
                              + (f"{row['mean_iterations']:.2f}" if row["mean_iterations"] is not None else "-")
                              + (f" ({row['not_converged']} not converged: sentinel mean "
                                 f"{row['mean_with_sentinel']:.0f}, off the paper's axes)"
                                 if row["not_converged"] else "")
                              for row in r["rows"]),
                  file=sys.stderr, flush=True)
    achieved = flops / total_s / 1e12
    out = {
        "metric": "local-solver study V-cycles/s (batched patch CG, omega=1/2 V-cycle, FP64)",
        "value": total_vc / total_s,
        "unit": "V-cycles/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": total_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{STUDY_WORKLOAD}: single 2^d-cell patches, every vertex moved by delta h in a "
                        f"random direction, one-cell jumps 1..1e8 and 1e4 with distortion, 20 per value, "
                        f"p in (3, 7, 15) for d = 2 and (3, 7) for d = 3, levels (3,1) / (7,3,1) / (15,7,3,1), damped Jacobi "
                        f"(degree-1 Chebyshev on [0.5, 3.5]) and Cartesian-reinforced smoothers, omega 1/2, "
                        f"CG to 1e-8 within 100 iterations, b ~ N(0,1)",
            "patches": {f"{d}d-p{p}": len(res[(d, p)]["X"]) for d, p in cases},
        },
        "tables": tables,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": None,
            "kernel": "patch_kernel<double,d,Levels<p,...,1>,pcg> for (d, p) in "
                      + ", ".join(f"({d}, {p})" for d, p in cases),
            "note": "a few hundred patches per call: latency-bound, far below a full GPU",
        },
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_study(res[(3, 7)])
    print(json.dumps(out, default=float))
    return 0


def cpu_baseline_study(r, budget_s=12.0):
    """The oracle's patch CG on a sample of the 3D p = 7 study's patches
    (patch matrices untimed), in V-cycles per second."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import fem, pmg
    from paper_2510_17785_amd.study import OMEGA_HALF_BOUNDS

    sample = [int(j) for j in np.random.default_rng(0).choice(len(r["X"]), 6, replace=False)]
    with threadpool_limits(limits=1):
        solvers = []
        for j in sample:
            s = pmg.LocalSolver(fem.PatchGeometry(r["X"][j], r["mu"][j]), r["levels"], cheb_degree=1)
            s.set_bounds([OMEGA_HALF_BOUNDS] * (len(r["levels"]) - 1))
            solvers.append(s)
        vc, solves, t0 = 0, 0, time.perf_counter()
        while True:
            for s, j in zip(solvers, sample):
                vc += s.pcg(r["b"][j], 1e-8, 100)[1]
                solves += 1
            if time.perf_counter() - t0 >= budget_s:
                break
        t = time.perf_counter() - t0
    return {"value": vc / t, "unit": "V-cycles/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(sample)} of the {len(r['X'])} 3D p=7 study patches, {solves} oracle CG "
                      f"solves ({vc} V-cycles) in {t:.1f} s (setup untimed)"}


GMRES_WORKLOAD = "gmres-2d-paper-order"


def bench_gmres(args):
    """GMRES with the GMG preconditioner in the paper's sweep order on its 2D
    mesh (32 x 32 cells, every interior vertex moved by 0.25 h in a random
    direction, all vertex patches, damped Jacobi omega = 1/2 in one local
    V-cycle, levels from 1, 3, 7, 15) at p = 3, 7, 15, to 1e-8 from a random
    right-hand side.  A step is the three solves.  Value: fine-level DoFs
    solved per second (sum over the three of DoFs / solve time)."""
    import numpy as np
    import torch

    import synth
    from paper_2510_17785_amd import GMGSolver

    dev = torch.device("cuda", 0)
    n, dim, delta = 32, 2, 0.25
    X = synth.make_sphere_distorted_mesh(dim, n, delta, 8025)
    om = np.array((0.5, 3.5 / 1.1))
    rows, total_s, total_dofs = [], 0.0, 0
    for p in (3, 7, 15):
        lv = (p,) + tuple(q for q in (15, 7, 3, 1) if q < p)
        G = GMGSolver(dim, n, p, X, np.ones(n ** dim), levels=lv, precision="fp64", cheb_degree=1,
                      bounds="fixed", with_boundary=True)
        for l in range(1, G.n_mesh_levels):
            S = G.smoother(l)
            S.set_bounds(np.broadcast_to(om, (S.n_patches, len(lv) - 1, 2)).copy())
        G.set_post_direction(+1)
        bh = synth.make_rhs(dim, n, p, p)   # N(0, 1) on interior nodes, zero on the boundary
        b = torch.tensor(bh, device=dev)
        for _ in range(args.warmup):
            G.gmres(b, 1e-8, 100)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = max(1, min(args.steps, 10))
        for _ in range(steps):
            _, it, rel = G.gmres(b, 1e-8, 100)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        dofs = (n * p - 1) ** dim
        rows.append({"p": p, "dofs": dofs, "iterations": it, "relres": rel, "solve_ms": sec * 1e3})
        total_s += sec
        total_dofs += dofs
        G.close()
        print(f"# gmres p={p}: {dofs} DoFs, {it} iterations, {sec * 1e3:.2f} ms", file=sys.stderr, flush=True)
    out = {
        "metric": "GMRES-GMG DoFs solved per second (paper sweep order, 2D, three degrees)",
        "value": total_dofs / total_s,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": max(1, min(args.steps, 10)),
        "warmup": args.warmup,
        "ms_per_step": total_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{GMRES_WORKLOAD}: 2D {n}^2 cells, every interior vertex moved by {delta} h "
                               f"in a random direction, all vertex patches, damped Jacobi omega 1/2, one "
                               f"local V-cycle, GMRES to 1e-8 with the same sweep order before and after "
                               f"the coarse correction, p = 3, 7, 15"},
        "solves": rows,
        "roofline": None,
        "note": "host-driven GMRES (one synchronisation per Gram-Schmidt product): a time-to-solution "
                "figure; the patch kernels it calls are the ones profiled for the sweep workloads",
    }
    print(json.dumps(out))
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-cg", action="store_true", help="skip the outer CG iteration check")
    ap.add_argument("--no-second", action="store_true",
                    help="skip the second record (the 32^3 Q7 jump workload) of the default run")
    ap.add_argument("--no-tune", action="store_true",
                    help="time the default launch shape (one workgroup per patch)")
    ap.add_argument("--launch", action="append", default=[],
                    help="PREC:GRID:MAP, a fixed launch shape instead of the autotuner's "
                         "(for profiler runs that must launch what a tuned run timed)")
    ap.add_argument("--train-patches", type=int, default=None,
                    help="random patches whose Lanczos bounds train the bound network "
                         "(default 100000 for the 32^3 Q6 learned-bounds workload, 50000 for the 32^3 Q7 "
                         "workload, else 6000)")
    ap.add_argument("--train-epochs", type=int, default=60)
    ap.add_argument("--only", choices=["fp32", "fp64"], default=None,
                    help="time one precision only (for profiler runs; prints no JSON line)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a device-to-device copy of this many bytes, 5 times (a "
                         "known-size kernel for calibrating the HBM byte counters)")
    args = ap.parse_args(argv)
    if args.copy_bytes:
        import torch
        n = args.copy_bytes // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(f"# copied {n * 8} bytes 5 times", file=sys.stderr)
        return 0
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the smoother is measured on one MI355X "
              "(a multi-GPU run would need a halo exchange per colour, which this library "
              "does not have)", file=sys.stderr)
        return 2

    import synth

    if args.workload == PCG_WORKLOAD:
        return bench_pcg(args)
    if args.workload == STUDY_WORKLOAD:
        return bench_study(args)
    if args.workload == GMRES_WORKLOAD:
        return bench_gmres(args)
    w = synth.workload(args.workload)
    if w.name == "3d-n24-q8-batch":
        return bench_batch(args, w)
    # the 32^3 Q7 jump workload (matrix cores on the hot path) as a second
    # record of the default run
    second = synth.workload(SECOND_WORKLOAD) if (args.workload == DEFAULT_WORKLOAD and not args.only
                                                  and not args.no_second) else None
    cases = [(w, synth.make_case(w))] + ([(second, synth.make_case(second))] if second else [])
    # the CPU baselines first, in processes forked before the GPU is touched
    cpu = {}
    if not args.no_cpu and not args.only:
        for wk, (X, mu, bh) in cases:
            cpu[wk.name] = cpu_baseline(wk, X, mu, bh)
            print(f"# cpu oracle {wk.name}: {cpu[wk.name]['value']:.3e} DoF/s on {cpu[wk.name]['cores']} "
                  f"cores, {cpu[wk.name]['one_core']['value']:.3e} on one", file=sys.stderr, flush=True)
    out = None
    for k, (wk, (X, mu, bh)) in enumerate(cases):
        rec = bench_sweep(args, wk, X, mu, bh, secondary=k > 0)
        if rec is None:
            return 0
        if wk.name in cpu:
            rec["cpu_baseline"] = cpu[wk.name]
        if out is None:
            out = rec
        else:
            out.setdefault("secondary", []).append(rec)
    print(json.dumps(out))
    return 0


def bench_sweep(args, w, X, mu, bh, secondary=False):
    """Sweeps of one mesh workload: FP32 local solver with learned bounds (the
    headline) against FP64 with Lanczos bounds (plus the BF16-input forms where
    they exist), the additive variant, the outer GMG-CG iteration check and the
    roofline of the FP32 kernel.  Returns the record (None for --only)."""
    import numpy as np
    import torch

    import synth
    from paper_2510_17785_amd import GMGSolver, PatchSmoother

    steps = args.steps if not secondary else max(5, min(args.steps, 10))
    if args.train_patches is None or secondary:
        train_patches = {"3d-n32-q6-learned": 100000, "3d-n32-q7-jump": 50000}.get(w.name, 6000)
    else:
        train_patches = args.train_patches
    dev = torch.device("cuda", 0)
    b = torch.tensor(bh, device=dev)

    net = None
    train = {}
    if args.only != "fp64":
        from paper_2510_17785_amd.learned import train_bound_network
        Xt, mut = synth.make_random_patches(w.dim, train_patches, w.alpha, w.mu_log10, 4000 + w.cfg)
        tr = train_bound_network(w.dim, w.p, w.levels, Xt, mut, epochs=args.train_epochs, batch=256,
                                 lr=2e-3, seed=1)
        net = tr
        train = {"patches": train_patches, "epochs": args.train_epochs,
                 "label_s": tr.label_seconds, "train_s": tr.train_seconds,
                 "val_rmse_ln": [float(x) for x in tr.val_rmse], "margin_ln": tr.margin}
        print(f"# {w.name} bound network: labels {tr.label_seconds:.2f} s, training {tr.train_seconds:.2f} s, "
              f"val rmse {tr.val_rmse}", file=sys.stderr, flush=True)

    def learned(S):
        return S.set_bounds_mlp(net.net, net.margin)

    res = {}
    variants = [("fp32", "learned"), ("fp64", "lanczos")]
    if has_bf16(w):
        variants += [("bf16", "learned"), ("bf16x3", "learned")]
    if args.only:
        variants = [v for v in variants if v[0] == args.only]
    for prec, bsrc in variants:
        t0 = time.perf_counter()
        S = PatchSmoother(w.dim, w.n, w.p, X, mu, levels=w.levels, precision=prec,
                          bounds="fixed" if bsrc == "learned" else "lanczos")
        fallback = learned(S) if bsrc == "learned" else None
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        u = torch.zeros_like(b)
        fixed = [x.split(":") for x in args.launch if x.split(":")[0] == prec]
        if fixed:
            S.set_launch(int(fixed[0][1]), int(fixed[0][2]))
        elif not args.no_tune:
            S.autotune(u, b)
        tuned_equal = None
        if tuple(S.launch) != (0, 0):
            # the timed shape gives the default shape's bits (one colour)
            shape = tuple(S.launch)
            u1, u2 = torch.zeros_like(b), torch.zeros_like(b)
            S.smooth_colors(u1, b, 0, 1)
            S.set_launch(0, 0)
            S.smooth_colors(u2, b, 0, 1)
            S.set_launch(*shape)
            torch.cuda.synchronize()
            tuned_equal = bool(torch.equal(u1, u2))
        sweep_ms, per_launch, wall = time_sweeps(S, u, b, steps, args.warmup, torch)
        res[prec] = dict(S=S, setup_s=setup_s, sweep_ms=sweep_ms, per_launch=per_launch,
                         dofs=S.n_interior_dofs, n_patches=S.n_patches, fallback=fallback,
                         launch=list(S.launch), tuned_equal=tuned_equal)
        print(f"# {w.name} {prec}+{bsrc}: sweep {sweep_ms:.4f} ms, setup {setup_s:.3f} s, "
              f"{S.n_interior_dofs * 1e3 / sweep_ms:.3e} DoF/s, launch {S.launch}", file=sys.stderr, flush=True)

    if args.only:
        return None
    # the additive variant on the FP32 handle: residuals and local solves of
    # all patches from one iterate in one launch each, then the damped
    # scatter colour by colour
    additive = None
    if "fp32" in res and not secondary:
        S32 = res["fp32"]["S"]
        u = torch.zeros_like(b)
        for _ in range(args.warmup):
            S32.smooth_additive(u, b, 0.5)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            S32.smooth_additive(u, b, 0.5)
        e1.record()
        torch.cuda.synchronize()
        ms_add = e0.elapsed_time(e1) / steps
        additive = {"ms_per_step": ms_add, "value": res["fp32"]["dofs"] / (ms_add / 1e3), "unit": "DoF/s",
                    "theta": 0.5, "note": "one additive sweep (all patches from one iterate), FP32 local "
                                          "solver with learned bounds; convergence per sweep differs from "
                                          "the multiplicative sweep"}
        print(f"# fp32 additive: sweep {ms_add:.4f} ms", file=sys.stderr, flush=True)
    cg = {}
    if not args.no_cg:
        cg_variants = [("fp64_lanczos", "fp64", "lanczos"), ("fp32_learned", "fp32", "learned")]
        if not secondary:
            cg_variants += [("fp32_lanczos", "fp32", "lanczos")]
        if has_bf16(w):
            cg_variants += [("bf16x3_learned", "bf16x3", "learned")]
            if not secondary:
                cg_variants += [("bf16_learned", "bf16", "learned")]
        if not secondary:
            # one interval for every patch and level: the envelope of the Lanczos bounds
            cg_variants += [("fp32_fixed", "fp32", "fixed")]
            # additive sweeps (damping 2^-d) as both smoothing steps
            cg_variants += [("fp32_learned_additive", "fp32", "learned")]
        for key, prec, bsrc in cg_variants:
            t0 = time.perf_counter()
            G = GMGSolver(w.dim, w.n, w.p, X, mu, levels=w.levels, precision=prec,
                          bounds="lanczos" if bsrc in ("lanczos", "fixed") else "fixed")
            nfb = 0
            if bsrc == "learned":
                for l in range(1, G.n_mesh_levels):
                    nfb += learned(G.smoother(l))
            elif bsrc == "fixed":
                for l in range(1, G.n_mesh_levels):
                    S_l = G.smoother(l)
                    lam = S_l.bounds()
                    env = np.array([lam[..., 0].min(), lam[..., 1].max()])
                    S_l.set_bounds(np.broadcast_to(env, lam.shape).copy())
            if key.endswith("_additive"):
                G.set_additive(0.5 ** w.dim)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x, it, rel = G.cg(b, rtol=w.rtol)
            torch.cuda.synchronize()
            cg[key] = {"iterations": it, "relres": rel, "setup_s": t1 - t0,
                       "solve_s": time.perf_counter() - t1}
            if bsrc == "learned":
                cg[key]["lanczos_fallback_patches"] = nfb
            G.close()
            print(f"# {w.name} cg {key}: {it} iterations, relres {rel:.2e}", file=sys.stderr, flush=True)
        cg["fp32_learned_within_one_of_fp64"] = (cg["fp32_learned"]["iterations"]
                                                 <= cg["fp64_lanczos"]["iterations"] + 1)

    r32 = res["fp32"]
    F, B = algorithmic_per_patch(w.dim, w.levels, 3, 4)
    total_launch_ms = float(np.sum(r32["per_launch"])) / steps
    n_launch = r32["S"].n_colors
    avg_launch_s = total_launch_ms / n_launch / 1e3
    patches_per_launch = r32["n_patches"] / n_launch
    achieved = F * patches_per_launch / avg_launch_s / 1e12
    mshare = mfma_flops_per_patch(w.dim, w.levels, 3) / F
    value = r32["dofs"] / (r32["sweep_ms"] / 1e3)
    value64 = res["fp64"]["dofs"] / (res["fp64"]["sweep_ms"] / 1e3)
    persistent = 0 < r32["launch"][0] < max(r32["S"].color_offsets[c + 1] - r32["S"].color_offsets[c]
                                            for c in range(r32["S"].n_colors))
    out = {
        "metric": "patch-smoother DoF/s: FP32-MFMA+learned vs FP64 plain, same outer CG iters",
        "value": value,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": r32["sweep_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: {w.dim}D {w.n}^{w.dim} cells perturbed by {w.alpha} h, Q{w.p}, "
                        f"mu={'1' if w.mu_log10 is None else '10^U' + str(tuple(w.mu_log10))}, "
                        f"{r32['n_patches']} vertex patches, local levels "
                        f"{'->'.join(map(str, w.levels))}, Chebyshev degree 3, N_MG=1, "
                        f"FP32 local solver with learned Chebyshev bounds vs FP64 local "
                        f"solver with Lanczos bounds (12 steps)",
            "interior_dofs": r32["dofs"],
            "sweep": f"forward, {2 ** w.dim} colours",
        },
        "fp64": {"value": value64, "unit": "DoF/s", "ms_per_step": res["fp64"]["sweep_ms"],
                 "speedup_fp32_over_fp64": value / value64},
        **{prec: {"value": res[prec]["dofs"] / (res[prec]["sweep_ms"] / 1e3), "unit": "DoF/s",
                  "ms_per_step": res[prec]["sweep_ms"],
                  "speedup_over_fp64": res["fp64"]["sweep_ms"] / res[prec]["sweep_ms"]}
           for prec in ("bf16", "bf16x3") if prec in res},
        "additive_fp32": additive,
        "vcycles_per_s": r32["n_patches"] / (r32["sweep_ms"] / 1e3),
        "launch_shapes": {p: res[p]["launch"] for p in res},
        "tuned_shape_equals_default_bitwise": {p: res[p]["tuned_equal"] for p in res},
        "setup_s": {f"{p}_{'lanczos' if p == 'fp64' else 'learned'}": res[p]["setup_s"] for p in res},
        "learned_bounds": dict(train, lanczos_fallback_patches=res["fp32"]["fallback"]),
        "outer_cg": cg,
        "roofline": {
            "bound": "mfma" if mshare > 0.5 else "alu",
            "achieved": achieved,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": measured_traffic(w.name),
            "valu_issue_frac": achieved / mixed_peak(mshare),
            "peak_parts": {"fp32_peak": FP32_PEAK_TFLOPS, "valu_fp32_unpacked": VALU_PEAK_TFLOPS,
                           "mfma_fp32": MFMA_FP32_PEAK_TFLOPS, "mfma_flop_share": mshare,
                           "issuable_peak": mixed_peak(mshare)},
            "kernel": f"patch_kernel<float,{w.dim},Levels<{','.join(map(str, w.levels))}>,smooth,"
                      f"{'persistent' if persistent else 'one workgroup per patch'}>",
            "launch_shape": r32["launch"],
            "algorithmic_flops_per_patch": F,
            "algorithmic_bytes_per_patch": B,
            "patches_per_launch": patches_per_launch,
            "avg_launch_ms": avg_launch_s * 1e3,
            "hbm_frac": B * patches_per_launch / avg_launch_s / 1e9 / HBM_PEAK_GBS,
        },
    }
    for r in res.values():
        r["S"].close()
    return out


if __name__ == "__main__":
    sys.exit(main())
