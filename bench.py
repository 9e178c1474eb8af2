#!/usr/bin/env python3
"""Benchmark of the inexact AF-IETI solve on one MI355X.

Workload (default): 3D compressible elasticity on the unit cube split into
2x2x2 trilinear patches (interior vertex moved by U(-0.05, 0.05)^3, seed 0),
splines p=3 C^2 with 32^3 elements per patch (35^3 basis functions x 3
components, 1,029,000 DOF), E=1, nu=0.3, trigonometric body force, u=0 on
z=0; MINRES to a preconditioned residual ratio of 1e-8 from x0=0.

One step = one full AF-IETI solve (prologue, MINRES with the FD/Schur
preconditioner, recovery) with inputs resident in HBM; assembly and FD setup
are outside the timed region.  The headline value is the FP32-FD solve time;
the FP64-FD solve, the FD-apply throughput, the stiffness-kernel roofline
and the CPU oracle baseline are reported on the same JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "AF-IETI solve s to 1e-8 rel.res (FP32-FD vs FP64-FD); FD-apply DOF/s"
# HBM bytes of one stiffness-operator application (k_mf_brick + k_mf_gather)
# read from the FETCH_SIZE / WRITE_SIZE counters (scaled by a 1 GiB device
# copy's readings): profiles/k_mf_stiffness_c2_traffic.md.  Valid for the
# kernels that were measured; None for workloads without such a run.
MEASURED_TRAFFIC = {"c2": 230.8e6}
# HBM bytes of one FP32 P_A^{-1} application (k_fdg_fwd + k_fdg_mid +
# k_fdg_bwd), from the same counters: profiles/fd_c2_fp32_counters.md
MEASURED_FD_TRAFFIC = {"c2": 36.98e6}
FP32_MFMA_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name):
    import workloads as W
    if name == "c2":
        prob = W.make_c2(seed=0)
        desc = ("3D unit cube, 2x2x2 trilinear patches (interior vertex +-0.05), p=3 C^2, "
                "32^3 elements/patch (35^3 basis x 3 comp), E=1 nu=0.3, trig load, u=0 on z=0")
    elif name == "c1":
        prob = W.make_c1(seed=0)
        desc = "2D unit square, 2x2 bilinear patches, p=2 C^1, 16^2 elements/patch, lambda=mu=1, u=0 on x=0"
    elif name == "c4":
        prob = W.make_c4(seed=0)
        desc = ("ragged batch of 32 3D problems: patch grids in {1,2,3}^3, 8..40 elements per direction, "
                "p in {2,3,4}, lognormal Lame, 8 trig modes, u=0 on z=0")
    elif name.startswith("c3"):
        p = int(name[2:]) if len(name) > 2 else 3
        prob = W.make_c3(seed=0, p=p)
        desc = f"3D unit cube, 4x4x4 patches, p={p} C^{p-1}, 24^3 elements/patch, lognormal Lame, 8 trig modes"
    elif name.startswith("nc"):
        p = int(name[2:]) if len(name) > 2 else 3
        prob = W.make_nonconforming(p=p)
        desc = (f"non-conforming box (0,1)x(0,3)x(0,1): three cubes of 4, 8, 16 elements per direction "
                f"(nested interfaces), p={p} C^{p-1}, steel, Dirichlet data of a manufactured solution")
    elif name.startswith("ws"):
        k = int(name[2:]) if len(name) > 2 else 4
        prob = W.make_weak_scaling(k=k, n_el=8, p=3)
        desc = (f"weak-scaling cube: {k}^3 unit-cube patches, p=3 C^2, 8^3 elements/patch, steel, "
                "manufactured solution, Dirichlet data on y=0,1 and z=0,1, tractions on x=0,1")
    else:
        raise SystemExit(f"unknown workload {name}")
    return prob, desc


def time_events(fn, reps):
    import torch
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def fd_flops(solver_prob):
    """Algorithmic flops of one P_A^{-1} application: per patch and
    component 2 n^d (sum_m n_m) multiply-adds forward and backward (the
    paper's 4 d n N per patch) plus the divide."""
    if isinstance(solver_prob, list):
        return sum(fd_flops(p) for p in solver_prob)
    total = 0
    for pd in solver_prob["patches"]:
        # basis functions on uniform open knots: n_el (p - reg) + reg + 1
        n = [e * (pd["p"] - pd["reg"]) + pd["reg"] + 1 for e in pd["n_el"]]
        N = 1
        for v in n:
            N *= v
        total += solver_prob["dim"] * (4 * N * sum(n) + N)
    return total


def stiffness_alg_flops(prob):
    """Algorithmic flops of one stiffness product A w: the assembled
    operator's 2 flops per stored coefficient, each row (component, node)
    coupling to the d (2p+1)^d coefficients of its stencil (Section 3, local
    matrices): 2 d (2p+1)^d per DOF."""
    if isinstance(prob, list):
        return sum(stiffness_alg_flops(q) for q in prob)
    d = prob["dim"]
    total = 0
    for pd in prob["patches"]:
        N = 1
        for e in pd["n_el"][:d]:
            N *= e * (pd["p"] - pd["reg"]) + pd["reg"] + 1
        total += d * N * 2 * d * (2 * pd["p"] + 1) ** d
    return total


def mf_flops(prob):
    """FP64 flops the matrix-free stiffness kernel executes per application
    (sum-factorised quadrature of the Section 3 bilinear form): per element brick
    of BE^3 elements with NB = BE + p basis functions and QB = BE (p + 1)
    Gauss points per direction, six univariate passes each way -- a
    multiply-add per Gauss point and supported basis function (p + 1 of
    them): 2 products along direction 1 on 3 NB^2 lines, 3 along direction 2
    on 3 NB QB lines, 3 along direction 3 on 3 QB^2 lines, forward and
    transposed -- plus 196 flops per Gauss point for the Jacobian of the
    trilinear map, its adjugate and determinant, the reciprocal of |det J|,
    the scaled stress and the flux."""
    if isinstance(prob, list):
        return sum(mf_flops(q) for q in prob)
    total = 0
    for pd in prob["patches"]:
        p = pd["p"]
        BE = 2 if p <= 4 else 1
        NB, QB = BE + p, BE * (p + 1)
        nb = 1
        for e in pd["n_el"]:
            nb *= -(-e // BE)
        fma = 3 * QB * (p + 1) * (2 * NB * NB + 3 * NB * QB + 3 * QB * QB)
        total += nb * (2 * 2 * fma + 196 * QB ** 3)
    return total


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(prob, gpu_iters, n_iters=2):
    """The oracle, untouched, on the host: ``n_iters`` MINRES iterations of
    the same problem (saddle operator, preconditioner, inner products and
    vector updates as in the oracle's MINRES), timed and scaled by the GPU
    iteration count (an extrapolated full solve); plus one full oracle solve
    of the small 2D workload (C1), timed end to end."""
    import numpy as np
    from threadpoolctl import threadpool_info
    import workloads as W
    from oracle.afieti import AFIETI
    o = AFIETI(prob)
    x = W.random_vector(o.n_dof + o.n_c, 5)
    o.apply_op(x)  # geometry tables (setup, not timed)
    t0 = time.perf_counter()
    for _ in range(n_iters):
        q = o.apply_op(x)
        z = o.apply_prec(q)
        d = float(q @ x) + float(z @ q)
        v = q - 0.5 * x - 0.25 * z
        x = x + 1e-3 * v + d * 0.0
    per_it = (time.perf_counter() - t0) / n_iters
    blas = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    oc1 = AFIETI(W.make_c1(seed=0))
    t0 = time.perf_counter()
    r1 = oc1.solve(tol=1e-8)
    c1_s = time.perf_counter() - t0
    return dict(value=per_it * gpu_iters, unit="s", cores=blas, kind="oracle",
                sample=f"{n_iters} MINRES iterations of the oracle on this workload ({per_it:.2f} s each: saddle "
                       f"operator, preconditioner, dots, updates), x {gpu_iters} iterations (extrapolated)",
                extrapolated=True, per_iteration_s=per_it, nproc=os.cpu_count(), cpu_model=_cpu_model(),
                threads="BLAS threads (dense FD products); the quadrature and sparse products run on one thread",
                c1_full_solve_s=c1_s, c1_iterations=int(r1["iters"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--fd-reps", type=int, default=100)
    ap.add_argument("--mv-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-fp32", action="store_true")
    ap.add_argument("--no-geometry", action="store_true",
                    help="skip the geometry-inclusion variant of the local solvers")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the method would shard by patch). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import workloads as W
    from paper_2001_09626_amd import Solver

    prob, desc = workload(args.workload)
    t = time.time()
    log(f"setup FP32-FD handle ({args.workload})")
    s32 = Solver(prob, fd_precision="fp32", tol=1e-8)
    torch.cuda.synchronize()
    setup32 = time.time() - t
    log(f"  setup {setup32:.1f}s n_dof={s32.n_dof} n_c={s32.n_c} stencil={s32.stiffness_bytes/1e9:.2f} GB")
    s64 = None
    if not args.only_fp32:
        t = time.time()
        log("setup FP64-FD handle")
        s64 = Solver(prob, fd_precision="fp64", tol=1e-8)
        torch.cuda.synchronize()
        log(f"  setup {time.time()-t:.1f}s")
    u32 = torch.empty(s32.n_dof, dtype=torch.float64, device="cuda")
    l32 = torch.empty(s32.n_c, dtype=torch.float64, device="cuda")
    for i in range(args.warmup):
        _, _, st = s32.solve(u=u32, lam=l32)
        log(f"warmup FP32-FD solve {i}: {st['iterations']} it, {st['ms']:.1f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters32 = []
    for i in range(args.steps):
        _, _, st = s32.solve(u=u32, lam=l32)
        iters32.append(st["iterations"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms32 = (t1 - t0) * 1e3 / args.steps
    log(f"FP32-FD solve: {ms32:.1f} ms/step, {iters32[-1]} iterations")

    out = {}
    if s64 is not None:
        u64 = torch.empty(s64.n_dof, dtype=torch.float64, device="cuda")
        l64 = torch.empty(s64.n_c, dtype=torch.float64, device="cuda")
        for i in range(args.warmup):
            s64.solve(u=u64, lam=l64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            _, _, st64 = s64.solve(u=u64, lam=l64)
        torch.cuda.synchronize()
        ms64 = (time.perf_counter() - t0) * 1e3 / args.steps
        log(f"FP64-FD solve: {ms64:.1f} ms/step, {st64['iterations']} iterations")
        rel = float(torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64))
        out.update(fp64_fd_solve_s=ms64 / 1e3, iterations_fp64_fd=st64["iterations"],
                   solve_speedup_fp32_vs_fp64=ms64 / ms32, rel_diff_u_fp32_vs_fp64=rel)

    # the geometry-inclusion local solvers (the variant of the paper's
    # numerical results), FP32 FD: setup (fit, d^2 pencils per patch,
    # scalings) and solve
    if not args.no_geometry:
        t = time.time()
        log("setup geometry-inclusion FP32-FD handle")
        sg = Solver(prob, fd_precision="fp32", tol=1e-8, precond="geo")
        torch.cuda.synchronize()
        setup_g = time.time() - t
        ug = torch.empty(sg.n_dof, dtype=torch.float64, device="cuda")
        lg = torch.empty(sg.n_c, dtype=torch.float64, device="cuda")
        for i in range(args.warmup):
            sg.solve(u=ug, lam=lg)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            _, _, stg = sg.solve(u=ug, lam=lg)
        torch.cuda.synchronize()
        msg_ = (time.perf_counter() - t0) * 1e3 / args.steps
        log(f"geometry-inclusion FP32-FD solve: {msg_:.1f} ms/step, {stg['iterations']} iterations "
            f"(setup {setup_g:.1f}s)")
        out["geometry_inclusion"] = dict(solve_s=msg_ / 1e3, iterations=stg["iterations"], setup_s=setup_g,
                                         fd_precision="fp32")
        sg.close()

    # FD-apply throughput (one apply over all patches and components)
    r = torch.from_numpy(W.random_vector(s32.n_dof, 3)).cuda()
    z = torch.empty_like(r)
    flops = fd_flops(prob)
    for name, s in (("fp32", s32), ("fp64", s64)):
        if s is None:
            continue
        s.apply_fd(r, z)
        ms = time_events(lambda: s.apply_fd(r, z), args.fd_reps)
        out[f"fd_apply_ms_{name}"] = ms
        out[f"fd_apply_dof_per_s_{name}"] = s.n_dof / (ms * 1e-3)
        out[f"fd_apply_tflops_{name}"] = flops / (ms * 1e-3) / 1e12
        if name == "fp32":
            out["fd_apply_frac_fp32_mfma_peak"] = flops / (ms * 1e-3) / 1e12 / FP32_MFMA_PEAK_TFLOPS
        log(f"FD apply {name}: {ms*1e3:.1f} us, {s.n_dof/(ms*1e-3)/1e9:.2f} GDOF/s")

    # stiffness matvec: the dominant kernel of every MINRES iteration,
    # timed with HIP events on the stream its kernels are launched on
    x = torch.from_numpy(W.random_vector(s32.n_dof, 4)).cuda()
    y = torch.empty_like(x)
    s32.apply("stiffness", x, y)
    mv_ms = time_events(lambda: s32.apply("stiffness", x, y), args.mv_reps)
    alg = stiffness_alg_flops(prob)
    if s32.stiffness_bytes == 0:
        # matrix-free: bound by FP64 vector arithmetic; achieved counts the
        # method's algorithmic flops (2 d (2p+1)^d per DOF), the flops the
        # quadrature kernel executes are reported beside them
        impl = mf_flops(prob)
        tfs = alg / (mv_ms * 1e-3) / 1e12
        log(f"stiffness matvec (matrix-free): {mv_ms:.3f} ms, {tfs:.2f} TFLOP/s algorithmic FP64, "
            f"{impl / (mv_ms * 1e-3) / 1e12:.2f} TFLOP/s executed")
        roof = dict(bound="alu", achieved=tfs, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s", frac=tfs / FP64_PEAK_TFLOPS,
                    traffic=MEASURED_TRAFFIC.get(args.workload), kernel="stiffness operator: k_mf_brick + k_mf_gather",
                    flops_per_launch=alg, ms_per_launch=mv_ms,
                    executed_flops_per_launch=impl,
                    executed_tflops=impl / (mv_ms * 1e-3) / 1e12,
                    executed_frac=impl / (mv_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                    algorithmic_bytes=16 * s32.n_dof,
                    note="achieved = 2 d (2p+1)^d flops per DOF (assembled-operator count) / time; "
                         "executed = the quadrature kernel's own flops")
    else:
        mv_bytes = s32.stiffness_bytes + 2 * 8 * s32.n_dof
        gbs = mv_bytes / (mv_ms * 1e-3) / 1e9
        log(f"stiffness matvec (assembled): {mv_ms:.3f} ms, {gbs:.0f} GB/s")
        roof = dict(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=gbs / HBM_PEAK_GBS,
                    traffic=None, kernel="k_stiffness", bytes_per_launch=mv_bytes, ms_per_launch=mv_ms,
                    flops_per_launch=alg)

    # FD apply against the FP32 matrix-core peak (4 d n flops per DOF)
    fd_roof = None
    if "fd_apply_ms_fp32" in out:
        a = flops / (out["fd_apply_ms_fp32"] * 1e-3) / 1e12
        fd_roof = dict(bound="mfma", achieved=a, peak=FP32_MFMA_PEAK_TFLOPS, unit="TFLOP/s",
                       frac=a / FP32_MFMA_PEAK_TFLOPS, kernel="FD apply, FP32 on the matrix cores",
                       traffic=MEASURED_FD_TRAFFIC.get(args.workload),
                       flops_per_launch=flops, ms_per_launch=out["fd_apply_ms_fp32"],
                       algorithmic_bytes=16 * s32.n_dof)

    # jump operator and projection: bandwidth-bound, algorithmic bytes of
    # their index and value streams
    bx = s32.export("B")
    nnz = int(len(bx) + np.count_nonzero(bx[:, 2] >= 0))
    c = torch.from_numpy(W.random_vector(s32.n_c, 6)).cuda()
    yc = torch.empty_like(c)
    jump = {}
    for name, src, dst, nbytes in (
            ("B", x, yc, s32.n_c * (8 + 8 + 8) + nnz * 8),          # plus/minus index, x values, y
            ("Bt", c, y, (s32.n_dof + 1) * 8 + nnz * (4 + 8 + 8) + s32.n_dof * 8),  # CSR ptr, (row, sign, x), y
            ("P_u", x, y, s32.n_dof * (8 + 8 + 8 + 8))):            # x twice, control points, y
        s32.apply(name, src, dst)
        ms = time_events(lambda: s32.apply(name, src, dst), args.mv_reps)
        gbs = nbytes / (ms * 1e-3) / 1e9
        jump[name] = dict(ms=ms, bytes=nbytes, gbs=gbs, frac=gbs / HBM_PEAK_GBS)
        log(f"{name}: {ms * 1e3:.1f} us, {gbs:.0f} GB/s ({100 * gbs / HBM_PEAK_GBS:.1f} % of HBM)")

    cpu = None
    if not args.no_cpu_baseline and args.workload != "c4":
        log("CPU oracle baseline (one MINRES iteration of the oracle)")
        cpu = cpu_baseline(prob, iters32[-1])
        log(f"  oracle {cpu['per_iteration_s']:.2f} s/iteration on {cpu['cores']} threads")

    line = {
        "metric": METRIC,
        "value": ms32 / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "fd_dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "name": args.workload, "n_dof": int(s32.n_dof),
                   "n_c": int(s32.n_c), "tol": 1e-8, "setup_s": setup32},
        "iterations_fp32_fd": iters32[-1],
        "fp32_fd_solve_s": ms32 / 1e3,
        **out,
        "roofline": roof,
        "fd_roofline": fd_roof,
        "jump_hbm": jump,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
