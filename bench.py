"""Benchmark: cell-wise Q_k operator apply + vertex-patch FDM inverse on one MI355X.

One step = fe_apply followed by patch_fdm_inverse on the 3D Q3 64^3 Cartesian
mesh (193^3 = 7,189,057 unique DoFs, 16.8M cell-wise entries), FP64, inputs
resident in HBM.  Four independent (x, y, r, z) buffer sets are rotated so
that the working set exceeds the 256 MB last-level cache.  The headline value
is unique DoFs per second of whole steps.  Also reported (not part of the
timed steps): the FP32 step, the Q7 32^3 step, per-kernel durations from HIP
events on the launch stream, the MG-PCG solves on Q7 32^3 (FP32 Chebyshev
patch-FDM smoother inside FP64 CG vs the plain FP64 Jacobi-MG solve), and the
CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps 100] [--warmup 1000] [--no-pcg] [--no-cpu]
"""
import argparse
import itertools
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GDoF/s apply+patch inverse (Q3/Q7, FP32 vs FP64); PCG s to 1e-10 rel. res."
HBM_PEAK_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # untimed steps before the timed ones: the GPU needs about a tenth of a second
    # of load to reach its steady clocks (Q3 64^3 FP64: 148 us per step after
    # 10 warmup steps, 136 us after 1000 or when timing 1000 steps)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--no-pcg", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-deformed", action="store_true")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper's cube solves (p = 2..5, 128^3)")
    ap.add_argument("--only-paper", action="store_true", help="run the paper's cube solves only")
    ap.add_argument("--only-step", action="store_true", help="time the headline step only (for profilers)")
    ap.add_argument("--with-copy", action="store_true", help="with --only-step: add a plain copy kernel of known size")
    ap.add_argument("--only-pcg", action="store_true", help="run the Q7 32^3 MG-PCG solves only (for profilers)")
    ap.add_argument("--only-deformed", action="store_true",
                    help="run the deformed Q7 64^3 part only (training and the four solves; for profilers)")
    ap.add_argument("--step-config", default="q3", choices=["q3", "q7", "q7f32", "q3f32"],
                    help="with --only-step: which step to run (Q3 64^3 or Q7 32^3, FP64 or FP32)")
    return ap.parse_args()


def make_inputs(fe, P, dtype, nsets, seed0):
    import torch
    from synthetic_inputs import uniform
    sets = []
    for i in range(nsets):
        xg = torch.as_tensor(uniform(P.n_dofs, seed=seed0 + 2 * i), dtype=torch.float64, device="cuda")
        x64 = P.cellvec(torch.float64)
        P.gather(xg, x64)
        x = x64.to(dtype)
        r = torch.as_tensor(uniform(P.len, seed=seed0 + 2 * i + 1), dtype=dtype, device="cuda")
        sets.append((x, P.cellvec(dtype), r, P.cellvec(dtype)))
        del xg, x64
    return sets


def time_steps(P, sets, steps, warmup):
    import torch

    def step(i):
        x, y, r, z = sets[i % len(sets)]
        P.apply(x, y)
        P.patch_inverse(r, z)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for i in range(steps):
        step(i)
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps   # ms per step


def kernel_times(fe, P, sets, reps):
    """Average duration (ms) of each kernel family over `reps` steps, HIP events on the launch stream."""
    import torch
    fe.prof_reset()
    fe.prof_enable(True)
    for i in range(reps):
        x, y, r, z = sets[i % len(sets)]
        P.apply(x, y)
        P.patch_inverse(r, z)
    torch.cuda.synchronize()
    fe.prof_enable(False)
    out = {}
    for name in ("apply", "fdm_patch", "fdm_sum", "fdm_fused", "fdm_lattice"):
        c, t = fe.prof_query(name)
        if c:
            out[name] = t / c
    fe.prof_reset()
    return out


def measured_traffic(family):
    """HBM bytes per launch of a kernel family from the committed counter summaries
    under profiles/ (FETCH_SIZE and WRITE_SIZE passes, calibrated on a plain copy),
    or None when none was taken on the kernel source as it is now."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            t = line.split()
            if not t or t[0] != "traffic":
                continue
            kv = dict(x.split("=", 1) for x in t[1:] if "=" in x)
            if kv.get("family") != family:
                continue
            src = os.path.join(ROOT, kv.get("source", ""))
            if not os.path.isfile(src):
                continue
            if source_digest(src) != kv.get("code_sha256"):
                continue
            return int(kv["fetch_bytes"]) + int(kv["write_bytes"])
    return None


def source_digest(path):
    """sha256 of a kernel source with its comments and blank lines removed, so
    that editing a comment does not invalidate counters taken on the code."""
    import hashlib
    import re
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    lines = [ln.rstrip() for ln in text.splitlines() if ln.strip()]
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def kernel_bytes(P, dt_bytes):
    """Algorithmic bytes per launch of each kernel family: every vector entry read once and
    written once, plus the patch-solution scratch of the two-pass kernels."""
    k, n = P.degree, P.n
    n_patches = (n - 1) ** 3
    vec = P.len * dt_bytes
    # patch solutions: k <= 3 split by cell slot (8 blocks of k^3 per patch),
    # k >= 4 patch-major ((2k-1)^3 per patch)
    wbuf = n_patches * (8 * k ** 3 if k <= 3 else (2 * k - 1) ** 3) * dt_bytes
    # the fused (k = 2) and lattice (k = 3) patch inverses read r and write z once
    return {"apply": 2 * vec, "fdm_patch": vec + wbuf, "fdm_sum": wbuf + vec, "fdm_fused": 2 * vec,
            "fdm_lattice": 2 * vec}


def bench_config(fe, degree, n, dtype, steps, warmup, nsets):
    import torch
    P = fe.Problem(3, degree, n, bc=1)
    sets = make_inputs(fe, P, dtype, nsets, seed0=0)
    ms = time_steps(P, sets, steps, warmup)
    kt = kernel_times(fe, P, sets, max(10, steps // 2))
    kb = kernel_bytes(P, 8 if dtype == torch.float64 else 4)
    res = {"ms_per_step": ms, "gdofs": P.n_dofs / (ms * 1e-3) / 1e9, "n_dofs": P.n_dofs,
           "kernel_ms": kt, "kernel_gbs": {k: kb[k] / (v * 1e-3) / 1e9 for k, v in kt.items()}}
    del sets
    P.close()
    torch.cuda.empty_cache()
    return res


def timed_solve(P, b, opts, name):
    """First solve (its setup: levels, diagonals, Lanczos estimates, per-patch factors, graph
    capture), then a second solve from zero with the setup cached; both reported."""
    x = P.cellvec()
    first = P.pcg_solve(b, x, opts, raise_on_error=False)
    x.zero_()
    rep = P.pcg_solve(b, x, opts, raise_on_error=False)
    log("pcg %s: %.4f s, %d iters, relres %.2e (first solve: setup %.3f s, solve %.4f s)"
        % (name, rep["t_solve"], rep["iters"], rep["relres"], first["t_setup"], first["t_solve"]))
    return {"seconds": rep["t_solve"], "iters": rep["iters"], "relres": rep["relres"],
            "first_setup_s": first["t_setup"], "first_solve_s": first["t_solve"],
            "converged": rep["converged"], "status": rep["status"]}


def bench_pcg(fe):
    """Q7 32^3, manufactured RHS, tol 1e-10: FP32 Chebyshev(3) patch-FDM MG inside FP64 CG vs FP64 Jacobi MG."""
    import torch
    P = fe.Problem(3, 7, 32, bc=1)
    b = P.cellvec()
    P.rhs_manufactured(b)
    out = {}
    for name, opts in (
            ("fp32_chebfdm_flexible", fe.default_opts(smoother=fe.SMOOTH_CHEB_FDM, inner=fe.F32, flexible=1,
                                                      nu_pre=1, nu_post=1, tol=1e-10)),
            ("fp64_chebfdm", fe.default_opts(smoother=fe.SMOOTH_CHEB_FDM, inner=fe.F64, nu_pre=1, nu_post=1,
                                             tol=1e-10)),
            ("fp64_jacobi_plain", fe.default_opts(smoother=fe.SMOOTH_JACOBI, inner=fe.F64, omega=0.7,
                                                  nu_pre=2, nu_post=2, tol=1e-10, maxit=400))):
        out[name] = timed_solve(P, b, opts, name)
    P.close()
    torch.cuda.empty_cache()
    return out


def bench_deformed_q7(fe):
    """The end-to-end case: Q7 64^3 deformed, model trained on 40,000 patches of three Q7 32^3 meshes."""
    return bench_deformed(fe, 7, 64, n_train=32, train_meshes=3, epochs=30, max_patches=40000)


def bench_deformed(fe, k, n, n_train, train_meshes, epochs, with_solve=True, max_patches=None):
    """Deformed, variable-coefficient mesh: general apply rate; MLP trained on the patches of
    other generated meshes (other amplitudes and coefficient fields; at most max_patches,
    sampled evenly over the meshes with a fixed seed); MG-PCG to 1e-10 with the plain FP64
    Jacobi smoother vs FP32 Chebyshev patch-FDM smoothers with averaged and learned factors."""
    import torch
    from synthetic_inputs import coefficient_modes, uniform
    out = {"workload": "Q%d %d^3 deformed (amp 0.1), coefficient exp(smooth field)" % (k, n)}
    t0 = time.perf_counter()
    feats, targs = [], []
    amps = [0.02 + 0.11 * i / max(1, train_meshes - 1) for i in range(train_meshes)]
    for i, amp in enumerate(amps):
        Pt = fe.Problem(3, k, n_train, geometry=fe.GEOM_DEFORMED, bc=1, deform_amp=amp,
                        coef=coefficient_modes(1000 + i))
        Xi, Ti = Pt.patch_features(), Pt.patch_fit_targets(sweeps=20)
        if max_patches is not None and Xi.shape[0] > max_patches // train_meshes:
            g = torch.Generator(device="cpu").manual_seed(11 + i)
            idx = torch.randperm(Xi.shape[0], generator=g)[: max_patches // train_meshes].to(Xi.device)
            Xi, Ti = Xi[idx], Ti[idx]
        feats.append(Xi)
        targs.append(Ti)
        Pt.close()
        del Pt
    X, T = torch.cat(feats), torch.cat(targs)
    out["train_patches"] = int(X.shape[0])
    out["targets_s"] = time.perf_counter() - t0
    P = fe.Problem(3, k, n, geometry=fe.GEOM_DEFORMED, bc=1, deform_amp=0.1, coef=coefficient_modes(2))
    out["unique_dofs"] = P.n_dofs
    # general apply rate: one (x, y) pair, and 4 rotated pairs (working set beyond the
    # 256 MB last-level cache: the HBM rate); metric stored per Gauss point (6 values
    # per entry streamed) or formed in the kernel (only the coefficient streamed)
    for (dtype, name), (mode, mtag) in itertools.product(((torch.float64, "fp64"), (torch.float32, "fp32")),
                                                         ((0, ""), (1, "_formed_metric"))):
        P.set_metric_mode(mode)
        s = 8 if dtype == torch.float64 else 4
        geo = 6 if mode == 0 else 1
        for nsets, tag in ((1, mtag), (4, mtag + "_rotated4")):
            xs = [torch.as_tensor(uniform(P.len, seed=7 + i), dtype=dtype, device="cuda") for i in range(nsets)]
            ys = [P.cellvec(dtype) for _ in range(nsets)]
            for i in range(3):
                P.apply(xs[i % nsets], ys[i % nsets])
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for i in range(12):
                P.apply(xs[i % nsets], ys[i % nsets])
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 12
            out["apply_" + name + tag] = {"ms": ms, "gdofs": P.n_dofs / ms / 1e6,
                                          "gbs_algorithmic": (2 * s + geo * s) * P.len / ms / 1e6}
            del xs, ys
    P.set_metric_mode(0)
    # model
    glorot = []
    for i, (no, ni) in enumerate([(64, 64), (64, 64), (12, 64)]):
        lim = (6.0 / (ni + no)) ** 0.5
        glorot += [uniform(no * ni, seed=20 + i, low=-lim, high=lim), [0.0] * no]
    import numpy as np
    p0 = torch.as_tensor(np.concatenate([np.asarray(g, dtype=np.float64) for g in glorot]),
                         dtype=torch.float32, device="cuda")
    P.mlp_set_params(p0)
    t1 = time.perf_counter()
    out["train_final_loss"] = P.mlp_train(X, T, epochs=epochs, batch=256, lr=2e-3, seed=5)
    out["train_s"] = time.perf_counter() - t1
    if with_solve:
        b = P.cellvec()
        P.rhs_manufactured(b)
        cases = (("fp64_jacobi_plain", fe.default_opts(smoother=fe.SMOOTH_JACOBI, inner=fe.F64, omega=0.0,
                                                       nu_pre=2, nu_post=2, tol=1e-10, maxit=400)),
                 ("fp32_chebfdm_averaged", fe.default_opts(smoother=fe.SMOOTH_CHEB_FDM, inner=fe.F32, flexible=1,
                                                           factors=1, nu_pre=1, nu_post=1, tol=1e-10)),
                 ("fp32_chebfdm_learned", fe.default_opts(smoother=fe.SMOOTH_CHEB_FDM, inner=fe.F32, flexible=1,
                                                          factors=2, nu_pre=1, nu_post=1, tol=1e-10)),
                 ("fp32_chebfdm_bestfit", fe.default_opts(smoother=fe.SMOOTH_CHEB_FDM, inner=fe.F32, flexible=1,
                                                          factors=3, nu_pre=1, nu_post=1, tol=1e-10)),
                 ("fp64_chebfdm_averaged", fe.default_opts(smoother=fe.SMOOTH_CHEB_FDM, inner=fe.F64,
                                                           factors=1, nu_pre=1, nu_post=1, tol=1e-10)),
                 ("fp64_chebfdm_learned", fe.default_opts(smoother=fe.SMOOTH_CHEB_FDM, inner=fe.F64,
                                                          factors=2, nu_pre=1, nu_post=1, tol=1e-10)))
        for name, opts in cases:
            out[name] = timed_solve(P, b, opts, "deformed Q%d %d^3 %s" % (k, n, name))
        # the same learned-factor and plain solves with the metric formed in the kernel
        P.set_metric_mode(1)
        for name, opts in cases:
            if name in ("fp32_chebfdm_learned", "fp64_jacobi_plain"):
                out[name + "_formed_metric"] = timed_solve(P, b, opts, "deformed Q%d %d^3 %s, formed metric"
                                                           % (k, n, name))
        P.set_metric_mode(0)
    P.close()
    torch.cuda.empty_cache()
    return out


PAPER_CUBE = {   # Table mg_solve_time (Sec. 6.2), cube rows, A100 80 GB, fp64: context only
    2: {"cg_iters": 8, "mg_mdofs": 522.1, "solve_mdofs": 44.7},
    3: {"cg_iters": 9, "mg_mdofs": 1147.0, "solve_mdofs": 99.5},
    4: {"cg_iters": 10, "mg_mdofs": 662.4, "solve_mdofs": 56.7},
    5: {"cg_iters": 11, "mg_mdofs": 996.5, "solve_mdofs": 77.0},
}


def bench_paper_cube(fe, n=128, degrees=(2, 3, 4, 5)):
    """The paper's cube solve (Sec. 6.2): masked Jacobi V-cycle (omega 0.7, one pre- and one
    post-sweep), FP64, CG until <r, M r> has fallen by 1e-14, on 128^3 cells.  MG throughput =
    DoFs / V-cycle time (events around 10 preconditioner applications), solve throughput =
    DoFs / solve time; DoFs both as the paper estimates them (cells p^3) and exact."""
    import torch
    out = {}
    for p in degrees:
        P = fe.Problem(3, p, n, bc=1)
        b = P.cellvec()
        P.rhs_manufactured(b)
        opts = fe.default_opts(smoother=fe.SMOOTH_JACOBI, inner=fe.F64, omega=0.7, nu_pre=1, nu_post=1,
                               stop=1, tol=1e-14, maxit=100)
        rec = timed_solve(P, b, opts, "paper cube p=%d %d^3" % (p, n))
        e = P.cellvec()
        for _ in range(2):
            P.vcycle(b, e, opts)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            P.vcycle(b, e, opts)
        e1.record()
        torch.cuda.synchronize()
        vc_s = e0.elapsed_time(e1) / 10 * 1e-3
        est = n ** 3 * p ** 3
        rec.update({"vcycle_s": vc_s, "dofs_exact": P.n_dofs, "dofs_paper_estimate": est,
                    "mg_mdofs": est / vc_s / 1e6, "solve_mdofs": est / rec["seconds"] / 1e6,
                    "mg_mdofs_exact": P.n_dofs / vc_s / 1e6, "solve_mdofs_exact": P.n_dofs / rec["seconds"] / 1e6,
                    "paper_a100": PAPER_CUBE[p]})
        log("paper cube p=%d: %d iters, V-cycle %.2f ms (%.0f MDoF/s), solve %.4f s (%.0f MDoF/s)"
            % (p, rec["iters"], vc_s * 1e3, rec["mg_mdofs"], rec["seconds"], rec["solve_mdofs"]))
        out["p%d" % p] = rec
        del b, e
        P.close()
        torch.cuda.empty_cache()
    return out


PAPER_ADAPTIVE = {   # Table mg_adaptive_solve_time (Sec. 6.3), cube, A100 80 GB, fp64: context only
    2: {"cg_iters": 9, "mg_mdofs": 574.2, "solve_mdofs": 52.3},
    3: {"cg_iters": 9, "mg_mdofs": 992.3, "solve_mdofs": 88.8},
    4: {"cg_iters": 10, "mg_mdofs": 605.9, "solve_mdofs": 51.8},
}


def bench_paper_adaptive(fe, degrees=(2, 3, 4), depth_degrees=(2, 3, 4, 5)):
    """Sec. 6.3 on the GPU path: local multigrid (masked Jacobi, omega 0.7, one pre- and one
    post-sweep) as the CG preconditioner on the cube refined toward a sphere surface (centre
    (1/2, 1/2, 1/2), radius 5/16, cells within one cell width of it), FP64, CG until <r, M r>
    has fallen by 1e-14.  (a) Throughput at 6 uniform + 4 adaptive levels (the scale of the
    paper's deepest cube: ~10^5 -- 10^6 cells on each adaptive level); DoFs as the paper
    estimates them, active cells x p^3.  (b) Iterations for 1..4 adaptive refinements at 5
    uniform levels (Table mg_adaptive_iters)."""
    import torch
    out = {"throughput": {}, "iterations_vs_depth": {}}
    opts = fe.default_opts(smoother=fe.SMOOTH_JACOBI, inner=fe.F64, omega=0.7, nu_pre=1, nu_post=1,
                           stop=1, tol=1e-14, maxit=100)
    for p in degrees:
        t0 = time.perf_counter()
        A = fe.Adaptive(p, 6, 4, fe.FEATURE_SPHERE, (0.5, 0.5, 0.5), 0.3125, 1.0)
        create_s = time.perf_counter() - t0
        b = A.vec()
        A.rhs_manufactured(b)
        x = A.vec()
        first = A.pcg(b, x, opts, raise_on_error=False)
        x.zero_()
        rep = A.pcg(b, x, opts, raise_on_error=False)
        z = A.vec()
        for _ in range(2):
            A.precondition(b, z, opts)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            A.precondition(b, z, opts)
        e1.record()
        torch.cuda.synchronize()
        vc_s = e0.elapsed_time(e1) / 10 * 1e-3
        est = A.active_cells * p ** 3
        rec = {"levels_cells": [A.level_cells(l) for l in range(A.n_levels)], "active_cells": A.active_cells,
               "dofs_paper_estimate": est, "create_s": create_s, "iters": rep["iters"],
               "seconds": rep["t_solve"], "first_solve_s": first["t_solve"], "status": rep["status"],
               "vcycle_s": vc_s, "mg_mdofs": est / vc_s / 1e6, "solve_mdofs": est / rep["t_solve"] / 1e6,
               "paper_a100": PAPER_ADAPTIVE[p]}
        log("paper adaptive p=%d: %d active cells, levels %s, setup %.2f s, %d iters, V-cycle %.2f ms (%.0f MDoF/s), "
            "solve %.4f s (%.0f MDoF/s)" % (p, A.active_cells, rec["levels_cells"], create_s, rep["iters"],
                                            vc_s * 1e3, rec["mg_mdofs"], rep["t_solve"], rec["solve_mdofs"]))
        out["throughput"]["p%d" % p] = rec
        del b, x, z
        A.close()
        torch.cuda.empty_cache()
    for p in depth_degrees:
        its = []
        for a in (1, 2, 3, 4):
            A = fe.Adaptive(p, 5, a, fe.FEATURE_SPHERE, (0.5, 0.5, 0.5), 0.3125, 1.0)
            b = A.vec()
            A.rhs_manufactured(b)
            x = A.vec()
            its.append(A.pcg(b, x, opts, raise_on_error=False)["iters"])
            del b, x
            A.close()
            torch.cuda.empty_cache()
        out["iterations_vs_depth"]["p%d" % p] = its
        log("paper adaptive p=%d: CG iterations for 1..4 adaptive refinements %s" % (p, its))
    return out


def copy_bandwidth():
    """A plain device copy (torch's elementwise copy kernel) over 4 rotated pairs of
    1 GiB buffers: the achievable HBM rate of a streaming kernel in this run, in GB/s
    (bytes read + written)."""
    import torch
    n = (1 << 30) // 8
    srcs = [torch.ones(n, dtype=torch.float64, device="cuda") for _ in range(4)]
    dsts = [torch.empty_like(s) for s in srcs]
    for i in range(4):
        dsts[i].copy_(srcs[i])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(20):
        dsts[i % 4].copy_(srcs[i % 4])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 20
    del srcs, dsts
    torch.cuda.empty_cache()
    return 2 * n * 8 / (ms * 1e-3) / 1e9


def cpu_baseline():
    """The oracle timed on the host cores: the plain C FP64 reference of the same
    step (cell-wise Dirichlet apply + vertex-patch inverse, their definitions
    written out, one OpenMP thread per independent output) on the full Q3 64^3
    workload; the numpy oracle on a 16^3 sample if the C oracle cannot be built."""
    import numpy as np
    from oracle.mesh import StructuredMesh
    from synthetic_inputs import uniform
    nproc = os.cpu_count()
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else nproc
    try:
        from oracle import c_oracle
        threads = c_oracle.max_threads()
    except Exception as e:   # no compiler: the numpy oracle on a sample
        log("C oracle unavailable (%s): numpy oracle on a 16^3 sample" % e)
        return cpu_baseline_numpy(nproc, affinity)
    k, n = 3, 64
    m = StructuredMesh(3, k, n)
    O = c_oracle.CartesianOracle(m)
    x = m.gather(uniform(m.n_global, seed=0)).ravel()
    r = uniform(m.n_cellwise, seed=1)
    y, z = np.empty_like(x), np.empty_like(r)
    reps = 0
    t0 = time.perf_counter()
    while True:
        O.apply_dirichlet(x, y)
        O.patch_inverse(r, z)
        reps += 1
        if time.perf_counter() - t0 > 12.0 and reps >= 2:
            break
    dt = (time.perf_counter() - t0) / reps
    return {"value": m.n_global / dt / 1e9, "unit": "GDoF/s", "cores": threads, "kind": "oracle",
            "nproc": nproc, "affinity_cpus": affinity,
            "sample": "Q3 64^3 (%d DoFs, the full workload) apply + patch inverse, FP64, C oracle with %d "
                      "OpenMP threads, %d repetitions in %.1f s" % (m.n_global, threads, reps, dt * reps)}


def cpu_baseline_numpy(nproc, affinity):
    """The numpy/scipy FP64 oracle, unmodified, on a 16^3 sample of the same workload."""
    from oracle.mesh import StructuredMesh
    from oracle.operators import apply_cellwise, assemble_csr, element_matrix_cartesian
    from oracle.patch import patch_inverse_cellwise
    from synthetic_inputs import uniform
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])   # BLAS pool the oracle uses
    except Exception:
        cores = 1
    k, n = 3, 16
    m = StructuredMesh(3, k, n)
    E = element_matrix_cartesian(3, k, m.h)
    A = assemble_csr(m, E)
    x = m.gather(uniform(m.n_global, seed=0))
    r = uniform(m.n_cellwise, seed=1).reshape(m.n_cells, m.n_local)
    reps = 0
    t0 = time.perf_counter()
    while True:
        apply_cellwise(m, E, x)
        patch_inverse_cellwise(A, m, r, shared=True)
        reps += 1
        if time.perf_counter() - t0 > 12.0:
            break
    dt = (time.perf_counter() - t0) / reps
    return {"value": m.n_global / dt / 1e9, "unit": "GDoF/s", "cores": cores, "kind": "oracle",
            "nproc": nproc, "affinity_cpus": affinity,
            "sample": "Q3 16^3 (%d DoFs) apply + patch inverse, FP64, numpy oracle, %d repetitions in %.1f s" %
                      (m.n_global, reps, dt * reps)}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    from paper_2607_03413_amd import fe

    if args.only_pcg:
        print(json.dumps(bench_pcg(fe)))
        return
    if args.only_deformed:
        print(json.dumps(bench_deformed_q7(fe)))
        return
    if args.only_paper:
        print(json.dumps({"cube": bench_paper_cube(fe), "adaptive": bench_paper_adaptive(fe)}))
        return
    if args.only_step and args.step_config != "q3":
        deg, n = (7, 32) if args.step_config.startswith("q7") else (3, 64)
        dtype = torch.float32 if args.step_config.endswith("f32") else torch.float64
        log("Q%d %d^3 %s step" % (deg, n, "FP32" if dtype == torch.float32 else "FP64"))
        print(json.dumps(bench_config(fe, deg, n, dtype, args.steps, args.warmup, nsets=4)))
        return
    log("Q3 64^3 FP64 step")
    main64 = bench_config(fe, 3, 64, torch.float64, args.steps, args.warmup, nsets=4)
    dom = max(main64["kernel_ms"], key=lambda k: main64["kernel_ms"][k])
    if args.only_step:
        if args.with_copy:
            # calibration for the HBM byte counters: a plain copy of a known size
            # (2 x 134,217,728 bytes per launch) next to the kernels of the step
            src = torch.ones(16777216, dtype=torch.float64, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(5):
                torch.mul(src, 1.5, out=dst)    # elementwise kernel: reads and writes 134,217,728 bytes
            torch.cuda.synchronize()
        print(json.dumps(main64))
        return
    log("Q3 64^3 FP32 step")
    main32 = bench_config(fe, 3, 64, torch.float32, args.steps, args.warmup, nsets=4)
    log("Q7 32^3 FP64 / FP32 steps")
    q7_64 = bench_config(fe, 7, 32, torch.float64, max(10, args.steps // 2), args.warmup, nsets=4)
    q7_32 = bench_config(fe, 7, 32, torch.float32, max(10, args.steps // 2), args.warmup, nsets=4)
    pcg = None if args.no_pcg else bench_pcg(fe)
    paper = paper_adaptive = None
    if not args.no_paper:
        log("paper's cube solves, p = 2..5 on 128^3 cells")
        paper = bench_paper_cube(fe)
        log("paper's adaptive cube (local smoothing)")
        paper_adaptive = bench_paper_adaptive(fe)
    copy_gbs = copy_bandwidth()
    log("plain copy: %.0f GB/s" % copy_gbs)
    deformed = {}
    if not args.no_deformed:
        log("deformed Q3 48^3 (apply, learned vs averaged factors)")
        deformed["q3_48cubed"] = bench_deformed(fe, 3, 48, n_train=24, train_meshes=2, epochs=30)
        log("deformed Q7 64^3 end-to-end solves")
        deformed["q7_64cubed"] = bench_deformed_q7(fe)
    cpu = None if args.no_cpu else cpu_baseline()

    # roofline entry for the dominant kernel of the headline step
    k_ms = main64["kernel_ms"][dom]
    P = fe.Problem(3, 3, 64, bc=1)
    bytes_dom = kernel_bytes(P, 8)[dom]
    P.close()
    achieved = bytes_dom / (k_ms * 1e-3) / 1e9
    roof = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom),
            "avg_launch_ms": round(k_ms, 5), "algorithmic_bytes": bytes_dom,
            "copy_gbs_measured": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4)}
    line = {
        "metric": METRIC, "value": round(main64["gdofs"], 4), "unit": "GDoF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(main64["ms_per_step"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "3D Poisson Q3 64^3 Cartesian, fe_apply + patch_fdm_inverse per step",
                   "unique_dofs": main64["n_dofs"], "precision": "fp64", "buffer_sets": 4},
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp32": {"value": round(main32["gdofs"], 4), "ms_per_step": round(main32["ms_per_step"], 5),
                 "kernel_ms": main32["kernel_ms"], "kernel_gbs": main32["kernel_gbs"]},
        "fp64_kernels": {"kernel_ms": main64["kernel_ms"], "kernel_gbs": main64["kernel_gbs"]},
        "q7_32cubed": {"fp64": {"value": round(q7_64["gdofs"], 4), "kernel_ms": q7_64["kernel_ms"]},
                       "fp32": {"value": round(q7_32["gdofs"], 4), "kernel_ms": q7_32["kernel_ms"]},
                       "unique_dofs": q7_64["n_dofs"]},
        "pcg_q7_32cubed": pcg,
        "paper_cube_128cubed": paper,
        "paper_adaptive_cube": paper_adaptive,
        "deformed": deformed,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
