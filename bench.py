"""Benchmark: factor + solve throughput (DOF/s) of spaLU on one MI355X.

A step is one whole pass of the hot path over one batch of synthetic input:
factorization (leaf elimination, per-level IDs and sparsification, segment
LU, separator elimination, merges) followed by the multi-RHS solve with FP64
iterative refinement to the workload's tolerance.  The matrix, right-hand
sides and nested-dissection plan are resident before the timed region
(nested dissection is a closed-form host step, timed and reported apart).

Default workload: the non-symmetric convection-diffusion operator
-0.01 Lap u + (1, 0.5) . grad u, first-order upwind, on the 2047 x 2047
interior grid (N = 4,190,209), eps = 1e-5, 64 right-hand sides uniform in
[-1, 1], classical FP64 refinement (x += M r) to 1e-8.  The headline
`value` is the learned form:
FP32 storage of the factor and FP32 MFMA separator Schur products (FP64
pivoted LU of diagonal blocks, ID CPQR and triangular solve, and refinement
residual), the solve sweeps captured as a HIP graph, and the trained rank
predictor choosing each segment's first sample count or keeping a segment
whole when it predicts no compression.  Beside it: the mixed form (the same
without the predictor) and the plain form (FP64 storage and FP64 MFMA,
adaptive sampling, direct per-level launches).  Each form uses the launch
shapes the autotuner cached for its workload, if any.

A form name with the suffix "-sym" (e.g. --forms learned-sym,plain-sym,plain
on a symmetric positive definite workload) runs that form in the symmetric
variant: one-sided IDs and L D L^T segment factors (Section 4.4.2).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--side", type=int, default=None)
    ap.add_argument("--nrhs", type=int, default=None)
    ap.add_argument("--forms", default=None,
                    help="comma-separated forms, the first one the headline (default: learned,mixed,plain; on the "
                         "symmetric positive definite workloads the symmetric learned form first, and on the 3D "
                         "Laplacian only FP32 forms, whose workspace fits at 127^3)")
    ap.add_argument("--cpu-side", type=int, default=None,
                    help="grid side of the oracle's sample (default 255 in 2D, 23 for the 3D Laplacian)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="direct launches in every form")
    ap.add_argument("--tune", action="store_true",
                    help="search the launch shapes of each form before its warm-up (untimed) and cache them")
    ap.add_argument("--no-tuning", action="store_true", help="the library's default launch shapes, not the cache")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device to device (4 dispatches of a plain copy kernel), to scale "
                         "the FETCH_SIZE / WRITE_SIZE counters of a counter run")
    ap.add_argument("--eps", type=float, default=None, help="override the workload's ID tolerance")
    ap.add_argument("--rho", type=float, default=0.5,
                    help="near-field radius factor of the hybrid sampling (near: distance <= max(1, rho * span))")
    ap.add_argument("--restart", type=int, default=None,
                    help="refinement corrections by flexible GMRES(restart); 0: classical x += M r (default: "
                         "GMRES(8) for the GRF diffusion and Helmholtz families, classical otherwise)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_form(S, P, nd, dev, form, steps, warmup, profile, graph=True, restart=8, rho=0.5, tuning="cache"):
    import numpy as np
    import torch
    base, sym = form[:-4] if form.endswith("-sym") else form, form.endswith("-sym")
    prec = S.FP64 if base == "plain" else S.FP32
    model = None
    if base == "learned":
        from paper_2408_14193_amd import rank_model
        model = rank_model.load(device=dev)
    rp = torch.from_numpy(P.indptr).to(dev)
    ci = torch.from_numpy(P.indices).to(dev)
    v = torch.from_numpy(P.data).to(dev)
    B = torch.from_numpy(np.ascontiguousarray(P.rhs.T)).to(dev)   # (nrhs, n): column-major n x nrhs
    X = torch.empty_like(B)
    tol = P.tol

    def step():
        t0 = time.perf_counter()
        F = S.Factor(nd, rp, ci, v, eps=P.eps, precision=prec, rank_model=model, rho=rho, symmetric=sym)
        t1 = time.perf_counter()
        info, rr = F.solve_into(B, X, tol=tol, max_iter=50, graph=(graph and base != "plain"), restart=restart)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return F, info, rr, t1 - t0, t2 - t1

    # launch shapes: the autotuner's cached choice for this workload (or,
    # with --tune, a fresh search before the warm-up), else the defaults
    from paper_2408_14193_amd import autotune
    key = autotune.workload_key(P.dims, prec, base == "learned", P.nrhs, P.eps, symmetric=sym)
    if tuning == "tune":
        def one():
            t = time.perf_counter()
            F, info, rr, _, _ = step()
            del F
            return time.perf_counter() - t, bool(info["converged"])
        shapes, source = autotune.tune(one, key, reps=3, log=log), "tuned"
    else:
        shapes = autotune.apply_cached(key) if tuning == "cache" else None
        source = "cache" if shapes is not None else "default"
        if shapes is None:
            shapes = S.set_tuning(**S.tuning_default())
    changed = {k: v for k, v in shapes.items() if v != S.tuning_default()[k]}
    log("[%s] launch shapes: %s %s" % (form, source, changed or "(defaults)"))

    # with profiling, the last warm-up step (untimed) times every kernel to
    # find the dominant one; the timed steps carry the events of that kernel
    # only, for its roofline; one more untimed step after them times every
    # kernel for the breakdown
    for i in range(warmup):
        if profile and i == warmup - 1:
            S.profile(True)
        F, info, rr, tf, ts = step()
        log("[%s] warmup %d: factor %.1f ms, solve %.1f ms, %d refinement steps, residual %.2e"
            % (form, i, tf * 1e3, ts * 1e3, info["iterations"], rr.max()))
        del F
    torch.cuda.synchronize()
    if profile and warmup > 0:
        first = S.profile_read()
        S.profile(True)
        S.profile_only(dominant_kernel(first))
    elif profile:
        S.profile(True)
    tfs, tss, its, res = [], [], [], []
    t0 = time.perf_counter()
    for i in range(steps):
        F, info, rr, tf, ts = step()
        tfs.append(tf)
        tss.append(ts)
        its.append(info["iterations"])
        res.append(float(rr.max()))
        last = F
        del F
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    finfo = dict(last.info)
    finfo["flops"], finfo["bytes"] = last.work()
    del last
    prof = S.profile_read() if profile else None
    breakdown = None
    if profile and warmup > 0:
        S.profile(True)
        F, *_ = step()
        del F
        torch.cuda.synchronize()
        breakdown = S.profile_read()
    if profile:
        S.profile(False)
    ms = (t1 - t0) * 1e3 / steps
    log("[%s] %d steps: %.1f ms/step (factor %.1f, solve %.1f), refinement %s, residual %.2e"
        % (form, steps, ms, 1e3 * sum(tfs) / steps, 1e3 * sum(tss) / steps, its, max(res)))
    return dict(ms_per_step=ms, factor_ms=1e3 * sum(tfs) / steps, solve_ms=1e3 * sum(tss) / steps,
                refine_iters=its, max_rel_residual=max(res), factor_info=finfo,
                converged=all(r <= tol for r in res), profile=prof,
                breakdown=breakdown if breakdown is not None else prof,
                breakdown_steps=1 if breakdown is not None else steps,
                tuning=dict(source=source, key=key, changed=changed), X=X.clone())


def measured_traffic(name, form):
    """HBM bytes per launch of kernel `name` from the committed counter runs
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size), or None
    when there is none for this kernel and form or its sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % name)
    if form.startswith("plain") or form.endswith("-sym") or not os.path.exists(path):
        return None
    d = json.load(open(path))
    h = hashlib.sha256()
    for src in d["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return d["traffic_bytes_per_launch"] if h.hexdigest() == d["sources_sha256"] else None


def dominant_kernel(prof):
    """Kernel step with the largest summed event time (the replayed solve
    graph, a composite of many kernels, is not a kernel)."""
    return max(((k, v) for k, v in prof.items() if k != "solve_sweep_graph"), key=lambda kv: kv[1]["ms"])[0]


def roofline(prof, form):
    """Dominant kernel of the timed steps' events; achieved = algorithmic
    bytes per launch / average launch time."""
    name = dominant_kernel(prof)
    st = prof[name]
    avg_ms = st["ms"] / st["launches"]
    bpl = st["bytes"] / st["launches"]
    fpl = st["flops"] / st["launches"]
    gbs = bpl / (avg_ms * 1e-3) / 1e9
    tfs = fpl / (avg_ms * 1e-3) / 1e12
    peak_f = FP64_PEAK_TFS   # every form computes in FP64 (the mixed forms store FP32)
    return dict(kernel=name, bound="hbm", achieved=round(gbs, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbs / HBM_PEAK_GBS, 5), traffic=measured_traffic(name, form),
                launches=st["launches"], avg_launch_ms=round(avg_ms, 4),
                bytes_per_launch=bpl, flops_per_launch=fpl,
                achieved_tflops=round(tfs, 4), flop_frac=round(tfs / peak_f, 5),
                share_of_step=None)


def host_cpu():
    """Logical CPUs of this host and the processor model (lscpu)."""
    import subprocess
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return os.cpu_count() or 1, model


def cpu_baseline(cfg, side, nrhs=None):
    """The FP64 oracle on a bounded sample of the same workload family, with
    the BLAS thread pool on every host core (the oracle's loops are Python
    and single-threaded; its dense products use the pool)."""
    from threadpoolctl import threadpool_info
    from oracle import spalu as O
    from oracle.nd import nd_order
    from workloads import make_config
    P = make_config(cfg, side=side, nrhs=nrhs)
    nd = nd_order(P.dims)
    ncpu, model = host_cpu()
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    t0 = time.perf_counter()
    F = O.factor(nd, P.scipy(), O.Opts(eps=P.eps))
    t1 = time.perf_counter()
    x, it, hist = O.solve(F, P.rhs, tol=P.tol, max_iter=50)
    t2 = time.perf_counter()
    n = P.n
    return dict(value=round(n / (t2 - t0), 2), unit="DOF/s", cores=threads, kind="oracle",
                host=dict(nproc=ncpu, model=model),
                sample="%s %s (%d DOF), %d RHS, eps %g, FP64, refinement to %g: factor %.1f s, "
                       "solve %.1f s (%d refinement steps, residual %.1e); BLAS threads %d of %d logical "
                       "CPUs (%s)" % (P.name, "x".join(map(str, P.dims)), n, P.nrhs, P.eps, P.tol,
                                      t1 - t0, t2 - t1, it, hist[-1].max(), threads, ncpu, model))


def main():
    a = parse()
    ws = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or ws != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    dev = torch.device("cuda:0")
    if a.copy_calibration > 0:
        nb = a.copy_calibration << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied %d bytes 4 times" % nb)
        return
    from paper_2408_14193_amd import spalu as S
    from workloads import make_config
    P = make_config(a.config, side=a.side, nrhs=a.nrhs)
    if a.restart is None:
        a.restart = 8 if a.config in (1, 4) else 0
    if a.eps is not None:
        P.eps = a.eps
    t0 = time.perf_counter()
    nd = S.ND(P.dims)
    t_nd = time.perf_counter() - t0
    log("workload %s %s: N=%d, nrhs=%d, eps=%g, tol=%g, L=%d, ND %.2f s (host)"
        % (P.name, P.dims, P.n, P.nrhs, P.eps, P.tol, nd.L, t_nd))
    if a.forms is None:
        a.forms = {0: "learned-sym,learned,mixed,plain", 1: "learned-sym,learned,mixed,plain",
                   3: "learned-sym,mixed-sym"}.get(a.config, "learned,mixed,plain")
    forms = a.forms.split(",")
    res = {}
    for i, f in enumerate(forms):
        res[f] = run_form(S, P, nd, dev, f, a.steps, a.warmup, profile=(i == 0), graph=not a.no_graph,
                          restart=a.restart, rho=a.rho,
                          tuning="tune" if a.tune else "off" if a.no_tuning else "cache")
    head = forms[0]
    r = res[head]
    value = P.n / (r["ms_per_step"] * 1e-3)
    roof = roofline(r["profile"], head)
    bd, bsteps = r["breakdown"], r["breakdown_steps"]
    total_ms = sum(st["ms"] for st in bd.values()) / bsteps
    roof["share_of_step"] = round(r["profile"][roof["kernel"]]["ms"] / a.steps / r["ms_per_step"], 4)
    out = {
        "metric": "DOF/s factor+solve to 1e-8 rel. residual, mixed/learned vs plain FP64",
        "value": round(value, 1),
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(r["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "storage": "f64" if head.startswith("plain") else "f32",
        "data": "synthetic",
        "config": {"workload": "%s %s, N=%d, %d RHS, eps=%g, refinement to %g, %s form"
                               % (P.name, "x".join(map(str, P.dims)), P.n, P.nrhs, P.eps, P.tol, head),
                   "n": P.n, "nrhs": P.nrhs, "eps": P.eps, "tol": P.tol, "levels": nd.L,
                   "refinement": ("fgmres(%d)" % a.restart) if a.restart > 0 else "classical",
                   "nd_host_s": round(t_nd, 3)},
        "factor_ms": round(r["factor_ms"], 3),
        "solve_ms": round(r["solve_ms"], 3),
        "refine_iters": r["refine_iters"],
        "max_rel_residual": r["max_rel_residual"],
        "converged": r["converged"],
        "launch_shapes": r["tuning"],
        "roofline": roof,
        # per-kernel event times of one fully profiled, untimed warm-up step
        "kernel_ms_per_step": {k: round(v["ms"] / bsteps, 4) for k, v in
                               sorted(bd.items(), key=lambda kv: -kv[1]["ms"])},
        "profiled_kernel_ms_per_step": round(total_ms, 3),
        "factor_stats": {k: r["factor_info"][k] for k in
                         ("sparsified", "sample_passes", "resampled", "max_front", "q_tilde",
                          "flops", "bytes", "workspace_bytes")},
    }
    # each form's solution against the plain FP64 form's (largest relative
    # difference over the right-hand sides), when the plain form ran
    err = {}
    if "plain" in res:
        import torch
        Xp = res["plain"]["X"]
        nrm = torch.linalg.vector_norm(Xp, dim=1)
        for f in forms:
            if f != "plain":
                d = torch.linalg.vector_norm(res[f]["X"] - Xp, dim=1) / nrm
                err[f] = float(d.max())
        out["max_rel_diff_vs_plain_fp64"] = err.get(head)
    for f in forms[1:]:
        rf = res[f]
        vf = P.n / (rf["ms_per_step"] * 1e-3)
        out["%s_form" % f] = {"value": round(vf, 1), "ms_per_step": round(rf["ms_per_step"], 3),
                              "factor_ms": round(rf["factor_ms"], 3), "solve_ms": round(rf["solve_ms"], 3),
                              "refine_iters": rf["refine_iters"],
                              "max_rel_residual": rf["max_rel_residual"], "converged": rf["converged"],
                              "launch_shapes": rf["tuning"]}
        if f in err:
            out["%s_form" % f]["max_rel_diff_vs_plain_fp64"] = err[f]
        out["ratio_%s_vs_%s" % (head, f)] = round(value / vf, 3)
    if not a.no_cpu:
        if a.cpu_side is None:
            a.cpu_side = 23 if a.config == 3 else 255
        log("cpu baseline: oracle on a side-%d sample ..." % a.cpu_side)
        out["cpu_baseline"] = cpu_baseline(a.config, a.cpu_side)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
