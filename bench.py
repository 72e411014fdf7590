#!/usr/bin/env python
"""Benchmark of the EDFA-preconditioned GMRES hot path on one MI355X.

Workload: the 64^3 full-tensor grid (262,144 cells, ~1.05M unknowns) with
K = k1 R diag(1, a^-1/2, a^-1) R^T per cell (Haar R, a log-uniform in [10, 100],
ln k1 a Gaussian random field, sigma 2, correlation length 8 cells), Dirichlet
p = 1 / 0 on x = 0 / 1, no flow elsewhere.  Synthetic, seeded, assembled once on the
device before timing (assembly is not part of the metric).

One step = EDFA stage 1 + stage 2 (dynamic patterns, n_add = 1, n_ent = 6,
post-filtration on H~ with tau = 1e-3) followed by right-preconditioned GMRES(50)
from x0 = 0 to a true relative residual <= 1e-8.  The launch-shape autotuner runs once
per preconditioner before the timed steps (its choices persist across re-setups).
``value`` is the mean wall time of one step in seconds for the FP64 path.  ``forms``
holds the same step with the FP32 preconditioner inside FP64 flexible GMRES and with
Bi-CGStab (the paper's solver); on request (--batched, --transient) also the 256-grid
batch and the 128x128x64 distorted-channel sequence of 10 steps with dt doubling from
1e-3 (FP64 and mixed; stage-2 refresh per step and full re-setup per step).
``roofline`` is the dominant sparse-product kernel of the 64^3 step, timed live with HIP
events inside the solve; ``families`` lists every product.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--batched] [--transient]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "setup+GMRES time to 1e-8 rel residual, FP64 vs mixed/batched; HBM GB/s"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def spmv_bytes(nnz, n):
    """Algorithmic bytes of y = A x in CSR (FP64 values, int32 indices): values and
    column indices once, row pointers once, x once, y once."""
    return 12 * nnz + 4 * (n + 1) + 8 * n + 8 * n


def print_tune_report(rep, tag):
    """One stderr line per timed matrix: the chosen kernel, its time and its rate on the
    algorithmic bytes (values and indices once, row pointers once, x and y once)."""
    for name, r in rep.items():
        vb = r["value_bytes"]
        nbytes = (4 + vb) * r["nnz"] + 4 * (r["rows"] + 1) + vb * (r["cols"] + r["rows"])
        t = r["us"][r["variant"]]
        alt = " ".join(f"{v}:{u:.1f}" for v, u in r["us"].items())
        lay = f"pad {r['sell_padding']:.2f}{' sorted' if r['sell_sorted'] else ''}"
        print(f"[tune {tag}] {name:8s} rows {r['rows']:8d} nnz {r['nnz']:9d} {lay:17s} "
              f"{r['variant']:8s} {t:7.1f} us {nbytes / t / 1e3:6.0f} GB/s  ({alt})",
              file=sys.stderr, flush=True)


def run_form(edfa, S, b, prm, steps, warmup, flexible, method="gmres", P=None):
    import torch
    if P is None:
        P = edfa.Precond(S, prm)
    # one-off choice of SpMV launch shapes, kept across the timed re-setups
    rep = P.autotune(report=True)
    print_tune_report(rep, ("fp32" if prm.precision == 1 else "fp64") + f" {method}")
    kw = dict(rtol=1e-8, restart=50, flexible=flexible, method=method, max_iter=5000)
    for _ in range(warmup):
        P.resetup()
        edfa.solve(S, P, b, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, pinfos = [], []
    for k in range(steps):
        P.resetup()
        x, info, st = edfa.solve(S, P, b, **kw)
        infos.append((info, st))
        pinfos.append(P.info())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # after the timed steps: one solve with events around the system products and the
    # applications, one with events around every product (the events themselves add a few
    # microseconds per product, so the timed steps run without them)
    _, i1, _ = edfa.solve(S, P, b, profile=1, **kw)
    _, i2, _ = edfa.solve(S, P, b, profile=2, **kw)
    info, st = infos[-1]
    for k in ("spmv_avg_ms", "spmv_count", "apply_avg_ms", "apply_count"):
        info[k] = i1[k]
    info["slot_ms"], info["slot_launches"] = i2["slot_ms"], i2["slot_launches"]
    info["apply_count_products"] = i2["apply_count"]
    return (t1 - t0) / steps, infos, pinfos, x, rep


def kernel_label(variant, what="the system matrix", role=0, value_bytes=8):
    """Kernel (as traces name it) that runs a product for a tuner choice."""
    kind, depth = variant.split("/")
    t = "double, double" if value_bytes == 8 else "float, float"
    if kind == "sell":
        return f"k_spmv_sell<{t}, {role}, {depth}>: SELL-64 SpMV with {what}"
    if kind == "chunk":
        return f"k_spmv_chunk<{t}, {depth}>: row-chunk SpMV with {what}"
    return (f"k_spmv_csr_vec<{t}, {kind[3:]}, {depth}>: CSR SpMV with {what}, "
            f"{kind[3:]} lanes per row")


def run_batched(edfa, inputs, steps, warmup):
    """The 256-grid batch (cube sides U{8..32}, sigma_lnK ~ U[0.5, 3]), EDFA dynamic (1, 4),
    each grid to a relative residual of 1e-8.  Three forms, each timed as setup + solve:
    the plain FP64 path grid by grid (one system per grid, one step), one batched FP64
    system, and the batched FP32-preconditioner FGMRES with graph-captured cycles."""
    import torch
    probs = inputs.batch_problems(256, 8, 32)
    cells = sum(p.n_cells for p in probs)
    prm64 = edfa.Params("dynamic", n_add=1, n_ent=4)
    prm32 = edfa.Params("dynamic", n_add=1, n_ent=4, precision=1)

    def timed(S, P, b, flexible, graph, k, w):
        for _ in range(w):
            P.resetup()
            edfa.solve(S, P, b, rtol=1e-8, restart=50, flexible=flexible, use_graph=graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            P.resetup()
            x, info, st = edfa.solve(S, P, b, rtol=1e-8, restart=50, flexible=flexible,
                                     use_graph=graph)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k, info, st

    # grid by grid, plain FP64 (systems assembled beforehand; one step after one warm-up)
    singles = []
    for p in probs:
        S1 = edfa.System(p)
        singles.append((S1, edfa.Precond(S1, prm64), S1.rhs()))
    for S1, P1, b1 in singles:
        edfa.solve(S1, P1, b1, rtol=1e-8, restart=50)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    conv_single = 0
    for S1, P1, b1 in singles:
        P1.resetup()
        x1, i1, st1 = edfa.solve(S1, P1, b1, rtol=1e-8, restart=50)
        conv_single += int(st1 == 0)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    del singles

    S = edfa.System(probs)
    b = S.rhs()
    P64 = edfa.Precond(S, prm64)
    P64.autotune()
    t64, i64, st64 = timed(S, P64, b, False, False, steps, warmup)
    del P64
    P32 = edfa.Precond(S, prm32)
    P32.autotune()
    t32, i32, st32 = timed(S, P32, b, True, True, steps, warmup)
    log(f"batch of 256: grid by grid {t_single:.3f} s, batched FP64 {t64:.3f} s, "
        f"batched mixed + graph {t32:.3f} s")
    return {"workload": "batch_256_lognormal_iso_8..32", "grids": 256, "cells": cells,
            "unknowns": S.info["n"],
            "grid_by_grid_fp64_s": t_single, "grid_by_grid_converged": conv_single,
            "batched_fp64_s": t64, "batched_fp64_converged": i64["converged"],
            "batched_fp64_iterations_max": i64["iterations"],
            "batched_mixed_graph_s": t32, "batched_mixed_graph_converged": i32["converged"],
            "batched_mixed_graph_iterations_max": i32["iterations"]}


def run_transient(edfa, inputs, nsteps=10):
    """128x128x64 distorted hexahedra with binary channels (contrast 1e6, 30% volume): a
    sequence of `nsteps` steps with dt doubling from 1e-3 (eq. delta_t_dyn with dt_mult = 2
    and no pressure goal), p_n the previous step's pressure, through edfa_transient.  The
    preconditioner is refreshed by stage 2 only (stage 1 does not depend on dt) or rebuilt
    fully every step; FP64 GMRES and the FP32-preconditioner FGMRES form.  Times are whole
    sequences (setup included); chi_inf per step and its mean are reported."""
    import torch
    prob = inputs.channel_problem(128, 128, 64, contrast=1e6, perturb=0.2, dt=1e-3)
    out = {"workload": "channels_distorted_128x128x64", "cells": prob.n_cells, "steps": nsteps,
           "channel_fraction": prob.meta.get("channel_fraction")}
    for name, prec, flex in (("fp64", 0, False), ("mixed", 1, True)):
        prm = edfa.Params("dynamic", n_add=1, n_ent=6, tau=1e-3, filt="post_H", precision=prec)
        for refresh, every in (("stage2", 0), ("full", 1)):
            S = edfa.System(prob)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P = edfa.Precond(S, prm)
            u, steps, st = edfa.transient(S, P, n_steps=nsteps, dt0=1e-3, dt_mult=2.0,
                                          porosity=inputs.PHI, stage1_every=every,
                                          flexible=flex)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            iters = [r["iterations"] for r in steps]
            chi = [r["chi_inf"] for r in steps]
            log(f"transient {name} refresh={refresh}: {t:.3f} s for {len(steps)} steps, "
                f"iterations {iters}")
            out[f"{name}_{refresh}"] = {
                "s": t, "iterations": iters, "converged_steps": sum(r["converged"] for r in steps),
                "dt": [r["dt"] for r in steps], "chi_inf": chi,
                "chi_inf_mean": sum(chi) / len(chi) if chi else 0.0,
                "setup_ms": [round(r["t_setup_ms"], 3) for r in steps],
                "solve_ms": [round(r["t_solve_ms"], 3) for r in steps]}
            del P, S
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(iters_gpu, n_full, ne_full, n_sample=16):
    """Time the oracle on a bounded sample of the workload family: the whole oracle pipeline
    on the n_sample^3 member (same field statistics, correlation length scaled with the
    grid), with the per-cell restricted solves of stage 1 spread over every core this
    process may run on (a process pool, the paper's parfor); stage 2 and GMRES as the oracle
    runs them.  The measured rates are scaled to the 64^3 step: setup per cell, solve per
    iteration and unknown at the GPU iteration count."""
    cores = len(os.sched_getaffinity(0))
    code = r"""
import json, sys, time
sys.path.insert(0, %r)
from paper_2009_13916_amd import inputs
from oracle import edfa, krylov, mhfe
if __name__ == "__main__":
    n = %d
    p = inputs.full_tensor_problem(n, sigma=2.0, corr=8.0 * n / 64)
    s = mhfe.assemble(p)
    prm = edfa.Params("dynamic", n_add=1, n_ent=6, tau=1e-3, filt="post_H")
    t0 = time.perf_counter(); st1 = edfa.stage1(s, prm, workers=%d); t1 = time.perf_counter()
    st2 = edfa.stage2(s, st1, prm); t2 = time.perf_counter()
    E = edfa.Edfa(s, prm, st1, st2); A = s.matrix()
    t3 = time.perf_counter(); r = krylov.gmres(lambda v: A @ v, E.apply, s.b, 1e-8, 50); t4 = time.perf_counter()
    print(json.dumps({"stage1": t1 - t0, "stage2": t2 - t1, "solve": t4 - t3,
                      "iters": r.iterations, "n": s.n, "ne": s.ne}))
""" % (ROOT, n_sample, cores)
    path = os.path.join("/tmp", f"edfa_cpu_baseline_{os.getpid()}.py")
    with open(path, "w") as f:
        f.write(code)
    try:
        out = subprocess.run([sys.executable, path], capture_output=True, text=True, timeout=900)
    finally:
        os.unlink(path)
    if out.returncode != 0:
        log("cpu baseline failed: " + out.stderr[-500:])
        return None
    d = json.loads(out.stdout.strip().splitlines()[-1])
    setup = (d["stage1"] + d["stage2"]) * ne_full / d["ne"]
    solve = d["solve"] / (d["iters"] * d["n"]) * iters_gpu * n_full
    return {"value": setup + solve, "unit": "s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": (f"oracle pipeline on the {n_sample}^3 member of the workload family "
                       f"({d['ne']} cells; stage 1 {d['stage1']:.2f} s over a pool of {cores} "
                       f"processes, stage 2 {d['stage2']:.2f} s and {d['iters']} GMRES "
                       f"iterations in {d['solve']:.2f} s in one process), setup scaled per "
                       f"cell and solve per iteration and unknown to 64^3 at the GPU iteration "
                       f"count ({iters_gpu})")}


COPY_BYTES = 1 << 30   # bytes read (and written) by the calibration copy
TRAFFIC = os.path.join(ROOT, "profiles", "spmv_kernels_full_tensor_64cubed_traffic.md")


def slot_bytes(r):
    """Algorithmic bytes of one product with a tuned matrix (values and indices once, row
    pointers once, x and y once)."""
    vb = r["value_bytes"]
    return (4 + vb) * r["nnz"] + 4 * (r["rows"] + 1) + vb * (r["cols"] + r["rows"])


def spmv_kernel_sha():
    """SHA-256 of the source of the sparse-product kernels (SELL, CSR and chunk kernels): a
    traffic figure measured on another version of them is not reported."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2009_13916_amd", "csrc", "sparse.hip")).read()
    a = src.index("void k_spmv_sell(")
    e = src.index("// Launch helper: the extended launch")
    return hashlib.sha256(src[a:e].encode()).hexdigest()[:16]


def measured_traffic(kernel, fam):
    """HBM bytes per launch of `kernel` (its trace name) over the matrices it multiplied in
    the profiled solve (`fam` rows), weighted by their launches, from the per-matrix figures
    of the committed PMC summary; None when the summary is absent, was taken on another
    version of the kernels, or lacks one of those matrices with this same kernel."""
    if not os.path.exists(TRAFFIC):
        return None
    txt = open(TRAFFIC).read()
    try:
        blob = txt[txt.index("```json") + 7:]
        d = json.loads(blob[:blob.index("```")])
    except ValueError:
        return None
    if d.get("kernel_sha") != spmv_kernel_sha():
        return None
    meas = d.get("matrices", {})
    tot = n = 0
    for f in fam:
        if f["kernel"] != kernel:
            continue
        m = meas.get(f["matrix"])
        if not m or m.get("kernel") != kernel:
            return None
        tot += m["hbm_bytes_per_launch"] * f["launches"]
        n += f["launches"]
    return tot / n if n else None


# Kernels of the products in the counter passes: those the tuner keeps on the 64^3 workload
# in unprofiled runs (under the counter passes every launch is serialised, which distorts
# the tuner's own timings, so the passes pin the kernels instead of tuning).
PROBE_VARIANTS = {"A": "sell/4", "G_F": "sell/4", "G_F^T": "sell/4", "A_ppi": "sell/4",
                  "A_pip": "sell/4", "M_L": "chunk/12", "M_U": "chunk/12"}


def probe(torch, edfa, S, b, what):
    """Launches counted by the FETCH_SIZE / WRITE_SIZE passes: the workload's preconditioner
    with the product kernels pinned to PROBE_VARIANTS, then 'spmv': 20 products with the
    system matrix, or 'apply': 20 applications.  Then one device copy of COPY_BYTES (reads
    and writes COPY_BYTES) that calibrates the counters.  Prints, per matrix, the
    algorithmic bytes and the kernel of its product, and the order of the products inside
    one application."""
    rec = {"probe": what, "launches": 20, "copy_bytes": COPY_BYTES, "kernel_sha": spmv_kernel_sha()}
    P = edfa.Precond(S, edfa.Params("dynamic", n_add=1, n_ent=6, tau=1e-3, filt="post_H"))
    for k, v in PROBE_VARIANTS.items():
        P.set_variant(v, k)
    torch.cuda.synchronize()
    if what == "spmv":
        for _ in range(20):
            S.spmv(b)   # the system matrix with the pinned kernel
        names = ["A"]
    else:
        for _ in range(20):
            P.apply(b)
        # order of the products inside one application (eq. EDFA_prec)
        rec["apply_order"] = ["G_F", "G_F^T", "A_ppi", "M_L", "M_U", "A_pip", "G_F", "G_F^T"]
        names = ["G_F", "G_F^T", "A_ppi", "M_L", "M_U", "A_pip"]
    pi, si = P.info(), S.info
    nfu, ne = si["nfu"], si["ne"]
    shape = {"A": (si["n"], si["n"], si["nnz"]),
             "G_F": (nfu, nfu, pi["nnz_GF"]), "G_F^T": (nfu, nfu, pi["nnz_GF"]),
             "A_ppi": (ne, nfu, si["nnz_block"][2]), "A_pip": (nfu, ne, si["nnz_block"][1]),
             "M_L": (ne, ne, pi["nnz_ML"]), "M_U": (ne, ne, pi["nnz_MU"])}
    rec["products"] = {}
    for k in names:
        r, c, z = shape[k]
        rec["products"][k] = {
            "bytes": slot_bytes({"value_bytes": 8, "rows": r, "cols": c, "nnz": z}), "rows": r,
            "kernel": kernel_label(PROBE_VARIANTS[k], k, 0 if k == "A" else 1).split(":")[0]}
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps(rec), flush=True)


def families(info, rep, apply_count):
    """Per matrix of a profiled solve: its kernel, algorithmic bytes, mean launch time (HIP
    events on the solve stream), rate and fraction of peak, and time per step; per kernel
    symbol: the totals.  Returns (per-matrix list, per-kernel dict)."""
    rows, kern = [], {}
    for name, ms in info["slot_ms"].items():
        if name not in rep:
            continue
        r = rep[name]
        n = info["slot_launches"][name]
        by = slot_bytes(r)
        label = kernel_label(r["variant"], name, 0 if name in ("A", "A^T") else 1,
                             r["value_bytes"])
        sym = label.split(":")[0]
        gbs = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        rows.append({"matrix": name, "kernel": sym, "bytes_per_launch": by,
                     "avg_launch_us": round(ms * 1e3, 2), "launches": n,
                     "per_apply": round(n / apply_count, 3) if apply_count else None,
                     "GB_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "ms_per_step": round(ms * n, 3)})
        k = kern.setdefault(sym, {"bytes": 0.0, "ms": 0.0, "launches": 0, "matrices": []})
        k["bytes"] += by * n
        k["ms"] += ms * n
        k["launches"] += n
        k["matrices"].append(name)
    return rows, kern


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=64, help="grid side (64 = the benchmark workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-bicgstab", action="store_true")
    # The 256-grid batch and the 128x128x64 sequence run only on request: a default run that
    # included them once ended in a GPU memory fault whose cause has not been found, so they
    # stay out of the default run until it is.  --no-batched / --no-transient are accepted
    # (and do nothing) for older command lines.
    ap.add_argument("--batched", action="store_true", help="also run the 256-grid batch forms")
    ap.add_argument("--transient", action="store_true",
                    help="also run the 128x128x64 ten-step sequence")
    ap.add_argument("--no-batched", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-transient", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--batched-only", action="store_true",
                    help="diagnostic: run only the 256-grid batch forms and print their record")
    ap.add_argument("--transient-only", action="store_true",
                    help="diagnostic: run only the 128x128x64 ten-step sequence")
    ap.add_argument("--probe", choices=["spmv", "apply"], default=None,
                    help="run only the launches that PMC passes count: 'spmv' = 20 system "
                         "products, 'apply' = setup and 20 preconditioner applications; "
                         "each then one plain copy of known size")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the solver does not "
              "shard a system over several GPUs.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2009_13916_amd import edfa, inputs
    edfa.load()
    torch.cuda.set_device(0)
    if args.transient_only:
        print(json.dumps({"forms": {"transient_128x128x64": run_transient(edfa, inputs)}}),
              flush=True)
        return
    if args.batched_only:
        print(json.dumps({"forms": {"batch_256": run_batched(edfa, inputs, args.steps,
                                                             args.warmup)}}), flush=True)
        return
    n = args.n
    log(f"building the {n}^3 full-tensor workload")
    prob = inputs.full_tensor_problem(n, sigma=2.0, corr=8.0 * n / 64)
    S = edfa.System(prob)
    b = S.rhs()
    torch.cuda.synchronize()
    if args.probe:
        probe(torch, edfa, S, b, args.probe)
        return
    nnz, N, ne = S.info["nnz"], S.info["n"], S.info["ne"]
    log(f"assembled: N={N} nnz={nnz}")
    prm = edfa.Params("dynamic", n_add=1, n_ent=6, tau=1e-3, filt="post_H")
    t64, infos, pinfos, x, rep64 = run_form(edfa, S, b, prm, args.steps, args.warmup,
                                            flexible=False)
    info, st = infos[-1]
    pi = pinfos[-1]
    log(f"fp64: {t64:.4f} s/step, {info['iterations']} iterations, relres {info['relres_true']:.2e}")
    log("preconditioner: " + ", ".join(f"{k} {v}" for k, v in pi.items()))
    forms = {"fp64": {"s_per_step": t64, "iterations": info["iterations"],
                      "relres_true": info["relres_true"], "converged": st == 0,
                      "stage1_ms": pi["t_stage1_ms"], "stage2_ms": pi["t_stage2_ms"],
                      "solve_ms": info["t_solve_ms"], "mu": pi["mu"], "colors": pi["n_colors"],
                      "nnz_H_raw": pi["nnz_H_raw"], "nnz_H": pi["nnz_H"],
                      "apply_avg_us": round(info["apply_avg_ms"] * 1e3, 2)}}
    if not args.no_mixed:
        prm32 = edfa.Params("dynamic", n_add=1, n_ent=6, tau=1e-3, filt="post_H", precision=1)
        t32, i32, p32, x32, rep32 = run_form(edfa, S, b, prm32, args.steps, args.warmup,
                                             flexible=True)
        inf32, st32 = i32[-1]
        fam32, _ = families(inf32, rep32, inf32["apply_count_products"])
        dp = (x32 - x)[S.info["nfu"]:].norm() / x[S.info["nfu"]:].norm()
        log(f"mixed: {t32:.4f} s/step, {inf32['iterations']} iterations")
        forms["mixed_fp32_precond_fgmres"] = {
            "s_per_step": t32, "iterations": inf32["iterations"], "relres_true": inf32["relres_true"],
            "converged": st32 == 0, "stage1_ms": p32[-1]["t_stage1_ms"],
            "stage2_ms": p32[-1]["t_stage2_ms"], "solve_ms": inf32["t_solve_ms"],
            "apply_avg_us": round(inf32["apply_avg_ms"] * 1e3, 2),
            "pressure_rel_diff_vs_fp64": float(dp), "families": fam32}
    if not args.no_bicgstab:
        tb, ib, pb, xb, _ = run_form(edfa, S, b, prm, args.steps, args.warmup, flexible=False,
                                     method="bicgstab")
        infb, stb = ib[-1]
        dpb = (xb - x)[S.info["nfu"]:].norm() / x[S.info["nfu"]:].norm()
        log(f"bicgstab: {tb:.4f} s/step, {infb['iterations']} iterations")
        forms["fp64_bicgstab"] = {
            "s_per_step": tb, "iterations": infb["iterations"], "relres_true": infb["relres_true"],
            "converged": stb == 0, "solve_ms": infb["t_solve_ms"],
            "pressure_rel_diff_vs_gmres": float(dpb)}
    off = "not in the default run (an unexplained GPU fault in a default run with it); --%s"
    if args.batched and not args.no_batched:
        forms["batch_256"] = run_batched(edfa, inputs, args.steps, args.warmup)
    else:
        forms["batch_256"] = {"skipped": off % "batched"}
    if args.transient and not args.no_transient:
        forms["transient_128x128x64"] = run_transient(edfa, inputs)
    else:
        forms["transient_128x128x64"] = {"skipped": off % "transient"}

    # per-matrix product timings of the last profiled FP64 step and the dominant kernel
    fam, kern = families(info, rep64, info["apply_count_products"])
    dom = max(kern, key=lambda k: kern[k]["ms"])
    K = kern[dom]
    achieved = K["bytes"] / (K["ms"] * 1e-3) / 1e9
    for f in sorted(fam, key=lambda r: -r["ms_per_step"]):
        log(f"product {f['matrix']:8s} {f['kernel']:40s} {f['avg_launch_us']:8.2f} us "
            f"{f['GB_s']:7.1f} GB/s ({f['frac']:.3f})  x{f['launches']}  {f['ms_per_step']:.2f} ms/step")
    apply_bytes = sum(f["bytes_per_launch"] * f["launches"] for f in fam
                      if f["matrix"] not in ("A", "A^T")) / max(1, info["apply_count_products"])
    apply_kernel_us = sum(f["avg_launch_us"] * f["launches"] for f in fam
                          if f["matrix"] not in ("A", "A^T")) / max(1, info["apply_count_products"])
    apply_gbs = apply_bytes / (info["apply_avg_ms"] * 1e-3) / 1e9 if info["apply_avg_ms"] else 0.0
    spmv_ms = info["spmv_avg_ms"]
    ab = spmv_bytes(nnz, N)
    out = {
        "metric": METRIC, "value": t64, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t64 * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"full_tensor_grf_{n}^3", "cells": ne, "unknowns": N, "nnz": nnz,
                   "edfa": "dynamic (n_add 1, n_ent 6), post-filtration on H~ 1e-3",
                   "krylov": "GMRES(50), x0 = 0", "rtol": 1e-8},
        "iterations": info["iterations"], "relres_true": info["relres_true"],
        "forms": forms,
        "roofline": {"bound": "hbm", "kernel": dom,
                     "matrices": K["matrices"],
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom, fam),
                     "bytes_per_launch": K["bytes"] / K["launches"],
                     "avg_launch_ms": K["ms"] / K["launches"], "launches": K["launches"]},
        "families": fam,
        "apply": {"bytes": apply_bytes, "avg_us": round(info["apply_avg_ms"] * 1e3, 2),
                  "GB_s": round(apply_gbs, 1), "frac": round(apply_gbs / HBM_PEAK_GBS, 4),
                  "launches": info["apply_count"],
                  "kernel_us": round(apply_kernel_us, 2),
                  "kernel_frac": round(apply_bytes / (apply_kernel_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)},
        "system_spmv": {"bytes": ab, "avg_us": round(spmv_ms * 1e3, 2),
                        "GB_s": round(ab / (spmv_ms * 1e-3) / 1e9, 1) if spmv_ms else 0.0},
    }
    if not args.no_cpu_baseline:
        log("timing the oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(info["iterations"], N, ne)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
