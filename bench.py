"""Benchmark: direct approximate factoring AW ~ V + right-preconditioned
BiCGSTAB on the 64^3 convection-diffusion workload (n = 262144, W pattern
pattern(A^2), V = diagonal + top-4 |A w0| rows of the lower triangle of the
shadow, unit-norm-v mode), learned vs plain W pattern, one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode unit_v|unit_w]

A step is one pass of the hot path on device-resident A and b: W pattern ->
factor (all columns) -> V assembly -> BiCGSTAB to 1e-8.  `value` is
columns factored and solved per second over the step; the factoring pass
alone, the solve, BiCGSTAB iterations and the learned-pattern variant are
reported beside it, with the factor kernel's roofline and the CPU oracle's
rate on the host cores.
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

import numpy as np  # noqa: E402

WORKLOAD = "convdiff3d_64"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6  # vector FP64, MI355X


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(A, Jri, lcount, sv):
    """Per-column compulsory traffic of the factoring pass, summed: gather of
    A(:, J_j) (values + row indices + the colptr pair of each column), the
    J_j read, the W write, the V write (values + rows) and r_j."""
    cn = np.diff(A.colptr).astype(np.int64)
    gathered = int(cn[Jri].sum())
    k = len(Jri)
    total = gathered * (sv + 4) + 8 * k + 4 * k + k * (sv + 4) + int(lcount.sum()) * (sv + 4) \
        + 8 * A.n
    return total, gathered


def algorithmic_flops(A, Jcp, Jri, lcount, mode):
    """FP64 operations of the factoring pass, summed over columns (complex
    counted as 4 real): the Gram matrix over the sparse B_j (each row r of
    B_j with c_r entries adds c_r (c_r + 1) to the Hermitian upper
    triangle), then for unit-norm v a Cholesky k^3/3, the triangular solves
    with 1 + l right-hand sides 2 k^2 (1 + l), H = B_L Y 2 l^2 k and an l x l
    Jacobi (7 sweeps of 6 l^3); for unit-norm w the downdate 2 l k^2 and two
    k x k Jacobi eigen-solves (7 sweeps of 6 k^3 each); plus the residual
    2 nnz(B_j)."""
    import scipy.sparse as sp
    n = A.n
    P = sp.csc_matrix((np.ones(A.nnz), A.rowidx, A.colptr), shape=(n, n))
    S = sp.csc_matrix((np.ones(len(Jri)), Jri, Jcp), shape=(n, n))
    C = (P @ S).tocsc()  # C[r, j] = number of columns of B_j holding row r
    c = C.data
    cols = np.repeat(np.arange(n), np.diff(C.indptr))
    gram = np.bincount(cols, weights=c * (c + 1.0), minlength=n)
    nnzb = np.bincount(cols, weights=c, minlength=n)
    k = np.diff(Jcp).astype(np.float64)
    l = np.asarray(lcount, dtype=np.float64)
    if mode == "unit_v":
        f = gram + k ** 3 / 3 + 2 * k ** 2 * (1 + l) + 2 * l ** 2 * k + 42 * l ** 3 + 2 * nnzb
    else:
        f = gram + 2 * l * k ** 2 + 84 * k ** 3 + 2 * nnzb
    return float(f.sum()) * (4.0 if A.is_complex else 1.0)


def kernel_source_sha(kernel):
    """sha256 over the sources a factor kernel is compiled from."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1208_3573_amd", "csrc")
    files = {"factor_small_kernel": ["factor_small.hip", "dcommon.h", "factor_kernels.h"],
             "factor_generic_kernel": ["factor_generic.hip", "dcommon.h", "factor_kernels.h"]}[kernel]
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload, mode):
    """HBM bytes per factoring pass from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel factor), or
    None when there is none or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}__{workload}_{mode}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != kernel_source_sha(kernel):
        return None
    try:
        return float(vals["traffic_bytes_per_pass"])
    except (KeyError, ValueError):
        return None


def copy_calibration():
    """A plain device copy of known size, for scaling rocprofv3's
    FETCH_SIZE / WRITE_SIZE counters: 3 launches, 1 GiB read + 1 GiB written
    each."""
    import torch
    nbytes = 1 << 30
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_launch": nbytes, "copy_bytes_written_per_launch": nbytes,
                      "launches": 3}), flush=True)


# Method variants on the 64^3 matrix (the rows beyond the headline
# configuration): Algorithm 1 with the paper's parameters (k = 3, tau_i = 0.1),
# Algorithm 2 with the Gauss-Seidel V_0, the Section 3.2 constraint, the
# Section 3.1 leverage rule, block diagonal V on the x-lines of the grid (64
# rows per block) with the pattern of D or the top-k rows of the block, and
# the left variant.
VARIANTS = {
    "alg1": dict(w="sparsified", v="topk_lower", v_count=5,
                 sparsify=dict(k=3, tau_i=0.1, p_i=0, tau_l=0.0, p_l=0)),
    "alg2_gs": dict(w="alg2_gs_lower", v="topk_lower", v_count=5),
    "stab": dict(w="A2", v="topk_lower", v_count=5, stab_r=2.0),
    "lev": dict(w="A2", v="lev_lower", v_count=5),
    "block_d": dict(w="A2", v="block", blocks=64),
    "block_topk": dict(w="A2", v="topk_block", v_count=5, blocks=64),
    "left": dict(w="A2", v="topk_lower", v_count=5, left=True),
}


def cpu_baseline(A, J, mode, v, l, upper, b):
    """The oracle as it stands, on all host cores, on the full workload once
    (factor + BiCGSTAB)."""
    import oracle
    nth = oracle.nthreads_default()
    t0 = time.perf_counter()
    F = oracle.factor(A, J, mode, v, l, nthreads=nth)
    t1 = time.perf_counter()
    _, info = oracle.bicgstab(A, b, F, upper=upper)
    t2 = time.perf_counter()
    return dict(value=A.n / (t2 - t0), unit="columns/s", cores=nth, kind="oracle",
                sample=f"full {WORKLOAD} workload once: factor {t1 - t0:.2f} s + "
                       f"BiCGSTAB {t2 - t1:.2f} s ({info.iters} its)",
                factor_cols_per_s=A.n / (t1 - t0), iters=info.iters)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="unit_v", choices=["unit_v", "unit_w"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--opt", action="append", default=[], metavar="KEY=VALUE",
                    help="library context option, e.g. trsv_waves=8")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in launch shapes instead of tuning them first")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the known-size copy used to scale the HBM counters")
    ap.add_argument("--variants", default="",
                    help="comma-separated extra configurations timed on the same matrix after "
                         "the main line (reported under 'variants'): " + ", ".join(VARIANTS))
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for {args.gpus}); the "
              "multi-GPU layout is described in DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1208_3573_amd import diaf
    from paper_1208_3573_amd import learned as LR

    cfg = synth.WORKLOADS[WORKLOAD]
    A = synth.workload_matrix(WORKLOAD)
    b = synth.rhs_ones(A)
    upper = cfg["v"].endswith("upper")
    ctx = diaf.Context(0)
    for kv in args.opt:
        k, v = kv.split("=", 1)
        ctx.set_option(k, int(v))
    dA = diaf.DeviceCSC.from_host(A)
    db = torch.from_numpy(b).cuda()
    x = torch.zeros_like(db)
    spec = diaf.make_spec(w=cfg["w"], v=cfg["v"], v_count=cfg["v_count"])
    tuned = None
    if not args.no_autotune:
        # launch shapes picked on this problem, before (and outside) the timed steps
        t0 = time.perf_counter()
        tuned = diaf.diaf_autotune(ctx, dA, spec, args.mode)
        tuned["seconds"] = time.perf_counter() - t0
        log(f"autotune: {tuned}")

    def step(spec_):
        t0 = time.perf_counter()
        F = diaf.diaf_factor(ctx, dA, spec_, args.mode)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        info = diaf.diaf_solve(ctx, dA, F, db, x, 1e-8, 1000)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        st = F.stats()
        return F, st, info, (t1 - t0) * 1e3, (t2 - t1) * 1e3

    for _ in range(args.warmup):
        F, st, info, fms, sms = step(spec)
        log(f"warmup: factor {fms:.1f} ms, solve {sms:.1f} ms, {info.iters} its")
        F.close()
    torch.cuda.synchronize()
    recs = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        F, st, info, fms, sms = step(spec)
        log(f"step: factor {fms:.1f} ms, solve {sms:.1f} ms, {info.iters} its")
        recs.append((st.ms_factor_kernels, st.ms_pattern, st.ms_factor, st.ms_assemble, fms, sms,
                     info.iters, info.relres_true, st.factor_launches))
        last = F
        if len(recs) < args.steps:
            F.close()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_step = t_total * 1e3 / args.steps
    R = np.array(recs, dtype=float)
    kern_ms = float(np.mean(R[:, 0]))
    factor_ms = float(np.mean(R[:, 4]))
    solve_ms = float(np.mean(R[:, 5]))
    iters = int(R[-1, 6])
    st = last.stats()
    levels = last.levels()  # diagnostic depth of the V solve, taken after the timed steps
    H = last.to_host()
    sv = 16 if A.is_complex else 8
    bytes_alg, gathered = algorithmic_bytes(A, H["Wri"], H["lcount"], sv)
    launches = max(1, int(R[-1, 8]))
    achieved = bytes_alg / (kern_ms * 1e-3) / 1e9
    flops_alg = algorithmic_flops(A, H["Wcp"], H["Wri"], H["lcount"], args.mode)
    tflops = flops_alg / (kern_ms * 1e-3) / 1e12
    kname = "factor_small_kernel" if (st.count_deferred == 0 and launches == 1) \
        else "factor_generic_kernel"
    traffic = measured_traffic(kname, WORKLOAD, args.mode)
    out = {
        "metric": "columns factored/s + factor+solve time to 1e-8, learned vs plain, 1 GPU",
        "value": A.n / (ms_step * 1e-3),
        "unit": "columns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": A.n, "nnz": A.nnz, "w_pattern": cfg["w"],
                   "v_pattern": f"{cfg['v']} l={cfg['v_count']}", "mode": args.mode,
                   "rhs": "A*ones", "rtol": 1e-8},
        "factor_ms": factor_ms,
        "factor_kernel_ms": kern_ms,
        "factor_cols_per_s": A.n / (factor_ms * 1e-3),
        "factor_kernel_cols_per_s": A.n / (kern_ms * 1e-3),
        "solve_ms": solve_ms,
        "bicgstab_iters": iters,
        "relres_true": float(R[-1, 7]),
        "nrm": st.nrm,
        "v_levels": levels,
        "autotuned": tuned,
        "roofline": ({"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": achieved / HBM_PEAK_GBS, "traffic": traffic}
                     if bytes_alg / (HBM_PEAK_GBS * 1e9) >= flops_alg / (FP64_PEAK_TFLOPS * 1e12)
                     else {"bound": "alu", "achieved": tflops, "peak": FP64_PEAK_TFLOPS,
                           "unit": "TFLOP/s", "frac": tflops / FP64_PEAK_TFLOPS,
                           "traffic": traffic}) | {
                     "kernel": kname, "bytes_per_pass": bytes_alg, "flops_per_pass": flops_alg,
                     "hbm_frac": achieved / HBM_PEAK_GBS,
                     "fp64_frac": tflops / FP64_PEAK_TFLOPS,
                     "launches_per_pass": launches},
    }
    last.close()

    if not args.no_learned:
        log("learned: preparing model")
        model, gate, gate_dom = LR.load_or_train(ctx, args.mode, log=log)
        lspec = diaf.make_spec(w="learned", v=cfg["v"], v_count=cfg["v_count"], model=model,
                               gate_tau=gate, gate_dom=gate_dom)
        for _ in range(args.warmup):
            F, lst, linfo, lf, ls = step(lspec)
            log(f"learned warmup: factor {lf:.1f} ms, solve {ls:.1f} ms, {linfo.iters} its, "
                f"flag {linfo.flag}, fell back {lst.count_fell_back}, nnz(W) {lst.nnz_w}")
            F.close()
        lrec = []
        for _ in range(args.steps):
            F, lst, linfo, lf, ls = step(lspec)
            log(f"learned step: factor {lf:.1f} ms, solve {ls:.1f} ms, {linfo.iters} its")
            lrec.append((lf, ls, linfo.iters, lst.count_fell_back, lst.nnz_w, F.levels()))
            F.close()
        L_ = np.array(lrec, dtype=float)
        out["learned"] = {"factor_ms": float(L_[:, 0].mean()), "solve_ms": float(L_[:, 1].mean()),
                          "e2e_ms": float((L_[:, 0] + L_[:, 1]).mean()),
                          "bicgstab_iters": int(L_[-1, 2]), "fell_back": int(L_[-1, 3]),
                          "nnz_w": int(L_[-1, 4]), "gate_tau": gate, "gate_dom": gate_dom,
                          "v_levels": int(L_[-1, 5])}
        out["plain"] = {"factor_ms": factor_ms, "solve_ms": solve_ms,
                        "e2e_ms": factor_ms + solve_ms, "bicgstab_iters": iters,
                        "nnz_w": int(len(H["Wri"])), "v_levels": int(levels)}
        model.close()

    if args.variants:
        out["variants"] = {}
        for name in [v.strip() for v in args.variants.split(",") if v.strip()]:
            kw = dict(VARIANTS[name])
            nb = kw.pop("blocks", None)
            if nb:
                kw["v_blocks"] = torch.arange(0, A.n + 1, nb, dtype=torch.int32, device="cuda")
            vspec = diaf.make_spec(**kw)
            rec = []
            for it in range(args.warmup + args.steps):
                F, vst, vinfo, vf, vs = step(vspec)
                log(f"variant {name}: factor {vf:.1f} ms (pattern {vst.ms_pattern:.2f}, kernels "
                    f"{vst.ms_factor_kernels:.2f}), solve {vs:.1f} ms, {vinfo.iters} its, "
                    f"flag {vinfo.flag}, relres_true {vinfo.relres_true:.2e}")
                if it >= args.warmup:
                    rec.append((vf, vs, vst.ms_pattern, vst.ms_factor_kernels, vinfo.iters,
                                vinfo.flag, vinfo.relres_true, vst.nnz_w, F.levels(), vst.nrm))
                F.close()
            Rv = np.array(rec, dtype=float)
            out["variants"][name] = {
                "spec": {k: (v if not hasattr(v, "shape") else f"blocks of {nb}")
                         for k, v in kw.items()},
                "factor_ms": float(Rv[:, 0].mean()), "solve_ms": float(Rv[:, 1].mean()),
                "e2e_ms": float((Rv[:, 0] + Rv[:, 1]).mean()),
                "pattern_ms": float(Rv[:, 2].mean()), "factor_kernel_ms": float(Rv[:, 3].mean()),
                "bicgstab_iters": int(Rv[-1, 4]), "flag": int(Rv[-1, 5]),
                "relres_true": float(Rv[-1, 6]), "nnz_w": int(Rv[-1, 7]),
                "v_levels": int(Rv[-1, 8]), "nrm_AW_minus_V": float(Rv[-1, 9])}

    if not args.no_cpu:
        log("cpu baseline: oracle on host cores")
        import oracle
        Jo = oracle.pattern_A2(A)
        out["cpu_baseline"] = cpu_baseline(A, Jo, args.mode, cfg["v"], cfg["v_count"], upper, b)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
