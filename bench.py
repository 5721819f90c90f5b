"""Benchmark: direct approximate factoring AW ~ V + right-preconditioned
BiCGSTAB on the 64^3 convection-diffusion workload (n = 262144, W pattern
pattern(A^2), V = diagonal + top-4 |A w0| rows of the lower triangle of the
shadow, unit-norm-v mode), learned vs plain W pattern, one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode unit_v|unit_w]
                    [--workload convdiff3d_64|random_1m]

A step is one pass of the hot path on device-resident A and b: W pattern ->
factor (all columns) -> V assembly -> BiCGSTAB to 1e-8.  `value` is
columns factored and solved per second over the step; the factoring pass
alone, the solve, BiCGSTAB iterations and the learned-pattern variant are
reported beside it, with the factor kernel's roofline and the CPU oracle's
rate on the host cores.

--workload random_1m: the random n = 10^6 matrix (lognormal column degrees,
W = pattern(A) plus the top-8 two-hop rows, V = diagonal + top-4 lower).
Its BiCGSTAB does not converge (30 % of the rows are not diagonally
dominant), so there a step is the factoring pass alone (W pattern ->
factor -> V assembly) and `value` is columns factored per second; the
solve is run once, outside the timed steps, only with --solve-maxit.
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
    """sha256 over the sources a factor kernel's code comes from."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1208_3573_amd", "csrc")
    # the kernel's own source and the header that defines its arguments
    # (factor_kernels.h holds only the launchers' declarations)
    files = {"factor_small_kernel": ["factor_small.hip", "dcommon.h"],
             "factor_mid_kernel": ["factor_mid.hip", "dcommon.h"],
             "factor_generic_kernel": ["factor_generic.hip", "dcommon.h"]}[kernel]
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
# configuration): Algorithm 1 with the paper's parameters (k = 3, tau_i = 0.1)
# and V_0 diagonal, or block diagonal on the x-lines (64 rows per block) with
# V block diagonal on the same blocks or the top-k lower rule,
# Algorithm 2 with the Gauss-Seidel V_0, the Section 3.2 constraint, the
# Section 3.1 leverage rule, block diagonal V on the x-lines of the grid (64
# rows per block) with the pattern of D or the top-k rows of the block, and
# the left variant.
VARIANTS = {
    "alg1": dict(w="sparsified", v="topk_lower", v_count=5,
                 sparsify=dict(k=3, tau_i=0.1, p_i=0, tau_l=0.0, p_l=0)),
    "alg1_block": dict(w="sparsified", v="block", blocks=64, v0_blocks=64,
                       sparsify=dict(k=3, tau_i=0.1, p_i=0, tau_l=0.0, p_l=0)),
    "alg1_block_topk": dict(w="sparsified", v="topk_lower", v_count=5, v0_blocks=64,
                            sparsify=dict(k=3, tau_i=0.1, p_i=0, tau_l=0.0, p_l=0)),
    "alg2_gs": dict(w="alg2_gs_lower", v="topk_lower", v_count=5),
    "stab": dict(w="A2", v="topk_lower", v_count=5, stab_r=2.0),
    "lev": dict(w="A2", v="lev_lower", v_count=5),
    "block_d": dict(w="A2", v="block", blocks=64),
    "block_topk": dict(w="A2", v="topk_block", v_count=5, blocks=64),
    "left": dict(w="A2", v="topk_lower", v_count=5, left=True),
}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, J, mode, v, l, upper, b, solve, runs=3, sample_all=None, sample_1=32768):
    """The oracle as it stands on the host cores: all cores, median of `runs`
    runs on the full workload (factor + BiCGSTAB when the workload solves)
    or on `sample_all` evenly spaced columns; and one core on `sample_1`
    evenly spaced columns (factoring only)."""
    import oracle
    nth = oracle.nthreads_default()
    cols_all = None if sample_all is None else np.linspace(0, A.n - 1, sample_all).astype(np.int32)
    ncols = A.n if cols_all is None else len(cols_all)
    rates, frates, its, fsec, ssec = [], [], None, [], []
    for _ in range(runs):
        t0 = time.perf_counter()
        F = oracle.factor(A, J, mode, v, l, nthreads=nth, cols=cols_all)
        t1 = time.perf_counter()
        if solve:
            _, info = oracle.bicgstab(A, b, F, upper=upper)
            its = info.iters
        t2 = time.perf_counter()
        rates.append(ncols / (t2 - t0))
        frates.append(ncols / (t1 - t0))
        fsec.append(t1 - t0)
        ssec.append(t2 - t1)
    cols_1 = np.linspace(0, A.n - 1, min(sample_1, A.n)).astype(np.int32)
    t0 = time.perf_counter()
    oracle.factor(A, J, mode, v, l, nthreads=1, cols=cols_1)
    one = len(cols_1) / (time.perf_counter() - t0)
    what = "full workload" if cols_all is None else f"{ncols} evenly spaced columns"
    sample = (f"{what}, median of {runs} runs on {nth} threads: factor "
              f"{float(np.median(fsec)):.2f} s" +
              (f" + BiCGSTAB {float(np.median(ssec)):.2f} s ({its} its)" if solve else "") +
              f"; 1 thread: factoring {len(cols_1)} evenly spaced columns")
    return dict(value=float(np.median(rates)), unit="columns/s", cores=nth, kind="oracle",
                sample=sample, cpu=cpu_model(), factor_cols_per_s=float(np.median(frates)),
                factor_cols_per_s_1core=one, iters=its)


def class_caps(st):
    """(|J_j|, gathered entries) capacities of the size classes the factoring
    pass used (the context's class table)."""
    return [(int(st.class_kcap[q]), int(st.class_tcap[q])) for q in range(8)
            if st.class_kcap[q] > 0]


def column_stats(A, Jcp, Jri, lcount, mode, sv, caps):
    """Per column: algorithmic bytes and flops (as algorithmic_bytes and
    algorithmic_flops count them), |J_j|, gathered entries and the shadow
    size m_j, from the symbolic product pattern(A) pattern(J)."""
    import scipy.sparse as sp
    n = A.n
    cn = np.diff(A.colptr).astype(np.int64)
    k = np.diff(Jcp).astype(np.int64)
    col = np.repeat(np.arange(n), k)
    t = np.bincount(col, weights=cn[Jri], minlength=n).astype(np.int64)
    l = np.asarray(lcount, dtype=np.int64)
    byt = t * (sv + 4) + 8 * k + 4 * k + k * (sv + 4) + l * (sv + 4) + 8
    P = sp.csc_matrix((np.ones(A.nnz), A.rowidx, A.colptr), shape=(n, n))
    S = sp.csc_matrix((np.ones(len(Jri)), Jri, Jcp), shape=(n, n))
    C = (P @ S).tocsc()
    m = np.diff(C.indptr).astype(np.int64)
    c = C.data
    ccol = np.repeat(np.arange(n), m)
    gram = np.bincount(ccol, weights=c * (c + 1.0), minlength=n)
    nnzb = np.bincount(ccol, weights=c, minlength=n)
    shared = np.bincount(ccol, weights=(c >= 2), minlength=n).astype(np.int64)
    kf, lf = k.astype(np.float64), l.astype(np.float64)
    if mode == "unit_v":
        fl = gram + kf ** 3 / 3 + 2 * kf ** 2 * (1 + lf) + 2 * lf ** 2 * kf + 42 * lf ** 3 + 2 * nnzb
    else:
        fl = gram + 2 * lf * kf ** 2 + 84 * kf ** 3 + 2 * nnzb
    fl = fl * (4.0 if A.is_complex else 1.0)
    cls = np.full(n, len(caps))
    for q in range(len(caps) - 1, -1, -1):
        cls[(k <= caps[q][0]) & (t <= caps[q][1])] = q
    return dict(bytes=byt, flops=fl, k=k, t=t, m=m, cls=cls, shared=shared, caps=caps)


def kernel_rooflines(cs, st, flags, mode, lmax, steps_factor, is_complex=False):
    """Per factor kernel: the columns it finished (the one-wave kernel keeps
    the columns with |J_j| <= 32, at most 256 gathered entries and a shadow
    of at most 64 rows, and for unit-norm w those whose block is not rank
    deficient; for unit-norm v the mid-size kernel takes the other columns
    with |J_j| <= 64 and at most 1024 gathered entries (complex: 32, 256)
    and at most 256 rows of two or more entries; the generic kernel takes
    the rest, per size class), their algorithmic bytes and flops, its device
    time per pass, and the fractions of the HBM and FP64 peaks."""
    k, t = cs["k"], cs["t"]
    small = (k <= 32) & (t <= 256) & (cs["m"] <= 64) & (lmax <= 8)
    if mode == "unit_w":
        small &= (flags & 1) == 0
    mid = np.zeros_like(small)
    if st.launches_mid:
        mk, mt = (32, 256) if is_complex else (64, 1024)
        mid = ~small & (k <= mk) & (t <= mt) & (cs["shared"] <= 256)
    out = {}
    if st.launches_mid:
        ms_mid = st.ms_mid_kernel / steps_factor
        b = float(cs["bytes"][mid].sum())
        f = float(cs["flops"][mid].sum())
        out["factor_mid_kernel"] = dict(
            cols=int(mid.sum()), cols_reported=int(st.cols_mid / steps_factor), ms=ms_mid,
            bytes=b, flops=f, gbs=b / (ms_mid * 1e-3) / 1e9,
            hbm_frac=b / (ms_mid * 1e-3) / (HBM_PEAK_GBS * 1e9),
            fp64_frac=f / (ms_mid * 1e-3) / (FP64_PEAK_TFLOPS * 1e12),
            waves_per_simd=st.occ_mid, launches=int(st.launches_mid / steps_factor))
    ms_small = st.ms_small_kernel / steps_factor
    if st.launches_small:
        b = float(cs["bytes"][small].sum())
        f = float(cs["flops"][small].sum())
        out["factor_small_kernel"] = dict(
            cols=int(small.sum()), cols_reported=int(st.cols_small / steps_factor), ms=ms_small,
            bytes=b, flops=f, gbs=b / (ms_small * 1e-3) / 1e9,
            hbm_frac=b / (ms_small * 1e-3) / (HBM_PEAK_GBS * 1e9),
            fp64_frac=f / (ms_small * 1e-3) / (FP64_PEAK_TFLOPS * 1e12),
            waves_per_simd=st.occ_small, launches=1)
    gen = ~small & ~mid
    ms_gen = sum(st.ms_generic_class[q] for q in range(8)) / steps_factor
    if ms_gen > 0:
        per = {}
        for q in range(len(cs["caps"])):
            if not st.launches_generic_class[q]:
                continue
            sel = gen & (cs["cls"] == q)
            msq = st.ms_generic_class[q] / steps_factor
            bq = float(cs["bytes"][sel].sum())
            per[str(q)] = dict(caps=cs["caps"][q], cols=int(sel.sum()),
                               cols_reported=int(st.cols_generic_class[q] / steps_factor),
                               ms=msq, gbs=bq / (msq * 1e-3) / 1e9,
                               waves_per_simd=st.occ_generic_class[q])
        b = float(cs["bytes"][gen].sum())
        f = float(cs["flops"][gen].sum())
        out["factor_generic_kernel"] = dict(
            cols=int(gen.sum()), ms=ms_gen, bytes=b, flops=f, gbs=b / (ms_gen * 1e-3) / 1e9,
            hbm_frac=b / (ms_gen * 1e-3) / (HBM_PEAK_GBS * 1e9),
            fp64_frac=f / (ms_gen * 1e-3) / (FP64_PEAK_TFLOPS * 1e12),
            launches=len(per), classes=per)
    return out


def density(H, nnzA):
    """rho = (nnz(W) + nnz(L_V) + nnz(U_V)) / nnz(A), the density the paper
    reports with its tables; a triangular V is its own LU factor, so the V
    part is nnz(V)."""
    return (len(H["Wri"]) + len(H["Vri"])) / nnzA


def learned_block_comparison(ctx, dA, db, x, n, steps, warmup, LR, diaf, torch):
    """Second basic algorithm (unit-norm w) with V block diagonal on the
    grid's x-lines (64-row blocks): plain pattern(A^2), plain pattern(A),
    the network trained on labels at dropping tolerance 0.1 with no gate
    and with its calibrated gates, and the 1-hop top-p rule at the learned
    mean |J_j| (p = mean |J_j| - 7 beyond pattern(A)).  Same tolerance 1e-8
    for all; medians over the timed steps."""
    N = round(n ** (1.0 / 3.0))
    vb = torch.arange(0, n + 1, N, dtype=torch.int32, device="cuda")
    model, gate, gate_dom = LR.load(ctx, LR.weights_path("unit_w", "block"))

    def run(spec_):
        rec = []
        for it in range(warmup + steps):
            t0 = time.perf_counter()
            F = diaf.diaf_factor(ctx, dA, spec_, "unit_w")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            info = diaf.diaf_solve(ctx, dA, F, db, x, 1e-8, 1000)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            st = F.stats()
            if it >= warmup:
                rec.append(((t1 - t0) * 1e3, (t2 - t1) * 1e3, st.ms_factor_kernels))
            F.close()
        R = np.median(np.array(rec), axis=0)
        return {"factor_ms": float(R[0]), "solve_ms": float(R[1]), "e2e_ms": float(R[0] + R[1]),
                "factor_kernel_ms": float(R[2]), "bicgstab_iters": int(info.iters),
                "flag": int(info.flag), "relres_true": float(info.relres_true),
                "nnz_w": int(st.nnz_w), "fell_back": int(st.count_fell_back)}

    res = {"plain_A2": run(diaf.make_spec(w="A2", v="block", v_blocks=vb)),
           "plain_A": run(diaf.make_spec(w="A", v="block", v_blocks=vb))}
    res["learned_ungated"] = run(diaf.make_spec(w="learned", v="block", v_blocks=vb,
                                                model=model))
    res["learned_gated"] = run(diaf.make_spec(w="learned", v="block", v_blocks=vb, model=model,
                                              gate_tau=gate, gate_dom=gate_dom))
    p = max(0, int(round(res["learned_ungated"]["nnz_w"] / n - 7)))
    res["ablation_1hop"] = run(diaf.make_spec(w="A_1hop_topk", w_topk=p, v="block",
                                              v_blocks=vb)) | {"p": p}
    res |= {"label_tau": 0.1, "gate_tau": gate, "gate_dom": gate_dom}
    model.close()
    for k, v in res.items():
        if isinstance(v, dict):
            log(f"learned unit_w block: {k}: e2e {v['e2e_ms']:.1f} ms, "
                f"{v['bicgstab_iters']} its, nnz(W) {v['nnz_w']}, fell back {v['fell_back']}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="unit_v", choices=["unit_v", "unit_w"])
    ap.add_argument("--workload", default=WORKLOAD, choices=["convdiff3d_64", "random_1m"])
    ap.add_argument("--solve-maxit", type=int, default=0,
                    help="random_1m: run BiCGSTAB once after the timed steps with this maxit")
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

    workload = args.workload
    solves = workload == "convdiff3d_64"
    cfg = synth.WORKLOADS[workload]
    A = synth.workload_matrix(workload)
    b = synth.rhs_ones(A)
    upper = cfg["v"].endswith("upper")
    ctx = diaf.Context(0)
    for kv in args.opt:
        k, v = kv.split("=", 1)
        ctx.set_option(k, int(v))
    dA = diaf.DeviceCSC.from_host(A)
    db = torch.from_numpy(b).cuda()
    x = torch.zeros_like(db)
    spec = diaf.make_spec(w=cfg["w"], v=cfg["v"], v_count=cfg["v_count"],
                          w_topk=cfg.get("w_topk", 0))
    tuned = None
    if not args.no_autotune:
        # launch shapes picked on this problem, before (and outside) the timed steps
        t0 = time.perf_counter()
        tuned = diaf.diaf_autotune(ctx, dA, spec, args.mode)
        tuned["seconds"] = time.perf_counter() - t0
        log(f"autotune: {tuned}")

    def step(spec_, solve=solves, maxit=1000):
        t0 = time.perf_counter()
        F = diaf.diaf_factor(ctx, dA, spec_, args.mode)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        info = None
        if solve:
            info = diaf.diaf_solve(ctx, dA, F, db, x, 1e-8, maxit)
            torch.cuda.synchronize()
        t2 = time.perf_counter()
        st = F.stats()
        return F, st, info, (t1 - t0) * 1e3, (t2 - t1) * 1e3

    def its(info):
        return f", {info.iters} its" if info is not None else ""

    for _ in range(args.warmup):
        F, st, info, fms, sms = step(spec)
        log(f"warmup: factor {fms:.1f} ms, solve {sms:.1f} ms{its(info)}")
        F.close()
    torch.cuda.synchronize()
    recs = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        F, st, info, fms, sms = step(spec)
        log(f"step: factor {fms:.1f} ms, solve {sms:.1f} ms{its(info)}")
        recs.append((st.ms_factor_kernels, st.ms_pattern, st.ms_factor, st.ms_assemble, fms, sms,
                     info.iters if info else 0, info.relres_true if info else np.nan,
                     st.factor_launches))
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
    levels = last.levels() if solves else None  # diagnostic, after the timed steps
    H = last.to_host()
    sv = 16 if A.is_complex else 8
    bytes_alg, gathered = algorithmic_bytes(A, H["Wri"], H["lcount"], sv)
    launches = max(1, int(R[-1, 8]))
    achieved = bytes_alg / (kern_ms * 1e-3) / 1e9
    flops_alg = algorithmic_flops(A, H["Wcp"], H["Wri"], H["lcount"], args.mode)
    tflops = flops_alg / (kern_ms * 1e-3) / 1e12
    cs = column_stats(A, H["Wcp"], H["Wri"], H["lcount"], args.mode, sv, class_caps(st))
    kr = kernel_rooflines(cs, st, H["flags"], args.mode, int(H["lcount"].max()), 1,
                          A.is_complex)
    # the dominant factor kernel of the pass and its roofline
    kname = max(kr, key=lambda q: kr[q]["ms"])
    K = kr[kname]
    hbm_bound = K["bytes"] / (HBM_PEAK_GBS * 1e9) >= K["flops"] / (FP64_PEAK_TFLOPS * 1e12)
    traffic = measured_traffic(kname, workload, args.mode)
    kach = K["bytes"] / (K["ms"] * 1e-3) / 1e9
    ktf = K["flops"] / (K["ms"] * 1e-3) / 1e12
    roof = ({"bound": "hbm", "achieved": kach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": kach / HBM_PEAK_GBS, "traffic": traffic} if hbm_bound else
            {"bound": "alu", "achieved": ktf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
             "frac": ktf / FP64_PEAK_TFLOPS, "traffic": traffic})
    roof |= {"kernel": kname, "bytes_per_pass": K["bytes"], "flops_per_pass": K["flops"],
             "ms_per_pass": K["ms"], "hbm_frac": K["hbm_frac"], "fp64_frac": K["fp64_frac"],
             "launches_per_pass": K["launches"],
             "waves_per_simd": K.get("waves_per_simd")}
    if traffic:
        roof["traffic_frac"] = traffic / (K["ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9)
    cfgd = {"workload": workload, "n": A.n, "nnz": A.nnz, "w_pattern": cfg["w"]
            + (f" top-{cfg['w_topk']}" if cfg.get("w_topk") else ""),
            "v_pattern": f"{cfg['v']} l={cfg['v_count']}", "mode": args.mode}
    if solves:
        cfgd |= {"rhs": "A*ones", "rtol": 1e-8}
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
        "config": cfgd,
        "step": "W pattern + factor + V assembly + BiCGSTAB to 1e-8" if solves
                else "W pattern + factor + V assembly (the solve does not converge on this matrix)",
        "factor_ms": factor_ms,
        "factor_kernel_ms": kern_ms,
        "pattern_ms": float(np.mean(R[:, 1])),
        "assemble_ms": float(np.mean(R[:, 3])),
        "factor_cols_per_s": A.n / (factor_ms * 1e-3),
        "factor_kernel_cols_per_s": A.n / (kern_ms * 1e-3),
        "nrm": st.nrm,
        "rho": density(H, A.nnz),
        "autotuned": tuned,
        "roofline": roof,
        "pass_roofline": {"bytes": bytes_alg, "gathered_entries": gathered, "flops": flops_alg,
                          "kernel_ms": kern_ms, "hbm_frac": achieved / HBM_PEAK_GBS,
                          "fp64_frac": tflops / FP64_PEAK_TFLOPS, "launches": launches},
        "kernels": kr,
    }
    if solves:
        out |= {"solve_ms": solve_ms, "bicgstab_iters": iters, "relres_true": float(R[-1, 7]),
                "v_levels": levels}
        # refactoring the same pattern (time stepping): the first call records
        # the factor launches, later ones replay them as one graph
        rt = []
        for _ in range(1 + max(3, args.steps)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            diaf.diaf_refactor(ctx, dA, last)
            torch.cuda.synchronize()
            rt.append((time.perf_counter() - t0) * 1e3)
        rst = last.stats()
        out["refactor"] = {"first_ms": rt[0], "replay_ms": float(np.median(rt[1:])),
                           "replay_kernels_ms": rst.ms_factor, "factor_ms": factor_ms,
                           "graph": bool(ctx.get_option("factor_graph"))
                           and args.mode == "unit_v"}
        log(f"refactor: first {rt[0]:.2f} ms, replay {np.median(rt[1:]):.2f} ms")
    last.close()

    if solves and not args.no_learned:
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
        out["learned_unit_w_block"] = learned_block_comparison(
            ctx, dA, db, x, A.n, args.steps, args.warmup, LR, diaf, torch)

    if not solves and args.solve_maxit > 0:
        F, _, info, fms, sms = step(spec, solve=True, maxit=args.solve_maxit)
        out["solve_once"] = {"maxit": args.solve_maxit, "iters": info.iters, "flag": info.flag,
                             "relres": info.relres, "relres_true": info.relres_true,
                             "ms": sms}
        F.close()

    if args.variants:
        out["variants"] = {}
        for name in [v.strip() for v in args.variants.split(",") if v.strip()]:
            kw = dict(VARIANTS[name])
            nb = kw.pop("blocks", None)
            if nb:
                kw["v_blocks"] = torch.arange(0, A.n + 1, nb, dtype=torch.int32, device="cuda")
            nb0 = kw.pop("v0_blocks", None)
            if nb0:
                kw["sparsify"] = dict(kw["sparsify"], v0_blocks=torch.arange(
                    0, A.n + 1, nb0, dtype=torch.int32, device="cuda"))
            vspec = diaf.make_spec(**kw)
            rec = []
            for it in range(args.warmup + args.steps):
                F, vst, vinfo, vf, vs = step(vspec, solve=True)
                log(f"variant {name}: factor {vf:.1f} ms (pattern {vst.ms_pattern:.2f}, kernels "
                    f"{vst.ms_factor_kernels:.2f}), solve {vs:.1f} ms, {vinfo.iters} its, "
                    f"flag {vinfo.flag}, relres_true {vinfo.relres_true:.2e}")
                if it >= args.warmup:
                    rec.append((vf, vs, vst.ms_pattern, vst.ms_factor_kernels, vinfo.iters,
                                vinfo.flag, vinfo.relres_true, vst.nnz_w, F.levels(), vst.nrm))
                F.close()
            Rv = np.array(rec, dtype=float)
            out["variants"][name] = {
                "spec": {k: (f"blocks of {nb}" if hasattr(v, "shape") else
                             {a: (f"blocks of {nb0}" if hasattr(b, "shape") else b)
                              for a, b in v.items()} if isinstance(v, dict) else v)
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
        if workload == "convdiff3d_64":
            Jo = oracle.pattern_A2(A)
            out["cpu_baseline"] = cpu_baseline(A, Jo, args.mode, cfg["v"], cfg["v_count"], upper,
                                               b, True)
        else:
            Jo = oracle.pattern_1hop(A, cfg["w_topk"])
            out["cpu_baseline"] = cpu_baseline(A, Jo, args.mode, cfg["v"], cfg["v_count"], upper,
                                               b, False, sample_all=200000, sample_1=20000)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
