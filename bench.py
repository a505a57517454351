"""Benchmark: MLFMA Z.x matvecs/s at N = 122,880 (PEC sphere, radius 4
wavelengths, 6-level tree) on one MI355X -- FP32 batched (complex64 far
field, complex128 near field; leaf, near-field and interpolation products on
the matrix cores; d0 4.5, p 10) against FP64 single-vector (d0 4, p 10, with
the two-box buffer at the two finest levels that its 1e-4 bound needs), each
with its relative 2-norm error against the CPU FP64 oracle on 1 % of the
rows (1,229, stored by tests/golden/make_oracle_rows.py; FP32: all 32 columns
of the batch).

One "step" is one apply of Z to a block of `--ncols` right-hand sides (the
whole hot path: near-field product, aggregation, interpolation, translation,
anterpolation, disaggregation).  Inputs are resident in HBM before timing
starts; the library launches on torch's current stream, which is what the
HIP events bracket.  Prints ONE JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12            # B/s
FP32_PEAK = 157.3e12         # flop/s, vector (256 CU x 128 lanes x 2 x 2.4 GHz)
FP64_PEAK = 78.6e12          # flop/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--ncols", type=int, default=32)
    ap.add_argument("--d0", type=float, default=4.5, help="digits (truncation rule) of the FP32 batched path")
    ap.add_argument("--p", type=int, default=10, help="interpolation points of the FP32 batched path")
    ap.add_argument("--wide", action="store_true", help="two-box buffer (wide near field) on the FP32 path")
    ap.add_argument("--no-autotune", action="store_true", help="default matrix-core shapes on the FP32 path")
    ap.add_argument("--d0-64", type=float, default=4.0, help="digits of the FP64 single-vector path")
    ap.add_argument("--p-64", type=int, default=10, help="interpolation points of the FP64 path")
    ap.add_argument("--narrow-64", action="store_true",
                    help="one-box buffer on the FP64 path (default: two-box buffer, for its 1e-4 bound)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration under rocprofv3)")
    ap.add_argument("--nlv", type=int, default=6)
    ap.add_argument("--rows", type=int, default=64, help="oracle rows timed for the CPU baseline")
    ap.add_argument("--err-cols", type=int, default=8, help="R x batch columns checked against the oracle rows")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle (no error, no CPU baseline)")
    ap.add_argument("--no-eigs", action="store_true", help="skip the eigenmodes-per-hour measurement")
    ap.add_argument("--no-sweep", action="store_true", help="skip the 8-wavenumber sweep measurement")
    ap.add_argument("--sweep-only", action="store_true",
                    help="only the one-pass 8-wavenumber sweep (profiling of its kernels): prints its record")
    ap.add_argument("--no-d0-3", action="store_true", help="skip the 3-digit truncation measurement")
    ap.add_argument("--no-sai", action="store_true", help="skip the SAI build and apply measurement")
    ap.add_argument("--no-cmp", action="store_true",
                    help="skip the Calderon-against-SAI inner iteration count (needs the SAI leg)")
    ap.add_argument("--no-track", action="store_true",
                    help="skip the plate frequency sweep with mode tracking")
    ap.add_argument("--no-r", action="store_true",
                    help="skip the R x measurement (sibling against standard translation lists)")
    return ap.parse_args()


def stage_model(st, nc, cb):
    """Algorithmic bytes and flops per apply, per stage, from the plan
    statistics.  cb = bytes per far-field complex number (8 FP32, 16 FP64)."""
    N = st["N"]
    lev = {x["l"]: x for x in st["levels"]}
    lf = max(lev)
    Kf = lev[lf]["K"]
    nleaf = lev[lf]["nbox"]
    p = st["interp_p"]
    m = {}
    # near-field values in complex128 on both paths (FP64 accumulation)
    m["near"] = dict(bytes=st["nnz_near"] * 16 + st["near_cols_total"] * 4 + 2 * N * nc * cb,
                     flops=8.0 * st["nnz_near"] * nc, fp="f64")
    m["aggregate"] = dict(bytes=N * 2 * Kf * cb + N * nc * cb + nleaf * 2 * Kf * nc * cb,
                          flops=8.0 * N * 2 * Kf * nc, fp="f32" if cb == 8 else "f64")
    m["disagg"] = dict(bytes=N * 2 * Kf * cb + nleaf * 2 * Kf * nc * cb + 2 * N * nc * cb,
                       flops=8.0 * N * 2 * Kf * nc, fp=m["aggregate"]["fp"])
    for l in range(2, lf + 1):
        L = lev[l]
        pat = L["nbox"] * 2 * L["K"] * nc * cb
        m[f"m2l_l{l}"] = dict(bytes=2 * pat + 343 * L["K"] * cb, flops=8.0 * L["far_pairs"] * 2 * L["K"] * nc,
                              fp=m["aggregate"]["fp"])
        if l < lf:
            C = lev[l + 1]
            cpat = C["nbox"] * 2 * C["K"] * nc * cb
            fl = C["nbox"] * nc * (2 * L["nt"] * C["np"] * p * 4 + 2 * L["K"] * p * 4 + 2 * L["K"] * 8)
            m[f"interp_l{l}"] = dict(bytes=cpat + pat, flops=float(fl), fp=m["aggregate"]["fp"])
            m[f"anterp_l{l + 1}"] = dict(bytes=2 * cpat + pat, flops=float(fl), fp=m["aggregate"]["fp"])
    m["permute"] = dict(bytes=2 * N * nc * cb, flops=0.0, fp=m["aggregate"]["fp"])
    return m


def roofline(stage, times, calls, model):
    mdl = model[stage]
    t = times[stage]["ms"] / times[stage]["calls"] * 1e-3
    peak_f = FP32_PEAK if mdl["fp"] == "f32" else FP64_PEAK
    intensity = mdl["flops"] / max(mdl["bytes"], 1)
    if intensity * HBM_PEAK > peak_f:           # above the ridge: arithmetic-bound
        return {"kernel": stage, "bound": "alu", "achieved": mdl["flops"] / t / 1e12, "peak": peak_f / 1e12,
                "unit": "TFLOP/s", "frac": mdl["flops"] / t / peak_f, "traffic": None,
                "avg_launch_ms": t * 1e3, "alg_flops": mdl["flops"], "alg_bytes": mdl["bytes"]}
    return {"kernel": stage, "bound": "hbm", "achieved": mdl["bytes"] / t / 1e9, "peak": HBM_PEAK / 1e9,
            "unit": "GB/s", "frac": mdl["bytes"] / t / HBM_PEAK, "traffic": None,
            "avg_launch_ms": t * 1e3, "alg_flops": mdl["flops"], "alg_bytes": mdl["bytes"]}


def measured_traffic(stage, path_tag, cfg):
    """HBM bytes per launch of a stage from the committed rocprofv3 --pmc
    summary (FETCH_SIZE x2 + WRITE_SIZE x1, copy-calibrated), or None when
    there is none for this stage or the kernel source changed since."""
    import hashlib
    f = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(f):
        return None
    rec = json.load(open(f)).get(f"{stage}/{path_tag}")
    if not rec or rec.get("config") != cfg:
        return None
    h = hashlib.sha256()
    for f in ("cm_apply.hip", "cm_mfma.hip"):
        h.update(open(os.path.join(ROOT, "paper_1412_1756_amd", "csrc", f), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return rec["read_bytes"] + rec["write_bytes"]


def inner_solves(op):
    """GMRES iterations per Arnoldi step (nii) of the characteristic-mode
    solve on this handle: IRA on Z^-1 R (eq. (24)) for 10 modes, 30 Arnoldi
    steps, inner GMRES(200) to 1e-3 (the paper's tolerance), FP64 far field,
    with no preconditioner, with the SAI (built by the caller) and with the
    Calderon preconditioner of eqs. (25)-(27) (refined handle one level
    deeper, p 6, d0 3: it only preconditions)."""
    import torch
    import workloads
    v0 = torch.tensor(workloads.cn01(op.N, 3), dtype=torch.complex128, device="cuda")
    res = {"nev": 10, "arnoldi_steps": 30, "gmres_tol": 1e-3, "far": "fp64"}
    t0 = time.perf_counter()
    info = op.cmp_build(nlv=op.stats()["nlv"] + 1, interp_p=6, d0=3.0)
    torch.cuda.synchronize()
    res["cmp_build_s"] = time.perf_counter() - t0
    res["cmp_refined_unknowns"] = info["N_refined"]
    for name, pc in (("none", False), ("sai", True), ("cmp", "cmp")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = op.eigs(10, 30, v0, tol=1e-6, maxrestart=0, gmres_restart=200, gmres_maxit=2000, gmres_tol=1e-3,
                    far="fp64", precond=pc, vectors=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[name] = {"gmres_per_arnoldi_step": r["gmres_iters"] / max(1, r["n_op"]), "seconds": dt,
                     "ms_per_gmres_iteration": dt * 1e3 / max(1, r["gmres_iters"]),
                     "inner_failures": r["inner_failures"]}
    return res


def _oracle_rows_times_x(args):
    """cpu_baseline worker: the oracle's rows `rows` of Z for workload
    `name`, applied to the seed-0 vector (one thread)."""
    name, rows = args
    os.environ["OMP_NUM_THREADS"] = "1"
    import workloads
    from oracle import efie
    V, F, spec = workloads.workload(name)
    if len(rows) == 0:
        return np.zeros(0, dtype=np.complex128)
    Zr = efie.rows_Z(V, F, spec["k"], np.asarray(rows))
    return Zr @ workloads.cn01(Zr.shape[1], 0)


def hbm_copy_rate(dev):
    """Achievable HBM bandwidth on this GPU: a plain 2 GiB device-to-device
    copy (2 x 2 GiB of traffic per copy), ten copies between HIP events."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.complex64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 10 * 2 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"GBps": gbs, "frac_of_peak": gbs * 1e9 / HBM_PEAK, "kernel": "device copy 2 GiB (torch copy_)"}


def sweep_rate(V, F, k0, ncols, steps, d0, p, shared=True):
    """The wavenumber-sweep workload: one handle at 8 wavenumbers 0.9 k0 ..
    1.1 k0 (a plan, tables and near field per wavenumber), a block of ncols
    columns with column j at wavenumber j mod 8, FP32 far field, autotuned;
    column-matvecs/s over `steps` applies between HIP events.  shared: the
    one-pass route (CM_FLAG_SWEEP_SHARED: sampling at 1.1 k0, slots of four
    columns per wavenumber, one tree pass), else one batched apply per
    wavenumber on its own stream."""
    import torch
    import workloads
    from paper_1412_1756_amd import Operator
    ks = list(np.linspace(0.9, 1.1, 8) * k0)
    t0 = time.perf_counter()
    sw = Operator(V, F, ks, nlv=6, d0=d0, interp_p=p, max_cols=ncols, autotune=True, sweep_shared=shared)
    t_build = time.perf_counter() - t0
    X = torch.tensor(workloads.cn01_block(sw.N, ncols, 100), dtype=torch.complex64, device="cuda")
    Y = torch.empty_like(X)
    kidx = np.arange(ncols, dtype=np.int32) % 8
    sw.apply(X, out=Y, k_index=kidx)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        sw.apply(X, out=Y, k_index=kidx)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    out = {"workload": "sphere_r4_n122880, 8 wavenumbers 0.9-1.1 k0, column j at j mod 8", "ncols": ncols,
           "route": "one pass" if shared else "per wavenumber", "ms_per_apply": ms,
           "column_matvecs_per_s": ncols * 1000.0 / ms, "setup_s": t_build, "d0": d0, "interp_p": p}
    if shared:
        st = sw.stats()
        out["one_pass_applies"] = st["sweep_one_pass_calls"]
        out["L_per_level"] = {lv["l"]: lv["L"] for lv in st["levels"] if lv["l"] >= 2}
        # one stage-timed pass (kernels one at a time), ms per apply per stage
        sw.stage_timing(True)
        for _ in range(3):
            sw.apply(X, out=Y, k_index=kidx)
        torch.cuda.synchronize()
        out["stage_ms"] = {k_: v["ms"] / 3 for k_, v in sw.stage_times().items()}
        sw.stage_timing(False)
    del sw
    torch.cuda.empty_cache()
    return out


def eigs_small(no_cpu):
    """Eigenmodes per hour on the 1,920-unknown sphere: the 10 smallest
    characteristic values by implicitly restarted Arnoldi on Z^-1 R with
    SAI-preconditioned GMRES inner solves, handle set-up + SAI build + IRA
    timed together; beside it the oracle's dense fill + QZ on the host cores."""
    import torch
    import workloads
    from paper_1412_1756_amd import Operator
    V, F, spec = workloads.workload("sphere_r0.5_n1920")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op = Operator(V, F, spec["k"], nlv=spec["nlv"], d0=6.0, interp_p=12, max_cols=1)
    op.sai_build(0.01, 0.014, 0.18)
    v0 = torch.tensor(workloads.cn01(op.N, 3), dtype=torch.complex128, device="cuda")
    r = op.eigs(10, 30, v0, tol=1e-6, maxrestart=30, gmres_tol=1e-8, vectors=False)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out = {"workload": "sphere_r0.5_n1920", "N": op.N, "modes": r["nconv"], "seconds": t,
           "modes_per_hour": r["nconv"] / t * 3600.0, "op_products": r["n_op"], "gmres_iters": r["gmres_iters"],
           "restarts": r["restarts"]}
    # the same modes by IRA on X^-1 R (eq. (14)): inner solves with X
    # unpreconditioned, and preconditioned by the SAI of X_near (SAI build timed)
    for key, pre in (("x_inverse_route", False), ("x_inverse_route_sai", True)):
        t0 = time.perf_counter()
        if pre:
            op.sai_build(0.01, 0.014, 0.18, part="X")
        rx = op.eigs(10, 30, v0, tol=1e-6, maxrestart=30, gmres_tol=1e-8, gmres_maxit=2000, route="X",
                     precond=pre, vectors=False)
        torch.cuda.synchronize()
        tx = time.perf_counter() - t0
        out[key] = {"seconds": tx, "modes": rx["nconv"], "op_products": rx["n_op"],
                    "gmres_iters": rx["gmres_iters"], "converged": rx["converged"],
                    "max_abs_diff_vs_z_route": float(np.max(np.abs(np.sort(rx["lam"].real)
                                                                   - np.sort(r["lam"].real))))}
    if not no_cpu:
        from threadpoolctl import threadpool_limits
        from oracle import efie, modes
        cores = os.cpu_count() or 1
        with threadpool_limits(limits=cores):
            t0 = time.perf_counter()
            Z = efie.dense_Z(V, F, spec["k"])
            lam = modes.qz_modes(Z.imag, Z.real, nev=10)
            tc = time.perf_counter() - t0
        out["max_abs_diff_vs_qz"] = float(np.max(np.abs(np.sort(r["lam"].real) - np.sort(lam.real))))
        out["cpu_oracle"] = {"seconds": tc, "modes_per_hour": 10 / tc * 3600.0, "cores": cores,
                             "kind": "oracle dense fill + QZ"}
    return out


def plate_sweep(solver="ira"):
    """The paper's plate sweep: a 1.0 m x 0.6 m PEC plate (1,085 RWG
    unknowns, 3 levels) over 220-380 MHz in 20 MHz steps, from the top
    frequency down (characteristic values grow in magnitude as the plate
    shrinks electrically, so the modes of 380 MHz stay among the computed
    ones); at each frequency handle set-up with dZ/dk tables, SAI build, IRA
    for eight modes and d lambda/dk, and the four smallest-|lambda| modes of
    380 MHz followed by modal correlation; timed end to end."""
    import torch
    import workloads
    from paper_1412_1756_amd import Operator
    from paper_1412_1756_amd.tracking import track_modes
    c0 = 299792458.0
    V, F = workloads.plate(25, 15, 0.04)
    freqs = [380e6 - 20e6 * i for i in range(9)]
    ks = [2 * np.pi * f / c0 for f in freqs]

    def make_op(k):
        return Operator(V, F, k, nlv=3, d0=6.0, interp_p=12, max_cols=16, deriv=True)

    N = make_op(ks[0]).N
    v0 = torch.tensor(workloads.cn01(N, 3), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if solver == "ira":
        t = track_modes(make_op, ks, 8, 24, v0, ntrack=4, tol=1e-6, maxrestart=60, gmres_tol=1e-8, gmres_maxit=3000)
    else:
        t = track_modes(make_op, ks, 8, 24, v0, ntrack=4, solver="jd", target=0.0, mmin=10, mmax=30, maxit=600,
                        tol=1e-6, inner_steps=20, precond=True)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    out = {"workload": "plate 1.0 m x 0.6 m, h 0.04 m", "N": N, "solver": solver,
           "freqs_MHz": [f / 1e6 for f in freqs], "modes_solved": 8, "modes_tracked": 4, "seconds": sec,
           "mode_points_per_hour": 8 * len(ks) / sec * 3600.0, "lam": np.round(t["lam"], 5).tolist(),
           "min_corr": float(t["corr"].min()), "max_pred_err": float(np.abs(t["lam"][1:] - t["pred"]).max()),
           "converged": all(t["converged"])}
    if solver == "ira":
        out["op_products"] = int(sum(t["n_op"]))
        out["inner_solves_redone_without_sai"] = t["inner_retries"]
    else:
        out["operator_applies"] = int(sum(t["n_op"]))
    return out


def jd_vs_ira_plate():
    """The four characteristic values nearest 0 of the 1.0 m x 0.6 m plate at
    300 MHz (1,085 unknowns, 3 levels, FP64) by Jacobi-Davidson on (X, R)
    (20 GMRES steps per correction, no inner solve with Z; unpreconditioned
    and right-preconditioned by i P) and by IRA on Z^-1 R (SAI-preconditioned
    inner solves), each timed from the built handle (the SAI build is counted
    where the SAI is used)."""
    import torch
    import workloads
    from paper_1412_1756_amd import Operator
    V, F = workloads.plate(25, 15, 0.04)
    k = 2 * np.pi * 300e6 / 299792458.0
    op = Operator(V, F, k, nlv=3, d0=6.0, interp_p=12, max_cols=1)
    v0 = torch.tensor(workloads.cn01(op.N, 3), dtype=torch.complex128, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = op.jd(4, v0, target=0.0, mmin=6, mmax=20, maxit=300, tol=1e-8, inner_steps=20, vectors=False)
    t_jd = time.perf_counter() - t0
    t0 = time.perf_counter()
    op.sai_build(0.01, 0.014, 0.18)
    t_sai = time.perf_counter() - t0
    e = op.eigs(4, 20, v0, tol=1e-8, maxrestart=60, gmres_tol=1e-10, vectors=False)
    t_ira = time.perf_counter() - t0
    t0 = time.perf_counter()
    rp = op.jd(4, v0, target=0.0, mmin=6, mmax=20, maxit=300, tol=1e-8, inner_steps=20, precond=True,
               vectors=False)
    t_jdp = time.perf_counter() - t0 + t_sai
    return {"workload": "plate 1.0 m x 0.6 m, h 0.04 m, 300 MHz", "N": op.N, "modes": 4,
            "jd": {"seconds": t_jd, "lam": np.sort(r["lam"]).round(6).tolist(), "outer": r["outer"],
                   "operator_applies": r["n_matvec"], "converged": r["converged"]},
            "jd_sai": {"seconds": t_jdp, "lam": np.sort(rp["lam"]).round(6).tolist(), "outer": rp["outer"],
                       "operator_applies": rp["n_matvec"], "converged": rp["converged"]},
            "ira": {"seconds": t_ira, "lam": np.sort(e["lam"].real).round(6).tolist(), "op_products": e["n_op"],
                    "gmres_iters": e["gmres_iters"], "operator_applies": e["n_matvec"],
                    "converged": e["converged"]}}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); sharding over several GPUs "
              "(Morton ranges of leaf boxes, pattern halos per level, a transpose where coarse levels "
              "split by direction) is not built", file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads
    from paper_1412_1756_amd import Operator

    name = "sphere_r4_n122880"
    V, F, spec = workloads.workload(name)
    k = spec["k"]
    dev = torch.device("cuda:0")
    if a.sweep_only:
        print(json.dumps({"sweep_8k": sweep_rate(V, F, k, a.ncols, a.steps, a.d0, a.p)}), flush=True)
        return
    op32 = Operator(V, F, k, nlv=a.nlv, d0=a.d0, interp_p=a.p, max_cols=max(a.ncols, 1), wide_near=a.wide,
                    autotune=not a.no_autotune)
    op64 = Operator(V, F, k, nlv=a.nlv, d0=a.d0_64, interp_p=a.p_64, max_cols=1, wide_near=not a.narrow_64)
    N = op32.N
    st = op32.stats()
    st64 = op64.stats()
    x1 = workloads.cn01(N, 0)
    Xh = workloads.cn01_block(N, a.ncols, 100)
    Xh[:, 0] = x1
    X32 = torch.tensor(Xh, dtype=torch.complex64, device=dev)
    X64 = torch.tensor(x1, dtype=torch.complex128, device=dev).reshape(N, 1)
    Y32 = torch.empty_like(X32)
    Y64 = torch.empty_like(X64)
    torch.cuda.synchronize()

    def timed(op, X, Y, steps, warm, stage_timing=True, opname="Z"):
        for _ in range(warm):
            op.apply(X, op=opname, out=Y)
        torch.cuda.synchronize()
        op.stage_timing(stage_timing)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            op.apply(X, op=opname, out=Y)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        times = op.stage_times() if stage_timing else {}
        op.stage_timing(False)
        return e0.elapsed_time(e1) / steps, wall, times

    # untimed-stage pass (pure throughput), then a pass with per-stage events
    ms32, wall32, _ = timed(op32, X32, Y32, a.steps, a.warmup, stage_timing=False)
    ms64, wall64, _ = timed(op64, X64, Y64, a.steps, a.warmup, stage_timing=False)
    _, _, times32 = timed(op32, X32, Y32, max(3, a.steps // 4), 1)
    _, _, times64 = timed(op64, X64, Y64, max(3, a.steps // 4), 1)
    ne = max(1, min(a.err_cols, a.ncols))
    r_out = None
    if not a.no_r:
        # R x (sin kernel) on the same batch: the sibling lists of the FP32 handle
        # against a handle with the standard MLFMA lists (same d0, p, tuning)
        YR = torch.empty_like(X32)
        msR, _, _ = timed(op32, X32, YR, a.steps, a.warmup, stage_timing=False, opname="R")
        yR = YR[:, :ne].cpu().numpy().astype(np.complex128)
        t0 = time.perf_counter()
        opS = Operator(V, F, k, nlv=a.nlv, d0=a.d0, interp_p=a.p, max_cols=max(a.ncols, 1), wide_near=a.wide,
                       autotune=not a.no_autotune, r_standard=True)
        t_setup_s = time.perf_counter() - t0
        msRs, _, _ = timed(opS, X32, YR, a.steps, a.warmup, stage_timing=False, opname="R")
        yRs = YR[:, :ne].cpu().numpy().astype(np.complex128)
        stS = opS.stats()
        del opS, YR
        torch.cuda.empty_cache()
        pairs = lambda s_: {L["l"]: L["farR_pairs"] for L in s_["levels"] if L["l"] >= 2}
        r_out = {"op": "R", "ncols": a.ncols, "dtype": "c64 far field / c128 near field",
                 "siblings": {"ms_per_apply": msR, "column_matvecs_per_s": a.ncols * 1000.0 / msR,
                              "translation_pairs": pairs(st)},
                 "standard": {"ms_per_apply": msRs, "column_matvecs_per_s": a.ncols * 1000.0 / msRs,
                              "translation_pairs": pairs(stS), "setup_s": t_setup_s}}
    if a.copy_calib:
        src = torch.empty(1 << 27, dtype=torch.complex64, device=dev)       # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    y32 = Y32[:, :ne].cpu().numpy().astype(np.complex128)
    y64 = Y64[:, 0].cpu().numpy()

    model32 = stage_model(st, a.ncols, 8)
    model64 = stage_model(st64, 1, 16)
    dom32 = max((s for s in times32 if s in model32), key=lambda s: times32[s]["ms"])
    dom64 = max((s for s in times64 if s in model64), key=lambda s: times64[s]["ms"])
    roof = roofline(dom32, times32, None, model32)
    roof64 = roofline(dom64, times64, None, model64)
    cfg32 = f"d0 {a.d0:g}, p {a.p}, {a.ncols} columns" + (", wide near" if a.wide else "") + \
        ("" if a.no_autotune else ", autotuned")
    cfg64 = f"d0 {a.d0_64:g}, p {a.p_64}, 1 columns" + ("" if a.narrow_64 else ", wide near")
    roof["traffic"] = measured_traffic(dom32, "fp32_batched", cfg32)
    roof64["traffic"] = measured_traffic(dom64, "fp64_single", cfg64)
    stage_frac = {s: round(v["ms"] / sum(u["ms"] for u in times32.values()), 4) for s, v in times32.items()}

    out = {
        "metric": "MLFMA Z·x matvecs/s at N=122,880: FP32 batched vs FP64 single, at stated rel err",
        "value": a.ncols * 1000.0 / ms32,
        "unit": "matvecs/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms32,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 far field / c128 near field",
        "data": "synthetic",
        "config": {"workload": name, "N": N, "nlv": a.nlv, "d0": a.d0, "interp_p": a.p, "ncols": a.ncols,
                   "wide_near": bool(a.wide), "nnz_near": st["nnz_near"],
                   "autotune": st.get("autotune"),
                   "k": k, "mesh": "icosphere nsub 6, radius 4 wavelengths"},
        "fp64_single": {"matvecs_per_s": 1000.0 / ms64, "ms_per_matvec": ms64, "dtype": "c128",
                        "d0": a.d0_64, "interp_p": a.p_64, "wide_near": not a.narrow_64,
                        "nnz_near": st64["nnz_near"], "roofline": roof64},
        "roofline": roof,
        "stage_fraction_fp32_batched": stage_frac,
        "stage_fraction_fp64_single": {s: round(v["ms"] / sum(u["ms"] for u in times64.values()), 4)
                                       for s, v in times64.items()},
        "stage_ms_fp32_batched": {s: round(v["ms"] / v["calls"], 4) for s, v in times32.items()},
        "stage_ms_fp64_single": {s: round(v["ms"] / v["calls"], 4) for s, v in times64.items()},
    }
    # errors against the stored oracle rows (1 % of the rows, seed 2, written by
    # tests/golden/make_oracle_rows.py from the oracle alone): the batch's
    # columns are the same seeded columns (seeds 100 + j, column 0 = seed 0)
    g = np.load(os.path.join(ROOT, "tests", "golden", f"oracle_rows_{name}.npz"))
    rows = g["rows"]
    gc = min(a.ncols, int(g["ncols"]))

    def errs(y, ref):
        e = y - ref
        return (float(np.linalg.norm(e) / np.linalg.norm(ref)),
                float(np.abs(e).max() / np.sqrt(np.mean(np.abs(ref) ** 2))))

    y32g = Y32[:, :gc].cpu().numpy().astype(np.complex128)[rows]
    e32, m32 = errs(y32g, g["Zx"][:, :gc])
    e64, m64 = errs(y64[rows], g["Zx"][:, 0])
    out["config"]["rel_err_fp32_batched"] = e32
    out["config"]["max_element_err_fp32_batched"] = m32
    out["config"]["rel_err_cols"] = gc
    out["config"]["rel_err_rows"] = int(rows.size)
    out["fp64_single"]["rel_err"] = e64
    out["fp64_single"]["max_element_err"] = m64
    out["config"]["rel_err_reference"] = "oracle rows tests/golden/oracle_rows_sphere_r4_n122880.npz"
    if r_out is not None:
        for key, yy in (("siblings", yR), ("standard", yRs)):
            r_out[key]["rel_err"] = errs(yy[rows], g["Rx"][:, :ne])[0]
    if not a.no_cpu:
        # the oracle itself on the host cores (one single-threaded process per
        # core, each filling its share of a bounded sample of rows and
        # applying them to x), extrapolated to one full Z.x
        import multiprocessing as mp
        cores = min(16, os.cpu_count() or 1)
        crow = np.sort(np.random.default_rng(2).choice(N, a.rows, replace=False))
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(cores) as pool:
            parts = pool.map(_oracle_rows_times_x, [(name, crow[i::cores]) for i in range(cores)])
        t_rows = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1.0 / (t_rows / a.rows * N), "unit": "matvecs/s", "cores": cores,
                               "kind": "oracle",
                               "sample": f"{a.rows} of {N} rows of Z filled by the FP64 oracle and applied to x "
                                         f"in {cores} processes ({t_rows:.1f} s wall, process start-up included), "
                                         f"extrapolated x N/{a.rows} to one full Z.x"}
    if r_out is not None:
        out["r_apply"] = r_out
    if not a.no_sai:
        # SAI preconditioner apply (FP64 CSR, the FP64 handle's near-field pattern)
        t0 = time.perf_counter()
        op64.sai_build(0.01, 0.014, 0.18)
        t_sai = time.perf_counter() - t0
        nnz_p = op64.sai_nnz()
        Ys = torch.empty_like(X64)
        op64.sai_apply(X64, out=Ys)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            op64.sai_apply(X64, out=Ys)
        e1.record()
        torch.cuda.synchronize()
        ms_sai = e0.elapsed_time(e1) / 20
        sai_bytes = nnz_p * 20 + (N + 1) * 8 + 2 * N * 16
        # SAI-preconditioned GMRES(50) on the FP64 handle: time per iteration
        # against the apply (the inner solves of the eigen-solvers)
        b = X64[:, 0].contiguous()
        op64.gmres(b, restart=50, maxit=50, tol=1e-12)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, its, rr, _ = op64.gmres(b, restart=50, maxit=200, tol=1e-12)
        torch.cuda.synchronize()
        t_g = time.perf_counter() - t0
        out["gmres_fp64"] = {"restart": 50, "iterations": its, "ms_per_iteration": t_g * 1e3 / its,
                             "apply_ms": ms64, "ratio_to_apply": t_g * 1e3 / its / ms64, "relres": rr}
        out["sai_apply"] = {"nnz": nnz_p, "ms": ms_sai, "alg_bytes": sai_bytes,
                            "GBps": sai_bytes / (ms_sai * 1e-3) / 1e9, "frac_of_hbm_peak": sai_bytes / (ms_sai * 1e-3) / HBM_PEAK,
                            "build_s": t_sai, "thresholds": [0.01, 0.014, 0.18]}
        if not a.no_cmp:
            out["inner_solves_sai_vs_cmp"] = inner_solves(op64)
    if not a.no_d0_3:
        # the workload's named truncation (3 digits, eq. (30)) on the same batch: faster, and
        # past the FP32 error bound on this tree (stated, not the headline)
        del op32
        torch.cuda.empty_cache()
        op3 = Operator(V, F, k, nlv=a.nlv, d0=3.0, interp_p=8, max_cols=max(a.ncols, 1), autotune=True)
        Y3 = torch.empty_like(X32)
        ms3, _, _ = timed(op3, X32, Y3, a.steps, a.warmup, stage_timing=False)
        d3 = {"d0": 3.0, "interp_p": 8, "ncols": a.ncols, "ms_per_apply": ms3,
              "column_matvecs_per_s": a.ncols * 1000.0 / ms3}
        d3["rel_err"] = errs(Y3[:, :gc].cpu().numpy().astype(np.complex128)[rows], g["Zx"][:, :gc])[0]
        out["fp32_batched_d0_3"] = d3
        del op3
        torch.cuda.empty_cache()
    if not a.copy_calib:   # the counter-calibration runs keep their single 1 GiB copy
        out["hbm_achievable"] = hbm_copy_rate(dev)
    if not a.no_sweep:
        del op64
        torch.cuda.empty_cache()
        out["sweep_8k"] = sweep_rate(V, F, k, a.ncols, max(3, a.steps // 2), a.d0, a.p)
        out["sweep_8k_per_wavenumber"] = sweep_rate(V, F, k, a.ncols, max(3, a.steps // 2), a.d0, a.p, shared=False)
    if not a.no_eigs:
        out["eigenmodes"] = eigs_small(a.no_cpu)
    if not a.no_track:
        out["plate_mode_sweep"] = plate_sweep()
        out["plate_mode_sweep_jd"] = plate_sweep("jd")
        out["plate_mode_sweep_jd"]["max_abs_diff_vs_ira_sweep"] = float(np.max(np.abs(
            np.array(out["plate_mode_sweep_jd"]["lam"]) - np.array(out["plate_mode_sweep"]["lam"]))))
        out["plate_jd_vs_ira"] = jd_vs_ira_plate()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
