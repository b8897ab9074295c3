"""Benchmark: time-to-tolerance and iterations per second of ME-GRBK for
A X B = C on one MI355X.

Workload: A 2000 x 500 and B 500 x 2000 with iid N(0,1) entries, X* 500 x 500
iid N(0,1), C = A X* B (data seed 2), X0 = 0, ME-GRBK (theta = 1/2), alpha =
1/||B||_2^2, stop at ||X - X*||_F/||X*||_F <= 1e-6. One step = the whole hot
path for that instance: plan set-up (row norms, A A^T, B^T B, alpha) and the
solve to tolerance. `value` is the job's updates per second over the timed
steps; `ms_per_step` is the time to tolerance. The same instance is also
solved in the FP32 and mixed forms (reported under "forms").

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import json
import os
import sys
import subprocess
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes_per_update(m, p, q, n, elem):
    # One update of the paper's form: read and write R (2 m n), read and
    # write X (2 p q), read B for R_i B^T and again for (R_i B^T) B (2 q n),
    # plus the selection / update vectors (m + n + p).
    return (2 * m * n + 2 * p * q + 2 * q * n + m + n + p) * elem


KERNEL_SOURCES = ["paper_2408_05444_amd/csrc/solver.hip", "paper_2408_05444_amd/csrc/select.h",
                  "paper_2408_05444_amd/csrc/exchange.h",
                  "paper_2408_05444_amd/csrc/device_common.h"]


def kernel_source_digest():
    """SHA-256 of the row solver's sources: its kernel file, the headers it is
    built from, and its parameter structs (the text of internal.h from
    `struct InstSlot` to the end of `struct SolveParams`)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    txt = open(os.path.join(ROOT, "paper_2408_05444_amd/csrc/internal.h")).read()
    a = txt.index("struct InstSlot")
    b = txt.index("};", txt.index("struct SolveParams")) + 2
    h.update(txt[a:b].encode())
    return h.hexdigest()


def measured_traffic(team_wgs, iters):
    """HBM bytes per launch of the solve kernel from the committed
    FETCH_SIZE / WRITE_SIZE counter record, each scaled by the same counter's
    reading on a copy kernel of known size. None when the kernel sources
    changed since the counters were taken, or the launch differs."""
    path = os.path.join(ROOT, "profiles", "solve_kernel_large_grbk_fp64_counters.json")
    try:
        rec = json.load(open(path))
        digest = kernel_source_digest()
    except (OSError, ValueError, KeyError):
        return None
    if digest != rec["source_sha256"]:
        return None
    if rec["team_wgs"] != team_wgs or rec["updates_per_launch"] != iters:
        return None
    cal = rec["calibration"]
    return (rec["fetch_size_kib_per_dispatch"] * 1024 * cal["fetch_scale"]
            + rec["write_size_kib_per_dispatch"] * 1024 * cal["write_scale"])


TS_BLOCK = 32   # block rows / columns of the two-sided form
MFMA_F64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
MFMA_BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 matrix peak


def gemm_forms(mek, torch, A, B, Xs, C, blur=None, reps=10):
    """The FP64 MFMA GEMMs of the set-up and the residual engine at the
    workload's sizes, timed with events on the stream they run on:
    A A^T (2000 x 2000 x 500) and R = C - (A X) B (2000 x 500 x 500, then
    2000 x 2000 x 500); with blur = (A, B, C, X) of the 3-channel image form,
    also its residual as one batched launch per product (3 x 512^3 twice)."""
    m, p = A.shape
    q, n = B.shape
    out = {}
    cases = {
        "gram_AAt": (lambda: mek.mek_gram(A, False), 2.0 * m * m * p),
        "residual_C-AXB": (lambda: mek.mek_residual(A, Xs, B, C), 2.0 * (m * p * q + m * q * n)),
    }
    if blur is not None:
        A3, B3, C3, X3 = blur
        nb, p3, q3 = X3.shape
        m3, n3 = A3.shape[0], B3.shape[1]
        cases["residual_blur3_batched"] = (lambda: mek.mek_residual_batched(A3, X3, B3, C3),
                                           2.0 * nb * (m3 * p3 * q3 + m3 * q3 * n3))
    # The split-BF16 residual engine of the FP32 and mixed iterations (BF16
    # matrix cores, FP32 accumulation): FP32 operands, 3 and 2 bf16 terms per
    # value (6 and 3 bf16 products per multiply-add). Its flop count is the
    # algorithmic 2 M N K per product; the bf16 work is 6x (3x) that.
    A32, B32 = A.float().contiguous(), B.float().contiguous()
    X32, C1 = Xs.float().contiguous()[None], C[None].contiguous()
    for P, mult in ((3, 6), (2, 3)):
        cases[f"split{P}_residual_C-AXB"] = (
            lambda P=P: mek.mek_residual_split(A32, X32, B32, C1, pieces=P),
            2.0 * (m * p * q + m * q * n), mult)
    if blur is not None:
        A3f, B3f, X3f = A3.float().contiguous(), B3.float().contiguous(), X3.float().contiguous()
        cases["split3_residual_blur3_batched"] = (
            lambda: mek.mek_residual_split(A3f, X3f, B3f, C3, pieces=3),
            2.0 * nb * (m3 * p3 * q3 + m3 * q3 * n3), 6)
    for name, case in cases.items():
        fn, flops = case[0], case[1]
        bf16 = len(case) > 2
        fn()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        sec = ev0.elapsed_time(ev1) * 1e-3 / reps
        tf = flops / sec / 1e12
        # Each call validates its pointers and synchronises, so this time
        # includes the call's own overhead: a lower bound on the kernels'
        # rate (the kernel trace in profiles/ gives the kernels alone).
        if bf16:
            tfb = tf * case[2]
            out[name] = {"ms_per_call": sec * 1e3, "tflops_incl_call": tf,
                         "bf16_tflops_incl_call": tfb, "peak_tflops": MFMA_BF16_PEAK_TFLOPS,
                         "frac_incl_call": tfb / MFMA_BF16_PEAK_TFLOPS}
        else:
            out[name] = {"ms_per_call": sec * 1e3, "tflops_incl_call": tf,
                         "peak_tflops": MFMA_F64_PEAK_TFLOPS,
                         "frac_incl_call": tf / MFMA_F64_PEAK_TFLOPS}
    return out


def cnn_forms(mek, torch, N=4, H=256, W=256, reps=20):
    """The warm-start network's convolutions at the training shape (batch 4,
    256 x 256): each layer shape's forward, input gradient and weight
    gradient, `reps` calls each, timed with events on the calls' stream
    (calls are stream ordered; the time includes the weight-reordering and
    partial-sum kernels of a call). FLOP = 2 N H W Cin Cout 9 per call."""
    import ctypes
    L = mek.lib()
    d = torch.device("cuda:0")
    g = torch.Generator(device=d)
    g.manual_seed(0)
    p = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None

    def bf16(C, nhwc):
        shape = (N, H, W, C) if nhwc else (N, C, H, W)
        return torch.randn(shape, generator=g, device=d).to(torch.bfloat16).view(torch.int16)

    x3, x32 = bf16(3, False), bf16(32, True)
    g3, g32 = bf16(3, False), bf16(32, True)
    y32 = torch.empty((N, H, W, 32), dtype=torch.int16, device=d)
    y3 = torch.empty((N, 3, H, W), dtype=torch.float64, device=d)
    w = {(o, c): (0.1 * torch.randn(o, c, 3, 3, generator=g, device=d)).to(torch.bfloat16).float()
         for o, c in [(32, 3), (32, 32), (3, 32)]}
    b = torch.zeros(32, device=d)
    dw = torch.empty(32 * 32 * 9, device=d)
    db = torch.empty(32, device=d)
    calls = {
        "fwd_3to32": (lambda: L.mek_cnn_conv3x3(N, 3, H, W, 32, p(x3), p(w[(32, 3)]), p(b), 1,
                                                p(y32), None, None, None), 3, 32),
        "fwd_32to32": (lambda: L.mek_cnn_conv3x3(N, 32, H, W, 32, p(x32), p(w[(32, 32)]), p(b), 1,
                                                 p(y32), None, None, None), 32, 32),
        "fwd_32to3": (lambda: L.mek_cnn_conv3x3(N, 32, H, W, 3, p(x32), p(w[(3, 32)]), p(b), 0,
                                                None, p(y3), None, None), 32, 3),
        "dgrad_32to32": (lambda: L.mek_cnn_conv3x3_grad_input(N, 32, H, W, 32, p(g32), p(x32),
                                                              p(w[(32, 32)]), p(y32), None), 32, 32),
        "dgrad_3to32": (lambda: L.mek_cnn_conv3x3_grad_input(N, 3, H, W, 32, p(g3), None,
                                                             p(w[(3, 32)]), p(y32), None), 3, 32),
        "wgrad_32x32": (lambda: L.mek_cnn_conv3x3_grad_weight(N, 32, H, W, 32, p(x32), p(g32),
                                                              p(x32), p(dw), p(db), None), 32, 32),
        "wgrad_3x32": (lambda: L.mek_cnn_conv3x3_grad_weight(N, 3, H, W, 32, p(x3), p(g32),
                                                             p(x32), p(dw), p(db), None), 3, 32),
    }
    out = {"batch": N, "height": H, "width": W}
    for name, (fn, ci, co) in calls.items():
        assert fn() == 0
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        tf = 2.0 * N * H * W * ci * co * 9 / (us * 1e-6) / 1e12
        out[name] = {"us_per_call": us, "tflops": tf, "frac_of_bf16_peak": tf / MFMA_BF16_PEAK_TFLOPS}
    return out


def blur_tensors(workloads, torch):
    """A, B (512 x 512 blur, shared), C and X* (3 x 512 x 512) on the GPU."""
    chans = workloads.blurred_image(512, 3, 2.0, seed=4, noise_std=1e-3)
    dev = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    return (t(chans[0].A), t(chans[0].B), t(np.stack([c.C for c in chans])),
            t(np.stack([c.X_star for c in chans])))


def blur_batch_forms(mek, workloads, torch):
    """The image-restoration form: 3 channels of a 512 x 512 image, banded
    Gaussian blur (sigma 2, 9 taps, rows summing to 1) on both sides, noise
    std 1e-3, a fixed budget of 100 m updates per channel (rel. error 1e-6
    is out of reach at this conditioning). One batched launch per form; the
    mixed form is compared with the FP64 iterate under the same indices."""
    A, B, C, Xs = blur_tensors(workloads, torch)
    K = 100 * 512
    out = {"budget_per_channel": K, "channels": 3}
    ref = None
    for prec in ["fp64", "mixed"]:
        plan = mek.mek_plan_create(A, B, precision=prec)
        kw = dict(variant="rgrbk", theta=0.8, max_iters=K, X_ref=Xs, seed=2408054440)
        if prec == "fp64":
            kw["hist_cap"] = K
        else:
            kw["replay_idx"] = ref
            kw["inner_iters"] = K // 8
        torch.cuda.synchronize()
        ts = time.perf_counter()
        code, res = mek.mek_solve_batched(plan, C, **kw)
        torch.cuda.synchronize()
        te = time.perf_counter() - ts
        its = sum(r.iters for r in res)
        out[prec] = {"time_s": te, "iters_per_s": its / te, "team_wgs": res[0].team_wgs,
                     "rel_err_vs_image": [r.rel_err for r in res],
                     "kernel_us_per_update": res[0].kernel_ms * 1e3 / max(res[0].iters, 1)}
        if prec == "fp64":
            ref = res[0].idx_hist.to(torch.int32).contiguous()
            X64 = torch.stack([r.X for r in res])
            # replaying channel 0's indices on every channel for the mixed form
            plan64 = plan
        else:
            _, r64 = mek.mek_solve_batched(plan64, C, variant="rgrbk", theta=0.8, max_iters=K,
                                           replay_idx=ref)
            X64r = torch.stack([r.X for r in r64])
            Xm = torch.stack([r.X for r in res])
            out[prec]["rel_diff_vs_fp64_same_indices"] = float(
                torch.linalg.norm(Xm - X64r) / torch.linalg.norm(X64r))
            out[prec]["passes"] = res[0].passes
            mek.mek_plan_destroy(plan64)
            mek.mek_plan_destroy(plan)
    # The sparse-aware update on the same channels, variant, budget and draws:
    # one work-group per channel.
    plan = mek.mek_plan_create(A, B, update="sparse")
    kw = dict(variant="rgrbk", theta=0.8, max_iters=K, X_ref=Xs, seed=2408054440, hist_cap=K)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    code, res = mek.mek_solve_batched(plan, C, **kw)
    torch.cuda.synchronize()
    te = time.perf_counter() - ts
    its = sum(r.iters for r in res)
    Xsp = torch.stack([r.X for r in res])
    same = int((res[0].idx_hist.to(torch.int32) == ref).sum())
    ka, kb, kbt, kg = mek.mek_plan_sparse_widths(plan)
    out["sparse_fp64"] = {
        "time_s": te, "iters_per_s": its / te, "work_groups": len(res),
        "rel_err_vs_image": [r.rel_err for r in res],
        "kernel_us_per_update": res[0].kernel_ms * 1e3 / max(res[0].iters, 1),
        "widths": [ka, kb, kbt, kg],
        "algorithmic_bytes_per_update": sparse_update_bytes(512, 512, 512, 512, ka, kb, kbt, kg),
        "rel_diff_vs_dense_fp64": float(torch.linalg.norm(Xsp - X64) / torch.linalg.norm(X64)),
        "same_indices_as_dense_channel0": same / K}
    mek.mek_plan_destroy(plan)
    out["discrepancy_stop"] = blur_discrepancy_forms(mek, workloads, torch, A, B, C, Xs)
    return out


def _psnr(X, Xs):
    """Peak signal-to-noise ratio of X against X* for images in [0, 1]."""
    mse = float(((X - Xs) ** 2).mean())
    return 10.0 * np.log10(1.0 / mse) if mse > 0 else float("inf")


def blur_discrepancy_forms(mek, workloads, torch, A, B, C, Xs):
    """The image form stopped by the discrepancy principle: each channel
    solved (ME-RGRBK theta 0.8) until ||C - A X B||_F <= 1.05 ||E||_F, with E
    the channel's added noise (rel. error 1e-6 against the image is out of
    reach, the blur being ill conditioned and C noisy), one solve per
    channel; the FP64 dense form, the mixed form and the FP64 sparse-aware
    form. Time to the stop and PSNR of the result against the image."""
    chans = workloads.blurred_image(512, 3, 2.0, seed=4, noise_std=1e-3)
    out = {}
    for name, prec, upd in [("fp64", "fp64", "dense"), ("mixed", "mixed", "dense"),
                            ("fp64_sparse", "fp64", "sparse")]:
        plan = mek.mek_plan_create(A, B, precision=prec, update=upd)
        per = []
        for c, ch in enumerate(chans):
            E = float(np.linalg.norm(ch.C - ch.A @ ch.X_star @ ch.B))
            tol = 1.05 * E / float(np.linalg.norm(ch.C))
            torch.cuda.synchronize()
            ts = time.perf_counter()
            r = mek.mek_solve(plan, C[c].contiguous(), variant="rgrbk", theta=0.8,
                              stop="rel_resid", tol=tol, max_iters=3_000_000,
                              seed=2408054440, instance=c)
            torch.cuda.synchronize()
            te = time.perf_counter() - ts
            per.append({"iters": r.iters, "time_s": te, "status": r.status,
                        "psnr_db": _psnr(r.X, Xs[c]),
                        "rel_err_vs_image": float(torch.linalg.norm(r.X - Xs[c]) /
                                                  torch.linalg.norm(Xs[c]))})
        mek.mek_plan_destroy(plan)
        out[name] = {"channels": per, "time_s": sum(x["time_s"] for x in per),
                     "mean_psnr_db": float(np.mean([x["psnr_db"] for x in per])),
                     "all_stopped": all(x["status"] == 0 for x in per)}
    blurred = [_psnr(torch.from_numpy(ch.C).to(A.device), Xs[c]) for c, ch in enumerate(chans)]
    out["psnr_blurred_db"] = float(np.mean(blurred))
    return out


def variant_sweep_forms(mek, workloads, torch, A, B, C, Xs, seed):
    """The variant sweep on the large workload: ME-GRBK, ME-RGRBK (theta 0.5
    and 1) and ME-MWRBK in FP64 (to relative error 1e-6) and FP32 (to 1e-5,
    residual refreshed from the iterate every 4 m updates); then ME-GRBK in FP64 on the rank-deficient case A = U V
    (rank 250, data seed 3) to 1e-6 against the least-norm solution
    A^+ C B^+ = V^T (V V^T)^-1 V X* (B has full row rank and U full column
    rank, so A^+ A is the projector onto the rows of V). Wall time of plan
    set-up + solve."""
    out = {}

    def run(key, A_, B_, C_, Xr, prec, v, th, tol):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        plan = mek.mek_plan_create(A_, B_, precision=prec)
        r = mek.mek_solve(plan, C_, variant=v, theta=th, stop="rel_err", tol=tol, X_ref=Xr,
                          max_iters=5_000_000, seed=seed)
        mek.mek_plan_destroy(plan)
        torch.cuda.synchronize()
        te = time.perf_counter() - ts
        out[key] = {"tol": tol, "time_to_tol_s": te, "iters": r.iters,
                    "iters_per_s": r.iters / te, "rel_err": r.rel_err, "status": r.status,
                    "kernel_us_per_update": r.kernel_ms * 1e3 / max(r.iters, 1)}

    for prec, tol in [("fp64", 1e-6), ("fp32", 1e-5)]:
        for v, th in [("grbk", 0.5), ("rgrbk", 0.5), ("rgrbk", 1.0), ("mwrbk", 0.5)]:
            run(f"{prec}_{v}_theta{th}", A, B, C, Xs, prec, v, th, tol)
    rd = workloads.large_rankdef()
    rng = np.random.default_rng(3)
    U = rng.standard_normal((2000, 250))
    V = rng.standard_normal((250, 500))
    assert np.allclose(U @ V, rd.A)
    Xln = V.T @ np.linalg.solve(V @ V.T, V @ rd.X_star)
    dev = A.device
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    run("fp64_grbk_rank250", t(rd.A), t(rd.B), t(rd.C), t(Xln), "fp64", "grbk", 0.5, 1e-6)
    return out


def paper_table_forms(mek, workloads, torch, trials=20):
    """The paper's Example 5.2 / Table 4 on its two Gaussian sets (Set 2: A
    140 x 30, B 70 x 160; Set 5: A 230 x 50, B 110 x 240) and Example 5.1 /
    Table 2 Set 2 (ME-BK, A 110 x 45, B 50 x 140, X0 = 1e-5 I), `trials`
    random instances each (data seeds of workloads.paper_table*), alpha =
    1/||B||_2^2, stop at squared relative error 1e-6 (relative error 1e-3)
    against X* (the limit here: A has full column rank and B full row rank).
    Per method: mean updates, mean wall time of a solve (plan set-up
    excluded, host checks and copies included), kernel time per update, and
    the paper's speed-up time(ME-RBK) / time(method)."""
    dev = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    out = {}

    def run(make, variants, X0_of=None):
        acc = {v: {"iters": [], "wall": [], "kms": []} for v in variants}
        for tr in range(trials):
            inst = make(tr)
            A, B, C, Xs = t(inst.A), t(inst.B), t(inst.C), t(inst.X_star)
            X0 = t(X0_of(inst)) if X0_of else None
            plan = mek.mek_plan_create(A, B)
            for v in variants:
                torch.cuda.synchronize()
                ts = time.perf_counter()
                r = mek.mek_solve(plan, C, X0=X0, variant=v, stop="rel_err", tol=1e-3,
                                  X_ref=Xs, max_iters=10 ** 7, seed=100 + tr)
                torch.cuda.synchronize()
                acc[v]["wall"].append(time.perf_counter() - ts)
                acc[v]["iters"].append(r.iters)
                acc[v]["kms"].append(r.kernel_ms)
                assert r.status == mek.MEK_OK
            mek.mek_plan_destroy(plan)
        res = {}
        for v in variants:
            its, wall, kms = (np.array(acc[v][k]) for k in ("iters", "wall", "kms"))
            res[v] = {"mean_iters": float(its.mean()), "mean_wall_ms": float(wall.mean() * 1e3),
                      "kernel_us_per_update": float(kms.sum() * 1e3 / its.sum())}
        if "rbk" in variants:
            for v in variants:
                res[v]["speedup_vs_rbk"] = res["rbk"]["mean_wall_ms"] / res[v]["mean_wall_ms"]
        return res

    out["table4_set2"] = run(workloads.paper_table3_set2, ["rbk", "grbk", "mwrbk"])
    out["table4_set5"] = run(workloads.paper_table3_set5, ["rbk", "grbk", "mwrbk"])
    out["table2_set2_bk"] = run(workloads.paper_table1_set2, ["bk"],
                                X0_of=lambda inst: 1e-5 * np.eye(*inst.X_star.shape))
    out["trials"] = trials
    return out


PAPER_IMAGES = [("face", 92, 92, 50_000), ("bird", 96, 96, 80_000),
                ("mandril", 125, 120, 100_000), ("barbara", 240, 192, 150_000)]


def paper_image_forms(mek, workloads, torch, names=("face", "bird", "mandril")):
    """The paper's colour-image example on synthetic images of its four
    sizes (h x w x 3, seed 7): A X A_c^T = C with A (hw x hw) the 2-D
    Gaussian blur (5 x 5 taps, sigma 6, zero padding; built on the GPU as
    T_w kron T_h), A_c the printed cross-channel matrix, no noise, X0 = 0,
    alpha = 1/||B||_2^2, the paper's update budgets, ME-RBK / ME-GRBK /
    ME-RGRBK (theta 0.8) / ME-MWRBK with the sparse-aware update (norms in
    device memory above 8192 rows). PSNR against the image (values in
    [0, 1]) for the blurred and the restored channels."""
    dev = torch.device("cuda:0")
    g = workloads.gaussian_taps(5, 6.0)
    Bm = torch.from_numpy(workloads.CROSS_CHANNEL.T.copy()).to(dev)
    out = {}
    for name, h, w, budget in PAPER_IMAGES:
        if name not in names:
            continue
        img = workloads.synthetic_image(h, w, 3, 7)
        X = torch.from_numpy(np.stack([img[c].T.reshape(-1) for c in range(3)], axis=1)).to(dev)
        Th = torch.from_numpy(workloads.blur_factor(h, g)).to(dev)
        Tw = torch.from_numpy(workloads.blur_factor(w, g)).to(dev)
        A = torch.kron(Tw, Th)
        # C = A X A_c^T, the blur applied per channel as T_h I T_w^T (= A vec(I)).
        Th_n, Tw_n = workloads.blur_factor(h, g), workloads.blur_factor(w, g)
        Cn = np.stack([(Th_n @ img[c] @ Tw_n.T).T.reshape(-1) for c in range(3)],
                      axis=1) @ workloads.CROSS_CHANNEL.T
        C = torch.from_numpy(np.ascontiguousarray(Cn)).to(dev)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        plan = mek.mek_plan_create(A, Bm, update="sparse")
        torch.cuda.synchronize()
        t_plan = time.perf_counter() - ts
        del A
        rows = {"pixels": h * w, "budget": budget, "plan_s": t_plan,
                "widths": list(mek.mek_plan_sparse_widths(plan)),
                "psnr_blurred": float(10 * np.log10(1.0 / np.mean((Cn - X.cpu().numpy()) ** 2)))}
        for v, th in [("rbk", 0.5), ("grbk", 0.5), ("rgrbk", 0.8), ("mwrbk", 0.5)]:
            torch.cuda.synchronize()
            ts = time.perf_counter()
            r = mek.mek_solve(plan, C, variant=v, theta=th, max_iters=budget, X_ref=X,
                              seed=2408054440)
            torch.cuda.synchronize()
            te = time.perf_counter() - ts
            mse = float(torch.mean((r.X - X) ** 2))
            rows[v] = {"time_s": te, "kernel_us_per_update": r.kernel_ms * 1e3 / max(r.iters, 1),
                       "iters": r.iters, "rel_err": r.rel_err,
                       "rel_resid": float(np.sqrt(r.resid2) / torch.linalg.norm(C)),
                       "psnr": float(10 * np.log10(1.0 / mse))}
            print(f"[bench] image {name} {v}: {te:.1f} s", file=sys.stderr, flush=True)
        mek.mek_plan_destroy(plan)
        out[name] = rows
    return out


def sparse_update_bytes(m, p, q, n, ka, kb, kbt, kg, elem=8):
    """Bytes one sparse-aware update moves: R_{i_k} read (n), the index and
    value of every ELL slot of B's rows and columns (q kb + n kbt), the
    changed rows of X read and written plus X_ref read (3 ka q) and the
    changed rows of R read and written (2 kg n)."""
    return elem * n + (elem + 4) * (q * kb + n * kbt) + 3 * elem * ka * q + 2 * elem * kg * n


def sparse_many_forms(mek, workloads, torch, image_counts=(32, 85), budget=100 * 512):
    """Many images at once with the sparse-aware update: n distinct 3-channel
    512 x 512 synthetic images (seeds 100..), the blur of the image form
    (sigma 2, 9 taps, noise 1e-3), every channel one instance of one launch
    (one work-group each), ME-RGRBK theta 0.8, `budget` updates per channel;
    for each n in image_counts (85 images = 255 channels: one per compute
    unit but one)."""
    out = {}
    dev = torch.device("cuda:0")
    for n_images in image_counts:
        Cs, Xs = [], []
        for i in range(n_images):
            for ch in workloads.blurred_image(512, 3, 2.0, seed=100 + i, noise_std=1e-3):
                Cs.append(ch.C)
                Xs.append(ch.X_star)
        A = torch.from_numpy(ch.A).to(dev)
        B = torch.from_numpy(ch.B).to(dev)
        C = torch.from_numpy(np.stack(Cs)).to(dev)
        X = torch.from_numpy(np.stack(Xs)).to(dev)
        del Cs, Xs
        plan = mek.mek_plan_create(A, B, update="sparse")
        torch.cuda.synchronize()
        ts = time.perf_counter()
        code, res = mek.mek_solve_batched(plan, C, variant="rgrbk", theta=0.8, max_iters=budget,
                                          X_ref=X, seed=2408054440)
        torch.cuda.synchronize()
        te = time.perf_counter() - ts
        its = sum(r.iters for r in res)
        ka, kb, kbt, kg = mek.mek_plan_sparse_widths(plan)
        per = sparse_update_bytes(512, 512, 512, 512, ka, kb, kbt, kg)
        kms = res[0].kernel_ms
        mek.mek_plan_destroy(plan)
        del C, X
        out[f"{3 * n_images}_channels"] = {
            "instances": len(res), "budget_per_instance": budget, "time_s": te,
            "iters_per_s": its / te, "kernel_ms": kms,
            "kernel_us_per_update_per_instance": kms * 1e3 / budget,
            "all_ran_budget": all(r.iters == budget for r in res),
            "mean_rel_err_vs_image": float(np.mean([r.rel_err for r in res])),
            "algorithmic_bytes_per_update": per,
            "achieved_GB_s": per * its / (kms * 1e-3) / 1e9}
    return out


def ragged_batch_forms(mek, workloads, torch, nb=64, budget=10_000):
    """The uneven-instance form: 64 independent consistent systems, m and n
    uniform in 128..1024, p and q in 64..512 (data seed 5), FP32 iterations
    (FP64 row norms, step size and stop test), a fixed budget of updates per
    instance. One ragged launch (mek_solve_multi) against the same instances
    solved one after another (mek_solve)."""
    insts = workloads.ragged_batch(nb, seed=5)
    dev = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    plans = [mek.mek_plan_create(t(i.A), t(i.B), precision="fp32") for i in insts]
    Cs = [t(i.C) for i in insts]
    kw = dict(variant="grbk", max_iters=budget, seed=2408054440)
    out = {"instances": nb, "budget_per_instance": budget, "precision": "fp32",
           "elements_of_R": int(sum(i.shape[0] * i.shape[3] for i in insts))}
    torch.cuda.synchronize()
    ts = time.perf_counter()
    code, res = mek.mek_solve_multi(plans, Cs, **kw)
    torch.cuda.synchronize()
    te = time.perf_counter() - ts
    its = sum(r.iters for r in res)
    out["one_launch"] = {"time_s": te, "iters_per_s": its / te,
                         "kernel_ms": res[0].kernel_ms, "work_groups": sum(r.team_wgs for r in res),
                         "all_ran_budget": all(r.iters == budget for r in res)}
    torch.cuda.synchronize()
    ts = time.perf_counter()
    its1 = 0
    for b, (P, C) in enumerate(zip(plans, Cs)):
        its1 += mek.mek_solve(P, C, instance=b, **kw).iters
    torch.cuda.synchronize()
    te1 = time.perf_counter() - ts
    out["one_after_another"] = {"time_s": te1, "iters_per_s": its1 / te1}
    out["speedup"] = te1 / te
    for P in plans:
        mek.mek_plan_destroy(P)
    return out


def ragged_tol_forms(mek, workloads, torch, nb=64, tol=1e-4, cap=100_000):
    """The uneven-instance form by its time-to-tolerance protocol: the same 64
    instances (data seed 5), FP32 iterations (FP64 norms, step, stop test),
    ME-GRBK to ||X - X_ref|| <= tol ||X_ref|| with X_ref = A^+ C B^+ (the
    oracle's pseudoinverses; != X* where m < p or n < q), per-instance cap
    `cap` updates. The measured set is the instances that reach the
    tolerance within the cap in a first ragged launch of all 64 (the plain
    form follows the same Philox trajectories). On that set: (1) plain, each
    instance alone (mek_solve, no residual refreshes: the arithmetic of a
    ragged launch); (2) one ragged launch with the library's default team
    sizes; (3) the same with team sizes from the autotuner (per-shape
    measured update times, the slowest instance's predicted time
    minimised), the stream-ordered call captured in a graph and replayed.
    Per instance: sizes, kappa(A) kappa(B), updates."""
    import oracle
    from paper_2408_05444_amd import autotune
    insts = workloads.ragged_batch(nb, seed=5)
    dev = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    per, Xr = [], []
    for i in insts:
        xr = oracle.least_norm(i.A, i.C, i.B)
        Xr.append(t(xr))
        sa = np.linalg.svd(i.A, compute_uv=False)
        sb = np.linalg.svd(i.B, compute_uv=False)
        per.append({"m": i.A.shape[0], "p": i.A.shape[1], "q": i.B.shape[0], "n": i.B.shape[1],
                    "kappa": float(sa[0] / sa[-1] * sb[0] / sb[-1])})
    dv = [(t(i.A), t(i.B), t(i.C)) for i in insts]
    kw = dict(variant="grbk", stop="rel_err", tol=tol, max_iters=cap, seed=2408054440)
    plans = [mek.mek_plan_create(A, B, precision="fp32") for A, B, _ in dv]
    _, first = mek.mek_solve_multi(plans, [c for _, _, c in dv], X_ref=Xr, **kw)
    for P in plans:
        mek.mek_plan_destroy(P)
    S = [b for b in range(nb) if first[b].status == 0]
    for b in range(nb):
        per[b]["iters_first_launch"] = first[b].iters
    # On the set, instance j (= S[j]) draws under Philox key (seed, j) in
    # every form, so the forms follow the same trajectories; the cap is
    # doubled so that a changed key does not drop an instance from the set.
    kw = dict(kw, max_iters=2 * cap)
    plain_t = []
    for j, b in enumerate(S):
        A, B, C = dv[b]
        plan = mek.mek_plan_create(A, B, precision="fp32")
        torch.cuda.synchronize()
        ts = time.perf_counter()
        r = mek.mek_solve(plan, C, X_ref=Xr[b], instance=j, refresh_period=-1, **kw)
        torch.cuda.synchronize()
        plain_t.append(time.perf_counter() - ts)
        mek.mek_plan_destroy(plan)
        per[b].update({"iters_plain": r.iters, "status_plain": r.status})
    out = {"instances": nb, "tol": tol, "cap": cap, "precision": "fp32",
           "measured_set": len(S), "per_instance": per,
           "plain": {"time_s": float(sum(plain_t)),
                     "updates": int(sum(per[b]["iters_plain"] for b in S)),
                     "all_reached_tol": all(per[b]["status_plain"] == 0 for b in S)}}
    out["plain"]["iters_per_s"] = out["plain"]["updates"] / out["plain"]["time_s"]

    def ragged(plans, label):
        Cs, Xs_ = [dv[b][2] for b in S], [Xr[b] for b in S]
        kwm = dict(kw)
        kwm["X_ref"] = Xs_
        torch.cuda.synchronize()
        ts = time.perf_counter()
        _, res = mek.mek_solve_multi(plans, Cs, **kwm)
        torch.cuda.synchronize()
        te = time.perf_counter() - ts
        upd = int(sum(r.iters for r in res))
        out[label] = {"time_s": te, "updates": upd, "iters_per_s": upd / te,
                      "all_reached_tol": all(r.status == 0 for r in res),
                      "teams": [r.team_wgs for r in res], "kernel_ms": res[0].kernel_ms}
        return res

    plans = [mek.mek_plan_create(dv[b][0], dv[b][1], precision="fp32") for b in S]
    ragged(plans, "batched_default_teams")
    for P in plans:
        mek.mek_plan_destroy(P)
    ts = time.perf_counter()
    table = autotune.Table()
    times = autotune.tune([dv[b] for b in S], "fp32", table, cus)
    teams = autotune.allocate(times, [per[b]["iters_plain"] for b in S], cus)
    out["autotuned_teams"] = teams
    out["autotune"] = {"time_s": time.perf_counter() - ts, "table": table.path,
                       "shapes_in_table": len(table.data)}
    plans = autotune.plans_for([dv[b] for b in S], "fp32", teams)
    ragged(plans, "batched_autotuned")
    # The autotuned launch captured in a graph and replayed.
    Cs, Xs_ = [dv[b][2] for b in S], [Xr[b] for b in S]
    kwa = dict(kw)
    kwa["X_ref"] = Xs_
    Xg, repg = mek.mek_solve_multi_async(plans, Cs, **kwa)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mek.mek_solve_multi_async(plans, Cs, X_out=Xg, reports=repg, **kwa)
    reps = []
    for _ in range(3):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        g.replay()
        torch.cuda.synchronize()
        reps.append(time.perf_counter() - ts)
    rd = [mek.read_device_report(repg[j]) for j in range(len(S))]
    upd = int(sum(d["iters"] for d in rd))
    tg = float(np.median(reps))
    out["batched_autotuned_graph"] = {"time_s": tg, "updates": upd, "iters_per_s": upd / tg,
                                      "all_reached_tol": all(d["status"] == 0 for d in rd),
                                      "replays": 3}
    for P in plans:
        mek.mek_plan_destroy(P)
    out["speedup_graph_vs_plain"] = out["plain"]["time_s"] / tg
    return out


def warm_start_forms(mek, workloads, torch, n_train=1024, n_test=512, epochs=20, lr=2e-3,
                     size=256, tau=1e-3):
    """The learned warm start: 3-channel 256 x 256 blurred images (sigma
    uniform on [1, 3], no noise; training seeds 100000 + i, held-out
    200000 + j), labels = the FP64 ME-GRBK iterate at relative residual tau
    (= 1e-3, the smallest of 1e-6..1e-3 that the X0 = 0 solve reaches
    within 1e6 updates on held-out images 0-7), computed by ragged launches
    of sparse-update plans; the network trained by the library's BF16
    kernels; then every channel of the held-out images solved to tau from
    X0 = 0 and from X0 = C + f(C), again in ragged sparse launches."""
    from paper_2408_05444_amd import warmstart
    dev = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    train = []
    for i in range(n_train):
        A, B, C, _, _ = workloads.warmstart_image(100000 + i, size=size)
        train.append((t(A), t(B), t(C)))
        if (i + 1) % 2000 == 0:
            print(f"[bench] warm start: {i + 1} training images made", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    labels = warmstart.solver_labels(mek, train, tau=tau, seed=2408054440)
    torch.cuda.synchronize()
    t_labels = time.perf_counter() - ts
    Cs = torch.stack([c for _, _, c in train])
    Ls = torch.stack(labels)
    del train, labels
    net = warmstart.WarmStartNet(seed=0)
    ts = time.perf_counter()
    hist = net.train(Cs, Ls, epochs=epochs, batch=4, lr=lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - ts
    del Cs, Ls
    held, sig = [], []
    for j in range(n_test):
        A, B, C, _, sigma = workloads.warmstart_image(200000 + j, size=size)
        held.append((t(A), t(B), t(C)))
        sig.append(sigma)
    r = warmstart.compare_warm_start(mek, net, held, tau=tau, seed=2408054440)
    iz, iw = np.array(r["iters_zero"]), np.array(r["iters_warm"])
    return {"tau_rel_resid": tau, "train_images": n_train, "epochs": epochs,
            "params": net.num_params(), "label_time_s": t_labels, "train_time_s": t_train,
            "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1],
            "held_out_images": n_test, "held_out_channels": int(iz.size),
            "mean_iters_zero": float(iz.mean()), "mean_iters_warm": float(iw.mean()),
            "iters_ratio": float(iw.mean() / iz.mean()),
            "median_iters_ratio_per_channel": float(np.median(iw / iz)),
            "time_to_tau_zero_s": r["time_zero_s"], "time_to_tau_warm_s": r["time_warm_s"],
            "time_ratio": r["time_warm_s"] / r["time_zero_s"],
            "all_reached_tau": all(s == 0 for s in r["status_zero"] + r["status_warm"]),
            "fallbacks": int(sum(r["fallback"])),
            "mean_start_rel_resid_warm": float(np.mean(r["start_rel_resid_warm"]))}


def _host_cpu():
    """Model name (lscpu) and logical CPU count of the host."""
    model = "unknown"
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    return model, os.cpu_count()


def _oracle_rate(oracle, inst, seed, updates, runs, omp, alpha):
    """Updates/s of the oracle's iteration loop: median over `runs` solves of
    `updates` ME-GRBK updates, each minus the median time of the set-up alone
    (row norms, Gram matrices, initial residual: a solve with 0 updates)."""
    kw = dict(variant="grbk", alpha=alpha, seed=seed, omp=omp, hist_cap=1)
    setup, total = [], []
    for _ in range(runs):
        t0 = time.perf_counter()
        oracle.solve(inst.A, inst.B, inst.C, max_iters=0, **kw)
        t1 = time.perf_counter()
        oracle.solve(inst.A, inst.B, inst.C, max_iters=updates, **kw)
        t2 = time.perf_counter()
        setup.append(t1 - t0)
        total.append(t2 - t1)
    loop = max(float(np.median(total)) - float(np.median(setup)), 1e-9)
    return updates / loop, float(np.median(setup))


def cpu_baseline(inst, seed, workloads):
    """The CPU oracle on this host, as it stands: the plain single-threaded
    build and the OpenMP build of the same source (row loops over all
    threads, identical results). Headline: the 2000 x 500 / 500 x 2000 FP64
    ME-GRBK instance, median of 5 windows of 200 updates (all threads) and of
    3 windows of 100 updates (one thread), set-up excluded. Also the
    100 x 40 / 40 x 100 instance's full time to rel. error 1e-6 (median of 5,
    one thread) and a 200-update window of one 512 x 512 blur channel."""
    import oracle
    alpha = oracle.spectral_alpha(inst.B)
    model, ncpu = _host_cpu()
    thr = oracle.threads(omp=True)
    rate_all, set_all = _oracle_rate(oracle, inst, seed, 200, 5, True, alpha)
    rate_one, set_one = _oracle_rate(oracle, inst, seed, 100, 3, False, alpha)
    c1 = workloads.small()
    a1 = oracle.spectral_alpha(c1.B)
    t1s, it1 = [], 0
    for _ in range(5):
        t0 = time.perf_counter()
        r = oracle.solve(c1.A, c1.B, c1.C, variant="grbk", alpha=a1, stop=oracle.STOP_REL_ERR,
                         tol=1e-6, Xref=c1.X_star, max_iters=10 ** 7, seed=seed, hist_cap=1)
        t1s.append(time.perf_counter() - t0)
        it1 = r.iters
    blur = workloads.blurred_image(512, 1, 2.0, seed=4, noise_std=1e-3)[0]
    rate_blur, _ = _oracle_rate(oracle, blur, seed, 200, 3, True, oracle.spectral_alpha(blur.B))
    return {"value": rate_all, "unit": "iters/s", "cores": thr, "kind": "oracle",
            "sample": f"ME-GRBK on the same 2000x500/500x2000 FP64 instance, OpenMP build on "
                      f"{thr} threads: median of 5 windows of 200 updates, set-up "
                      f"({set_all:.2f} s) excluded",
            "host": {"cpu_model": model, "logical_cpus": ncpu},
            "single_thread": {"value": rate_one, "unit": "iters/s", "cores": 1,
                              "sample": "median of 3 windows of 100 updates, set-up "
                                        f"({set_one:.2f} s) excluded"},
            "small_100x40_time_to_1e-6": {"time_s": float(np.median(t1s)), "iters": it1,
                                          "iters_per_s": it1 / float(np.median(t1s)),
                                          "cores": 1, "runs": 5},
            "blur512_one_channel": {"value": rate_blur, "unit": "iters/s", "cores": thr,
                                    "sample": "median of 3 windows of 200 ME-GRBK updates, "
                                              "set-up excluded"}}


def twosided_form(mek, torch, A, B, C, Xs):
    """The two-sided block projection (s = t = 32, theta = 1/2) on the large
    instance to relative error 1e-6, plan set-up included in the time."""
    torch.cuda.synchronize()
    ts = time.perf_counter()
    plan = mek.mek_plan_create(A, B)
    try:
        r = mek.mek_solve(plan, C, variant="twosided", theta=0.5, block_rows=TS_BLOCK,
                          block_cols=TS_BLOCK, stop="rel_err", tol=1e-6, X_ref=Xs,
                          max_iters=1_000_000)
    finally:
        mek.mek_plan_destroy(plan)
    torch.cuda.synchronize()
    te = time.perf_counter() - ts
    return {"tol": 1e-6, "block": [TS_BLOCK, TS_BLOCK], "theta": 0.5, "time_to_tol_s": te,
            "steps": r.iters, "rel_err": r.rel_err, "status": r.status,
            "kernel_us_per_step": r.kernel_ms * 1e3 / max(r.iters, 1)}


def small_forms(mek, workloads, torch, reps=7):
    """Plain ME-GRBK on A 100 x 40, B 40 x 100, X* 40 x 40 iid N(0, 1) (data
    seed 1), C = A X* B, X0 = 0, FP64, alpha = 1/||B||_2^2 from the oracle's
    SVD passed explicitly, stopped at ||X - X*||_F <= 1e-6 ||X*||_F (checked
    before every update). Time to tolerance (plan made once; median over
    `reps` solves, host wait and report copy included) and kernel time."""
    import oracle
    inst = workloads.small()
    alpha = oracle.spectral_alpha(inst.B)
    dev = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    A, B, C, Xs = t(inst.A), t(inst.B), t(inst.C), t(inst.X_star)
    plan = mek.mek_plan_create(A, B, alpha=alpha)
    kw = dict(variant="grbk", alpha=alpha, stop="rel_err", tol=1e-6, X_ref=Xs,
              max_iters=10 ** 7, seed=2408054440)
    mek.mek_solve(plan, C, **kw)
    walls, res = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        res = mek.mek_solve(plan, C, **kw)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - ts)
    mek.mek_plan_destroy(plan)
    w = float(np.median(walls))
    return {"tol": 1e-6, "iters": res.iters, "status": res.status, "rel_err": res.rel_err,
            "time_to_tol_s": w, "iters_per_s": res.iters / w, "team_wgs": res.team_wgs,
            "kernel_us_per_update": res.kernel_ms * 1e3 / max(res.iters, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--variant", default="grbk")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--gemm-only", action="store_true",
                    help="only time the FP64 MFMA GEMMs of the set-up and residual engine at the "
                         "workload's sizes (for a kernel trace) and print them")
    ap.add_argument("--warm-start-only", action="store_true",
                    help="only run the learned warm-start form and print it")
    ap.add_argument("--train-images", type=int, default=0,
                    help="warm-start form: training images (0: the default)")
    ap.add_argument("--test-images", type=int, default=0,
                    help="warm-start form: held-out images (0: the default)")
    ap.add_argument("--epochs", type=int, default=0, help="warm-start form: epochs (0: the default)")
    ap.add_argument("--sweep-only", action="store_true",
                    help="only run the variant sweep on the large workload and print it")
    ap.add_argument("--image-only", action="store_true",
                    help="only run the paper's colour-image model at its image sizes and print it")
    ap.add_argument("--images", default="",
                    help="with --image-only: comma-separated sizes by the paper's image names "
                         "(face, bird, mandril, barbara)")
    ap.add_argument("--paper-only", action="store_true",
                    help="only run the paper's Table 4 / Table 2 Gaussian sets and print them")
    ap.add_argument("--sparse-only", action="store_true",
                    help="only run the image forms (dense and sparse-aware updates) and print them")
    ap.add_argument("--cnn-only", action="store_true",
                    help="only time the warm-start network's convolutions at batch 4, 256 x 256")
    ap.add_argument("--twosided-only", action="store_true",
                    help="only run the two-sided block projection to 1e-6 and print it")
    ap.add_argument("--ragged-only", action="store_true",
                    help="only run the uneven-instance batch form and print it")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB device-to-device once (a known-size kernel for scaling "
                         "the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; multi-GPU runs are not part of it "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": src.numel() * 8}), flush=True)
        return
    import paper_2408_05444_amd as mek
    import workloads

    inst = workloads.large()
    m, p, q, n = inst.shape
    dev = torch.device("cuda:0")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    A, B, C, Xs = t(inst.A), t(inst.B), t(inst.C), t(inst.X_star)
    seed = 2408054440
    torch.cuda.synchronize()
    if args.warm_start_only:
        kw = {}
        if args.train_images:
            kw["n_train"] = args.train_images
        if args.test_images:
            kw["n_test"] = args.test_images
        if args.epochs:
            kw["epochs"] = args.epochs
        print(json.dumps({"warm_start": warm_start_forms(mek, workloads, torch, **kw)}), flush=True)
        return
    if args.sweep_only:
        print(json.dumps({"variant_sweep": variant_sweep_forms(mek, workloads, torch, A, B, C, Xs,
                                                               seed)}), flush=True)
        return
    if args.image_only:
        names = args.images.split(",") if args.images else ("face", "bird", "mandril")
        print(json.dumps({"paper_images": paper_image_forms(mek, workloads, torch, names)}),
              flush=True)
        return
    if args.paper_only:
        print(json.dumps({"paper_tables": paper_table_forms(mek, workloads, torch)}), flush=True)
        return
    if args.sparse_only:
        print(json.dumps({"blur3_batched": blur_batch_forms(mek, workloads, torch),
                          "blur_sparse_many": sparse_many_forms(mek, workloads, torch)}),
              flush=True)
        return
    if args.cnn_only:
        print(json.dumps({"cnn_convolutions": cnn_forms(mek, torch)}), flush=True)
        return
    if args.twosided_only:
        print(json.dumps({"twosided": twosided_form(mek, torch, A, B, C, Xs)}), flush=True)
        return
    if args.ragged_only:
        print(json.dumps({"ragged64_fp32": ragged_batch_forms(mek, workloads, torch),
                          "ragged64_fp32_to_tol": ragged_tol_forms(mek, workloads, torch)}),
              flush=True)
        return
    if args.gemm_only:
        print(json.dumps({"gemm_mfma_f64": gemm_forms(mek, torch, A, B, Xs, C,
                                                      blur=blur_tensors(workloads, torch))}),
              flush=True)
        return

    def step(precision="fp64", tol=1e-6, max_iters=5_000_000):
        plan = mek.mek_plan_create(A, B, precision=precision)
        res = mek.mek_solve(plan, C, variant=args.variant, stop="rel_err", tol=tol, X_ref=Xs,
                            max_iters=max_iters, seed=seed)
        mek.mek_plan_destroy(plan)
        return res

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    iters = sum(r.iters for r in results)
    kernel_ms = sum(r.kernel_ms for r in results)
    ok = all(r.status == mek.MEK_OK for r in results)
    bpu = algorithmic_bytes_per_update(m, p, q, n, 8)
    achieved = bpu * iters / (kernel_ms * 1e-3) / 1e9
    line = {
        "metric": "time-to-rel-err 1e-6 & iters/s: ME-GRBK plain GPU vs mixed/batched/warm-start",
        "value": iters / elapsed,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded iid N(0,1) A, B, X*; C = A X* B)",
        "config": {"workload": "ME-GRBK theta=1/2, A 2000x500, B 500x2000, X* 500x500, "
                               "consistent, X0=0, stop ||X-X*||/||X*|| <= 1e-6",
                   "m": m, "p": p, "q": q, "n": n, "variant": args.variant,
                   "iters_to_tol": results[-1].iters, "rel_err": results[-1].rel_err,
                   "converged": ok, "team_wgs": results[-1].team_wgs,
                   "r_in_lds": results[-1].r_in_lds},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(results[-1].team_wgs, results[-1].iters)
                     if args.variant == "grbk" else None,
                     "traffic_unit": "bytes per launch (one launch = one solve)",
                     "kernel": "solve_kernel<double,LDS>",
                     "kernel_us_per_update": kernel_ms * 1e3 / max(iters, 1),
                     "algorithmic_bytes_per_update": bpu},
    }
    # The update is bound by the latency of its exchanges between work-groups,
    # not by bandwidth (R lives in LDS): the same team's exchanges and block
    # collectives alone, timed by the library, give the floor under it.
    floor = mek.mek_exchange_floor(results[-1].team_wgs, m, n, q, rounds=20000)
    line["roofline"]["regime"] = ("latency: the exchanges between the team's work-groups "
                                  "(R stays in LDS, 0.67 MB per update crosses HBM)")
    line["roofline"]["latency_floor_us_per_update"] = floor
    line["roofline"]["latency_frac"] = floor / (kernel_ms * 1e3 / max(iters, 1))
    if not args.no_forms:
        forms = {}
        # FP32 (residual refreshed from the iterate every 4 m updates on the
        # split-BF16 engine) is timed to its target 1e-5; mixed to 1e-6.
        for prec, tol, cap in [("fp32", 1e-5, 1_000_000), ("mixed", 1e-6, 5_000_000)]:
            torch.cuda.synchronize()
            ts = time.perf_counter()
            r = step(prec, tol, cap)
            torch.cuda.synchronize()
            te = time.perf_counter() - ts
            forms[prec] = {"tol": tol, "time_to_tol_s": te, "iters": r.iters,
                           "iters_per_s": r.iters / te, "rel_err": r.rel_err, "status": r.status,
                           "passes": r.passes}
        forms["fp64"] = {"tol": 1e-6, "time_to_tol_s": elapsed / args.steps,
                         "iters": results[-1].iters,
                         "iters_per_s": iters / elapsed, "rel_err": results[-1].rel_err,
                         "status": results[-1].status}
        forms["twosided"] = twosided_form(mek, torch, A, B, C, Xs)
        # Each form reports to stderr when it ends (the run takes minutes).
        for name, fn in [
                ("small_100x40", lambda: small_forms(mek, workloads, torch)),
                ("variant_sweep", lambda: variant_sweep_forms(mek, workloads, torch, A, B, C, Xs, seed)),
                ("blur3_batched", lambda: blur_batch_forms(mek, workloads, torch)),
                ("blur_sparse_many", lambda: sparse_many_forms(mek, workloads, torch)),
                ("paper_tables", lambda: paper_table_forms(mek, workloads, torch)),
                ("paper_images", lambda: paper_image_forms(mek, workloads, torch)),
                ("ragged64_fp32", lambda: ragged_batch_forms(mek, workloads, torch)),
                ("ragged64_fp32_to_tol", lambda: ragged_tol_forms(mek, workloads, torch)),
                ("warm_start", lambda: warm_start_forms(mek, workloads, torch))]:
            t0 = time.perf_counter()
            forms[name] = fn()
            print(f"[bench] form {name} done in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                  flush=True)
        line["forms"] = forms
        line["gemm_mfma_f64"] = gemm_forms(mek, torch, A, B, Xs, C,
                                           blur=blur_tensors(workloads, torch))
        line["cnn_convolutions"] = cnn_forms(mek, torch)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(inst, seed, workloads)
    torch.cuda.synchronize()   # nothing of ours is in flight at interpreter exit
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
