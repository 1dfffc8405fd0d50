#!/usr/bin/env python3
"""Throughput of randomized LUPP ID + CUR on one MI355X.

Workload (poly8192): A = U diag(s) V^T, 8192 x 8192, s_i = i^-2, U and V
Haar-orthonormal (seeded, generated on the GPU with torch, rounded to FP32
storage), Gaussian embedding Omega of l = k + 16 = 272 rows, k = 256.

One step = one pass of the whole path over the resident inputs:
  sketch X = Omega A  ->  column LUPP on X (J, factors)  ->  Z (+1 FP64
  refinement in the FP32/BF16 modes)  ->  CUR (LUPP on C -> I, stable U)
  ->  ID and CUR residuals.
Modes: f64 (the FP32 values of A promoted to FP64; FP64 everywhere, the
paper's arithmetic), f32 (FP32 storage and arithmetic for sketch/LUPP), bf16
(A and Omega stored BF16; BF16 MFMA sketch, FP32 LUPP, FP64 Z/U).

Prints one JSON line.  `value` is decompositions per second of the main
mode (default f64) with the inputs already in HBM, back-to-back steps (the
256 MB last-level cache warm); `cold` repeats the step with a 512 MiB
buffer written between steps.  `roofline` describes the call that takes the
most time per step; `cpu_baseline` times the FP64 numpy oracle on the host
cores on one decomposition of the same workload (all threads, and one
thread); `parity` compares every mode's outputs with the FP64 oracle on the
same stored values; `configs` runs the two precision forms at their own
sizes (16384^2 BF16, k = 512; 65536 x 4096 with the FP8 sketch, k = 384).

Before the timed region the script runs plain device-to-device copies of
CALIB_MIB MiB (an elementwise kernel that reads and writes exactly that many
bytes), timed with events: the measured HBM ceiling.  Hardware byte
counters taken over this same command are scaled by what they read for that
copy.  `roofline.traffic` is filled from the counter summary committed under
profiles/ only while the LUPP source file still has the hash recorded there,
else it is null.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

M = N = 8192
K = 256
L = 272
PEAK_HBM = 8.0e12  # B/s, MI355X HBM3E
PEAK_MFMA = {"bf16": 2.5e15, "f32": 157.3e12, "f64": 78.6e12}  # dense FLOP/s
CALIB_MIB = 512
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lupp_poly8192_traffic.json")
LUPP_SOURCE = os.path.join(ROOT, "paper_2104_05877_amd", "csrc", "lupp.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", default="f64", choices=["bf16", "f32", "f64"],
                    help="main mode: its step is `value` (f64 is the paper's arithmetic)")
    ap.add_argument("--reports-mode", default="bf16", choices=["bf16", "f32", "f64"],
                    help="storage of the input the reports of the added rows run on")
    ap.add_argument("--cold-steps", type=int, default=10,
                    help="steps of the main mode with the last-level cache flushed between steps")
    ap.add_argument("--no-parity", action="store_true", help="skip the oracle comparison of every mode")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the precision forms at their own sizes")
    ap.add_argument("--other-steps", type=int, default=8, help="timed steps of the other two modes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--only-main", action="store_true", help="time the main mode only")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-rank report")
    ap.add_argument("--no-overlap", action="store_true",
                    help="report the sequential step as the value (no concurrent Z / CUR branches)")
    ap.add_argument("--two-sided-only", action="store_true",
                    help="run only the Alg. 3 and Rand-CPQR reports on the main mode's input (for profiling)")
    ap.add_argument("--sketch-shapes-only", action="store_true",
                    help="run only the sketch report on the 16384^2 BF16 and 65536 x 4096 FP8 "
                         "shapes (for profiling; no poly8192 input)")
    ap.add_argument("--sparse-only", action="store_true",
                    help="run only the CSC sketches of the SNN matrix, without the pivoting "
                         "(for profiling; no poly8192 input)")
    ap.add_argument("--learned-only", action="store_true",
                    help="run only the learned-rank report (no poly8192 input)")
    ap.add_argument("--input-cache", default=None,
                    help="folder: load the FP32 workload from it if stored there, else "
                         "generate it and store it (lets profiled runs skip the QR-based "
                         "generation)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="no GPU work: turn two rocprofv3 --pmc csv folders (FETCH_SIZE, "
                         "WRITE_SIZE) of a --only-main run into the recorded LUPP traffic")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_inputs(torch, seed, cache=None):
    from paper_2104_05877_amd import inputs

    path = os.path.join(cache, f"poly8192_seed{seed}.pt") if cache else None
    if path and os.path.exists(path):
        d = torch.load(path, weights_only=True)
        # stored as the contiguous transposes (n x m and m x l)
        a32 = d["a_t"].cuda().T
        om32 = d["om_t"].cuda().T
    else:
        a32, om32 = inputs.torch_poly8192(seed, "cuda", M, N, L)
        if path:
            os.makedirs(cache, exist_ok=True)
            torch.save({"a_t": a32.T.cpu(), "om_t": om32.T.cpu()}, path)
    out = {
        "f32": (a32, om32),
        "f64": (a32.T.contiguous().double().T, om32.T.contiguous().double().T),
        "bf16": (a32.T.contiguous().bfloat16().T, om32.T.contiguous().bfloat16().T),
    }
    torch.cuda.synchronize()
    return out


def run_mode(torch, R, ctx, A, Om, steps, warmup):
    """Time `steps` full steps; per-call HIP-event times on the context stream."""
    refine = 0 if A.dtype == torch.float64 else 1
    stream = ctx.stream
    names = ["sketch", "select_columns", "id_coeffs", "cur", "residual_id", "residual_cur"]
    decomp = names[:4]  # sketch .. CUR; the residuals are reported on top

    def step(ev):
        ev[0].record(stream)
        X = R.rpid_sketch(ctx, A, Om)
        ev[1].record(stream)
        J, Lf, Uf, diag, keff, st = R.rpid_select_columns(ctx, X, K, sync=False)
        ev[2].record(stream)
        Z, _ = R.rpid_id_coeffs(ctx, X, K, J, Lf, Uf, refine_steps=refine)
        ev[3].record(stream)
        I, U, keff_i, st_i = R.rpid_cur(ctx, A, K, J)
        ev[4].record(stream)
        rid = R.rpid_residual(ctx, R.RESIDUAL_ID, A, K, J, Z=Z)
        ev[5].record(stream)
        rcur = R.rpid_residual(ctx, R.RESIDUAL_CUR, A, K, J, I=I, U=U)
        ev[6].record(stream)
        return rid, rcur, st_i, J, I, X, Z, U, Lf, Uf

    def mk():
        return [torch.cuda.Event(enable_timing=True) for _ in range(7)]

    for _ in range(warmup):
        step(mk())
    torch.cuda.synchronize()
    evs = [mk() for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        out = step(evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = {n: 0.0 for n in names}
    step_ms, decomp_ms = [], []
    for ev in evs:
        for j, n in enumerate(names):
            per[n] += ev[j].elapsed_time(ev[j + 1]) / steps  # ms
        step_ms.append(ev[0].elapsed_time(ev[6]))
        decomp_ms.append(ev[0].elapsed_time(ev[4]))
    rid, rcur, st_i, J, I, X, Z, U, Lf, Uf = out
    import numpy as np

    return dict(ms_per_step=(t1 - t0) * 1e3 / steps, per_call_ms=per, rid=rid, rcur=rcur,
                status_cur=st_i, J=J.cpu().numpy(), I=I.cpu().numpy(),
                X=X.double().cpu().numpy(), Z=Z.cpu().numpy(), U=U.cpu().numpy(),
                Lf=Lf.double().cpu().numpy(), Uf=Uf.double().cpu().numpy(),
                step_ms_p10_p50_p90=[float(np.percentile(step_ms, q)) for q in (10, 50, 90)],
                decomp_ms_p10_p50_p90=[float(np.percentile(decomp_ms, q)) for q in (10, 50, 90)])


def overlapped_steps(torch, R, ctx, ctx2, A, Om, steps, warmup):
    """Wall time per step of the same path with Z and the ID residual on a
    second context and stream, concurrent with the CUR step and its residual
    (rpid.decompose_overlapped; bitwise the same outputs).  Returns (ms per
    step, the last step's outputs)."""
    for _ in range(warmup):
        R.decompose_overlapped(ctx, ctx2, A, Om, K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = R.decompose_overlapped(ctx, ctx2, A, Om, K)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, out


def sketch_loop(torch, R, ctx, A, Om, reps=20):
    """GPU time per sketch call (Omega transpose, streaming GEMM, split-K sum)
    over `reps` back-to-back calls, so the host runs ahead and no launch gap
    between calls is counted."""
    for _ in range(3):
        R.rpid_sketch(ctx, A, Om)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(ctx.stream)
    for _ in range(reps):
        R.rpid_sketch(ctx, A, Om)
    e1.record(ctx.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def sketch_shapes_report(torch, R, ctx, reps=10):
    """The sketch call on the two larger sketch workloads, random operands
    (timing does not depend on the values): A 16384 x 16384 BF16 with l = 544
    (arithmetic intensity above the BF16 ridge, so the MFMA rate bounds it),
    and the FP8 sketch of a 65536 x 4096 FP32 matrix with l = 400 (the call
    includes the per-column E4M3 quantisation of A, a read of 4mn and a write
    of mn bytes).  GPU time per call back to back; utilisation = 2lmn flops per
    call over the dense MFMA peak of the operand type."""
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    out = {}
    for name, (m, n, l, fp8) in {"bf16_16384x16384_l544": (16384, 16384, 544, False),
                                 "fp8_65536x4096_l400": (65536, 4096, 400, True)}.items():
        if fp8:
            A = torch.randn((n, m), device="cuda", generator=g).abs_().T
            Om = torch.randn((m, l), device="cuda", generator=g).T
            call, peak = (lambda: R.rpid_sketch_fp8(ctx, A, Om)), 5.0e15
        else:
            A = torch.randn((n, m), device="cuda", generator=g).to(torch.bfloat16).T
            Om = torch.randn((m, l), device="cuda", generator=g).to(torch.bfloat16).T
            call, peak = (lambda: R.rpid_sketch(ctx, A, Om)), PEAK_MFMA["bf16"]
        for _ in range(2):
            call()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(reps):
            call()
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms_per_call": ms, "tflops": 2.0 * l * m * n / (ms * 1e-3) / 1e12,
                     "mfma_util": 2.0 * l * m * n / (ms * 1e-3) / peak}
        del A, Om
        torch.cuda.empty_cache()
    return out


def power_report(torch, R, ctx, A, Om, plain):
    """Rand-LUPP-1piter: the row sketch X = Omega A^T A (eq. def_power_iter,
    q = 1) in place of Omega A, same l, same Omega values.  GPU time per
    power-sketch call back to back, and the ID/CUR residuals of one full
    decomposition on it beside those of the plain sketch."""
    refine = 0 if A.dtype == torch.float64 else 1
    for _ in range(2):
        R.rpid_sketch_power1(ctx, A, Om)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record(ctx.stream)
    for _ in range(reps):
        X = R.rpid_sketch_power1(ctx, A, Om)
    e1.record(ctx.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    J, Lf, Uf, diag, keff, st = R.rpid_select_columns(ctx, X, K)
    Z, _ = R.rpid_id_coeffs(ctx, X, K, J, Lf, Uf, refine_steps=refine)
    I, U, keff_i, st_i = R.rpid_cur(ctx, A, K, J)
    rid = R.rpid_residual(ctx, R.RESIDUAL_ID, A, K, J, Z=Z)
    rcur = R.rpid_residual(ctx, R.RESIDUAL_CUR, A, K, J, I=I, U=U)
    # Rand-CPQR-1piter on the same power sketch (column-pivoted QR, its own Z)
    Jq, Rq, _, _, stq = R.rpid_select_columns_cpqr(ctx, X, K)
    rid_q = R.rpid_residual(ctx, R.RESIDUAL_ID, A, K, Jq, Z=R.rpid_id_coeffs_cpqr(ctx, K, Jq, Rq))
    return {"sketch_power1_ms": ms, "sketch_ms": plain["per_call_ms"]["sketch"],
            "residual_id": rid, "residual_cur": rcur,
            "residual_id_plain": plain["rid"], "residual_cur_plain": plain["rcur"],
            "residual_id_cpqr_1piter": rid_q,
            "status_columns": st, "status_rows": st_i}


def two_sided_report(torch, R, ctx, A, Gam, plain):
    """Alg. 3 on the same input: X = Gamma A and Y^T = Omega A^T in one
    call (BF16: one pass over A in row blocks), LUPP on both, then the
    sketch-only estimates (row ID from Y, core S^{-1}) beside the stable CUR
    of the same indices.  GPU times per call back to back."""
    from paper_2104_05877_amd import inputs

    Om = inputs.torch_gaussian(L, N, 1234, A.device, dtype=A.dtype).T.contiguous().T
    refine = 0 if A.dtype == torch.float64 else 1

    def timed(fn, reps=10):
        for _ in range(2):
            out = fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(reps):
            out = fn()
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1) / reps

    (X, Yt), ms_two = timed(lambda: R.rpid_sketch_two_sided(ctx, A, Gam, Om))
    _, ms_plain = timed(lambda: R.rpid_sketch(ctx, A, Gam))

    def select_both():
        cj = R.rpid_select_columns(ctx, X, K, sync=False)
        ci = R.rpid_select_columns(ctx, Yt, K, sync=False)
        return cj, ci

    ((J, Lf, Uf, _, _, _), (I, Li, Ui, _, _, _)), ms_sel = timed(select_both, reps=5)
    Z, _ = R.rpid_id_coeffs(ctx, X, K, J, Lf, Uf, refine_steps=refine)
    Zy, _ = R.rpid_id_coeffs(ctx, Yt, K, I, Li, Ui, refine_steps=refine)
    (Us, st), ms_core = timed(lambda: R.rpid_cur_sketch(ctx, A, K, J, I), reps=5)
    Ist, Ust, _, _ = R.rpid_cur(ctx, A, K, J)  # Alg. 2's row indices, stable core, for reference
    return {
        "two_sided_sketch_ms": ms_two, "plain_sketch_ms": ms_plain,
        "select_columns_and_rows_ms": ms_sel, "cur_sketch_core_ms": ms_core,
        "indices_only_ms": ms_two + ms_sel,
        "residual_id": R.rpid_residual(ctx, R.RESIDUAL_ID, A, K, J, Z=Z),
        "residual_row_id": R.rpid_residual(ctx, R.RESIDUAL_ROW_ID, A, K, None, Z=Zy, I=I),
        "residual_cur_sketch_core": R.rpid_residual(ctx, R.RESIDUAL_CUR, A, K, J, I=I, U=Us),
        "residual_cur_alg2_stable": R.rpid_residual(ctx, R.RESIDUAL_CUR, A, K, J, I=Ist, U=Ust),
        "status_core": st,
    }


def cpqr_report(torch, R, ctx, A, Om, plain):
    """Rand-CPQR on the same sketch as Rand-LUPP (the paper's comparison):
    GPU time of the column-pivoted QR (k steps) and of its Z, and the ID
    residual of its pivots beside Rand-LUPP's."""
    X = R.rpid_sketch(ctx, A, Om)

    def timed(fn, reps=5):
        out = fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(reps):
            out = fn()
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1) / reps

    (J, Rf, diag, _, _), ms_qr = timed(lambda: R.rpid_select_columns_cpqr(ctx, X, K, sync=False))
    Z, ms_z = timed(lambda: R.rpid_id_coeffs_cpqr(ctx, K, J, Rf))
    rid = R.rpid_residual(ctx, R.RESIDUAL_ID, A, K, J, Z=Z)
    # Rand-LUPP's pivots with the least-squares Z over all l rows (the same Z
    # formula as CPQR's), for a like-for-like comparison of the pivots
    Jl, _, _, _, _, _ = R.rpid_select_columns(ctx, X, K)
    Zls, ms_ls = timed(lambda: R.rpid_id_coeffs_ls(ctx, X, K, Jl))
    rid_ls = R.rpid_residual(ctx, R.RESIDUAL_ID, A, K, Jl, Z=Zls)
    out = {"cpqr_ms": ms_qr, "cpqr_us_per_pivot": ms_qr * 1e3 / K, "id_coeffs_cpqr_ms": ms_z,
           "residual_id_cpqr": rid, "residual_id_lupp_least_squares_z": rid_ls, "id_coeffs_ls_ms": ms_ls}
    if plain is not None:
        out.update({"lupp_select_columns_ms": plain["per_call_ms"]["select_columns"],
                    "lupp_id_coeffs_ms": plain["per_call_ms"]["id_coeffs"], "residual_id_lupp": plain["rid"]})
    return out


def sparse_report(torch, R, ctx, A, Om):
    """Sparse and structured sketches (Sec. 2.2): the sparse sign embedding
    (zeta = 8, scale 1/sqrt(8)) and the SRTT on the main dense input, and the CSC sketch of
    an SNN matrix (eq. snn-def) 65536 x 65536, r = 400, s_i = 2/i (i <= 100)
    then 1/i, x_i and y_i with 0.1 % nonzeros (FP32 values, l = 272, Gaussian
    and sparse sign embeddings), followed by Rand-LUPP's column selection."""
    import numpy as np

    from paper_2104_05877_amd import inputs

    def timed(fn, reps=5):
        out = fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(reps):
            out = fn()
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1) / reps

    rng = np.random.default_rng(99)
    m = A.shape[0]
    rows, signs = inputs.sparse_sign_draws(rng, m, L, 8)
    rows_d, signs_d = torch.from_numpy(rows).cuda(), torch.from_numpy(signs).cuda()
    _, ms_ss_dense = timed(lambda: R.rpid_sketch_sparse_sign(ctx, A, rows_d, signs_d, L, 8 ** -0.5))
    _, ms_gauss_dense = timed(lambda: R.rpid_sketch(ctx, A, Om))
    perm, phi, sel = inputs.srtt_draws(rng, m, L)
    pd, fd, sd = torch.from_numpy(perm).cuda(), torch.from_numpy(phi).cuda(), torch.from_numpy(sel).cuda()
    _, ms_srtt_dense = timed(lambda: R.rpid_sketch_srtt(ctx, A, pd, fd, sd))
    rep = {"sparse_sign_dense_ms": ms_ss_dense, "gaussian_dense_ms": ms_gauss_dense, "srtt_dense_ms": ms_srtt_dense}
    rep.update(csc_report(torch, R, ctx, rng))
    return rep


def csc_report(torch, R, ctx, rng, with_selection=True):
    """CSC sketches of the SNN matrix 65536 x 65536 (r = 400, s_i = 2/i for
    i <= 100 then 1/i, 0.1 % nonzeros, FP32 values, l = 272) with a Gaussian
    and with a sparse sign embedding (zeta = 8, applied as a sparse operator),
    then Rand-LUPP's column selection on the Gaussian sketch."""
    import numpy as np

    from paper_2104_05877_amd import inputs

    def timed(fn, reps=20):
        out = fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(reps):
            out = fn()
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1) / reps

    ms_ = 65536
    i = np.arange(1, 401, dtype=np.float64)
    sv = np.where(i <= 100, 2.0 / i, 1.0 / i)
    cp, ri, va = inputs.snn_csc(np.random.default_rng(98), ms_, ms_, sv, 0.001)
    Ac = R.CSC(torch.from_numpy(cp).cuda(), torch.from_numpy(ri).cuda(), torch.from_numpy(va).float().cuda(), ms_, ms_)
    G = inputs.torch_gaussian(L, ms_, 97, "cuda", dtype=torch.float32).T.contiguous().T
    X, ms_csc = timed(lambda: R.rpid_sketch_csc(ctx, Ac, G))
    r2, s2 = inputs.sparse_sign_draws(rng, ms_, L, 8)
    r2d, s2d = torch.from_numpy(r2).cuda(), torch.from_numpy(s2).cuda()
    _, ms_csc_ss = timed(lambda: R.rpid_sketch_csc_sparse_sign(ctx, Ac, r2d, s2d, L, 8 ** -0.5))
    rep = {"snn65536_nnz": int(len(va)), "csc_gaussian_sketch_ms": ms_csc, "csc_sparse_sign_sketch_ms": ms_csc_ss,
           "csc_gaussian_gflops": 2.0 * len(va) * L / (ms_csc * 1e-3) / 1e9}
    if with_selection:
        (J, _, _, _, _, _), ms_sel = timed(lambda: R.rpid_select_columns(ctx, X, K, sync=False), reps=3)
        rep["csc_select_columns_ms"] = ms_sel
    return rep


def calibration_copy(torch, reps=5):
    """Elementwise kernels that read CALIB_MIB MiB and write CALIB_MIB MiB
    (a negating copy: a plain same-dtype copy would go to the DMA engines),
    outside any timed region.  Returns the best rate over `reps` launches in
    bytes per second (read + write), the measured HBM ceiling (2 x 512 MiB
    does not fit the 256 MB last-level cache)."""
    n = CALIB_MIB * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        torch.neg(src, out=dst)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    return 2.0 * CALIB_MIB * (1 << 20) / (best * 1e-3)


def cold_sketch(torch, R, ctx, A, Om, reps=10):
    """The sketch call alone with the last-level cache flushed before each
    call (a 512 MiB buffer written and synchronised outside the events):
    (p10, p50, p90) ms."""
    import numpy as np

    flush = torch.empty(CALIB_MIB * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    out = []
    for i in range(reps + 1):
        flush.fill_(float(i))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        R.rpid_sketch(ctx, A, Om)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        if i > 0:
            out.append(e0.elapsed_time(e1))
    del flush
    return [float(np.percentile(out, q)) for q in (10, 50, 90)]


def cold_steps(torch, R, ctx, A, Om, steps):
    """The sequential step with the last-level cache flushed before each
    step: a 512 MiB buffer is written between steps, outside the events
    that bracket the step.  Per-step times (ms)."""
    import numpy as np

    refine = 0 if A.dtype == torch.float64 else 1
    flush = torch.empty(CALIB_MIB * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    out = []
    for i in range(steps + 1):
        flush.fill_(float(i))
        torch.cuda.synchronize()  # the flush is done before the step starts
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        X = R.rpid_sketch(ctx, A, Om)
        J, Lf, Uf, _, _, _ = R.rpid_select_columns(ctx, X, K, sync=False)
        Z, _ = R.rpid_id_coeffs(ctx, X, K, J, Lf, Uf, refine_steps=refine)
        I, U, _, _ = R.rpid_cur(ctx, A, K, J)
        R.rpid_residual(ctx, R.RESIDUAL_ID, A, K, J, Z=Z)
        R.rpid_residual(ctx, R.RESIDUAL_CUR, A, K, J, I=I, U=U)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        if i > 0:
            out.append(e0.elapsed_time(e1))
    del flush
    return [float(np.percentile(out, q)) for q in (10, 50, 90)]


def _counter_rows(folder):
    import csv
    import glob

    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {folder}")
    per = {}
    for fn in files:
        with open(fn, newline="") as f:
            for r in csv.DictReader(f):
                key = (fn, r["Dispatch_Id"])
                e = per.setdefault(key, {"kernel": r["Kernel_Name"], "value": 0.0})
                e["value"] += float(r["Counter_Value"])
    return list(per.values())


def summarize_counters(fetch_dir, write_dir, mode):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the LUPP launches of a
    --only-main run in `mode`, scaled by what the same counters read for the
    calibration copy (CALIB_MIB MiB read, CALIB_MIB MiB written); recorded
    per mode."""
    out = {}
    for name, folder in (("fetch", fetch_dir), ("write", write_dir)):
        rows = _counter_rows(folder)
        calib = [r["value"] for r in rows if "neg" in r["kernel"].lower()]
        lupp = [r["value"] for r in rows if "lupp_panel_kernel" in r["kernel"]]
        if not calib or not lupp:
            raise SystemExit(f"{name}: calibration copy or LUPP dispatches missing")
        kib_expected = CALIB_MIB * 1024.0
        factor = kib_expected / max(calib)
        out[name] = {"calib_kib": max(calib), "factor": factor,
                     "lupp_kib_mean": sum(lupp) / len(lupp), "lupp_launches": len(lupp),
                     "lupp_bytes_per_launch": sum(lupp) / len(lupp) * 1024.0 * factor}
    with open(LUPP_SOURCE, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    elem = "double" if mode == "f64" else "float"
    rec = {"kernel": f"lupp_panel_kernel<{elem}> on 8192 x 256 panels ({mode} mode)", "mode": mode,
           "source_sha256": sha, "counters": out,
           "hbm_bytes_per_launch": out["fetch"]["lupp_bytes_per_launch"]
           + out["write"]["lupp_bytes_per_launch"]}
    try:
        with open(TRAFFIC_FILE) as f:
            allrec = json.load(f)
    except (OSError, ValueError):
        allrec = {}
    allrec[mode] = rec
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(allrec, f, indent=1)
    print(json.dumps(rec, indent=1))


def recorded_traffic(mode):
    """Counter-measured HBM bytes per LUPP launch in `mode`, if recorded for
    this source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f).get(mode)
        with open(LUPP_SOURCE, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError, AttributeError):
        return None
    if not rec or rec.get("source_sha256") != sha:
        return None
    return rec


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(torch, A, Om, threads_one=True):
    """The FP64 oracle, untuned, on the host: one decomposition (sketch, LUPP,
    Z, CUR) plus its ID and CUR residuals on the same stored values, with
    every BLAS thread and again with one thread.  GFLOP/s count the dominant
    terms 2mn(l + 3k): the sketch, W = Q_C^T A and the two residual
    products."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    import oracle.rpid_oracle as O

    a = np.asfortranarray(A.double().cpu().numpy())
    om = np.asfortranarray(Om.double().cpu().numpy())

    def one():
        t0 = time.perf_counter()
        d = O.decompose(a, om, K, gaps=True)
        r = O.residuals(a, d["J"], Z=d["Z"], I=d["I"], U=d["U"], only=("id", "cur"))
        return time.perf_counter() - t0, d, r

    t, d, r = one()
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    t1 = None
    if threads_one:
        with threadpool_limits(1):
            t1, _, _ = one()
    flops = 2.0 * M * N * (L + 3 * K)
    return dict(seconds=t, seconds_1thread=t1, threads=threads, gflops=flops / t / 1e9,
                gflops_1thread=(flops / t1 / 1e9) if t1 else None, rid=r["id"], rcur=r["cur"],
                oracle=d, nproc=os.cpu_count(), cpu_model=_cpu_model())


def _rel(a, b):
    import numpy as np

    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def parity_report(res, o, name):
    """A mode's last step against the FP64 oracle on the same stored values:
    pivot prefix, overlap, equality; errors of X, Z, U; residual ratios; and
    the column LUPP on the kernel's own X against the fixed-arithmetic
    oracle in the kernel's precision (bit for bit: pivots, L', U')."""
    import numpy as np

    import oracle.rpid_oracle as O

    J, I = res["J"].astype(np.int64), res["I"].astype(np.int64)
    same_j = J == o["J"]
    pj = int(np.argmin(same_j)) if not same_j.all() else K
    same_i = I == o["I"] if len(o.get("I", [])) == K else np.zeros(K, bool)
    pi = int(np.argmin(same_i)) if not same_i.all() else K
    dt = np.float64 if name == "f64" else np.float32
    f = O.lupp_colwise_fma(res["X"], K, dt)
    out = {"J_equal": bool(pj == K), "I_equal": bool(pi == K), "J_prefix": pj, "I_prefix": pi,
           "J_overlap": len(np.intersect1d(J, o["J"])) / K, "I_overlap": len(np.intersect1d(I, o["I"])) / K,
           "X_rel_err": _rel(res["X"], o["X"]),
           "lupp_bitexact_vs_fixed_arithmetic_oracle": bool(
               np.array_equal(J, f["J"]) and np.array_equal(res["Lf"], f["L"].astype(np.float64))
               and np.array_equal(res["Uf"], f["U"].astype(np.float64))),
           "ratio_id": res["rid"] / o["res"]["id"], "ratio_cur": res["rcur"] / o["res"]["cur"],
           "oracle_id": o["res"]["id"], "oracle_cur": o["res"]["cur"]}
    if pj == K:
        out["Z_rel_err"] = _rel(res["Z"], o["Z"])
        if pi == K:
            out["U_rel_err"] = _rel(res["U"], o["U"])
    return out


def configs_report(torch, R, ctx, reps=3):
    """The two precision forms at their own sizes, end to end (GPU time per
    call back to back; residuals of the last call):
    * 16384 x 16384 stored BF16 (rank-512 Gaussian factors + 1e-4 N(0,1)),
      k = 512, l = 544: BF16 sketch, FP32 LUPP, Z with one FP64 refinement
      step, CUR, both residuals;
    * 65536 x 4096 FP32, |F||G| (rank 384) + uniform[0, 1e-3], k = 384,
      l = 400: FP8 sketch, FP32 LUPP, Z (one refinement), CUR, CUR residual."""
    from paper_2104_05877_amd import inputs

    def timed(fn):
        out = fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        for _ in range(reps):
            out = fn()
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1) / reps

    rep = {}
    m = n = 16384
    k, l = 512, 544
    A = inputs.torch_lowrank_noise(m, n, k, 1e-4, 9, "cuda").T.contiguous().bfloat16().T
    Om = inputs.torch_gaussian(l, m, 10, "cuda").T.contiguous().bfloat16().T

    def c2():
        X = R.rpid_sketch(ctx, A, Om)
        J, Lf, Uf, _, _, _ = R.rpid_select_columns(ctx, X, k, sync=False)
        Z, _ = R.rpid_id_coeffs(ctx, X, k, J, Lf, Uf, refine_steps=1)
        I, U, _, st = R.rpid_cur(ctx, A, k, J)
        return J, Z, I, U, st

    (J, Z, I, U, st), ms = timed(c2)
    rep["bf16_16384x16384_k512_l544"] = {
        "ms_per_decomposition": ms, "status_rows": st,
        "residual_id": R.rpid_residual(ctx, R.RESIDUAL_ID, A, k, J, Z=Z),
        "residual_cur": R.rpid_residual(ctx, R.RESIDUAL_CUR, A, k, J, I=I, U=U)}
    del A, Om, J, Z, I, U
    torch.cuda.empty_cache()
    m, n, k, l = 65536, 4096, 384, 400
    A = inputs.torch_nonneg_lowrank(m, n, k, 1e-3, 5, "cuda")
    Om = inputs.torch_gaussian(l, m, 6, "cuda", dtype=torch.float32)

    def c3():
        X = R.rpid_sketch_fp8(ctx, A, Om)
        J, Lf, Uf, _, _, _ = R.rpid_select_columns(ctx, X, k, sync=False)
        Z, _ = R.rpid_id_coeffs(ctx, X, k, J, Lf, Uf, refine_steps=1)
        I, U, _, st = R.rpid_cur(ctx, A, k, J)
        return J, Z, I, U, st

    (J, Z, I, U, st), ms = timed(c3)
    rep["fp8_65536x4096_k384_l400"] = {
        "ms_per_decomposition": ms, "status_rows": st,
        "residual_id": R.rpid_residual(ctx, R.RESIDUAL_ID, A, k, J, Z=Z),
        "residual_cur": R.rpid_residual(ctx, R.RESIDUAL_CUR, A, k, J, I=I, U=U)}
    del A, Om
    torch.cuda.empty_cache()
    return rep


# learned-rank report on the learned form's own workload: a seeded stream of
# matrices with m, n uniform in [2048, 8192] and exponential (rate log-uniform
# in [1e-3, 1e-1]) or polynomial (power uniform in [0.5, 3]) spectra, BF16
# sketches of l = 512 rows, tolerance 1e-4 on the relative ID residual.  The
# first 80 % of the stream (by index) trains the network (its last
# LEARN_CALIB matrices calibrate the output shift), the last 20 % is held out.
LEARN_TOL, LEARN_L, LEARN_N, LEARN_CALIB, LEARN_K0 = 1e-4, 512, 400, 64, 8


def learned_report(torch, ctx):
    """Labels k* (smallest rank whose FP64 ID meets the tolerance, up to the
    library's rank cap, by bisection on one FP64 sketch) for every matrix;
    the network trained on the training part; then, on each held-out matrix,
    the tolerance reached three ways, each answer checked by the FP64
    residual: BF16 profile + network + plain path from k_hat (doubling on a
    miss, past l up to the cap), the plain FP64 path with rank doubling from
    LEARN_K0, and the pivot-ratio threshold rule on the same profile.  Times
    are wall-clock per matrix, the BF16 copies of A and Omega included in
    the two profile-based paths."""
    import numpy as np

    from paper_2104_05877_amd import inputs, learned as Lr

    cap = Lr.RANK_CAP
    n_test = LEARN_N // 5
    n_train = LEARN_N - n_test
    n_fit = n_train - LEARN_CALIB

    def case(idx):
        A64, Om64, _, _, fam = inputs.torch_stream_case(idx, cap, "cuda", 0, with_lo=False)
        return A64, Om64, fam

    def lo_copies(A64, Om64):
        return A64.T.contiguous().bfloat16().T, Om64[:LEARN_L].T.contiguous().bfloat16().T

    t0 = time.perf_counter()
    feats, labels = [], []
    for idx in range(n_train):
        A64, Om64, _ = case(idx)
        k, _ = Lr.rank_label(ctx, A64, Om64, LEARN_TOL, cap)
        A16, Om16 = lo_copies(A64, Om64)
        feats.append(Lr.profile_features(ctx, A16, Om16, LEARN_L))
        labels.append(k)
        del A64, Om64, A16, Om16
        if (idx + 1) % 40 == 0:
            log(f"learned: labelled {idx + 1} of {n_train} training matrices ({time.perf_counter() - t0:.0f} s)")
    t_labels = time.perf_counter() - t0
    F = torch.stack(feats)
    T = torch.tensor([Lr.target_of(k, cap) for k in labels], dtype=torch.float32, device="cuda")
    net = Lr.RankNet(ctx, seed=1)
    t0 = time.perf_counter()
    hist = net.fit(F[:n_fit].contiguous(), T[:n_fit].contiguous(), epochs=300, batch=32, lr=2e-3, tau=0.5,
                   seed=2)
    y_cal = net.predict(F[n_fit:].contiguous()).cpu().tolist()
    shift = Lr.calibrate_shift(y_cal, labels[n_fit:], cap)
    t_train = time.perf_counter() - t0
    log(f"learned: {n_train} training matrices labelled in {t_labels:.1f} s, shift {shift:+.2f}")

    r = {key: [] for key in ("t_l", "t_d", "t_t", "a_l", "a_d", "a_t", "khat_ratio", "kl_ratio", "kd_ratio",
                             "kt_ratio", "ks")}
    met, same_outcome = 0, 0
    for idx in range(n_train, LEARN_N):
        A64, Om64, fam = case(idx)
        ks, _ = Lr.rank_label(ctx, A64, Om64, LEARN_TOL, cap)
        kd, ad, sd = Lr.solve_doubling(ctx, A64, Om64, LEARN_TOL, LEARN_K0, cap)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        A16, Om16 = lo_copies(A64, Om64)
        torch.cuda.synchronize()
        t_copy = time.perf_counter() - tc
        kl, al, sl, khat = Lr.solve_learned(ctx, net, A64, Om64, A16, Om16, LEARN_TOL, LEARN_L, cap, shift)
        kt, at, st, _ = Lr.solve_threshold(ctx, A64, Om64, A16, Om16, LEARN_TOL, LEARN_L, cap)
        r["t_l"].append(sl + t_copy)
        r["t_d"].append(sd)
        r["t_t"].append(st + t_copy)
        r["a_l"].append(al)
        r["a_d"].append(ad)
        r["a_t"].append(at)
        r["ks"].append(ks)
        same_outcome += int((kl is None) == (kd is None) == (kt is None))
        if ks is not None:
            met += int(khat >= ks)
            r["khat_ratio"].append(khat / ks)
            for key, kk in (("kl_ratio", kl), ("kd_ratio", kd), ("kt_ratio", kt)):
                if kk is not None:
                    r[key].append(kk / ks)
        else:
            met += int(khat >= cap)
        del A64, Om64, A16, Om16
        if (idx + 1 - n_train) % 20 == 0:
            log(f"learned: {idx + 1 - n_train} of {n_test} held-out matrices solved")
    all_labels = labels + r["ks"]

    def med(v):
        return float(np.median(v)) if v else None

    return {
        "workload": "stream of %d matrices (%d train incl. %d calibration, %d held out), m, n uniform in "
                    "[2048, 8192], exp rate log-uniform in [1e-3, 1e-1] or poly power uniform in [0.5, 3], "
                    "BF16 sketch l = %d, tol %g, ranks up to %d" % (LEARN_N, n_train, LEARN_CALIB, n_test, LEARN_L,
                                                                    LEARN_TOL, cap),
        "censored_beyond_l": float(np.mean([k is None or k > LEARN_L for k in all_labels])),
        "censored_beyond_cap": float(np.mean([k is None for k in all_labels])),
        "label_seconds_train": t_labels, "train_seconds": t_train,
        "train_loss_first_last": [hist[0], hist[-1]], "calibrated_shift_log2": shift,
        "ms_per_matrix_learned": 1e3 * float(np.mean(r["t_l"])),
        "ms_per_matrix_fp64_doubling": 1e3 * float(np.mean(r["t_d"])),
        "ms_per_matrix_threshold_rule": 1e3 * float(np.mean(r["t_t"])),
        "speedup_learned_vs_fp64_doubling": float(np.sum(r["t_d"]) / np.sum(r["t_l"])),
        "speedup_threshold_vs_fp64_doubling": float(np.sum(r["t_d"]) / np.sum(r["t_t"])),
        "fp64_attempts_learned": float(np.mean(r["a_l"])),
        "fp64_attempts_doubling": float(np.mean(r["a_d"])),
        "fp64_attempts_threshold": float(np.mean(r["a_t"])),
        "met_without_fallback": met / n_test,
        "same_outcome_all_three": same_outcome / n_test,
        "khat_over_kstar_median": med(r["khat_ratio"]),
        "kfinal_over_kstar_median": {"learned": med(r["kl_ratio"]), "doubling": med(r["kd_ratio"]),
                                     "threshold": med(r["kt_ratio"])},
    }


def main():
    args = parse()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, args.mode)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the path runs on one GPU (how it would shard is described, not run); --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2104_05877_amd import rpid as R

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.sketch_shapes_only:
        ctx = R.Context(0)
        rep = sketch_shapes_report(torch, R, ctx)
        ctx.close()
        print(json.dumps({"sketch_shapes": rep}), flush=True)
        return
    if args.sparse_only:
        import numpy as np

        ctx = R.Context(0)
        rep = csc_report(torch, R, ctx, np.random.default_rng(99), with_selection=False)
        ctx.close()
        print(json.dumps({"sparse": rep}), flush=True)
        return
    if args.learned_only:
        ctx = R.Context(0)
        rep = learned_report(torch, ctx)
        ctx.close()
        print(json.dumps({"learned_rank": rep}), flush=True)
        return
    log("generating poly8192 inputs on the GPU")
    data = make_inputs(torch, args.seed, args.input_cache)
    hbm_measured = calibration_copy(torch)
    log(f"calibration copy: {hbm_measured / 1e9:.0f} GB/s (read + write)")
    ctx = R.Context(0)
    if args.two_sided_only:
        A, Om = data[args.reports_mode]
        rep = two_sided_report(torch, R, ctx, A, Om, None)
        rep_qr = cpqr_report(torch, R, ctx, A, Om, None)
        rep_sp = sparse_report(torch, R, ctx, A, Om)
        ctx.close()
        print(json.dumps({"mode": args.reports_mode, "two_sided": rep, "cpqr": rep_qr, "sparse": rep_sp}),
              flush=True)
        return
    results = {}
    order = [args.mode] + [m for m in ("f64", "f32", "bf16") if m != args.mode]
    if args.only_main:
        order = [args.mode]
    for mode in order:
        A, Om = data[mode]
        steps = args.steps if mode == args.mode else args.other_steps
        warm = args.warmup if mode == args.mode else 1
        log(f"mode {mode}: warmup {warm}, steps {steps}")
        results[mode] = run_mode(torch, R, ctx, A, Om, steps, warm)
        log(f"mode {mode}: {results[mode]['ms_per_step']:.3f} ms/step  per-call {results[mode]['per_call_ms']}")

    main_r = results[args.mode]
    per = main_r["per_call_ms"]
    ctx2 = R.Context(0, stream=torch.cuda.Stream(device=0))
    ov = {}
    for mode in order:
        ov[mode] = overlapped_steps(torch, R, ctx, ctx2, *data[mode],
                                    args.steps if mode == args.mode else args.other_steps,
                                    args.warmup if mode == args.mode else 1)
    ctx2.close()
    ov_ms, ov_out = ov[args.mode]
    ov_same = bool(np.array_equal(ov_out["J"].cpu().numpy(), main_r["J"])
                   and np.array_equal(ov_out["I"].cpu().numpy(), main_r["I"])
                   and ov_out["residual_id"] == main_r["rid"] and ov_out["residual_cur"] == main_r["rcur"])
    log(f"overlapped step: {ov_ms:.3f} ms (sequential {main_r['ms_per_step']:.3f}), same outputs {ov_same}")
    step_ms = main_r["ms_per_step"] if args.no_overlap else ov_ms
    cold = cold_steps(torch, R, ctx, *data[args.mode], args.cold_steps) if args.cold_steps > 0 else None
    sk_loop_ms = sketch_loop(torch, R, ctx, *data[args.mode])
    sk_cold = {m: cold_sketch(torch, R, ctx, *data[m]) for m in order}

    # The call with the largest time per step and its one dominant kernel:
    # the sketch GEMM, the LUPP panel kernel (select_columns), or the
    # residual product (residual_id / residual_cur).
    es = 8 if args.mode == "f64" else 4
    a_es = {"f64": 8, "f32": 4, "bf16": 2}[args.mode]
    peak_mfma = PEAK_MFMA[args.mode]
    cands = {
        "select_columns": dict(kernel="lupp_panel_kernel (column LUPP of X^T, 8192 x 256)", bound="hbm",
                               work=N * K * es + N * K * es + K * K * es,
                               note="algorithmic bytes: panel read, L' and U' written"),
        "sketch": dict(kernel="sketch GEMM (X = Omega A, 272 x 8192 x 8192)",
                       bound="hbm" if args.mode == "bf16" else "mfma",
                       work=(M * N * a_es + L * M * a_es + L * N * es) if args.mode == "bf16" else 2.0 * L * M * N,
                       note="bf16: bytes of A, Omega and X; else 2lmn flops"),
        "residual_id": dict(kernel="residual product ||A - C Z||_F (8192 x 8192, inner 256)",
                            bound="hbm" if args.mode == "bf16" else "mfma",
                            work=(M * N * a_es) if args.mode == "bf16" else 2.0 * M * N * K,
                            note="bf16: bytes of A; else 2mnk flops"),
        "residual_cur": dict(kernel="residual product ||A - (C U) R||_F (8192 x 8192, inner 256)",
                             bound="hbm" if args.mode == "bf16" else "mfma",
                             work=(M * N * a_es) if args.mode == "bf16" else 2.0 * M * N * K,
                             note="bf16: bytes of A; else 2mnk flops"),
    }
    dom = max(cands, key=lambda c: per[c])
    c = cands[dom]
    t_dom = per[dom] * 1e-3
    if c["bound"] == "hbm":
        ach = c["work"] / t_dom
        traffic = None
        if dom == "select_columns":
            rec = recorded_traffic(args.mode)
            if rec is not None:
                traffic = rec["hbm_bytes_per_launch"]
        roof = {"kernel": c["kernel"], "call": dom, "bound": "hbm", "achieved": ach / 1e9,
                "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": ach / PEAK_HBM,
                "frac_of_measured_hbm": ach / hbm_measured, "traffic": traffic,
                "algorithmic_per_launch": c["work"], "algorithmic": c["note"], "avg_ms": per[dom]}
    else:
        ach = c["work"] / t_dom
        roof = {"kernel": c["kernel"], "call": dom, "bound": "mfma", "achieved": ach / 1e12,
                "peak": peak_mfma / 1e12, "unit": "TFLOP/s", "frac": ach / peak_mfma, "traffic": None,
                "algorithmic_per_launch": c["work"], "algorithmic": c["note"], "avg_ms": per[dom]}
    roof["lupp_us_per_pivot"] = per["select_columns"] * 1e3 / K
    sketch_mfma = 2.0 * L * M * N / (sk_loop_ms * 1e-3) / peak_mfma

    line = {
        "metric": "ID+CUR decomps/sec & sketch-GEMM MFMA util at 8192^2, k=256; BF16 vs FP64",
        "value": 1e3 / step_ms,
        "unit": "decomps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.mode,
        "data": "synthetic",
        "config": {"workload": "poly8192", "m": M, "n": N, "k": K, "l": L,
                   "spectrum": "s_i = i^-2, Haar U and V, FP32 storage", "mode": args.mode,
                   "step": "sketch + LUPP(X^T) + Z + CUR(LUPP(C), U) + ID/CUR residuals",
                   "schedule": ("sequential" if args.no_overlap else
                                "Z and ID residual on a second stream, concurrent with CUR and its residual")},
        "step_ms_sequential": main_r["ms_per_step"],
        "step_ms_overlapped": ov_ms,
        "overlapped_outputs_equal_sequential": ov_same,
        "cold_step_ms_p10_p50_p90": cold,
        "hbm_measured_GBps": hbm_measured / 1e9,
        "sketch_mfma_util": sketch_mfma,
        "sketch_ms_back_to_back": sk_loop_ms,
        "sketch_ms_cold_p10_p50_p90": sk_cold,
        "sketch_mfma_util_cold": {m: 2.0 * L * M * N / (v[1] * 1e-3) / PEAK_MFMA[m] for m, v in sk_cold.items()},
        "modes": {m: {"decomps_per_s": 1e3 / ov[m][0], "ms_per_step_overlapped": ov[m][0],
                      "ms_per_step_sequential": r["ms_per_step"],
                      "step_ms_p10_p50_p90": r["step_ms_p10_p50_p90"],
                      "per_call_ms": r["per_call_ms"], "residual_id": r["rid"],
                      "residual_cur": r["rcur"]} for m, r in results.items()},
        "speedup_bf16_vs_f64": (ov["f64"][0] / ov["bf16"][0] if "f64" in ov and "bf16" in ov else None),
        "decomp_only": {m: {"decomps_per_s": 1e3 / r["decomp_ms_p10_p50_p90"][1],
                            "ms_p10_p50_p90": r["decomp_ms_p10_p50_p90"]} for m, r in results.items()},
        "roofline": roof,
    }
    rdata = data[args.reports_mode]
    rres = results.get(args.reports_mode, main_r)
    if not args.only_main:
        log(f"power-iteration report (Rand-LUPP-1piter), {args.reports_mode} input")
        line["power_iteration"] = power_report(torch, R, ctx, *rdata, rres)
        log("two-sided report (Alg. 3)")
        line["two_sided"] = two_sided_report(torch, R, ctx, *rdata, rres)
        log("Rand-CPQR report")
        line["cpqr"] = cpqr_report(torch, R, ctx, *rdata, rres)
        log("sparse-sketch report")
        line["sparse"] = sparse_report(torch, R, ctx, *rdata)
        log("sketch on the larger sketch workloads")
        line["sketch_shapes"] = sketch_shapes_report(torch, R, ctx)
        line["reports_mode"] = args.reports_mode
    if not args.no_configs and not args.only_main:
        log("precision forms at their own sizes")
        line["configs"] = configs_report(torch, R, ctx)
    if not args.no_learned and not args.only_main:
        log("learned-rank report")
        line["learned_rank"] = learned_report(torch, ctx)
    if not args.no_cpu_baseline:
        log("cpu baseline: FP64 oracle on one decomposition of the same workload")
        A, Om = data[args.mode]
        cb = cpu_baseline(torch, A, Om)
        line["cpu_baseline"] = {"value": 1.0 / cb["seconds"], "unit": "decomps/s",
                                "cores": cb["threads"], "kind": "oracle",
                                "sample": "1 decomposition + ID/CUR residuals of poly8192 "
                                          f"({args.mode} storage values promoted to FP64), "
                                          f"{cb['seconds']:.2f} s on {cb['threads']} BLAS threads",
                                "nproc": cb["nproc"], "cpu_model": cb["cpu_model"],
                                "gflops": cb["gflops"], "seconds_1thread": cb["seconds_1thread"],
                                "value_1thread": (1.0 / cb["seconds_1thread"]) if cb["seconds_1thread"] else None,
                                "gflops_1thread": cb["gflops_1thread"],
                                "flops_counted": "2mn(l + 3k): sketch, Q_C^T A, both residual products"}
        if not args.no_parity:
            log("parity of every mode against the FP64 oracle on the same stored values")
            o32 = cb["oracle"]
            o32["res"] = {"id": cb["rid"], "cur": cb["rcur"]}
            par = {}
            if args.mode in ("f64", "f32"):
                for mode in ("f64", "f32"):
                    if mode in results:
                        par[mode] = parity_report(results[mode], o32, mode)
            if "bf16" in results:
                import oracle.rpid_oracle as O

                ab = np.asfortranarray(data["bf16"][0].double().cpu().numpy())
                omb = np.asfortranarray(data["bf16"][1].double().cpu().numpy())
                ob = O.decompose(ab, omb, K)
                ob["res"] = O.residuals(ab, ob["J"], Z=ob["Z"], I=ob["I"], U=ob["U"], only=("id", "cur"))
                par["bf16"] = parity_report(results["bf16"], ob, "bf16")
            line["parity"] = par
            line["residual_ratio_vs_oracle"] = {
                "id": main_r["rid"] / cb["rid"], "cur": main_r["rcur"] / cb["rcur"],
                "oracle_id": cb["rid"], "oracle_cur": cb["rcur"],
                "J_equal": bool(np.array_equal(main_r["J"], cb["oracle"]["J"])),
                "I_equal": bool(np.array_equal(main_r["I"], cb["oracle"]["I"]))}
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
