"""Benchmark: one CCSD amplitude iteration on one MI355X.

A step is one pass of the whole iteration (eq. CC_general residual with the
particle ladder built from density-fitting tiles, ring, intermediates,
denominator step, DIIS, energy) for the nocc=40, nvir=360, naux=1200 system in
complex FP64, with the inputs resident in HBM before the timed region.

Prints one JSON line.  value = ladder algorithmic TFLOP per iteration (tile
build 2*naux*P_v^2 + contraction P_o*P_v^2 complex multiply-adds, 8 flops
each) divided by the wall time of a whole iteration.  roofline = the ladder
tile-build kernel (the dominant kernel), timed with HIP events on the
library's stream during the timed region.  cpu_baseline = the CPU oracle's
particle-ladder term on a bounded sample of rows of the same system.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA = 78.6  # TFLOP/s, MI355X dense FP64 matrix
PEAK_FP32_MFMA = 157.3  # TFLOP/s, MI355X dense FP32 matrix
PEAK_BF16_MFMA = 2516.6  # TFLOP/s, MI355X dense BF16 matrix
WORKLOAD = dict(nocc=40, nvir=360, naux=1200, seed=0)


# HBM bytes per ladder-build launch (mean over the 359 launches of one iteration),
# from one rocprofv3 pass each of FETCH_SIZE and WRITE_SIZE, scaled by what the
# counters read for a plain 1 GiB device copy (fetch x2.000, write x1.000), and
# the kernel's MFMA-busy fraction and clock from a third pass.
# They hold for the FP64 GETT source they were taken with: `gett_source_sha256`
# hashes gett.hip up to the BF16x3 section, and the figure is reported as null
# once that text differs.
TRAFFIC = {"gett_source_sha256": "8bb8d67aeb59ee0bfa310edb2ecfd55e3877387fe5ad0c7983b8f0d45a1aa591",
           "fetch_bytes": 8.1345e9, "write_bytes": 0.3770e9,
           "mfma_busy": 0.716, "clock_ghz": 2.31}
GETT_SRC = os.path.join(ROOT, "paper_2103_08473_amd", "csrc", "gett.hip")
BF16_MARK = "// BF16x3 complex GETT"


def gett_fp64_source_sha256():
    import hashlib
    with open(GETT_SRC, "rb") as f:
        text = f.read()
    cut = text.find(BF16_MARK.encode())
    return hashlib.sha256(text[:cut] if cut >= 0 else text).hexdigest()


def measured_traffic():
    """Counter-derived HBM bytes per launch, or None if the kernel changed since."""
    if gett_fp64_source_sha256() != TRAFFIC["gett_source_sha256"]:
        return None
    return TRAFFIC["fetch_bytes"] + TRAFFIC["write_bytes"]


def measured_mfma_busy():
    """MFMA-busy fraction of the tile-build kernel from SQ_VALU_MFMA_BUSY_CYCLES over
    GRBM_GUI_ACTIVE x 1024 SIMDs (a separate rocprofv3 pass), and the clock that
    GRBM_GUI_ACTIVE implies; None if the kernel changed since."""
    if gett_fp64_source_sha256() != TRAFFIC["gett_source_sha256"]:
        return None
    return {"mfma_busy": TRAFFIC["mfma_busy"], "clock_ghz": TRAFFIC["clock_ghz"]}


def ladder_build_flops(o, v, X):
    Pv = v * (v - 1) / 2
    return 8.0 * 2.0 * X * Pv * Pv


def ladder_build_bytes(o, v, X):
    """Mean algorithmic HBM bytes of one tile-build launch (FP64 complex): read the
    factor rows of a (v x X) and of all b > a ((v-a-1) v x X), write the v (v-a-1) v tile."""
    rows_b = (v - 1) / 2.0  # mean of v-a-1 over a = 0..v-2
    return 16.0 * (v * X + rows_b * v * X + v * rows_b * v)


def cpu_baseline(eps, B, o, budget_s=20.0):
    """Time the oracle's particle-ladder rows on the host, until ~budget_s of work."""
    import numpy as np
    from oracle.ccsd import ladder_rows
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    n = eps.size
    v = n - o
    X = B.shape[0]
    rng = np.random.default_rng(5)
    tau = rng.standard_normal((o, o, v, v)) + 1j * rng.standard_normal((o, o, v, v))
    Po, Pv = o * (o - 1) / 2, v * (v - 1) / 2
    t0 = time.perf_counter()
    rows = 0
    flops = 0.0
    while time.perf_counter() - t0 < budget_s and rows < v - 1:
        ladder_rows(B, o, tau, rows, rows + 1)
        flops += 8.0 * (v - rows - 1) * (2.0 * X * Pv + Po * Pv)
        rows += 1
    dt = time.perf_counter() - t0
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
            "sample": "oracle particle ladder (1/2 sum <ab||cd> tau_ij^cd, <ab||cd> built from B) "
                      "for virtual rows a=0..%d of the 40/360/1200 system, %.1f s; flops counted "
                      "as the GPU ladder's algorithmic work for those rows" % (rows - 1, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="first run one plain device-to-device copy of this many GiB (a known-size "
                         "kernel to scale hardware byte counters by)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2103_08473_amd import exacc
    from paper_2103_08473_amd.synth import make_system

    o, v, X = WORKLOAD["nocc"], WORKLOAD["nvir"], WORKLOAD["naux"]
    eps, B = make_system(o, v, X, seed=WORKLOAD["seed"])
    torch.cuda.set_device(0)
    if args.copy_calibration_gib > 0:
        nel = int(args.copy_calibration_gib * (1 << 30)) // 8
        src_t = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst_t = torch.empty_like(src_t)
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        del src_t, dst_t
    eps_d = torch.from_numpy(eps).cuda()
    B_d = torch.from_numpy(B).cuda()
    stream = torch.cuda.Stream()
    def progress(msg):
        print("bench: " + msg, file=sys.stderr, flush=True)

    progress("fp64 CCSD iterations")
    cc = exacc.CCSD(eps_d, B_d, o, stream=stream.cuda_stream, timing=1, tol=1e-9)
    for _ in range(args.warmup):
        cc.iterate(1)
    cc.stage_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for _ in range(args.steps):
        st, _, res, conv = cc.iterate(1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stages = cc.stage_times(reset=True)
    E = cc.energy()
    # Lambda equations (App. D) on the same handle, at these amplitudes: the first step
    # also builds the transformed-Hamiltonian pieces, so it is the warm-up
    lam = {}
    if not args.no_mixed:
        progress("lambda iterations")
        cc.lambda_iterate(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            cc.lambda_iterate(1)
        torch.cuda.synchronize()
        dtl = (time.perf_counter() - t0) / args.steps
        sl = cc.stage_times(reset=True)
        lam = {"lambda_fp64": {
            "s_per_iter": round(dtl, 4),
            "ccsd_iteration_time_ratio": round((dt / args.steps) / dtl, 3),
            "stage_ms_per_iter": {k: round(t / (args.steps + 1), 2) for k, t in sl.items()}}}
    cc.close()

    # CCD (the paper's CCDOUBLES) and CC2 variants: same system, FP64
    ccd = {}
    if not args.no_mixed:
        for name, kw in (("ccd_fp64", {"doubles_only": 1}), ("cc2_fp64", {"cc2": 1})):
            progress(name)
            cd = exacc.CCSD(eps_d, B_d, o, stream=stream.cuda_stream, timing=1, tol=1e-9, **kw)
            for _ in range(args.warmup):
                cd.iterate(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                cd.iterate(1)
            torch.cuda.synchronize()
            dtc = (time.perf_counter() - t0) / args.steps
            cd.close()
            ccd[name] = {"s_per_iter": round(dtc, 4),
                         "ccsd_iteration_time_ratio": round((dt / args.steps) / dtc, 3)}

    # DF-factor generation (the step before the iteration) for the same spinor count:
    # nao = 600 AO functions, nspinor = o + v = 400, naux = X.  Inputs made on the device
    # with torch (J = L K, V = L L^T, orthonormal C); not part of the timed product.
    dfleg = {}
    if not args.no_mixed:
        try:
            progress("df factors")
            g = torch.Generator(device="cuda").manual_seed(5)
            nao, nsp = 600, o + v
            K = torch.randn((X, nao, nao), dtype=torch.complex128, device="cuda", generator=g) * 0.05
            K = 0.5 * (K + K.transpose(1, 2).conj())
            Lm = torch.eye(X, dtype=torch.float64, device="cuda") + torch.tril(
                torch.randn((X, X), dtype=torch.float64, device="cuda", generator=g), -1) * (0.3 / X ** 0.5)
            J = (Lm.to(torch.complex128) @ K.reshape(X, -1)).reshape(X, nao, nao).contiguous()
            del K
            Vm = (Lm @ Lm.T).contiguous()
            Cq = torch.linalg.qr(torch.randn((nao, nao), dtype=torch.complex128, device="cuda",
                                             generator=g))[0][:, :nsp].contiguous()
            exacc.df_factors(Cq, J, Vm)                      # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Bdf, nsit = exacc.df_factors(Cq, J, Vm)
            torch.cuda.synchronize()
            dtd = time.perf_counter() - t0
            fl = 8.0 * (X * nsp * nao * nao + X * nsp * nsp * nao + X * X * nsp * nsp + nsit * 3.0 * X ** 3)
            dfleg = {"df_factors": {"nao": nao, "nspinor": nsp, "naux": X, "seconds": round(dtd, 4),
                                    "newton_schulz_steps": nsit, "tflops": round(fl / dtd / 1e12, 3),
                                    "flops_counted": "complex GEMM work, 8 flops per multiply-add"}}
            del J, Vm, Cq, Bdf, Lm
            torch.cuda.empty_cache()
        except Exception as ex:  # the headline line must still print
            dfleg = {"df_factors": {"error": str(ex)[:200]}}

    mixed = {}
    if not args.no_mixed:
        # same system, low-precision phases of the mixed schedules
        for name, prec in (("mixed_fp32", exacc.MIXED_FP32), ("mixed_bf16x3", exacc.MIXED_BF16X3)):
            progress(name)
            cm = exacc.CCSD(eps_d, B_d, o, stream=stream.cuda_stream, timing=1, tol=1e-9,
                            precision=prec)
            for _ in range(args.warmup):
                cm.iterate(1)
            cm.stage_times(reset=True)
            assert cm.phase()[0]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                cm.iterate(1)
            torch.cuda.synchronize()
            dtm = (time.perf_counter() - t0) / args.steps
            sm = cm.stage_times(reset=True)
            cm.close()
            bms = sm.get("ladder_build", float("nan")) / args.steps
            btf = ladder_build_flops(o, v, X) / (bms * 1e-3) / 1e12
            mixed[name] = {
                "phase": ("fp32" if prec == exacc.MIXED_FP32 else "bf16x3 ladder, fp32 other")
                         + " contractions, fp64 assembly/DIIS/energy",
                "s_per_iter": round(dtm, 4),
                "ladder_tflops_per_iter": round(exacc.ladder_flops(o, v, X) / dtm / 1e12, 3),
                "speedup_vs_fp64": round((dt / args.steps) / dtm, 3),
                "ladder_build_tflops": round(btf, 3),
                "stage_ms_per_iter": {k: round(t / args.steps, 2) for k, t in sm.items()}}
            if prec == exacc.MIXED_FP32:
                mixed[name]["ladder_build_frac_fp32_peak"] = round(btf / PEAK_FP32_MFMA, 4)
            else:  # 4 real products x 3 split terms = 12 bf16 MFMA products (24 flops) per
                # complex multiply-add, against 8 algorithmic flops
                mixed[name]["ladder_build_hw_frac_bf16_peak"] = round(btf * 24 / 8 / PEAK_BF16_MFMA, 4)
    del B_d

    s_per_iter = dt / args.steps
    lad = exacc.ladder_flops(o, v, X)
    value = lad / s_per_iter / 1e12
    build_ms = stages.get("ladder_build", float("nan")) / args.steps
    contract_ms = stages.get("ladder_contract", float("nan")) / args.steps
    achieved = ladder_build_flops(o, v, X) / (build_ms * 1e-3) / 1e12
    ladder_ms = build_ms + contract_ms + stages.get("ladder_antisym", 0.0) / args.steps
    out = {
        "metric": "ladder TFLOP/s + s/CCSD iter, FP64 vs mixed at |dE|<=1e-7 Eh; p99 solve latency",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * s_per_iter, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "CCSD iteration, complex FP64, nocc=40 nvir=360 naux=1200 seed 0 "
                               "(size-scaled sigma_B = 0.00663), DIIS(8)",
                   "nocc": o, "nvir": v, "naux": X, "precision": "fp64"},
        "s_per_iter": round(s_per_iter, 4),
        "ladder_tflops_kernels": round(lad / (ladder_ms * 1e-3) / 1e12, 3),
        "dense_equiv_tflops": round(8.0 * o * o * v ** 4 / s_per_iter / 1e12, 3),
        "residual_last": res,
        "energy": [E.real, E.imag],
        "stage_ms_per_iter": {k: round(t / args.steps, 2) for k, t in stages.items()},
        "roofline": {"bound": "mfma", "kernel": "ladder tile build (GETT kind 1)",
                     "achieved": round(achieved, 3), "peak": PEAK_FP64_MFMA, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP64_MFMA, 4), "traffic": measured_traffic(),
                     "traffic_unit": "bytes per launch (HBM, counter-derived)",
                     "algorithmic_bytes_per_launch": ladder_build_bytes(o, v, X),
                     "flops_counted": "8 real flops per complex multiply-add (algorithmic); the "
                                      "kernel's 3-multiplication complex product issues 6",
                     "hw_frac": round(0.75 * achieved / PEAK_FP64_MFMA, 4),
                     "counters": measured_mfma_busy()},
    }
    out.update(lam)
    out.update(dfleg)
    out.update(ccd)
    out.update(mixed)
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(eps, B, o)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
