"""Converged CCSD solves of one system in several precision modes, compared.

Runs the solves one after another (one handle resident at a time, so the
largest systems fit), each to ||Delta|| <= tol, and reports per mode the
iteration count (and how many ran FP32/BF16x3 contractions), the time to
solution, the mean seconds per low-precision and per FP64 iteration, and
against the first mode's solve: |dE| (complex, Hartree), max |dT1|, max |dT2|
and the speedup.

    python -m paper_2103_08473_amd.solve_report --nocc 40 --nvir 360 --naux 1200

Systems too large for two solves in one run are compared across runs: the
first run keeps the energy, all of t1 and a sample of t2 (`--save`), the
second compares against that file (`--ref`).  The t2 sample is 1M unique
(i<j, a<b) entries drawn with a fixed seed plus the 500k entries of largest
magnitude in the saved solve, so max |dT2| is taken over the sample.

    python -m paper_2103_08473_amd.solve_report --nocc 60 --nvir 540 --naux 1800 \\
        --modes mixed_bf16x3 --save bf16.npz
    python -m paper_2103_08473_amd.solve_report --nocc 60 --nvir 540 --naux 1800 \\
        --modes fp64 --ref bf16.npz
"""
from __future__ import annotations

import argparse
import json
import sys
import time

START = time.time()

import numpy as np  # noqa: E402

from . import exacc  # noqa: E402
from .synth import make_system  # noqa: E402

MODES = {"fp64": exacc.FP64, "mixed_fp32": exacc.MIXED_FP32, "mixed_bf16x3": exacc.MIXED_BF16X3}
SAMPLE_SEED, SAMPLE_RANDOM, SAMPLE_TOP = 2024, 1_000_000, 500_000


def triples_flops(o, v, X):
    """Algorithmic flops of exacc_ccsd_triples: the <ab||ie> tiles packed over a<b
    (2 o P_v v X complex multiply-adds) and, per occupied triple, the two packed parts of W,
    3 P_v v^2 (sum over e, a<b) + 3 o v P_v (sum over m, b<c), 8 flops each."""
    ntrip = o * (o - 1) * (o - 2) / 6
    Pv = v * (v - 1) / 2
    return 8.0 * (2.0 * o * Pv * v * X + ntrip * (3.0 * Pv * v * v + 3.0 * o * v * Pv))


def solve(eps_d, B_d, nocc, mode, tol, diis, max_iter, log, time_limit=None, triples=False,
          lam=False, **extra):
    import torch
    t0 = time.perf_counter()
    cc = exacc.CCSD(eps_d, B_d, nocc, precision=MODES[mode], tol=tol, diis_size=diis,
                    max_iter=max_iter, timing=0, **extra)
    t_create = time.perf_counter() - t0
    hist = []
    conv = False
    t1 = time.perf_counter()
    for it in range(1, max_iter + 1):
        ph = ("fp64", "low", "dc")[cc.phase()[0]]
        ti = time.perf_counter()
        st, _, r, conv = cc.iterate(1)
        E = cc.energy()
        hist.append((it, ph, E.real, E.imag, r, time.perf_counter() - ti))
        log("  %-13s it %3d %-4s E %.12f %+.3e i  |D| %.3e  t %.1fs" % (
            mode, it, ph, E.real, E.imag, r, time.perf_counter() - t1))
        if conv or st == exacc.ERR_DIVERGED:
            break
        if time_limit is not None and time.time() - START > time_limit:
            log("  stopping: time limit")
            break
    torch.cuda.synchronize()
    t_iter = time.perf_counter() - t1
    tri = None
    if triples:
        t0 = time.perf_counter()
        e4, et, em = cc.triples()
        dtt = time.perf_counter() - t0
        o, v, X = nocc, eps_d.numel() - nocc, B_d.shape[0]
        tri = {"E(+T)": e4, "E((T))": et, "E(-T)": em, "seconds": round(dtt, 3),
               "tflops": round(triples_flops(o, v, X) / dtt / 1e12, 3)}
        log("  triples %s" % json.dumps(tri))
    lres = None
    if lam:
        t0 = time.perf_counter()
        lhist = []
        lconv = False
        for _ in range(max_iter):
            ti = time.perf_counter()
            st, _, r, lconv = cc.lambda_iterate(1)
            lhist.append((r, time.perf_counter() - ti))
            log("  lambda it %3d |D| %.3e  t %.1fs" % (len(lhist), r, time.perf_counter() - t0))
            if lconv or st == exacc.ERR_DIVERGED:
                break
        dtl = time.perf_counter() - t0
        g = cc.density()
        n = g.shape[0]
        herm = 0.5 * (g + g.conj().T)
        lres = {"converged": lconv, "iterations": len(lhist), "seconds": round(dtl, 3),
                "first_iteration_s": round(lhist[0][1], 3) if lhist else None,
                "s_per_iter_after_first": round(float(np.mean([x[1] for x in lhist[1:]])), 4)
                if len(lhist) > 1 else None,
                "residual": lhist[-1][0] if lhist else None,
                "density_trace": [float(np.trace(g).real), float(np.trace(g).imag)],
                "density_hermitian_part_max_offdiag": float(np.abs(herm - np.diag(np.diag(herm))).max())
                if n > 1 else 0.0}
        log("  lambda %s" % json.dumps(lres))
    t1a, t2a = cc.amplitudes()
    cc.close()
    low_t = [h[5] for h in hist if h[1] == "low"]
    hi_t = [h[5] for h in hist if h[1] == "fp64"]
    dc_t = [h[5] for h in hist if h[1] == "dc"]
    return {"energy": [E.real, E.imag], "converged": conv, "iterations": len(hist),
            "low_precision_iterations": len(low_t), "defect_corrected_iterations": len(dc_t),
            "s_per_dc_iter": round(float(np.mean(dc_t)), 4) if dc_t else None,
            "create_s": round(t_create, 3),
            "iterate_s": round(t_iter, 3), "s_per_iter": round(t_iter / max(1, len(hist)), 4),
            "s_per_low_iter": round(float(np.mean(low_t)), 4) if low_t else None,
            "s_per_fp64_iter": round(float(np.mean(hi_t)), 4) if hi_t else None,
            "residual": hist[-1][4] if hist else None,
            "triples": tri, "lambda": lres, "history": hist}, t1a, t2a


def random_unique_t2(o, v, n, seed=SAMPLE_SEED):
    """Flat indices into t2[o][o][v][v] of about n distinct entries with i<j and a<b."""
    rng = np.random.default_rng(seed)
    i, j = rng.integers(0, o, 4 * n), rng.integers(0, o, 4 * n)
    a, b = rng.integers(0, v, 4 * n), rng.integers(0, v, 4 * n)
    keep = (i < j) & (a < b)
    return np.unique(((i[keep] * o + j[keep]) * v + a[keep]) * v + b[keep])[:n]


def save_solution(path, res, t1, t2, o, v):
    flat = t2.reshape(-1)
    ridx = random_unique_t2(o, v, SAMPLE_RANDOM)
    top = min(SAMPLE_TOP, flat.size)
    tidx = np.argpartition(np.abs(flat), -top)[-top:]
    np.savez(path, energy=np.array(res["energy"]), t1=t1, rand_idx=ridx, rand_val=flat[ridx],
             top_idx=tidx, top_val=flat[tidx])


def compare_saved(path, res, t1, t2, o, v):
    ref = np.load(path)
    flat = t2.reshape(-1)
    ridx = random_unique_t2(o, v, SAMPLE_RANDOM)
    if not np.array_equal(ridx, ref["rand_idx"]):
        raise ValueError("sample indices differ from %s" % path)
    tidx = ref["top_idx"]
    E = complex(*res["energy"])
    return {"ref": path, "abs_dE": abs(E - complex(*ref["energy"])),
            "max_dT1": float(np.abs(t1 - ref["t1"]).max()),
            "max_dT2_sampled": float(max(np.abs(flat[ridx] - ref["rand_val"]).max(),
                                         np.abs(flat[tidx] - ref["top_val"]).max())),
            "sampled_t2_entries": int(ridx.size + tidx.size)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nocc", type=int, default=40)
    ap.add_argument("--nvir", type=int, default=360)
    ap.add_argument("--naux", type=int, default=1200)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--diis", type=int, default=8)
    ap.add_argument("--max-iter", type=int, default=60)
    ap.add_argument("--modes", default="fp64,mixed_fp32,mixed_bf16x3")
    ap.add_argument("--switch-tol", type=float, default=None,
                    help="mixed modes: ||Delta|| below which FP64 contractions start")
    ap.add_argument("--sigma", type=float, default=None,
                    help="width of the DF factor entries (default: the generator's size rule)")
    ap.add_argument("--save", default=None, help="keep E, t1 and a t2 sample of the first mode here")
    ap.add_argument("--ref", default=None, help="compare every mode with a solve kept by --save")
    ap.add_argument("--triples", action="store_true",
                    help="after each solve, E(+T), E((T)) and E(-T) (App. C) with their time")
    ap.add_argument("--triples-block", type=int, default=0,
                    help="occupied block size n_red of the triples loops (0: as large as fits)")
    ap.add_argument("--lambda", dest="lam", action="store_true",
                    help="after each solve, the Lambda equations (App. D) and the density (App. E)")
    ap.add_argument("--ladder-group-nvir", type=int, default=None,
                    help="opts.ladder_group_nvir (all ladder rows in one product up to this nvir)")
    ap.add_argument("--time-limit", type=float, default=None,
                    help="stop iterating once this many seconds have passed since start-up")
    args = ap.parse_args()
    import torch

    def log(s):
        print(s, flush=True)
        sys.stdout.flush()

    o, v, X = args.nocc, args.nvir, args.naux
    log("generating (%d, %d, %d) seed %d" % (o, v, X, args.seed))
    eps, B = make_system(o, v, X, seed=args.seed, sigma=args.sigma)
    eps_d = torch.from_numpy(eps).cuda()
    B_d = torch.from_numpy(B).cuda()
    del B
    out = {"system": {"nocc": o, "nvir": v, "naux": X, "seed": args.seed, "sigma": args.sigma,
                      "tol": args.tol, "diis": args.diis}, "modes": {}}
    ref = None
    for mode in args.modes.split(","):
        log("solve %s" % mode)
        extra = {} if args.switch_tol is None else {"mixed_switch_tol": args.switch_tol}
        if args.triples_block:
            extra["triples_occ_block"] = args.triples_block
        if args.ladder_group_nvir is not None:
            extra["ladder_group_nvir"] = args.ladder_group_nvir
        res, t1, t2 = solve(eps_d, B_d, o, mode, args.tol, args.diis, args.max_iter, log,
                            time_limit=args.time_limit, triples=args.triples, lam=args.lam, **extra)
        if args.ref:
            res.update(compare_saved(args.ref, res, t1, t2, o, v))
        if args.save and not out["modes"]:
            save_solution(args.save, res, t1, t2, o, v)
        if ref is None:
            ref = (res, t1, t2)
        else:
            r0, r1, r2 = ref
            res["abs_dE_vs_" + list(out["modes"])[0]] = abs(complex(*res["energy"]) - complex(*r0["energy"]))
            res["max_dT1"] = float(np.abs(t1 - r1).max())
            res["max_dT2"] = float(np.abs(t2 - r2).max())
            res["speedup_time_to_solution"] = round(r0["iterate_s"] / res["iterate_s"], 3)
        del t1, t2
        hist = res.pop("history")
        res["last_iterations"] = hist[-3:]
        out["modes"][mode] = res
        log(json.dumps({mode: res}))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
