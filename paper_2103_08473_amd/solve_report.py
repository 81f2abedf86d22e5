"""Converged CCSD solves of one system in several precision modes, compared.

Runs the solves one after another (one handle resident at a time, so the
largest systems fit), each to ||Delta|| <= tol, and reports per mode the
iteration count (and how many ran FP32/BF16x3 contractions), the time to
solution, and against the FP64 solve: |dE| (complex, Hartree), max |dT1|,
max |dT2| and the speedup.

    python -m paper_2103_08473_amd.solve_report --nocc 40 --nvir 360 --naux 1200
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import exacc
from .synth import make_system

MODES = {"fp64": exacc.FP64, "mixed_fp32": exacc.MIXED_FP32, "mixed_bf16x3": exacc.MIXED_BF16X3}


def solve(eps_d, B_d, nocc, mode, tol, diis, max_iter, log):
    import torch
    t0 = time.perf_counter()
    cc = exacc.CCSD(eps_d, B_d, nocc, precision=MODES[mode], tol=tol, diis_size=diis,
                    max_iter=max_iter, timing=0)
    t_create = time.perf_counter() - t0
    hist = []
    n_low = 0
    conv = False
    t1 = time.perf_counter()
    for it in range(1, max_iter + 1):
        low = cc.phase()[0]
        st, _, r, conv = cc.iterate(1)
        E = cc.energy()
        n_low += int(low)
        hist.append((it, "low" if low else "fp64", E.real, E.imag, r))
        log("  %-13s it %3d %-4s E %.12f %+.3e i  |D| %.3e  t %.1fs" % (
            mode, it, "low" if low else "fp64", E.real, E.imag, r, time.perf_counter() - t1))
        if conv or st == exacc.ERR_DIVERGED:
            break
    torch.cuda.synchronize()
    t_iter = time.perf_counter() - t1
    t1a, t2a = cc.amplitudes()
    cc.close()
    return {"energy": [E.real, E.imag], "converged": conv, "iterations": len(hist),
            "low_precision_iterations": n_low, "create_s": round(t_create, 3),
            "iterate_s": round(t_iter, 3), "s_per_iter": round(t_iter / max(1, len(hist)), 4),
            "history": hist}, t1a, t2a


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
    ap.add_argument("--sigma", type=float, default=None,
                    help="width of the DF factor entries (default: the generator's size rule)")
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
                      "tol": args.tol,
                      "diis": args.diis}, "modes": {}}
    ref = None
    for mode in args.modes.split(","):
        log("solve %s" % mode)
        res, t1, t2 = solve(eps_d, B_d, o, mode, args.tol, args.diis, args.max_iter, log)
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
